"""GPU parity of several-element SNAP (snap_set_elements +
snap_compute_elements) against the oracle's snap_elements, element by
element and pair by pair, with the tolerances of the one-element parity
tests; the one-element case against snap_compute bit for bit; a bad type
reported by snap_sync_status."""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

E_REL = 1e-11
F_ABS = 1e-10


def _setup(name):
    import torch
    from paper_2011_12875_amd import snapmi
    pos, box, types, rad, wt, f, beta, tj = wl.make_elements(name)
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    pot.set_elements(rad, wt, f)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    dev = dict(pos=torch.as_tensor(pos, device="cuda"),
               types=torch.as_tensor(types, dtype=torch.int32, device="cuda"),
               beta=torch.as_tensor(beta, device="cuda"))
    return pos, box, types, rad, wt, f, beta, tj, pot, nl, dev


@pytest.mark.parametrize("name", ["bcc128_2j4_3el", "bcc2000_2j8_2el"])
def test_elements_parity(name):
    print("case", name, flush=True)
    pos, box, types, rad, wt, f, beta, tj, pot, nl, dev = _setup(name)
    out = pot.compute_elements(dev["pos"], box, nl, dev["types"], dev["beta"], bispectrum=True,
                               pair_derivs=True)
    pot.sync_status()
    o = oracle.snap_elements(pos, box, tj, types, rad, wt, f, beta)
    E = out["energy"].cpu().numpy()
    scale = np.maximum(np.abs(o["E"]), np.abs(o["E"]).mean())
    assert (np.abs(E - o["E"]) / scale).max() <= E_REL
    assert np.abs(out["force"].cpu().numpy() - o["F"]).max() <= F_ABS
    B = out["bispectrum"].cpu().numpy()
    assert (np.abs(B - o["B"]) / np.maximum(np.abs(o["B"]), 1.0)).max() <= E_REL
    # pair derivatives by (i, k); the GPU list (to rcut) may hold pairs the
    # oracle's (to the largest pair cutoff) does not: those must be zero
    off, nbr = nl.off.cpu().numpy(), nl.nbr.cpu().numpy()[:nl.npairs]
    dE = out["dE"].cpu().numpy()
    ref = {}
    for i in range(len(pos)):
        for t in range(o["off"][i], o["off"][i + 1]):
            ref[(i, int(o["nbr"][t]))] = o["dE"][t]
    worst = 0.0
    for i in range(len(pos)):
        for t in range(off[i], off[i + 1]):
            r = ref.get((i, int(nbr[t])))
            worst = max(worst, np.abs(dE[t] - (r if r is not None else 0.0)).max())
    assert worst <= F_ABS
    # both elements' pair cutoffs are exercised: some listed pairs are beyond
    # their own cutoff (zero derivative) and some inside
    assert (np.abs(dE).sum(1) == 0.0).any() and (np.abs(dE).sum(1) > 0.0).any()
    # the virial from these pair derivatives (pairs beyond their cutoff add 0)
    W = pot.virial(dev["pos"], box, nl, out["dE"])
    Wref, _ = oracle.virial(pos, box, o["off"], o["nbr"], o["dE"])
    W = W.cpu().numpy().reshape(3, 3)
    assert np.abs(W - Wref).max() <= 1e-10 * np.abs(Wref).max()


def test_one_element_equals_snap_compute():
    """One element of radius rcut with rcutfac 1/2 and weight 1: the same bits
    as snap_compute."""
    import torch
    from paper_2011_12875_amd import snapmi
    pos, box, beta, tj = wl.make("bcc2000_2j8")
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    tpos = torch.as_tensor(pos, device="cuda")
    tb = torch.as_tensor(beta, device="cuda")
    a = pot.compute(tpos, box, nl, tb, bispectrum=True, pair_derivs=True)
    pot.set_elements([wl.RCUT], [1.0], 0.5)
    types = torch.zeros(len(pos), dtype=torch.int32, device="cuda")
    b = pot.compute_elements(tpos, box, nl, types, tb.reshape(1, -1).contiguous(),
                             bispectrum=True, pair_derivs=True)
    pot.sync_status()
    for k in ("energy", "force", "bispectrum", "dE"):
        assert torch.equal(a[k], b[k]), k


def test_bad_type_reported():
    import torch
    from paper_2011_12875_amd import snapmi
    pos, box, types, rad, wt, f, beta, tj, pot, nl, dev = _setup("bcc128_2j4_3el")
    bad = dev["types"].clone()
    bad[5] = 3
    pot.compute_elements(dev["pos"], box, nl, bad, dev["beta"])
    with pytest.raises(snapmi.SnapError):
        pot.sync_status()
    # the error is cleared; a good call is clean again
    pot.compute_elements(dev["pos"], box, nl, dev["types"], dev["beta"])
    pot.sync_status()
    torch.cuda.synchronize()


def test_elements_isolated_and_open_box():
    """Open box, two elements: a dimer inside its pair cutoff, a dimer of the
    same distance beyond it (smaller radii), and an isolated atom."""
    import torch
    from paper_2011_12875_amd import snapmi
    pos = np.array([[0.0, 0.0, 0.0], [2.9, 0.3, -0.2],        # A-A at ~2.92 < 2*1.6
                    [20.0, 0.0, 0.0], [22.9, 0.3, -0.2],      # B-B at ~2.92 > 2*1.4
                    [40.0, 5.0, 5.0]])
    types = np.array([0, 0, 1, 1, 0], dtype=np.int32)
    box = np.zeros(3)
    rad, wt, f, tj = np.array([1.6, 1.4]), np.array([1.0, 0.8]), 1.0, 6
    beta = np.stack([wl.beta(wl.ncoeff(tj), 50), wl.beta(wl.ncoeff(tj), 51)])
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    pot.set_elements(rad, wt, f)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    out = pot.compute_elements(torch.as_tensor(pos, device="cuda"), box, nl,
                               torch.as_tensor(types, device="cuda"),
                               torch.as_tensor(beta, device="cuda"), bispectrum=True)
    pot.sync_status()
    o = oracle.snap_elements(pos, box, tj, types, rad, wt, f, beta)
    E = out["energy"].cpu().numpy()
    scale = np.maximum(np.abs(o["E"]), np.abs(o["E"]).mean())
    assert (np.abs(E - o["E"]) / scale).max() <= E_REL
    assert np.abs(out["force"].cpu().numpy() - o["F"]).max() <= F_ABS
    F = out["force"].cpu().numpy()
    assert np.abs(F[0]).max() > 0.0 and np.all(F[2:] == 0.0)
