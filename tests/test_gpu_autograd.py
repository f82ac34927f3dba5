"""Autograd: the hand-written adjoint behind torch.autograd.Function.

Checked against central differences of the GPU energy itself (h = 1e-5 A on
64 random atoms of the 2000-atom 2J=8 workload, local energies so that
rounding stays well below the difference), torch's gradcheck at small size,
and the oracle's forces and bispectra.
"""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _setup(name):
    import torch
    from paper_2011_12875_amd import snapmi
    pos, box, beta, tj = wl.make(name)
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    return torch, pot, nl, pos, box, beta, tj


def test_forces_and_beta_gradient_match_oracle():
    torch, pot, nl, pos, box, beta, tj = _setup("bcc2000_2j8")
    from paper_2011_12875_amd.autograd import snap_energy
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda", requires_grad=True)
    E = snap_energy(tpos, tbeta, pot, box, nl)
    E.sum().backward()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta, want_dE=False)
    assert np.abs(-tpos.grad.cpu().numpy() - o["F"]).max() <= 1e-10
    gb = tbeta.grad.cpu().numpy()
    ref = o["B"].sum(0)
    assert np.abs(gb - ref).max() <= 1e-11 * np.abs(ref).max()


def test_weighted_loss_gradient_matches_oracle():
    """L = sum_i g_i E_i with random g: dL/dr = -F of coefficients g_i beta."""
    torch, pot, nl, pos, box, beta, tj = _setup("bcc128_2j4")
    from paper_2011_12875_amd.autograd import snap_energy
    g = np.random.default_rng(3).normal(size=len(pos))
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda", requires_grad=True)
    E = snap_energy(tpos, tbeta, pot, box, nl)
    (E * torch.tensor(g, device="cuda")).sum().backward()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=g[:, None] * beta[None, :], want_dE=False)
    ob = oracle.snap(pos, box, tj, wl.RCUT, beta=beta, want_dE=False)
    assert np.abs(-tpos.grad.cpu().numpy() - o["F"]).max() <= 1e-10
    assert np.abs(tbeta.grad.cpu().numpy() - g @ ob["B"]).max() <= 1e-11 * np.abs(g @ ob["B"]).max()


def test_central_differences_64_atoms():
    """dE/dr by central differences (h = 1e-5 A) on 64 random atoms."""
    torch, pot, nl, pos, box, beta, tj = _setup("bcc2000_2j8")
    from paper_2011_12875_amd.autograd import snap_energy
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda")
    E = snap_energy(tpos, tbeta, pot, box, nl)
    E.sum().backward()
    grad = tpos.grad.cpu().numpy()
    off, nbr = nl.off.cpu().numpy(), nl.nbr.cpu().numpy()
    atoms = np.random.default_rng(8).choice(len(pos), 64, replace=False)
    h = 1e-5
    worst = 0.0
    with torch.no_grad():
        for k in atoms:
            local = torch.tensor(np.concatenate([[k], nbr[off[k]:off[k + 1]]]), device="cuda")
            for al in range(3):
                pp = tpos.detach().clone()
                pm = tpos.detach().clone()
                pp[k, al] += h
                pm[k, al] -= h
                ep = snap_energy(pp, tbeta, pot, box, nl)[local].sum().item()
                em = snap_energy(pm, tbeta, pot, box, nl)[local].sum().item()
                worst = max(worst, abs((ep - em) / (2 * h) - grad[k, al]))
    assert worst <= 1e-6, worst


def test_gradcheck_small():
    torch, _, _, _, _, _, _ = _setup("bcc128_2j4")
    from paper_2011_12875_amd import snapmi
    from paper_2011_12875_amd.autograd import snap_energy
    pos, box = wl.cluster(8, 2.6, seed=4)
    tj = 4
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    beta = wl.beta(wl.ncoeff(tj), 5)
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda", requires_grad=True)
    f = lambda p, b: snap_energy(p, b, pot, box, nl)
    assert torch.autograd.gradcheck(f, (tpos, tbeta), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_backward_after_intervening_call():
    """A compute() between forward and backward must not corrupt the
    gradient (the forward is replayed)."""
    torch, pot, nl, pos, box, beta, tj = _setup("bcc128_2j4")
    from paper_2011_12875_amd.autograd import snap_energy
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda")
    E = snap_energy(tpos, tbeta, pot, box, nl)
    other = torch.tensor(wl.bcc(4, 0.2, 77)[0], device="cuda")
    pot.compute(other, box, nl, tbeta)
    E.sum().backward()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta, want_dE=False)
    assert np.abs(-tpos.grad.cpu().numpy() - o["F"]).max() <= 1e-10


def test_per_atom_beta_gradient_and_determinism():
    """Per-atom coefficients: dL/dbeta_i = g_i B_i; shared coefficients: the
    fixed-order reduction gives bit-identical repeats."""
    torch, pot, nl, pos, box, beta, tj = _setup("bcc128_2j4")
    from paper_2011_12875_amd.autograd import snap_energy
    g = np.random.default_rng(9).normal(size=len(pos))
    bat = np.tile(beta, (len(pos), 1)) * (1.0 + 0.1 * np.random.default_rng(10).normal(
        size=(len(pos), 1)))
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tb = torch.tensor(bat, device="cuda", requires_grad=True)
    E = snap_energy(tpos, tb, pot, box, nl)
    (E * torch.tensor(g, device="cuda")).sum().backward()
    ob = oracle.snap(pos, box, tj, wl.RCUT, beta=bat, want_dE=False)
    ref = g[:, None] * ob["B"]
    assert np.abs(tb.grad.cpu().numpy() - ref).max() <= 1e-11 * np.abs(ref).max()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=g[:, None] * bat, want_dE=False)
    assert np.abs(-tpos.grad.cpu().numpy() - o["F"]).max() <= 1e-10
    gt = torch.tensor(g, device="cuda")
    B = torch.tensor(ob["B"], device="cuda")
    r1 = pot.beta_grad(gt, B).cpu().numpy()
    r2 = pot.beta_grad(gt, B).cpu().numpy()
    assert np.array_equal(r1, r2)
    assert np.abs(r1 - g @ ob["B"]).max() <= 1e-12 * np.abs(g @ ob["B"]).max()


def test_double_backward_raises():
    """The adjoint is once-differentiable: a second derivative through it
    raises instead of silently returning a gradient without a graph."""
    torch, pot, nl, pos, box, beta, tj = _setup("bcc128_2j4")
    from paper_2011_12875_amd.autograd import snap_energy
    tpos = torch.tensor(pos, device="cuda", requires_grad=True)
    tbeta = torch.tensor(beta, device="cuda")
    E = snap_energy(tpos, tbeta, pot, box, nl)
    (gpos,) = torch.autograd.grad(E.sum(), tpos, create_graph=True)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(gpos.pow(2).sum(), tpos)
