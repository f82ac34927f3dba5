"""Pins of the oracle's virial W = dE_total/d(strain) = sum_p dE_p (x) r_ik
(CPU only): central finite differences of the oracle's energy under a
homogeneous strain r -> (I + eps) r -- the full tensor on an isolated
cluster, the diagonal on a periodic crystal (box scaled with the atoms) --
and the symmetry of W that rotational invariance of the energy implies."""
import numpy as np

import oracle
from paper_2011_12875_amd import workloads as wl


def _strain_fd(pos, box, tj, beta, a, b, h=1e-6):
    def energy(s):
        e = np.zeros((3, 3))
        e[a, b] = s
        m = np.eye(3) + e
        bx = np.array([box[d] * m[d, d] if box[d] > 0 else 0.0 for d in range(3)])
        return oracle.snap(pos @ m.T, bx, tj, wl.RCUT, beta=beta, want_dE=False)["E"].sum()
    return (energy(h) - energy(-h)) / (2 * h)


def test_virial_full_tensor_on_cluster():
    pos, box = wl.cluster(12, 3.2, seed=31)
    beta = wl.beta(14, 32)
    o = oracle.snap(pos, box, 4, wl.RCUT, beta=beta)
    W, Wa = oracle.virial(pos, box, o["off"], o["nbr"], o["dE"])
    for a in range(3):
        for b in range(3):
            assert abs(W[a, b] - _strain_fd(pos, box, 4, beta, a, b)) <= 1e-8 * np.abs(W).max()
    np.testing.assert_allclose(Wa.sum(0), W, rtol=0, atol=1e-12 * np.abs(W).max())


def test_virial_diagonal_on_periodic_crystal():
    pos, box = wl.bcc(3, 0.1, 33)
    beta = wl.beta(14, 34)
    o = oracle.snap(pos, box, 4, wl.RCUT, beta=beta)
    W, _ = oracle.virial(pos, box, o["off"], o["nbr"], o["dE"])
    for a in range(3):
        assert abs(W[a, a] - _strain_fd(pos, box, 4, beta, a, a)) <= 1e-7 * np.abs(W).max()


def test_virial_is_symmetric():
    """Rotational invariance: the antisymmetric part (a torque) vanishes."""
    for pos, box in (wl.cluster(12, 3.2, seed=35), wl.bcc(3, 0.1, 36)):
        o = oracle.snap(pos, box, 6, wl.RCUT, beta=wl.beta(30, 37))
        W, _ = oracle.virial(pos, box, o["off"], o["nbr"], o["dE"])
        assert np.abs(W - W.T).max() <= 1e-11 * np.abs(W).max()
