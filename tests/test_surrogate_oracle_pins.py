"""Pins of the surrogate oracle (CPU only) against what the mathematics fixes:
central finite differences of the network and of the SNAP oracle's
bispectrum, a closed-form special case of the network, Adam's closed forms
for a constant gradient, linearity of eq. (snapatomenergy) in the
coefficients (forces from the Jacobian equal the SNAP oracle's direct forces
with per-atom coefficients), and the transpose identity of the force
pull-back."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as so
from paper_2011_12875_amd import workloads as wl


def _params(nin, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, scale / np.sqrt(nin), (64, nin))
    W2 = rng.normal(0, scale / np.sqrt(64), (64, 64))
    return np.concatenate([W1.ravel(), rng.normal(0, 0.3, 64), W2.ravel(), rng.normal(0, 0.3, 64),
                           rng.normal(0, 0.3, 64), [0.7]])


def _norm(nin, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.normal(0, 1, nin), rng.uniform(0.5, 2.0, nin)])


def test_network_special_case_closed_form():
    """W1 = [I; 0], W2 = I, zero biases, w3 = 1 on the first nin units:
    E = sum_k silu(silu(x_k)) with silu(h) = h / (1 + exp(-h))."""
    nin = 14
    p = np.zeros(so.nparams(nin))
    W1, b1, W2, b2, w3, b3 = (np.zeros((64, nin)), np.zeros(64), np.eye(64), np.zeros(64),
                              np.zeros(64), 0.0)
    W1[:nin, :nin] = np.eye(nin)
    w3[:nin] = 1.0
    p[:] = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])
    B = np.random.default_rng(1).normal(0, 2, (7, nin))
    norm = np.stack([np.zeros(nin), np.ones(nin)])
    s = lambda h: h / (1.0 + np.exp(-h))
    np.testing.assert_allclose(so.energy(p, norm, B), s(s(B)).sum(1), rtol=1e-14, atol=1e-14)
    E, _ = so.energy_and_grad(p, norm, B)
    np.testing.assert_allclose(E, s(s(B)).sum(1), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("nin", [5, 14])
def test_input_gradient_finite_differences(nin):
    p, norm = _params(nin, 2), _norm(nin, 3)
    B = np.random.default_rng(4).normal(0, 1, (6, nin))
    _, g = so.energy_and_grad(p, norm, B)
    h = 1e-6
    fd = np.zeros_like(B)
    for k in range(nin):
        Bp, Bm = B.copy(), B.copy()
        Bp[:, k] += h
        Bm[:, k] -= h
        fd[:, k] = (so.energy(p, norm, Bp) - so.energy(p, norm, Bm)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-8)


def test_parameter_gradient_finite_differences():
    """Phi = sum r E + v . g, differentiated in every parameter block."""
    nin = 5
    p, norm = _params(nin, 5), _norm(nin, 6)
    rng = np.random.default_rng(7)
    B = rng.normal(0, 1, (9, nin))
    r = rng.normal(0, 1, 9)
    v = rng.normal(0, 1, (9, nin))
    grad = so.param_grad(p, norm, B, r, v)

    def phi(q):
        E, g = so.energy_and_grad(q, norm, B)
        return float(r @ E + (v * g).sum())

    # a few parameters from each block: W1, b1, W2, b2, w3, b3
    W1, B1, W2, B2, W3, B3 = 0, 64 * nin, 64 * nin + 64, 64 * nin + 64 + 4096, \
        64 * nin + 128 + 4096, 64 * nin + 192 + 4096
    idx = [W1 + 3, W1 + 200, B1 + 5, W2 + 17, W2 + 4000, B2 + 63, W3 + 9, B3]
    h = 1e-6
    for k in idx:
        qp, qm = p.copy(), p.copy()
        qp[k] += h
        qm[k] -= h
        fd = (phi(qp) - phi(qm)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, grad[k])
    # the energy-only gradient of b3 is sum r
    assert abs(so.param_grad(p, norm, B, r)[B3] - r.sum()) <= 1e-12


def test_adam_closed_forms():
    """Constant gradient: m_hat = g and v_hat = g^2 at every step, so each step
    moves theta by lr g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    th0 = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    lr, eps = 1e-2, 1e-8
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        th, m, v = so.adam(th, m, v, g, lr, t, eps=eps)
        np.testing.assert_allclose(th, th0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)


def _cluster():
    pos, box = wl.cluster(10, 3.0, seed=21)
    return pos, box


def test_jacobian_finite_differences():
    """J_p = dB_i/dr_ik: moving neighbour k moves r_ik one for one."""
    pos, box = _cluster()
    B, off, nbr, J = so.jacobian(pos, box, 4, wl.RCUT)
    h = 1e-5
    rng = np.random.default_rng(9)
    for p in rng.choice(len(nbr), 6, replace=False):
        i = int(np.searchsorted(off, p, side="right") - 1)
        k = int(nbr[p])
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, a] += h
            pm[k, a] -= h
            bp = oracle.snap(pp, box, 4, wl.RCUT, beta=np.zeros(14), want_dE=False)["B"][i]
            bm = oracle.snap(pm, box, 4, wl.RCUT, beta=np.zeros(14), want_dE=False)["B"][i]
            np.testing.assert_allclose(J[p, :, a], (bp - bm) / (2 * h), rtol=1e-6, atol=1e-8)


def test_jacobian_forces_equal_direct_snap_forces():
    """E_i = g_i . B_i is SNAP with per-atom coefficients g_i: the forces and
    pair derivatives from J must equal the oracle's direct ones."""
    pos, box = _cluster()
    B, off, nbr, J = so.jacobian(pos, box, 4, wl.RCUT)
    g = np.random.default_rng(10).normal(0, 0.2, (len(pos), 14))
    dE, F = so.jacobian_forces(off, nbr, J, g)
    o = oracle.snap(pos, box, 4, wl.RCUT, beta=g)
    np.testing.assert_allclose(dE, o["dE"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(F, o["F"], rtol=0, atol=1e-12)
    assert np.abs(F.sum(0)).max() < 1e-12


def test_jacobian_adjoint_is_the_transpose():
    """<v(lam), g> = <lam, F(g)> for the linear map g -> F."""
    pos, box = _cluster()
    _, off, nbr, J = so.jacobian(pos, box, 4, wl.RCUT)
    rng = np.random.default_rng(11)
    for _ in range(3):
        g = rng.normal(0, 1, (len(pos), 14))
        lam = rng.normal(0, 1, (len(pos), 3))
        _, F = so.jacobian_forces(off, nbr, J, g)
        v = so.jacobian_adjoint(off, nbr, J, lam)
        assert abs((v * g).sum() - (lam * F).sum()) <= 1e-12 * max(1.0, abs((lam * F).sum()))


def test_residuals_are_the_loss_derivatives():
    rng = np.random.default_rng(12)
    E, Er = rng.normal(0, 1, 5), rng.normal(0, 1, 5)
    F, Fr = rng.normal(0, 1, (5, 3)), rng.normal(0, 1, (5, 3))
    wE, wF = 0.3, 1.7
    L = lambda e, f: wE * ((e - Er) ** 2).sum() + wF * ((f - Fr) ** 2).sum()
    rE, lam, se, sf = so.residuals(E, Er, F, Fr, wE, wF)
    h = 1e-6
    for i in range(5):
        ep, em = E.copy(), E.copy()
        ep[i] += h
        em[i] -= h
        assert abs((L(ep, F) - L(em, F)) / (2 * h) - rE[i]) < 1e-7
    fp = F.copy()
    fp[2, 1] += h
    fm = F.copy()
    fm[2, 1] -= h
    assert abs((L(E, fp) - L(E, fm)) / (2 * h) - lam[2, 1]) < 1e-7
    assert abs(wE * se + wF * sf - L(E, F)) < 1e-12
