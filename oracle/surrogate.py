"""Plain FP64 CPU oracle for the learned surrogate -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; the product path never does, and this
module imports nothing from it.

What it computes, and from what:
  * the network E_i = f(x_i), x_i = (B_i - mean) * scale, with two hidden
    layers of 64 SiLU units (silu(h) = h / (1 + exp(-h))) and a linear output,
    parameters packed as W1[64][nin], b1[64], W2[64][64], b2[64], w3[64], b3;
    evaluated with plain float64 array operations;
  * g_i = dE_i/dB_i and the parameter gradient of
    Phi = sum_i r_i E_i + v_i . g_i by torch's CPU automatic differentiation in
    float64 (a double backward for the second term), not by hand-written
    derivatives;
  * Adam as stated by Kingma and Ba (2015), Algorithm 1;
  * the descriptor Jacobian J_p = dB_i/dr_ik of pair p = (i -> k), from the
    SNAP oracle's literal dB/dr (eq. (dbidrk)) with one unit coefficient
    vector per component, so that dE_p with beta = e_l is column l of J_p;
  * forces of per-atom energies from J_p, F_i = sum_{p = (i->k)} dE_p minus
    the same over pairs (k->i), dE_p = J_p^T g_i; and the pull-back of a force
    loss to g;
  * the squared-error loss of energies and forces and its derivatives.
"""
from __future__ import annotations

import numpy as np

from . import snap as snap_oracle
from . import components as snap_components

H = 64


def nparams(nin: int) -> int:
    return H * nin + H + H * H + H + H + 1


def unpack(params, nin):
    """(W1 [64, nin], b1 [64], W2 [64, 64], b2 [64], w3 [64], b3) views."""
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (nparams(nin),)
    o = 0
    W1 = p[o:o + H * nin].reshape(H, nin); o += H * nin
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def _silu(h):
    return h / (1.0 + np.exp(-h))


def standardise(B, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(B, dtype=np.float64) - norm[0]) * norm[1]


def energy(params, norm, B):
    """E_i of the network, float64 [n]."""
    B = np.asarray(B, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(params, B.shape[1])
    x = standardise(B, norm)
    a1 = _silu(x @ W1.T + b1)
    a2 = _silu(a1 @ W2.T + b2)
    return a2 @ w3 + b3


def _torch_net(theta, norm, B, nin):
    import torch
    o = 0
    W1 = theta[o:o + H * nin].reshape(H, nin); o += H * nin
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    x = (B - norm[0]) * norm[1]
    silu = torch.nn.functional.silu
    return silu(silu(x @ W1.T + b1) @ W2.T + b2) @ w3 + b3


def energy_and_grad(params, norm, B):
    """(E_i [n], g_i = dE_i/dB_i [n, nin]) by automatic differentiation."""
    import torch
    B = np.asarray(B, dtype=np.float64)
    nin = B.shape[1]
    theta = torch.tensor(np.asarray(params, dtype=np.float64))
    tn = torch.tensor(np.asarray(norm, dtype=np.float64))
    tB = torch.tensor(B, requires_grad=True)
    E = _torch_net(theta, tn, tB, nin)
    (g,) = torch.autograd.grad(E.sum(), tB)
    return E.detach().numpy(), g.numpy()


def param_grad(params, norm, B, dl_de, dl_dg=None):
    """d/dtheta of sum_i dl_de_i E_i + dl_dg_i . g_i (float64 [nparams])."""
    import torch
    B = np.asarray(B, dtype=np.float64)
    nin = B.shape[1]
    theta = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    tn = torch.tensor(np.asarray(norm, dtype=np.float64))
    tB = torch.tensor(B, requires_grad=True)
    E = _torch_net(theta, tn, tB, nin)
    phi = (torch.tensor(np.asarray(dl_de, dtype=np.float64)) * E).sum()
    if dl_dg is not None:
        (g,) = torch.autograd.grad(E.sum(), tB, create_graph=True)
        phi = phi + (torch.tensor(np.asarray(dl_dg, dtype=np.float64)) * g).sum()
    (gt,) = torch.autograd.grad(phi, theta)
    return gt.numpy()


def adam(params, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam; returns (params, m, v), all float64."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * np.square(grad)
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


def jacobian(pos, box, twojmax, rcut, rfac0=0.99363, rmin0=0.0, switch_flag=1, wself=1.0):
    """B [n, N_B], off, nbr and J [P, N_B, 3] with J[p, l] = dB_il/dr_ik."""
    nb = len(snap_components(twojmax))
    J = None
    for l in range(nb):
        e_l = np.zeros(nb)
        e_l[l] = 1.0
        o = snap_oracle(pos, box, twojmax, rcut, rfac0, rmin0, switch_flag, wself, beta=e_l)
        if J is None:
            J = np.zeros((len(o["nbr"]), nb, 3))
            B, off, nbr = o["B"], o["off"], o["nbr"]
        J[:, l, :] = o["dE"]
    return B, off, nbr, J


def pair_owner(off):
    off = np.asarray(off)
    return np.repeat(np.arange(len(off) - 1), np.diff(off))


def jacobian_forces(off, nbr, J, g):
    """(dE [P, 3], F [n, 3]) for per-atom input gradients g [n, nin]."""
    own = pair_owner(off)
    dE = np.einsum("plk,pl->pk", np.asarray(J, dtype=np.float64), np.asarray(g)[own])
    F = np.zeros((len(off) - 1, 3))
    np.add.at(F, own, dE)
    np.add.at(F, np.asarray(nbr), -dE)
    return dE, F


def jacobian_adjoint(off, nbr, J, lam):
    """dL/dg [n, nin] for dL/dF = lam [n, 3]."""
    own = pair_owner(off)
    lam = np.asarray(lam, dtype=np.float64)
    d = lam[own] - lam[np.asarray(nbr)]
    vp = np.einsum("plk,pk->pl", np.asarray(J, dtype=np.float64), d)
    v = np.zeros((len(off) - 1, np.asarray(J).shape[1]))
    np.add.at(v, own, vp)
    return v


def residuals(E, Eref, F, Fref, wE, wF):
    """(dL/dE, dL/dF, sum (E-Eref)^2, sum |F-Fref|^2) of
    L = wE sum (E - Eref)^2 + wF sum |F - Fref|^2."""
    dE = np.asarray(E) - np.asarray(Eref)
    dF = np.asarray(F) - np.asarray(Fref)
    return 2.0 * wE * dE, 2.0 * wF * dF, float(np.sum(dE * dE)), float(np.sum(dF * dF))
