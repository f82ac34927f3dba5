"""Surrogate kernels on the GPU against the surrogate oracle (CPU, float64).

Tolerances follow from the arithmetic of each kernel:
  * the network runs in FP32 (weights, activations, accumulation over at most
    64 terms per dot product): outputs are compared with
    |gpu - oracle| <= 3e-5 * max|oracle| (64 terms x 2^-24 unit roundoff,
    three layers, with room for the hardware exp);
  * the parameter gradient adds FP32 sums over up to 64 atoms per block and
    over blocks: 1e-4 * max|oracle|;
  * J_p is stored in FP32 after an FP64 evaluation: |dJ| <= 2^-23 |J| plus
    the FP64 error of the adjoint stages (1e-12 of the scale);
  * forces and pull-backs from J are FP64 sums of FP32 J entries: bounded by
    2^-23 times the same sums taken over absolute values;
  * residuals are plain FP64: 1e-14 relative.
"""
import numpy as np
import pytest

import oracle
from oracle import surrogate as so
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -23


def _torch():
    import torch
    from paper_2011_12875_amd import snapmi
    return torch, snapmi


def _params(nin, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.normal(0, 1 / np.sqrt(nin), 64 * nin), rng.normal(0, 0.3, 64),
                           rng.normal(0, 1 / 8, 4096), rng.normal(0, 0.3, 64),
                           rng.normal(0, 0.3, 64), [0.4]]).astype(np.float32)


def _norm(nin, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.normal(0, 3, nin), rng.uniform(0.2, 2.0, nin)]).astype(np.float32)


def _inputs(nin, n, seed, norm):
    rng = np.random.default_rng(seed)
    return norm[0] + rng.normal(0, 1.5, (n, nin)) / norm[1]


@pytest.mark.parametrize("nin", [5, 14, 30])
@pytest.mark.parametrize("n", [1, 65, 1000])
def test_mlp_forward_matches_oracle(nin, n):
    torch, snapmi = _torch()
    p, norm = _params(nin, 1), _norm(nin, 2)
    B = _inputs(nin, n, 3, norm)
    E, g = snapmi.mlp_forward(torch.tensor(p, device="cuda"), torch.tensor(norm, device="cuda"),
                              torch.tensor(B, device="cuda"))
    Eo, go = so.energy_and_grad(p.astype(np.float64), norm.astype(np.float64), B)
    assert np.abs(E.cpu().numpy() - Eo).max() <= 3e-5 * np.abs(Eo).max()
    assert np.abs(g.cpu().numpy() - go).max() <= 3e-5 * np.abs(go).max()


def test_mlp_range_gate():
    torch, snapmi = _torch()
    nin = 14
    p, norm = _params(nin, 4), np.stack([np.zeros(nin), np.ones(nin)]).astype(np.float32)
    bounds = torch.tensor(np.stack([-np.ones(nin), np.ones(nin)]).astype(np.float32), device="cuda")
    tp, tn = torch.tensor(p, device="cuda"), torch.tensor(norm, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    B = np.random.default_rng(5).uniform(-1.09, 1.09, (300, nin))
    snapmi.mlp_forward(tp, tn, torch.tensor(B, device="cuda"), bounds, 0.05, flag)
    assert int(flag.item()) == 0  # inside [-1.1, 1.1]
    for bad in (1.15, -1.2, np.nan):
        B2 = B.copy()
        B2[217, 9] = bad
        flag.zero_()
        snapmi.mlp_forward(tp, tn, torch.tensor(B2, device="cuda"), bounds, 0.05, flag)
        assert int(flag.item()) == 1, bad


@pytest.mark.parametrize("nin", [5, 14])
@pytest.mark.parametrize("n", [1, 64, 200])
@pytest.mark.parametrize("with_g", [False, True])
def test_mlp_param_grad_matches_oracle(nin, n, with_g):
    torch, snapmi = _torch()
    p, norm = _params(nin, 6), _norm(nin, 7)
    B = _inputs(nin, n, 8, norm)
    rng = np.random.default_rng(9)
    r = rng.normal(0, 1, n)
    v = rng.normal(0, 1, (n, nin)) / norm[1] if with_g else None
    tv = torch.tensor(v, device="cuda") if with_g else None
    gr = snapmi.mlp_grad(torch.tensor(p, device="cuda"), torch.tensor(norm, device="cuda"),
                         torch.tensor(B, device="cuda"), torch.tensor(r, device="cuda"), tv)
    go = so.param_grad(p.astype(np.float64), norm.astype(np.float64), B, r, v)
    assert np.abs(gr.cpu().numpy() - go).max() <= 1e-4 * np.abs(go).max()


def test_mlp_param_grad_is_deterministic():
    torch, snapmi = _torch()
    nin, n = 14, 5000
    p, norm = _params(nin, 10), _norm(nin, 11)
    args = [torch.tensor(p, device="cuda"), torch.tensor(norm, device="cuda"),
            torch.tensor(_inputs(nin, n, 12, norm), device="cuda"),
            torch.tensor(np.random.default_rng(13).normal(0, 1, n), device="cuda"),
            torch.tensor(np.random.default_rng(14).normal(0, 1, (n, nin)), device="cuda")]
    a = snapmi.mlp_grad(*args).cpu().numpy()
    b = snapmi.mlp_grad(*args).cpu().numpy()
    assert np.array_equal(a, b)


def test_mlp_param_grad_empty_is_zero():
    torch, snapmi = _torch()
    nin = 14
    p, norm = _params(nin, 15), _norm(nin, 16)
    gr = snapmi.mlp_grad(torch.tensor(p, device="cuda"), torch.tensor(norm, device="cuda"),
                         torch.zeros((0, nin), dtype=torch.float64, device="cuda"),
                         torch.zeros(0, dtype=torch.float64, device="cuda"),
                         grad=torch.full((p.size,), 7.0, device="cuda"))
    assert float(gr.abs().max()) == 0.0


def test_adam_matches_oracle():
    torch, snapmi = _torch()
    rng = np.random.default_rng(17)
    npar = 5185
    th = rng.normal(0, 1, npar).astype(np.float32)
    tth = torch.tensor(th, device="cuda")
    m = torch.zeros(npar, device="cuda")
    v = torch.zeros(npar, device="cuda")
    oth, om, ov = th.astype(np.float64), np.zeros(npar), np.zeros(npar)
    for step in range(1, 4):
        g = rng.normal(0, 1, npar).astype(np.float32)
        snapmi.adam_step(tth, m, v, torch.tensor(g, device="cuda"), 1e-3, step)
        oth, om, ov = so.adam(oth, om, ov, g.astype(np.float64), 1e-3, step)
    assert np.abs(tth.cpu().numpy() - oth).max() <= 1e-6 * np.abs(oth).max()


def _jac_case(name):
    if name == "bcc128":
        pos, box = wl.bcc(4, 0.05, 1)
    elif name == "cluster":
        pos, box = wl.cluster(30, 5.0, seed=18)
        pos = np.concatenate([pos, [[40.0, 40.0, 40.0]]])  # one atom without neighbours
    return pos, box


@pytest.mark.parametrize("case", ["bcc128", "cluster"])
def test_jacobian_matches_oracle(case):
    torch, snapmi = _torch()
    pos, box = _jac_case(case)
    pot = snapmi.SnapPotential(4, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    B, J = pot.jacobian(torch.tensor(pos, device="cuda"), box, nl)
    Bo, off, nbr, Jo = so.jacobian(pos, box, 4, wl.RCUT)
    assert np.array_equal(nl.off.cpu().numpy(), off) and np.array_equal(
        nl.nbr.cpu().numpy()[:nl.npairs], nbr)
    assert np.abs(B.cpu().numpy() - Bo).max() <= 1e-12 * np.abs(Bo).max()
    Jg = J.cpu().numpy()[:nl.npairs].astype(np.float64)
    assert np.all(np.abs(Jg - Jo) <= U32 * np.abs(Jo) + 1e-12 * np.abs(Jo).max())


def _abs_forces(off, nbr, J, g):
    own = so.pair_owner(off)
    s = np.einsum("plk,pl->pk", np.abs(J), np.abs(g)[own])
    S = np.zeros((len(off) - 1, 3))
    np.add.at(S, own, s)
    np.add.at(S, nbr, s)
    return S


def test_jacobian_forces_and_adjoint_match_oracle():
    torch, snapmi = _torch()
    pos, box = _jac_case("bcc128")
    pot = snapmi.SnapPotential(4, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    _, J = pot.jacobian(torch.tensor(pos, device="cuda"), box, nl)
    _, off, nbr, Jo = so.jacobian(pos, box, 4, wl.RCUT)
    rng = np.random.default_rng(19)
    g = rng.normal(0, 0.3, (len(pos), 14))
    lam = rng.normal(0, 1, (len(pos), 3))
    F = snapmi.jacobian_forces(nl, J, torch.tensor(g, device="cuda")).cpu().numpy()
    _, Fo = so.jacobian_forces(off, nbr, Jo, g)
    S = _abs_forces(off, nbr, Jo, g)
    assert np.all(np.abs(F - Fo) <= 2 * U32 * S + 1e-13)
    vg = snapmi.jacobian_adjoint(nl, J, torch.tensor(lam, device="cuda"), 14).cpu().numpy()
    vo = so.jacobian_adjoint(off, nbr, Jo, lam)
    own = so.pair_owner(off)
    Sv = np.zeros_like(vo)
    np.add.at(Sv, own, np.einsum("plk,pk->pl", np.abs(Jo),
                                 np.abs(lam[own]) + np.abs(lam[nbr])))
    assert np.all(np.abs(vg - vo) <= 2 * U32 * Sv + 1e-13)


def test_fit_residuals_match_oracle():
    torch, snapmi = _torch()
    rng = np.random.default_rng(20)
    n = 700
    E, Er = rng.normal(0, 1, n), rng.normal(0, 1, n)
    F, Fr = rng.normal(0, 1, (n, 3)), rng.normal(0, 1, (n, 3))
    t = lambda a: torch.tensor(a, device="cuda")
    rE, lam, sums = snapmi.fit_residuals(t(E), t(Er), t(F), t(Fr), 0.3, 1.7)
    orE, olam, se, sf = so.residuals(E, Er, F, Fr, 0.3, 1.7)
    assert np.abs(rE.cpu().numpy() - orE).max() <= 1e-14 * np.abs(orE).max()
    assert np.abs(lam.cpu().numpy() - olam).max() <= 1e-14 * np.abs(olam).max()
    s = sums.cpu().numpy().sum(0)
    assert abs(s[0] - se) <= 1e-13 * se and abs(s[1] - sf) <= 1e-13 * sf


def _untrained_surrogate(torch, snapmi, B_train):
    from paper_2011_12875_amd import surrogate as sg
    nin = B_train.shape[1]
    mean, std = B_train.mean(0), B_train.std(0)
    net = sg.Network.initial(nin, mean, std, 0.0, 1.0, seed=3)
    x = (B_train - mean) / std
    net.bounds = torch.tensor(np.stack([x.min(0), x.max(0)]).astype(np.float32), device="cuda")
    return net


def test_surrogate_forces_match_oracle_chain():
    """Adjoint route (snap_backward with beta = g) against the oracle chain:
    the oracle's B, the oracle network's g, the oracle's forces with per-atom
    coefficients g; and against the Jacobian route on the GPU."""
    torch, snapmi = _torch()
    from paper_2011_12875_amd import surrogate as sg
    pos, box = wl.bcc(4, 0.1, 21)
    o4 = oracle.snap(pos, box, 4, wl.RCUT, beta=np.zeros(14), want_dE=False)
    net = _untrained_surrogate(torch, snapmi, o4["B"])
    pot4, pot8 = snapmi.SnapPotential(4, wl.RCUT), snapmi.SnapPotential(8, wl.RCUT)
    beta8 = wl.surrogate_target_beta()
    sp = sg.SurrogatePotential(net, pot4, pot8, beta8)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    tpos = torch.tensor(pos, device="cuda")
    out = sp.compute(tpos, box, nl)
    assert not out["fallback"]
    st = net.state()
    Eo, go = so.energy_and_grad(st["params"].astype(np.float64), st["norm"].astype(np.float64),
                                o4["B"])
    of = oracle.snap(pos, box, 4, wl.RCUT, beta=go, want_dE=False)
    F = out["force"].cpu().numpy()
    assert np.abs(out["energy"].cpu().numpy() - Eo).max() <= 3e-5 * np.abs(Eo).max()
    assert np.abs(F - of["F"]).max() <= 3e-5 * np.abs(of["F"]).max()
    _, J = pot4.jacobian(tpos, box, nl)
    Ez, Bz = pot4.forward(tpos, box, nl, torch.zeros(14, dtype=torch.float64, device="cuda"))
    En, Bn = pot4.forward(tpos, box, nl, None)  # B only
    assert En is None and torch.equal(Bz, Bn)
    E2, g2 = net.forward(Bn, gate=False)
    F2 = snapmi.jacobian_forces(nl, J, g2).cpu().numpy()
    assert np.abs(F - F2).max() <= 1e-6 * np.abs(F).max()


def test_fallback_on_out_of_range_configuration():
    torch, snapmi = _torch()
    from paper_2011_12875_amd import surrogate as sg
    pot4, pot8 = snapmi.SnapPotential(4, wl.RCUT), snapmi.SnapPotential(8, wl.RCUT)
    beta8 = wl.surrogate_target_beta()
    Btr = np.concatenate([oracle.snap(wl.surrogate_config(c)[0], wl.surrogate_config(c)[1], 4,
                                      wl.RCUT, beta=np.zeros(14), want_dE=False)["B"]
                          for c in range(6)])
    net = _untrained_surrogate(torch, snapmi, Btr)
    net.margin = 0.05
    sp = sg.SurrogatePotential(net, pot4, pot8, beta8)
    tb8 = torch.tensor(beta8, device="cuda")
    # an in-range configuration (a training one) does not fall back
    pos, box, _ = wl.surrogate_config(0)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    assert not sp.compute(torch.tensor(pos, device="cuda"), box, nl)["fallback"]
    # sigma = 0.35 A is outside the training range of the descriptors
    pos, box = wl.bcc(10, wl.SURROGATE["sigma_ood"], wl.SURROGATE["ood_seed"])
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    tpos = torch.tensor(pos, device="cuda")
    out = sp.compute(tpos, box, nl)
    assert out["fallback"]
    ref = pot8.compute(tpos, box, nl, tb8)
    assert torch.equal(out["force"], ref["force"]) and torch.equal(out["energy"], ref["energy"])
    j = sp.judge(tpos, box, nl, out)
    assert j["force_rmse"] == 0.0 and j["fallback"]


def test_gate_flags_alternate_and_deferred_check():
    """The two gate flags: an in-range, an out-of-range, then an in-range
    configuration again (the tripped flag is cleared by the call after the
    next, without any clearing kernel), each checked with the deferred
    read-back; the out-of-range one resolves to plain 2J = 8 SNAP."""
    torch, snapmi = _torch()
    from paper_2011_12875_amd import surrogate as sg
    pot4, pot8 = snapmi.SnapPotential(4, wl.RCUT), snapmi.SnapPotential(8, wl.RCUT)
    beta8 = wl.surrogate_target_beta()
    Btr = np.concatenate([oracle.snap(wl.surrogate_config(c)[0], wl.surrogate_config(c)[1], 4,
                                      wl.RCUT, beta=np.zeros(14), want_dE=False)["B"]
                          for c in range(6)])
    net = _untrained_surrogate(torch, snapmi, Btr)
    net.margin = 0.05
    sp = sg.SurrogatePotential(net, pot4, pot8, beta8)
    pin, bin_, _ = wl.surrogate_config(0)
    nl_in = snapmi.NeighborList.build(pin, bin_, wl.RCUT)
    pout, bout = wl.bcc(10, wl.SURROGATE["sigma_ood"], wl.SURROGATE["ood_seed"])
    nl_out = snapmi.NeighborList.build(pout, bout, wl.RCUT)
    tin, tout = torch.tensor(pin, device="cuda"), torch.tensor(pout, device="cuda")
    seq = [(tin, bin_, nl_in, False), (tout, bout, nl_out, True), (tin, bin_, nl_in, False),
           (tin, bin_, nl_in, False), (tout, bout, nl_out, True), (tout, bout, nl_out, True),
           (tin, bin_, nl_in, False)]
    for tpos, box, nl, want in seq:
        out = sp.resolve(sp.compute(tpos, box, nl, check="deferred"))
        assert out["fallback"] == want
        if want:
            ref = pot8.compute(tpos, box, nl, torch.tensor(beta8, device="cuda"))
            assert torch.equal(out["force"], ref["force"])


def test_training_reduces_loss_and_beats_linear_model():
    """A short training (1000 configurations, 4000 Adam steps): the held-out
    force error falls, and the trained network beats the linear 2J = 4 model
    fitted by least squares to the same loss on held-out configurations."""
    torch, snapmi = _torch()
    from paper_2011_12875_amd import surrogate as sg
    pot4, pot8 = snapmi.SnapPotential(4, wl.RCUT), snapmi.SnapPotential(8, wl.RCUT)
    beta8 = wl.surrogate_target_beta()
    tr, va, te = wl.surrogate_split()
    dtr = sg.make_surrogate_data(tr[:1000], pot8, beta8, pot4)
    dte = sg.make_surrogate_data(te[:200], pot8, beta8, pot4)
    cfg = sg.TrainConfig(epochs=100, batch_configs=25, eval_every=20)
    net0 = sg.Network.initial(14, *[t.cpu().numpy() for t in sg.input_statistics(dtr)[:2]],
                              *sg.input_statistics(dtr)[2:], seed=cfg.seed)
    r0 = sg.evaluate(net0, dte)
    net, hist = sg.train(dtr, cfg, dte)
    r = sg.evaluate(net, dte)
    lin = sg.evaluate_linear(*sg.fit_linear(dtr), dte)
    print("initial", r0, "trained", r, "linear", lin, flush=True)
    assert r["force_rmse"] < 0.5 * r0["force_rmse"]
    assert hist[-1]["force_rmse"] <= hist[0]["force_rmse"]
    assert r["force_rmse"] < lin["force_rmse"]
