"""Learned surrogate of a high-order SNAP potential.

The energy of eq. (snapatomenergy) is linear in the bispectrum and its forces
come from the adjoint Y of eq. (y) (Sec. IV), which accepts any per-atom
coefficient vector.  The surrogate keeps that machinery and replaces the
linear map: a per-atom network E_i = f(B_i) on the 14 components of the
cheap 2J = 4 bispectrum, trained on energies and forces of a 2J = 8 potential
computed by the same library.  Its forces are the 2J = 4 adjoint with
per-atom coefficients g_i = dE_i/dB_i.

Every arithmetic step runs in the library's kernels (include/snapmi.h):
  data      snap_compute at 2J = 8 (labels E_i, F_i) and snap_jacobian at
            2J = 4 (B_i and J_p = dB_i/dr_ik per pair, FP32);
  training  snap_mlp_forward -> snap_jacobian_forces -> snap_fit_residuals ->
            snap_jacobian_adjoint -> snap_mlp_grad -> snap_adam_step;
  inference snap_forward (2J = 4) -> snap_mlp_forward (with the range gate)
            -> snap_backward with beta = g; configurations outside the
            training range are evaluated by plain 2J = 8 SNAP instead, and
            plain 2J = 8 SNAP is the judge of any evaluation.
torch provides device memory, the stream, and host-side bookkeeping (batch
index arrays, statistics of the training inputs, the small least-squares
solve of the linear reference model).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import snapmi
from . import workloads as wl

HIDDEN = 64


class _NL:
    """A neighbour list given by device tensors (a batch of configurations)."""

    def __init__(self, off, nbr, rev):
        self.off, self.nbr, self.rev = off, nbr, rev
        self.n = int(off.numel()) - 1
        self.npairs = int(nbr.numel())


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
class Network:
    """Parameters of the per-atom network and its input standardisation."""

    def __init__(self, params, norm, bounds=None, margin=0.05):
        import torch
        self.nin = int(norm.shape[1])
        self.params = params.to(torch.float32).contiguous()
        self.norm = norm.to(torch.float32).contiguous()
        self.bounds = None if bounds is None else bounds.to(torch.float32).contiguous()
        self.margin = float(margin)
        assert self.params.numel() == snapmi.mlp_nparams(self.nin)

    @classmethod
    def initial(cls, nin, mean, std, e_mean, e_std, seed=0, device="cuda"):
        """Random initial weights (variance 1/fan-in), output scaled to the
        spread of the energies and shifted to their mean."""
        import torch
        rng = np.random.default_rng(seed)
        W1 = rng.normal(0, 1 / np.sqrt(nin), (HIDDEN, nin))
        W2 = rng.normal(0, 1 / np.sqrt(HIDDEN), (HIDDEN, HIDDEN))
        w3 = rng.normal(0, e_std / np.sqrt(HIDDEN), HIDDEN)
        p = np.concatenate([W1.ravel(), np.zeros(HIDDEN), W2.ravel(), np.zeros(HIDDEN), w3,
                            [e_mean]])
        scale = 1.0 / np.maximum(np.asarray(std, dtype=np.float64), 1e-12)
        norm = np.stack([np.asarray(mean, dtype=np.float64), scale])
        return cls(torch.tensor(p, device=device), torch.tensor(norm, device=device))

    def forward(self, B, flag=None, energy=None, grad_b=None, gate=True, clear_flag=None):
        return snapmi.mlp_forward(self.params, self.norm, B,
                                  self.bounds if gate else None, self.margin, flag,
                                  energy, grad_b, clear_flag)

    def state(self):
        return {"params": self.params.cpu().numpy(), "norm": self.norm.cpu().numpy(),
                "bounds": None if self.bounds is None else self.bounds.cpu().numpy(),
                "margin": self.margin}


# ---------------------------------------------------------------------------
# training data
# ---------------------------------------------------------------------------
@dataclass
class Dataset:
    """Configurations of one box, concatenated on the device, with labels
    from the 2J = 8 potential and 2J = 4 descriptors and Jacobians."""
    box: np.ndarray
    natoms: np.ndarray          # per configuration
    npairs: np.ndarray
    a_off: np.ndarray           # atom offset of each configuration
    p_off: np.ndarray           # pair offset of each configuration
    off: object                 # device CSR over all configurations
    nbr: object
    rev: object
    B: object                   # [N, 14] float64
    J: object                   # [P, 14, 3] float32
    E: object                   # [N] float64 labels
    F: object                   # [N, 3] float64 labels
    sigma: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n(self):
        return int(self.a_off[-1])

    def batch(self, c0, c1):
        """Neighbour list (local indices), atom and pair ranges of
        configurations c0 .. c1-1."""
        a0, a1 = int(self.a_off[c0]), int(self.a_off[c1])
        p0, p1 = int(self.p_off[c0]), int(self.p_off[c1])
        off = (self.off[a0:a1 + 1] - p0).contiguous()
        nbr = (self.nbr[p0:p1] - a0).contiguous()
        rev = (self.rev[p0:p1] - p0).contiguous()
        return _NL(off, nbr, rev), (a0, a1), (p0, p1)


def build_dataset(configs, pot8, beta8, pot4, chunk=500, device="cuda"):
    """configs: list of (pos, box) sharing one box.  Labels and descriptors
    are computed on the device in chunks of configurations."""
    import torch
    box = np.asarray(configs[0][1], dtype=np.float64)
    offs, nbrs, revs, nat, npr = [], [], [], [], []
    for pos, bx in configs:
        assert np.allclose(bx, box)
        o, nb, rv = snapmi.build_neighbors(pos, box, pot4.rcut)
        offs.append(o)
        nbrs.append(nb)
        revs.append(rv)
        nat.append(len(pos))
        npr.append(len(nb))
    nat, npr = np.array(nat), np.array(npr)
    a_off = np.concatenate([[0], np.cumsum(nat)])
    p_off = np.concatenate([[0], np.cumsum(npr)])
    off = np.concatenate([[0]] + [o[1:] + p_off[c] for c, o in enumerate(offs)]).astype(np.int32)
    nbr = np.concatenate([nb + a_off[c] for c, nb in enumerate(nbrs)]).astype(np.int32)
    rev = np.concatenate([rv + p_off[c] for c, rv in enumerate(revs)]).astype(np.int32)
    pos_all = np.concatenate([p for p, _ in configs])
    N, P = int(a_off[-1]), int(p_off[-1])
    d_off = torch.as_tensor(off, device=device)
    d_nbr = torch.as_tensor(nbr, device=device)
    d_rev = torch.as_tensor(rev, device=device)
    nin = pot4.ncoeff
    B = torch.empty((N, nin), dtype=torch.float64, device=device)
    J = torch.empty((max(P, 1), nin, 3), dtype=torch.float32, device=device)
    E = torch.empty(N, dtype=torch.float64, device=device)
    F = torch.empty((N, 3), dtype=torch.float64, device=device)
    tb8 = torch.as_tensor(np.asarray(beta8, dtype=np.float64), device=device)
    for c0 in range(0, len(configs), chunk):
        c1 = min(len(configs), c0 + chunk)
        a0, a1, p0, p1 = int(a_off[c0]), int(a_off[c1]), int(p_off[c0]), int(p_off[c1])
        nl = _NL((d_off[a0:a1 + 1] - p0).contiguous(), (d_nbr[p0:p1] - a0).contiguous(),
                 (d_rev[p0:p1] - p0).contiguous())
        tpos = torch.as_tensor(pos_all[a0:a1], device=device)
        out = {"energy": E[a0:a1], "force": F[a0:a1]}
        pot8.compute(tpos, box, nl, tb8, out=out)
        pot4.jacobian(tpos, box, nl, bispectrum=B[a0:a1], jac=J[p0:p1])
    pot8.sync_status()
    pot4.sync_status()
    return Dataset(box, nat, npr, a_off, p_off, d_off, d_nbr, d_rev, B, J, E, F)


def make_surrogate_data(indices, pot8, beta8, pot4, chunk=500):
    cfgs, sig = [], []
    for c in indices:
        pos, box, s = wl.surrogate_config(int(c))
        cfgs.append((pos, box))
        sig.append(s)
    d = build_dataset(cfgs, pot8, beta8, pot4, chunk)
    d.sigma = np.array(sig)
    return d


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------
@dataclass
class TrainConfig:
    epochs: int = 100
    batch_configs: int = 50
    lr: float = 2e-3
    lr_final: float = 2e-5
    w_energy: float = 1.0     # per atom, eV^-2
    w_force: float = 1.0      # per force component, (eV/A)^-2
    seed: int = 0
    margin: float = 0.05
    eval_every: int = 10


def input_statistics(data: Dataset):
    """Mean, standard deviation, min and max of the training descriptors and
    the mean and spread of the energies (bookkeeping on the device)."""
    B = data.B
    mean = B.mean(0)
    std = B.std(0)
    return mean, std, data.E.mean().item(), data.E.std().item()


def evaluate(net: Network, data: Dataset, batch_configs=200):
    """Energy and force RMSE of the network on a dataset (the same kernels as
    training, without the gradient)."""
    import torch
    se = sf = 0.0
    for c0 in range(0, len(data.natoms), batch_configs):
        c1 = min(len(data.natoms), c0 + batch_configs)
        nl, (a0, a1), (p0, p1) = data.batch(c0, c1)
        E, g = net.forward(data.B[a0:a1], gate=False)
        F = snapmi.jacobian_forces(nl, data.J[p0:p1], g)
        _, _, sums = snapmi.fit_residuals(E, data.E[a0:a1], F, data.F[a0:a1], 1.0, 1.0)
        s = sums.sum(0).cpu().numpy()
        se += s[0]
        sf += s[1]
    n = data.n
    return {"energy_rmse": float(np.sqrt(se / n)), "force_rmse": float(np.sqrt(sf / (3 * n)))}


def train(train_data: Dataset, cfg: TrainConfig = TrainConfig(), val_data: Dataset | None = None,
          log=None):
    """Train the network with the library's kernels; returns (net, history)."""
    import torch
    dev = train_data.B.device
    nin = int(train_data.B.shape[1])
    mean, std, e_mean, e_std = input_statistics(train_data)
    net = Network.initial(nin, mean.cpu().numpy(), std.cpu().numpy(), e_mean, e_std, cfg.seed,
                          device=dev)
    # range of the standardised training inputs, for the inference gate
    x = (train_data.B - mean) / std
    net.bounds = torch.stack([x.min(0).values, x.max(0).values]).to(torch.float32).contiguous()
    net.margin = cfg.margin
    del x
    np_ = net.params.numel()
    m = torch.zeros(np_, dtype=torch.float32, device=dev)
    v = torch.zeros(np_, dtype=torch.float32, device=dev)
    nconf = len(train_data.natoms)
    bounds = list(range(0, nconf, cfg.batch_configs)) + [nconf]
    batches = [train_data.batch(bounds[k], bounds[k + 1]) for k in range(len(bounds) - 1)]
    amax = max(a1 - a0 for _, (a0, a1), _ in batches)
    pmax = max(p1 - p0 for _, _, (p0, p1) in batches)
    f64 = dict(dtype=torch.float64, device=dev)
    bufE = torch.empty(amax, **f64)
    bufg = torch.empty((amax, nin), **f64)
    bufF = torch.empty((amax, 3), **f64)
    bufdE = torch.empty((max(pmax, 1), 3), **f64)
    bufr = torch.empty(amax, **f64)
    buflam = torch.empty((amax, 3), **f64)
    bufv = torch.empty((amax, nin), **f64)
    bufs = torch.empty(((amax + 255) // 256, 2), **f64)
    work = torch.empty(snapmi.mlp_workspace(nin, amax), dtype=torch.float32, device=dev)
    grad = torch.empty(np_, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(cfg.seed + 1)
    nsteps = cfg.epochs * len(batches)
    decay = (cfg.lr_final / cfg.lr) ** (1.0 / max(1, nsteps - 1))
    history = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(cfg.epochs):
        for k in rng.permutation(len(batches)):
            nl, (a0, a1), (p0, p1) = batches[k]
            n = a1 - a0
            wE = cfg.w_energy / n
            wF = cfg.w_force / (3 * n)
            E, g = net.forward(train_data.B[a0:a1], energy=bufE[:n], grad_b=bufg[:n], gate=False)
            F = snapmi.jacobian_forces(nl, train_data.J[p0:p1], g, dE=bufdE[:max(p1 - p0, 1)],
                                       force=bufF[:n])
            rE, lam, _ = snapmi.fit_residuals(E, train_data.E[a0:a1], F, train_data.F[a0:a1], wE,
                                              wF, bufr[:n], buflam[:n], bufs)
            vg = snapmi.jacobian_adjoint(nl, train_data.J[p0:p1], lam, nin, out=bufv[:n])
            snapmi.mlp_grad(net.params, net.norm, train_data.B[a0:a1], rE, vg, work, grad)
            step += 1
            snapmi.adam_step(net.params, m, v, grad, cfg.lr * decay ** (step - 1), step)
        if val_data is not None and ((ep + 1) % cfg.eval_every == 0 or ep + 1 == cfg.epochs):
            r = evaluate(net, val_data)
            r.update(epoch=ep + 1, seconds=time.perf_counter() - t0)
            history.append(r)
            if log:
                log(r)
    torch.cuda.synchronize()
    return net, history


# ---------------------------------------------------------------------------
# the method without the network: linear 2J = 4 SNAP fitted by least squares
# ---------------------------------------------------------------------------
def fit_linear(data: Dataset, w_energy=1.0, w_force=1.0, batch_configs=200):
    """Coefficients (beta [N_B], constant) of E_i = beta . B_i + c minimising
    the same weighted energy + force loss.  Force columns come from the
    Jacobian kernels with unit coefficient vectors."""
    import torch
    dev = data.B.device
    nb = int(data.B.shape[1])
    A = torch.zeros((nb + 1, nb + 1), dtype=torch.float64, device=dev)
    y = torch.zeros(nb + 1, dtype=torch.float64, device=dev)
    for c0 in range(0, len(data.natoms), batch_configs):
        c1 = min(len(data.natoms), c0 + batch_configs)
        nl, (a0, a1), (p0, p1) = data.batch(c0, c1)
        n = a1 - a0
        Xe = torch.cat([data.B[a0:a1], torch.ones((n, 1), dtype=torch.float64, device=dev)], 1)
        cols = []
        for l in range(nb):
            g = torch.zeros((n, nb), dtype=torch.float64, device=dev)
            g[:, l] = 1.0
            cols.append(snapmi.jacobian_forces(nl, data.J[p0:p1], g).reshape(-1))
        Xf = torch.stack(cols + [torch.zeros(3 * n, dtype=torch.float64, device=dev)], 1)
        A += w_energy * Xe.T @ Xe + w_force * Xf.T @ Xf
        y += w_energy * Xe.T @ data.E[a0:a1] + w_force * Xf.T @ data.F[a0:a1].reshape(-1)
    sol = torch.linalg.solve(A.cpu(), y.cpu()).numpy()
    return sol[:nb], float(sol[nb])


def evaluate_linear(beta, const, data: Dataset, batch_configs=200):
    import torch
    dev = data.B.device
    tb = torch.as_tensor(np.asarray(beta, dtype=np.float64), device=dev)
    se = sf = 0.0
    for c0 in range(0, len(data.natoms), batch_configs):
        c1 = min(len(data.natoms), c0 + batch_configs)
        nl, (a0, a1), (p0, p1) = data.batch(c0, c1)
        n = a1 - a0
        E = (data.B[a0:a1] @ tb + const).contiguous()
        g = tb.expand(n, -1).contiguous()
        F = snapmi.jacobian_forces(nl, data.J[p0:p1], g)
        _, _, sums = snapmi.fit_residuals(E, data.E[a0:a1], F, data.F[a0:a1], 1.0, 1.0)
        s = sums.sum(0).cpu().numpy()
        se += s[0]
        sf += s[1]
    return {"energy_rmse": float(np.sqrt(se / data.n)),
            "force_rmse": float(np.sqrt(sf / (3 * data.n)))}


# ---------------------------------------------------------------------------
# inference with the range gate, the fallback and the judge
# ---------------------------------------------------------------------------
class SurrogatePotential:
    """E and F from the network on 2J = 4 descriptors; configurations with
    descriptors outside the training range (widened by the margin) fall back
    to plain SNAP with the target coefficients at the high order.

    The range gate writes one of two device flags, alternately: the network
    kernel sets this call's flag and clears the other one for the next call,
    so no separate clearing kernel runs.  The flag is copied to pinned host
    memory behind the step on the same stream; compute(check=True) waits for
    it, compute(check="deferred") returns at once with the check pending and
    resolve() settles it later (a fallback evaluation replaces the result if
    the gate tripped), so that the host never waits inside a step."""

    def __init__(self, net: Network, pot4, pot8, beta8):
        import torch
        self.net, self.pot4, self.pot8 = net, pot4, pot8
        self.beta8 = torch.as_tensor(np.asarray(beta8, dtype=np.float64), device="cuda")
        self.flags = torch.zeros(2, dtype=torch.int32, device="cuda")
        self.host_flags = torch.zeros(2, dtype=torch.int32).pin_memory()
        self.slot = 0
        self._bufs = {}

    def _buffers(self, n):
        import torch
        if self._bufs.get("n") != n:
            f64 = dict(dtype=torch.float64, device="cuda")
            self._bufs = {"n": n, "E": torch.empty(n, **f64),
                          "g": torch.empty((n, self.pot4.ncoeff), **f64),
                          "ones": torch.ones(n, **f64), "F": torch.empty((n, 3), **f64),
                          "B": torch.empty((n, self.pot4.ncoeff), **f64)}
        return self._bufs

    def compute(self, pos, box, nl, check=True):
        """Returns {"energy", "force", "fallback"}.  check=True: the gate is
        read back (the host waits for the step) and a tripped gate gives the
        fallback result; check="deferred": the read-back is enqueued and the
        result carries it as "pending" (see resolve); check=False: the gate
        is evaluated on the device but not read."""
        import torch
        b = self._buffers(pos.shape[0])
        s = self.slot
        self.slot ^= 1
        _, B = self.pot4.forward(pos, box, nl, None, bispectrum=b["B"])
        E, g = self.net.forward(B, flag=self.flags[s:s + 1], energy=b["E"], grad_b=b["g"],
                                clear_flag=self.flags[1 - s:2 - s])
        F = self.pot4.backward(pos, box, nl, g, b["ones"], force=b["F"])
        out = {"energy": E, "force": F, "fallback": False}
        if not check:
            return out
        self.host_flags[s:s + 1].copy_(self.flags[s:s + 1], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        out["pending"] = (ev, s, pos, box, nl)
        if check == "deferred":
            return out
        return self.resolve(out)

    def resolve(self, out):
        """Settle a pending gate check: wait for its read-back and, if the
        gate tripped, replace the result by plain SNAP at the high order."""
        pend = out.pop("pending", None)
        if pend is None:
            return out
        ev, s, pos, box, nl = pend
        ev.synchronize()
        if int(self.host_flags[s]):
            o8 = self.pot8.compute(pos, box, nl, self.beta8)
            out.update({"energy": o8["energy"], "force": o8["force"], "fallback": True})
        return out

    def judge(self, pos, box, nl, out=None):
        """Plain high-order SNAP on the same configuration: force RMSE and
        maximum error of an evaluation, and the reference force RMS."""
        if out is None:
            out = self.compute(pos, box, nl)
        ref = self.pot8.compute(pos, box, nl, self.beta8)
        dF = (out["force"] - ref["force"])
        dE = (out["energy"] - ref["energy"])
        return {"force_rmse": float(dF.pow(2).mean().sqrt()),
                "force_max_err": float(dF.abs().max()),
                "ref_force_rms": float(ref["force"].pow(2).mean().sqrt()),
                "energy_rmse_per_atom": float(dE.pow(2).mean().sqrt()),
                "fallback": bool(out["fallback"])}
