"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no SNAP arithmetic: it only draws positions and
coefficients.  The paper measures on a tungsten SNAP input (2000 atoms, 26
neighbours per atom, Sec. II.C and Table I) whose trained coefficients are
not available; a body-centred-cubic lattice with the same shape stands in for
it: lattice constant 3.1803 A, so the first three shells (8 at 2.754 A, 6 at
3.180 A, 12 at 4.498 A) give 26 neighbours inside rcut = 4.73 A, the next
shell sits at 5.274 A.  Coefficients are drawn from N(0, 0.1^2) (0.1 is the
standard deviation).
"""
from __future__ import annotations

import numpy as np

A_BCC = 3.1803
RCUT = 4.73
RFAC0 = 0.99363
RMIN0 = 0.0


def bcc(ncell, sigma: float, seed: int, a: float = A_BCC, open_axes=()):
    """BCC crystal of ncell^3 cubic cells (or nx x ny x nz for a tuple: an
    orthorhombic box) with Gaussian displacements.

    Atom order is cell-major: index = ((ix*ny + iy)*nz + iz)*2 + basis.
    Returns (pos [N,3] float64 wrapped into [0, L), box [3]); the axes in
    open_axes are not periodic (box entry 0, positions not wrapped).
    """
    nx, ny, nz = (ncell, ncell, ncell) if np.isscalar(ncell) else tuple(ncell)
    rng = np.random.default_rng(seed)
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    corner = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    sites = (corner[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    L = np.array([nx, ny, nz], dtype=np.float64) * a
    pos = sites + rng.normal(0.0, sigma, size=sites.shape)
    for d in range(3):
        if d in open_axes:
            L[d] = 0.0
        else:
            pos[:, d] = np.mod(pos[:, d], L[d])
    return np.ascontiguousarray(pos), L


def bcc_with_vacancies(ncell: int, nvac: int, sigma: float, vac_seed: int, pos_seed: int,
                       a: float = A_BCC):
    """BCC crystal with nvac sites removed at random, then displaced."""
    sites, box = bcc(ncell, 0.0, 0, a)
    rng_v = np.random.default_rng(vac_seed)
    drop = rng_v.choice(len(sites), size=nvac, replace=False)
    keep = np.setdiff1d(np.arange(len(sites)), drop)
    sites = sites[keep]
    rng = np.random.default_rng(pos_seed)
    pos = np.mod(sites + rng.normal(0.0, sigma, size=sites.shape), box[0])
    return np.ascontiguousarray(pos), box


def cluster(natoms: int, radius: float, seed: int, min_dist: float = 1.8):
    """Random isolated cluster inside a sphere (non-periodic box)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < natoms:
        p = rng.uniform(-radius, radius, size=3)
        if np.linalg.norm(p) > radius:
            continue
        if all(np.linalg.norm(p - q) >= min_dist for q in pts):
            pts.append(p)
    return np.ascontiguousarray(np.array(pts)), np.array([0.0, 0.0, 0.0])


def beta(ncoeff: int, seed: int, sd: float = 0.1, natoms: int | None = None):
    """Linear coefficients ~ N(0, sd^2): shape [ncoeff] or [natoms, ncoeff]."""
    rng = np.random.default_rng(seed)
    shape = (ncoeff,) if natoms is None else (natoms, ncoeff)
    return rng.normal(0.0, sd, size=shape)


def quadratic_alpha(ncoeff: int, seed: int, scale: float = 1e-4):
    """Synthetic quadratic coefficients: scale (G + G^T)/2 with G ~ N(0, 1)
    (symmetric, [ncoeff, ncoeff]).  With bispectra of rms ~40 at the BCC
    workloads, 1e-4 makes the quadratic energy comparable to the linear one."""
    g = np.random.default_rng(seed).normal(0.0, 1.0, size=(ncoeff, ncoeff))
    return scale * 0.5 * (g + g.T)


def ncoeff(twojmax: int) -> int:
    """Number of bispectrum components for a given twojmax (counting only)."""
    n = 0
    for j1 in range(twojmax + 1):
        for j2 in range(j1 + 1):
            for j in range(j1 - j2, min(twojmax, j1 + j2) + 1, 2):
                if j >= j1:
                    n += 1
    return n


# Named workloads (sizes of the paper's benchmark and its variations).
WORKLOADS = {
    # 128 atoms, 2J=4: small parity case
    "bcc128_2j4": dict(ncell=4, sigma=0.05, pos_seed=1, beta_seed=2, twojmax=4),
    # 2000 atoms, 26 neighbours, 2J=8: the paper's benchmark shape
    "bcc2000_2j8": dict(ncell=10, sigma=0.05, pos_seed=3, beta_seed=4, twojmax=8),
    # same positions, 2J=14 (204 components)
    "bcc2000_2j14": dict(ncell=10, sigma=0.05, pos_seed=3, beta_seed=5, twojmax=14),
    # 16000 sites, 800 vacancies, sigma 0.15: uneven 16-30 neighbours
    "bcc15200vac_2j8": dict(ncell=20, nvac=800, sigma=0.15, vac_seed=6, pos_seed=7, beta_seed=4,
                            twojmax=8),
}


# Several elements (synthetic; the paper's benchmark has one element): the
# positions of a one-element workload, each atom given an element at random
# (fraction frac of element 1), per-element radius and density weight, pair
# cutoff rcutfac (R_t_i + R_t_k) (the largest, 2 * 2.365, is RCUT), and
# coefficients per element.
ELEMENT_WORKLOADS = {
    "bcc2000_2j8_2el": dict(base="bcc2000_2j8", radius=(2.365, 2.05), weight=(1.0, 0.62),
                            rcutfac=1.0, frac=0.5, type_seed=14, beta_seed=15),
    "bcc128_2j4_3el": dict(base="bcc128_2j4", radius=(2.365, 2.05, 2.2), weight=(1.0, 0.62, 1.3),
                           rcutfac=1.0, frac=None, type_seed=16, beta_seed=17),
}


def make_elements(name: str):
    """(pos, box, types int32 [n], radius, weight, rcutfac, beta [nelem, N_B],
    twojmax) for a named several-element workload."""
    w = ELEMENT_WORKLOADS[name]
    pos, box, _, tj = make(w["base"])
    nelem = len(w["radius"])
    rng = np.random.default_rng(w["type_seed"])
    if w["frac"] is not None and nelem == 2:
        types = (rng.random(len(pos)) < w["frac"]).astype(np.int32)
    else:
        types = rng.integers(0, nelem, len(pos)).astype(np.int32)
    b = np.stack([beta(ncoeff(tj), w["beta_seed"] + e) for e in range(nelem)])
    return (pos, box, types, np.array(w["radius"]), np.array(w["weight"]), w["rcutfac"], b, tj)


def make(name: str):
    """Return (pos, box, beta, twojmax) for a named workload."""
    w = WORKLOADS[name]
    if "nvac" in w:
        pos, box = bcc_with_vacancies(w["ncell"], w["nvac"], w["sigma"], w["vac_seed"], w["pos_seed"])
    else:
        pos, box = bcc(w["ncell"], w["sigma"], w["pos_seed"])
    b = beta(ncoeff(w["twojmax"]), w["beta_seed"])
    return pos, box, b, w["twojmax"]


# ---------------------------------------------------------------------------
# Learned surrogate: training configurations, target coefficients, inference
# and out-of-range configurations.
# ---------------------------------------------------------------------------
SURROGATE = dict(
    ncell_train=5,          # 250 atoms per configuration, L = 15.9015 A
    n_configs=10000,
    sigma_range=(0.02, 0.2),
    config_seed0=10000,     # configuration c draws sigma_c and positions from seed 10000 + c
    split_seed=11,
    split=(8000, 1000, 1000),
    target_seed=9,          # target coefficients of the 2J = 8 potential
    target_decay=0.3,       # per unit of J above 4, in amplitude: decay ** ((J - 4) / 2)
    model_twojmax=4,
    label_twojmax=8,
    ncell_infer=20, sigma_infer=0.1, infer_seed=12,   # 16000 atoms
    sigma_ood=0.35, ood_seed=13,
)


def components(twojmax: int):
    """(J1, J2, J) of each bispectrum component in the library's order
    (counting only)."""
    out = []
    for j1 in range(twojmax + 1):
        for j2 in range(j1 + 1):
            for j in range(j1 - j2, min(twojmax, j1 + j2) + 1, 2):
                if j >= j1:
                    out.append((j1, j2, j))
    return out


def surrogate_config(c: int, ncell: int | None = None):
    """Training configuration c: BCC of ncell^3 cells (5 by default) with
    Gaussian displacements of a width sigma_c ~ U(sigma_range); sigma_c and
    the displacements come from seed config_seed0 + c.  Returns (pos, box,
    sigma_c)."""
    s = SURROGATE
    ncell = ncell or s["ncell_train"]
    sites, box = bcc(ncell, 0.0, 0)
    rng = np.random.default_rng(s["config_seed0"] + c)
    sigma = rng.uniform(*s["sigma_range"])
    pos = np.mod(sites + rng.normal(0.0, sigma, size=sites.shape), box[0])
    return np.ascontiguousarray(pos), box, sigma


def surrogate_split():
    """(train, val, test) configuration indices."""
    s = SURROGATE
    perm = np.random.default_rng(s["split_seed"]).permutation(s["n_configs"])
    a, b, _ = s["split"]
    return perm[:a], perm[a:a + b], perm[a + b:]


def surrogate_target_beta(decay: float | None = None):
    """Target coefficients of the 2J = 8 potential: N(0, 0.1^2) draws from
    target_seed, scaled by decay ** ((J - 4) / 2) for components whose J
    exceeds 4 (decay = 1 leaves them undamped)."""
    s = SURROGATE
    decay = s["target_decay"] if decay is None else decay
    b = beta(ncoeff(s["label_twojmax"]), s["target_seed"])
    damp = np.array([decay ** (max(0, j - 4) / 2.0) for (_, _, j) in components(s["label_twojmax"])])
    return b * damp


def surrogate_inference_config(ood: bool = False):
    """The 16000-atom inference configuration (sigma 0.1) or, with ood, the
    out-of-range one (sigma 0.35)."""
    s = SURROGATE
    if ood:
        return bcc(s["ncell_infer"], s["sigma_ood"], s["ood_seed"])
    return bcc(s["ncell_infer"], s["sigma_infer"], s["infer_seed"])
