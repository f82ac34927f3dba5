/*
 * snapmi.h -- C ABI of the MI355X (gfx950) SNAP energy-and-force library.
 *
 * The library evaluates the SNAP potential of Gayatri et al., "Rapid
 * Exploration of Optimization Strategies on Advanced Architectures using
 * TestSNAP and LAMMPS" (arXiv 2011.12875), in FP64, with the adjoint
 * formulation of its Sec. IV:
 *   compute_U  -- eq. (u): per-pair hyperspherical harmonics by the
 *                 recursion of eq. (hysphrecur), summed per atom (Sec. VI);
 *   compute_Y  -- eq. (y): Clebsch-Gordan products of eq. (z) weighted by
 *                 the linear coefficients and accumulated into Y_j;
 *   compute_dE -- eq. (snapforce2): per-pair dE = Y : dU^* (Sec. VI,
 *                 "compute_fused_dE"), kept per pair as in Sec. IV;
 *   update_forces -- the per-pair derivatives scattered to atoms.
 * The energy E_i of eq. (snapatomenergy) is returned per atom.
 *
 * Conventions used throughout:
 *   - units: positions and lengths in Angstrom; beta and energies in eV;
 *     forces and pair derivatives in eV/Angstrom;
 *   - twojmax is 2J of the paper (twice the maximum angular momentum);
 *     N_B (snap_ncoeff) bispectrum components are ordered J1 ascending,
 *     J2 = 0..J1, then J ascending, with J2 <= J1 <= J, the triangle rule
 *     and J1+J2+J even (the enumeration of Sec. II.A);
 *   - the neighbour list is a FULL list in CSR form: the pairs of atom i are
 *     p = off[i] .. off[i+1]-1, pair p = (i -> nbr[p]), and rev[p] is the
 *     index of the reverse pair (nbr[p] -> i).  Pairs with r >= rcut are
 *     allowed (a skin) and contribute nothing; i must not appear in its own
 *     list.  Orthorhombic box; box[d] <= 0 means dimension d is not
 *     periodic; a periodic edge must be at least 2*rcut (minimum image);
 *   - "dev" pointers are HIP device pointers, "host" pointers are ordinary
 *     host memory.  The caller owns every buffer it passes; the library owns
 *     its context (tables and workspace) until snap_destroy;
 *   - every call returns SNAP_OK (0) or a negative error code and never
 *     aborts; snap_last_error() gives a message for the last failure of the
 *     calling thread.
 */
#ifndef SNAPMI_H
#define SNAPMI_H

#ifdef __cplusplus
extern "C" {
#endif

#define SNAP_OK 0
#define SNAP_EINVAL (-1) /* an argument is out of range                        */
#define SNAP_EBOX (-2)   /* periodic box edge shorter than 2*rcut              */
#define SNAP_ENBR (-3)   /* neighbour list inconsistent (index, self, reverse) */
#define SNAP_EGEOM (-4)  /* coincident atoms (r < 1e-10 A) or non-finite data  */
#define SNAP_ENOMEM (-5) /* device or host allocation failed                   */
#define SNAP_EDEV (-6)   /* HIP runtime error or no usable gfx950 device       */

#define SNAP_MAX_TWOJMAX 14

typedef struct snap_ctx snap_ctx;

/* Parameters of the potential (Sec. II.A; the 3-sphere map, switching
 * function and self-contribution that the paper omits are fixed here):
 *   theta0 = rfac0 * pi * (r - rmin0) / (rcut - rmin0);
 *   f_c(r) = (cos(pi (r - rmin0)/(rcut - rmin0)) + 1)/2 for rmin0 < r < rcut,
 *            1 for r <= rmin0, and 1 everywhere if switch_flag == 0;
 *   U_j    = wself * identity + sum over neighbours of f_c u_j.           */
typedef struct {
    int twojmax;       /* 0 .. SNAP_MAX_TWOJMAX                               */
    double rcut;       /* > 0                                                 */
    double rfac0;      /* (0, 1]                                              */
    double rmin0;      /* [0, rcut)                                           */
    int switch_flag;   /* 0 or 1                                              */
    double wself;      /* self weight on the diagonal of every U_j (1.0)     */
    int dedr_dirs;     /* directions per lane in compute_dE: 1 or 3 (0: auto,
                        * 3 up to 2J = 6, 1 above)                            */
    int y_kernel;      /* compute_Y variant: 0 auto (the measured faster: rows
                        * through the texture path), 1 rows through the texture
                        * path, 2 U staged in LDS (2 <= 2J <= 8, else as 1)  */
    int dedr_kernel;   /* compute_dE variant: 0 auto (2), 1 tangent form
                        * (one derivative recursion per direction, dedr_dirs
                        * directions per lane), 2 generator form (one walk
                        * of the recursion per pair, three sums independent of
                        * the direction) with Y~ staged in LDS and, from
                        * 2J = 5, the columns split over two wavefronts, 3 as
                        * 2 with Y~ read through the texture path, 4 as 2 with
                        * one wavefront per block of pairs                   */
    int dedr_waves;    /* generator form: wavefronts that split the columns
                        * of a block of 64 pairs, 1 .. 4 (0: auto, 1 up to
                        * 2J = 4, else 2; 3 at 2J = 7 and 8 when the pair
                        * blocks number at most four per compute unit)      */
    int u_kernel;      /* compute_U variant: 0 auto (1), 1 one workgroup per
                        * column of the stored half (two pairs per lane, seed
                        * paths), 2 one pair per lane walking every column,
                        * 3 lanes over the elements of a level, one wavefront
                        * per atom, level J - 1 in LDS (Sec. VI)            */
} snap_params;

/* Create a context for one parameter set.  Builds the host index tables
 * (half-matrix layout of Sec. VI, Clebsch-Gordan coefficients, the Y
 * contraction program); device tables are uploaded on first use.  wself = 1,
 * dedr_dirs = auto.  *out receives the context (owned by the library).
 * Errors: SNAP_EINVAL for out-of-range parameters, SNAP_ENOMEM. */
int snap_setup(int twojmax, double rcut, double rfac0, double rmin0, int switch_flag,
               snap_ctx **out);

/* As snap_setup with every field of snap_params. */
int snap_setup_ex(const snap_params *p, snap_ctx **out);

/* Release the context, its tables and its device workspace. NULL is a no-op. */
int snap_destroy(snap_ctx *c);

/* Number of bispectrum components N_B (14, 55, 204 for 2J = 4, 8, 14;
 * Sec. II.C).  Returns a negative code for a NULL context. */
int snap_ncoeff(const snap_ctx *c);

/* Number of stored (half-matrix) elements of U_j and Y_j over all j: the
 * elements (J, p, q) with q <= J/2 (Sec. VI, symmetry halving). */
int snap_nhalf(const snap_ctx *c);

/* Host copy of a table, for inspection and tests.  which:
 *   0: components, int[3*N_B] (J1, J2, J)
 *   1: half elements, int[3*nhalf] (J, p, q) in storage order
 *   2: Clebsch-Gordan values used on the device, double, one per
 *      (J1, J2, J, M1, M2) in the order of snap_table(3)
 *   3: the keys of table 2, int[5 * count]
 *   4: sizes of the compute_Y program per atom, int[4]: Clebsch-Gordan
 *      products, partial sums (contribution, row, column), contributions
 *      and rows of Y
 * buf has room for cap elements of the table's type; returns the number of
 * elements of the table (which may exceed cap: nothing beyond cap is
 * written), or SNAP_EINVAL. */
int snap_table(const snap_ctx *c, int which, void *buf, int cap);

/* Build a full neighbour list on the host with a cell list (r < rcut).
 *   pos_host[n][3], box[3] as above;
 *   off[n+1], nbr[cap], rev[cap] receive the CSR list (host memory);
 *   *npairs receives the pair count.  Within each atom the neighbours are
 *   sorted by index.  Returns SNAP_OK, SNAP_ENOMEM if cap is too small
 *   (*npairs then holds the required size), SNAP_EBOX, SNAP_EINVAL. */
int snap_build_neighbors(const double *pos_host, int n, const double box[3], double rcut, int *off,
                         int *nbr, int *rev, int cap, int *npairs);

/* Check a host neighbour list: indices in range, no self pairs, off
 * non-decreasing with off[0] = 0 and off[n] = npairs, and rev consistent
 * (rev[rev[p]] == p and the reverse pair joins the same two atoms).
 * Returns SNAP_OK or SNAP_ENBR. */
int snap_check_neighbors(int n, const int *off, const int *nbr, const int *rev, int npairs);

/* SNAP energies and forces (the stage sequence of Sec. IV, Listing 5).
 *   n, npairs       atom and pair counts (host ints; npairs == off[n]);
 *   pos   dev  double[n][3]
 *   box   host double[3]
 *   off   dev  int[n+1], nbr dev int[npairs], rev dev int[npairs]
 *   beta  dev  double[N_B] (per_atom_beta == 0) or double[n][N_B]
 *   energy dev double[n]        E_i (eq. snapatomenergy)
 *   force  dev double[n][3]     F_i = -dE/dr_i
 *   bispec dev double[n][N_B] or NULL: the bispectrum B_i (eq. z)
 *   dE_pair dev double[npairs][3] or NULL: dE_i/dr_ik of pair (i -> k)
 *   stream  hipStream_t (NULL = default stream)
 * Work is enqueued on the stream and the call returns without waiting.
 * Coincident atoms are detected on the device and reported by the next
 * snap_sync_status.  Sizes: n <= 2^24, npairs <= 2^30, and
 * 16 (twojmax + 1) npad < 2^31 with npad = n rounded up to 64 (a row of U_J
 * is addressed with 32-bit byte counts: at most 8 947 840 atoms at 2J = 14,
 * 14 913 024 at 2J = 8).  Errors: SNAP_EINVAL (also for sizes beyond these
 * limits), SNAP_EBOX, SNAP_ENOMEM, SNAP_EDEV. */
int snap_compute(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                 const int *off, const int *nbr, const int *rev, const double *beta,
                 int per_atom_beta, double *energy, double *force, double *bispec,
                 double *dE_pair, void *stream);

/* snap_compute without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * snap_compute; the workspace (U, Y, per-row energy shares, pair derivatives
 * unless dE_pair is given, pair->atom map) is carved from one static device
 * array of 64 MiB per GPU, held until the process ends (2000 atoms at
 * 2J = 14 fit; the call needs about 16 (N_full + N_half) npad + 8 rows npad
 * + 28 npairs bytes).  The call allocates nothing: the context's constant
 * tables must already be on the device (one earlier snap_compute or
 * snap_forward on this context, on the current device), else SNAP_EINVAL;
 * sizes beyond the array are refused with SNAP_EINVAL.  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other threads) race; it does not change the workspace snap_backward and
 * snap_copy_workspace use. */
int snap_compute_noalloc(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                         const int *off, const int *nbr, const int *rev, const double *beta,
                         int per_atom_beta, double *energy, double *force, double *bispec,
                         double *dE_pair, void *stream);

/* Quadratic SNAP: the energy of eq. (snapatomenergy) extended to second
 * order in the bispectrum,
 *   E_i = beta . B_i + (1/2) B_i^T alpha B_i,
 * with forces from the adjoint stages run with the per-atom coefficients
 * g_i = dE_i/dB_i = beta + (1/2)(alpha + alpha^T) B_i (Sec. IV: Y takes any
 * per-atom coefficient vector, so any E_i = f(B_i) gets its forces this way).
 *   beta  dev double[N_B];  alpha dev double[N_B][N_B] (row-major; only its
 *         symmetric part matters)
 * Other arguments, outputs and errors as snap_compute (energy is the
 * quadratic E_i; bispec, if not NULL, receives B_i).  Stages: compute_U,
 * bispectrum, the energy and g_i, compute_Y, compute_dE, update_forces.  The
 * U_j of the call are kept as by snap_compute. */
int snap_compute_quadratic(snap_ctx *c, int n, int npairs, const double *pos,
                           const double box[3], const int *off, const int *nbr, const int *rev,
                           const double *beta, const double *alpha, double *energy,
                           double *force, double *bispec, double *dE_pair, void *stream);

/* Several elements (the density weights and per-element radii that
 * Sec. II.A leaves out of eq. (u), deferring to the SNAP reference it
 * cites).  Element e has radius[e] > 0 and density weight weight[e]; the pair
 * (i, k) has the cutoff R_ik = rcutfac (radius[t_i] + radius[t_k]), used in
 * its 3-sphere map and switching function, and enters U_i as
 * weight[t_k] f_c(r_ik) u_j(r_ik); pairs with r_ik >= R_ik contribute
 * nothing.  The largest cutoff 2 rcutfac max(radius) must not exceed the
 * context's rcut, which stays the neighbour-list cutoff.  Host arrays of
 * nelem (1..64) entries, copied; nelem = 0 removes the elements.
 * Errors: SNAP_EINVAL. */
int snap_set_elements(snap_ctx *c, int nelem, const double *radius, const double *weight,
                      double rcutfac);

/* snap_compute for several elements (after snap_set_elements):
 *   type  dev int[n], the element of each atom (0..nelem-1; a type out of
 *         range is reported by the next snap_sync_status as SNAP_EINVAL)
 *   beta  dev double[nelem][N_B], the coefficients of each element: E_i uses
 *         those of atom i's element (eq. snapatomenergy per element)
 * Other arguments, outputs and errors as snap_compute; the neighbour list is
 * built to the context's rcut. */
int snap_compute_elements(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                          const int *off, const int *nbr, const int *rev, const int *type,
                          const double *beta, double *energy, double *force, double *bispec,
                          double *dE_pair, void *stream);

/* The forward half used by automatic differentiation: compute_U and the
 * bispectrum only.  energy = sum_l beta_l B_l per atom; energy may be NULL
 * (then beta is not read and may be NULL too).  Other arguments as in
 * snap_compute; the context keeps U_j of this call for snap_backward. */
int snap_forward(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                 const int *off, const int *nbr, const int *rev, const double *beta,
                 int per_atom_beta, double *energy, double *bispec, void *stream);

/* The reverse sweep (Sec. IV: the adjoint Y is reverse-mode differentiation
 * of B with respect to U): given g_i = dL/dE_i (dev double[n]), computes
 * force = -dL/dr (dev double[n][3]) with Y built from the per-atom
 * coefficients g_i * beta, using the U_j and pair->atom map kept by the last
 * snap_forward (or snap_compute, snap_jacobian) on the same context and
 * stream.  That call must have had the same n and npairs, and no call that
 * grew the context's workspace may have come in between; otherwise
 * SNAP_EINVAL and nothing is enqueued.  dE_pair as in snap_compute (may be
 * NULL). */
int snap_backward(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                  const int *off, const int *nbr, const int *rev, const double *beta,
                  int per_atom_beta, const double *grad_energy, double *force, double *dE_pair,
                  void *stream);

/* Virial of the pair derivatives of a previous snap_compute (dE_pair, dev
 * double[npairs][3]): the derivative of the total energy with respect to a
 * homogeneous strain r -> (I + eps) r,
 *   virial[3a + b] = sum over pairs p = (i -> k) of dE_p[a] * r_ik[b]
 * (r_ik by minimum image; eq. (snapforce2) gives dE_p per pair, Sec. IV keeps
 * it, and this is the reduction such per-pair storage serves).  virial dev
 * double[9] (row-major 3 x 3), virial_atom dev double[n][9] or NULL: the
 * shares of the pairs of each atom i.  The sums are taken in a fixed order
 * (deterministic).  pos, box, off, nbr as in snap_compute. */
int snap_virial(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                const int *off, const int *nbr, const double *dE_pair, double *virial_atom,
                double *virial, void *stream);

/* Copy an internal per-atom array of the last call into dst (dev memory):
 * which = 0: U_j, which = 1: Y_j.  Layout: double[nhalf][n][2] (element-
 * major, re/im interleaved), elements in the order of snap_table(1).  n must
 * be the atom count of the last forward-type call (it sizes dst); otherwise
 * SNAP_EINVAL. */
int snap_copy_workspace(snap_ctx *c, int which, int n, double *dst, void *stream);

/* Derivative of the weighted energy L = sum_i g_i E_i, E_i = beta . B_i
 * (eq. (snapatomenergy)), with respect to the coefficients: the backward
 * pass of automatic differentiation for beta (Sec. IV treats the adjoint as
 * reverse-mode differentiation; this is its coefficient part).
 *   grad_energy dev double[n]      g_i
 *   bispec      dev double[n][N_B] B_i (from snap_forward or snap_compute)
 *   per_atom = 0: grad_beta dev double[N_B] = sum_i g_i B_i, summed per block
 *                 of 256 atoms and then over the blocks, always in the same
 *                 order (deterministic);
 *   per_atom = 1: grad_beta dev double[n][N_B] = g_i B_i.
 * Errors: SNAP_EINVAL, SNAP_ENOMEM, SNAP_EDEV. */
int snap_beta_grad(snap_ctx *c, int n, const double *grad_energy, const double *bispec,
                   int per_atom, double *grad_beta, void *stream);

/* Stage timing with HIP events recorded on the call's stream, around each
 * stage of every later snap_compute / snap_forward / snap_backward while
 * enabled (enable = 1), off again with enable = 0 (the default).  Stages:
 * 0 compute_U, 1 compute_Y, 2 compute_dE, 3 update_forces (+ energy),
 * 4 bispectrum.  Recording adds one event per stage boundary; the kernels
 * themselves are unchanged. */
int snap_profile(snap_ctx *c, int enable);

/* Wait for the recorded events and return, per stage, the summed elapsed
 * milliseconds (ms[5], host) and the number of launches (launches[5], host)
 * since the last call; then clear the record. */
int snap_stage_times(snap_ctx *c, double ms[5], int launches[5]);

/* Wait for the stream and report a device-side error of the previous calls
 * (SNAP_EGEOM for coincident atoms), clearing it.  SNAP_OK otherwise. */
int snap_sync_status(snap_ctx *c, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *snap_last_error(void);

/* ------------------------------------------------------------------------
 * Learned surrogate on cheap descriptors
 *
 * Eq. (snapatomenergy) is linear in the bispectrum; Sec. IV obtains forces
 * from per-atom coefficients through the adjoint Y of eq. (y), and that route
 * takes any per-atom coefficient vector.  The surrogate replaces beta . B_i by
 * a small network of B_i computed at a low twojmax, E_i = f(x_i) with
 * x_i = (B_i - mean) * scale, and gets its forces from the same adjoint with
 * coefficients g_i = dE_i/dB_i (snap_backward with beta = g,
 * per_atom_beta = 1 and grad_energy = 1).
 *
 * Network: nin -> 64 -> 64 -> 1, SiLU (silu(h) = h / (1 + exp(-h))) after
 * both hidden layers, FP32 weights and FP32 accumulation; nin = 5, 14 or 30
 * (N_B at 2J = 2, 4, 6).  params is one float array, row-major:
 * W1[64][nin], b1[64], W2[64][64], b2[64], w3[64], b3 (snap_mlp_nparams
 * floats).  norm is float[2][nin]: mean, then scale (1 / standard deviation).
 * All pointers below are dev unless marked host; calls enqueue on stream and
 * return without waiting.
 * ------------------------------------------------------------------------ */

/* Parameter count of the network for nin inputs (5185 for nin = 14), or
 * SNAP_EINVAL for an unsupported nin. */
int snap_mlp_nparams(int nin);

/* Floats of workspace snap_mlp_grad needs for n atoms (< 0 on bad input). */
long long snap_mlp_workspace(int nin, int n);

/* Energies and input gradients of the network.
 *   bispec  double[n][nin]   B_i
 *   energy  double[n]        E_i = f(x_i)
 *   grad_b  double[n][nin]   g_i = dE_i/dB_i
 *   bounds  float[2][nin] or NULL: per input, the low and high end of the
 *           range seen in training, in standardised units.  If any x_i,k lies
 *           outside [lo - margin (hi - lo), hi + margin (hi - lo)] or is not
 *           finite, *ood_flag is set to 1 (it is never cleared here).
 *   ood_flag int[1] or NULL.
 *   clear_flag int[1] or NULL: set to 0 by the launch, for the next call
 *           (two flags used alternately need no separate clearing; it must
 *           not be ood_flag).
 * Errors: SNAP_EINVAL, SNAP_EDEV. */
int snap_mlp_forward(int nin, int n, const float *params, const float *norm,
                     const float *bounds, float margin, const double *bispec, double *energy,
                     double *grad_b, int *ood_flag, int *clear_flag, void *stream);

/* Parameter gradient of  Phi = sum_i dl_de_i E_i + dl_dg_i . g_i  (grad,
 * float[nparams], overwritten): back-propagation for the first term,
 * forward-over-reverse differentiation for the second, so that a loss on
 * energies and on forces (through dl_dg, see snap_jacobian_adjoint) is
 * differentiated exactly.  dl_de double[n]; dl_dg double[n][nin] or NULL;
 * work float[snap_mlp_workspace(nin, n)].  Per-block partial sums are added in
 * a fixed order: the result is deterministic.  Errors: SNAP_EINVAL, SNAP_EDEV. */
int snap_mlp_grad(int nin, int n, const float *params, const float *norm, const double *bispec,
                  const double *dl_de, const double *dl_dg, float *work, float *grad,
                  void *stream);

/* One Adam step (Kingma and Ba, 2015) on np parameters: m and v (float[np],
 * zero before step 1) are the moment estimates, step >= 1 the step number for
 * the bias corrections 1 - beta^step.  Errors: SNAP_EINVAL, SNAP_EDEV. */
int snap_adam_step(int np, float *params, float *m, float *v, const float *grad, float lr,
                   float beta1, float beta2, float eps, int step, void *stream);

/* Descriptor Jacobian: the bispectrum B_i (eq. (z)) and, per pair
 * p = (i -> k), J_p = dB_i/dr_ik (eq. (dbidrk), kept per neighbour as the
 * compute_dB stage of Sec. II.B does, here obtained from the adjoint stages
 * with one unit coefficient vector per component: compute_Y with beta = e_l,
 * then compute_dE).
 *   bispec double[n][N_B] or NULL;  jac float[npairs][N_B][3].
 * Other arguments as in snap_compute.  Keeps U_j like snap_forward. */
int snap_jacobian(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                  const int *off, const int *nbr, const int *rev, double *bispec, float *jac,
                  void *stream);

/* Forces of per-atom energies with input gradients g_i from a stored
 * Jacobian: dE_p = J_p^T g_i per pair (dE_pair double[npairs][3], written),
 * then update_forces as in snap_compute (force double[n][3]).  off, rev as in
 * snap_compute; jac float[npairs][nin][3]; grad_b double[n][nin]. */
int snap_jacobian_forces(int nin, int n, int npairs, const int *off, const int *rev,
                         const float *jac, const double *grad_b, double *dE_pair, double *force,
                         void *stream);

/* Reverse of snap_jacobian_forces: for dl_dforce = dL/dF (double[n][3]),
 * dl_dg_i = sum over pairs p = (i -> k) of J_p (dl_dforce_i - dl_dforce_k)
 * (double[n][nin]). */
int snap_jacobian_adjoint(int nin, int n, int npairs, const int *off, const int *nbr,
                          const float *jac, const double *dl_dforce, double *dl_dg, void *stream);

/* Residuals of the loss L = w_energy sum_i (E_i - Eref_i)^2
 *                          + w_force sum_i |F_i - Fref_i|^2:
 * dl_de double[n] = 2 w_energy (E - Eref), dl_dforce double[n][3] =
 * 2 w_force (F - Fref), and sums double[ceil(n/256)][2], per block of 256
 * atoms, of (E - Eref)^2 and |F - Fref|^2. */
int snap_fit_residuals(int n, const double *energy, const double *energy_ref,
                       const double *force, const double *force_ref, double w_energy,
                       double w_force, double *dl_de, double *dl_dforce, double *sums,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SNAPMI_H */
