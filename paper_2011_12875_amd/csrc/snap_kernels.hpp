// snap_kernels.hpp -- launch interface between the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "snap_tables.hpp"

namespace snapmi {

struct Geom {
    double rcut, rfac0, rmin0, wself;
    double box[3];
    double ibox[3];  // 1 / box (0 on open axes)
    int switch_flag;
    // several elements (type == nullptr: one element, cutoff rcut, unit
    // weights): the pair (i, k) has the cutoff rcutfac (erad[t_i] + erad[t_k])
    // and density weight ewt[t_k]; device arrays
    const int *type = nullptr;
    const double *erad = nullptr, *ewt = nullptr;
    double rcutfac = 0.0;
    int nelem = 0;
};

// Device copies of the tables of one context.
struct DevTables {
    double *unscale_y = nullptr;
    int *half2full = nullptr;
    UInfo *uinfo = nullptr;
    BTerm *bterms = nullptr;
    BItem *bitems = nullptr;
    int *bl_begin = nullptr;
    YContrib *ycontrib = nullptr;
    YRowC *yrows = nullptr;
    double *ycp = nullptr, *ycq = nullptr, *nfull = nullptr;
    double *onehot = nullptr;  // identity [nb][nb]: unit coefficient vectors
    int nyrows = 0;
    int nhalf = 0;  // stored-half elements per atom (the row length of Y~)
    int ncu = 0;    // compute units of the device
    // LDS-staged compute_Y (used when y_lds is set and 2J is in range)
    YLContrib *ylcontrib = nullptr;
    double *ylcp = nullptr;
    YLTask *yltask = nullptr;
    YLGroup *ylgroup = nullptr;
    int yl_task_off[kYLdsGroupings] = {-1, -1, -1, -1};
    int yl_group_off[kYLdsGroupings] = {-1, -1, -1, -1};
    long yl_cost_total = 0;
    bool y_lds = false;           // the tables are on the device
    bool y_lds_selected = false;  // and the LDS kernel is the one to run
};
// smallest 2J for which the LDS-staged compute_Y is built
constexpr int kYLdsMinTJ = 2;

// Per-call device workspace.  U is element-major, U[e * npad + atom] (npad =
// n rounded up to 64), full matrices (sum (J+1)^2 elements): compute_Y reads
// one element of 64 consecutive atoms per load.  Y holds the scaled stored
// half atom-major, Y[atom * nhalf + e]: compute_dE reads the elements of one
// atom (a lane's, or a wavefront's) at immediate offsets from one base.
struct Work {
    double2 *U = nullptr, *Y = nullptr;
    double *dE = nullptr;
    double *Epart = nullptr;  // [nyrows][npad] per-row shares of the energy
    int *pair_atom = nullptr;
    int *flag = nullptr;
    int npad = 0;
};

// variant 1: one workgroup per column of the stored half; 2: one pair per lane;
// 3: lanes over the elements of a level
hipError_t launch_compute_u(int twojmax, int variant, int n, int npad, const double *pos,
                            const int *off, const int *nbr, const DevTables &T, const Geom &g,
                            double2 *U, int *pair_atom, int *flag, hipStream_t s);

// coefficients: beta[nb] shared, beta[n][nb] per atom (per_atom_beta), or
// beta[nelem][nb] per element of btype[n] (btype not NULL)
hipError_t launch_compute_y(int twojmax, int n, int npad, const double2 *U, double2 *Y,
                            const DevTables &T, const double *beta, int per_atom_beta, int nb,
                            const int *btype, int nelem, const double *gscale, double *Epart,
                            hipStream_t s);

// B (and, when energy is not NULL, energy = beta . B); nfull = number of full
// U elements (small 2J stage U in LDS)
hipError_t launch_bispectrum(int n, int npad, const double2 *U, const DevTables &T, int nb,
                             double *B, const double *beta, int per_atom_beta, double *energy,
                             hipStream_t s, int nfull);

// tangent form (snap_dedr.hip); nh = row length of the atom-major Y~
hipError_t launch_dedr_low(int twojmax, int dirs, int npairs, int nh, const double *pos,
                           const int *nbr, const int *pair_atom, const double2 *Y,
                           const DevTables &T, const Geom &g, double *dE, hipStream_t s);
hipError_t launch_dedr_high(int twojmax, int dirs, int npairs, int npad, const double *pos,
                            const int *nbr, const int *pair_atom, const double2 *Y,
                            const DevTables &T, const Geom &g, double *dE, hipStream_t s);
inline hipError_t launch_dedr(int twojmax, int dirs, int npairs, int npad, const double *pos,
                              const int *nbr, const int *pair_atom, const double2 *Y,
                              const DevTables &T, const Geom &g, double *dE, hipStream_t s)
{
    return twojmax <= 8
               ? launch_dedr_low(twojmax, dirs, npairs, npad, pos, nbr, pair_atom, Y, T, g, dE, s)
               : launch_dedr_high(twojmax, dirs, npairs, npad, pos, nbr, pair_atom, Y, T, g, dE, s);
}

// compute_dE in the generator form (snap_dedr_gen.hip): mapping 0 with the
// block's rows of Y~ staged in LDS, 1 read through the texture path; waves =
// wavefronts per block of pairs (0: auto); ncu = compute units (blocks are
// sized so that every unit runs the same number); nh = row length of the
// atom-major Y~
hipError_t launch_dedr_gen(int twojmax, int mapping, int waves, int ncu, int npairs, int nh,
                           const double *pos, const int *nbr, const int *pair_atom,
                           const double2 *Y, const Geom &g, double *dE, hipStream_t s);

// the static workspace of snap_compute_noalloc (snap_static.hip): its size,
// this device's address of it (looked up once per device), and the zeroing of
// the padding atoms of U (element-major) and Y (atom-major)
size_t static_scratch_bytes();
hipError_t static_scratch(void **out);
hipError_t launch_zero_padding(double2 *U, int nfull, double2 *Y, int nhalf, int n, int npad,
                               hipStream_t s);

hipError_t launch_gather(int n, int npad, int nrows, const int *off, const int *rev,
                         const double *dE, const double *Epart, double *energy, double *force,
                         hipStream_t s);

// virial W[a][b] = sum_p dE_p[a] r_ik[b]: per atom into watom[n][9] (if not
// NULL), per block of 256 atoms into partial[ceil(n/256)][9], total into out[9]
hipError_t launch_virial(int n, const double *pos, const int *off, const int *nbr, const Geom &g,
                         const double *dE, double *watom, double *partial, double *out,
                         hipStream_t s);

// quadratic SNAP: energy[n] = beta . B_i + B_i^T alpha B_i / 2 and
// g[n][nb] = beta + (alpha + alpha^T) B_i / 2 (B [n][nb], alpha [nb][nb])
hipError_t launch_quadratic(int n, int nb, const double *B, const double *beta,
                            const double *alpha, double *energy, double *g, hipStream_t s);

// dE/dbeta of sum_i g_i E_i: out[nb] = sum_i g_i B[i][:] in a fixed order
// (part: beta_grad_blocks(n) * nb doubles), or out[n][nb] = g_i B[i][:]
int beta_grad_blocks(int n);
hipError_t launch_beta_grad(int n, int nb, const double *g, const double *B, int per_atom,
                            double *part, double *out, hipStream_t s);

// dst[e][atom][re/im] = scale[e] * src[map[e] * se + atom * sa] for atom < n
// (element-major: se = npad, sa = 1; atom-major: se = 1, sa = row length)
hipError_t launch_unscale(int n, int se, int sa, int nhalf, const double2 *src, const int *map,
                          const double *scale, double *dst, hipStream_t s);

// ---------------------------------------------------------------------------
// surrogate network and descriptor Jacobian (snap_mlp.hip)
// ---------------------------------------------------------------------------
constexpr int kMlpHidden = 64;     // width of both hidden layers
constexpr int kMlpGradAtoms = 64;  // atoms per block of the parameter gradient

bool mlp_supported(int nin);
int mlp_nparams(int nin);
// floats of workspace launch_mlp_grad needs for n atoms
size_t mlp_grad_workspace(int nin, int n);

hipError_t launch_mlp_forward(int nin, int n, const float *prm, const float *norm,
                              const float *bounds, float margin, const double *B, double *E,
                              double *g, int *flag, int *clear_flag, hipStream_t s);
hipError_t launch_mlp_grad(int nin, int n, const float *prm, const float *norm, const double *B,
                           const double *rE, const double *v, float *work, float *grad,
                           hipStream_t s);
hipError_t launch_adam(int np, float *prm, float *m, float *v, const float *grad, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_pack_jac(int npairs, int nb, int l, const double *dE, float *jac, hipStream_t s);
hipError_t launch_jac_force(int nin, int n, int npairs, const int *off, const float *jac,
                            const double *g, double *dE, hipStream_t s);
hipError_t launch_jac_adjoint(int nin, int n, const int *off, const int *nbr, const float *jac,
                              const double *lam, double *v, hipStream_t s);
hipError_t launch_residuals(int n, const double *E, const double *Eref, const double *F,
                            const double *Fref, double wE, double wF, double *rE, double *lam,
                            double *sums, hipStream_t s);

}  // namespace snapmi
