// snap_mlp.hip -- kernels of the learned surrogate: a per-atom network
// nin -> 64 -> 64 -> 1 with SiLU activations on standardised bispectrum
// components, E_i = f(x_i), x_i = (B_i - mean) * scale, FP32 weights and FP32
// accumulation, and what training it needs.
//
//   k_mlp_forward_w E_i, g_i = dE_i/dB_i (the per-atom coefficients that the
//                   SNAP adjoint turns into forces) and an out-of-range flag;
//   k_mlp_grad      per block of 64 atoms, d/dtheta of
//                   sum_i r_i E_i + v_i . g_i  for given r_i and v_i: ordinary
//                   back-propagation for the energy term and
//                   forward-over-reverse for the force term;
//   k_reduce_rows   sums the per-block gradients in a fixed order (the result
//                   does not depend on scheduling);
//   k_adam          one Adam step;
//   k_pack_jac      stores one component of the descriptor Jacobian
//                   J_p = dB_i/dr_ik (pair p = i -> k), FP32;
//   k_jac_force     dE_p = J_p^T g_i (forces then follow from update_forces);
//   k_jac_adjoint   v_i = sum_{p of i} J_p (lambda_i - lambda_k): a force
//                   loss with dL/dF = lambda, pulled back to g;
//   k_residuals     r_i, lambda_i and the squared errors of a weighted
//                   energy + force loss.
// Lanes are atoms (or pairs); the weights are read with wavefront-uniform
// addresses, so they come through the scalar cache.
#include <hip/hip_runtime.h>

#include "snap_kernels.hpp"

namespace snapmi {

namespace {

constexpr int H = kMlpHidden;
constexpr int T = kMlpGradAtoms;
constexpr int HP = H + 1;  // padded LDS row: lanes reading [lane][k] hit distinct banks

template <int NIN>
struct MlpLayout {
    static constexpr int W1 = 0;               // W1[j][k], j < H, k < NIN
    static constexpr int B1 = W1 + H * NIN;
    static constexpr int W2 = B1 + H;          // W2[j][k], j, k < H
    static constexpr int B2 = W2 + H * H;
    static constexpr int W3 = B2 + H;          // w3[j]
    static constexpr int B3 = W3 + H;
    static constexpr int NP = B3 + 1;
};

// silu(h) = h s, s = 1/(1+exp(-h)); silu' = s (1 + h (1 - s));
// silu'' = s (1 - s) (2 + h (1 - 2 s)).
__device__ __forceinline__ void silu3(float h, float &a, float &d1, float &d2)
{
    const float s = 1.0f / (1.0f + __expf(-h));
    a = h * s;
    d1 = s * (1.0f + h * (1.0f - s));
    d2 = s * (1.0f - s) * (2.0f + h * (1.0f - 2.0f * s));
}

__device__ __forceinline__ void silu2(float h, float &a, float &d1)
{
    const float s = 1.0f / (1.0f + __expf(-h));
    a = h * s;
    d1 = s * (1.0f + h * (1.0f - s));
}

// The network on a workgroup of four wavefronts and 64 atoms (lane = atom
// in every wavefront): E_i, g_i = dE_i/dB_i and the range gate.  Wavefront
// w computes hidden units
// 16w .. 16w+15 of both layers, so the weights stay wavefront-uniform
// (scalar loads) while four times as many wavefronts share the work.
// Activations and partial sums are exchanged through LDS (unit-major,
// atom-contiguous rows: conflict-free).
constexpr int kFwdWaves = 4;
constexpr int kFwdUnits = H / kFwdWaves;

template <int NIN>
__global__ __launch_bounds__(64 * kFwdWaves) void k_mlp_forward_w(
    int n, const float *__restrict__ prm, const float *__restrict__ norm,
    const float *__restrict__ bounds, float margin, const double *__restrict__ B,
    double *__restrict__ E, double *__restrict__ g, int *__restrict__ flag,
    int *__restrict__ clear_flag)
{
    using L = MlpLayout<NIN>;
    // the flag of the next call (no workgroup of this launch touches it)
    if (clear_flag && blockIdx.x == 0 && threadIdx.x == 0) clear_flag[0] = 0;
    __shared__ float a1s[H][64];               // a1 of the block's atoms
    __shared__ float part[kFwdWaves][H][64];   // per-wave partial dE/da1, then dE/dx
    __shared__ float es[kFwdWaves][64];        // per-wave partial energies
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int u0 = w * kFwdUnits;
    const int i = blockIdx.x * 64 + lane;
    const int ia = i < n ? i : n - 1;
    float x[NIN];
    bool out = false;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
        x[k] = (float)((B[(size_t)ia * NIN + k] - (double)norm[k]) * (double)norm[NIN + k]);
        if (bounds && w == 0) {
            const float lo = bounds[k], hi = bounds[NIN + k], wd = margin * (hi - lo);
            out |= !(x[k] >= lo - wd && x[k] <= hi + wd);  // also catches NaN
        }
    }
    // layer 1, own units
    float s1[kFwdUnits];
#pragma unroll
    for (int jj = 0; jj < kFwdUnits; ++jj) {
        const int j = u0 + jj;
        float h = prm[L::B1 + j];
#pragma unroll
        for (int k = 0; k < NIN; ++k) h += prm[L::W1 + j * NIN + k] * x[k];
        float a;
        silu2(h, a, s1[jj]);
        a1s[j][lane] = a;
    }
    __syncthreads();
    // layer 2, own units; partial back-propagation to all of a1
    float a1[H], d1[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        a1[k] = a1s[k][lane];
        d1[k] = 0.0f;
    }
    float e = 0.0f;
    for (int jj = 0; jj < kFwdUnits; ++jj) {
        const int j = u0 + jj;
        float h = prm[L::B2 + j];
#pragma unroll
        for (int k = 0; k < H; ++k) h += prm[L::W2 + j * H + k] * a1[k];
        float a2, s2;
        silu2(h, a2, s2);
        const float w3 = prm[L::W3 + j];
        e += w3 * a2;
        const float d2 = w3 * s2;
#pragma unroll
        for (int k = 0; k < H; ++k) d1[k] += prm[L::W2 + j * H + k] * d2;
    }
#pragma unroll
    for (int k = 0; k < H; ++k) part[w][k][lane] = d1[k];
    es[w][lane] = e;
    __syncthreads();
    // own units of layer 1: sum the four partials, through silu', to dE/dx
    float gx[NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) gx[m] = 0.0f;
#pragma unroll
    for (int jj = 0; jj < kFwdUnits; ++jj) {
        const int j = u0 + jj;
        float d = 0.0f;
#pragma unroll
        for (int v = 0; v < kFwdWaves; ++v) d += part[v][j][lane];
        d *= s1[jj];
#pragma unroll
        for (int m = 0; m < NIN; ++m) gx[m] += prm[L::W1 + j * NIN + m] * d;
    }
    __syncthreads();  // everyone has read part: reuse it for dE/dx
#pragma unroll
    for (int m = 0; m < NIN; ++m) part[w][m][lane] = gx[m];
    __syncthreads();
    if (w == 0 && i < n) {
        float et = prm[L::B3];
#pragma unroll
        for (int v = 0; v < kFwdWaves; ++v) et += es[v][lane];
        E[i] = (double)et;
#pragma unroll
        for (int m = 0; m < NIN; ++m) {
            float gm = 0.0f;
#pragma unroll
            for (int v = 0; v < kFwdWaves; ++v) gm += part[v][m][lane];
            g[(size_t)i * NIN + m] = (double)gm * (double)norm[NIN + m];
        }
        if (out && flag) flag[0] = 1;
    }
}

// Per-atom vectors of one block, kept for the parameter sums.
template <int NIN>
struct GradLds {
    float a1[T][HP];    // a1
    float ad1[T][HP];   // tangent of a1 along u
    float d2[T][HP];    // dPhi/dh2
    float t2[T][HP];    // dPhi/d(tangent of h2)
    float q3[T][HP];    // dPhi/dw3
    float h1b[T][HP];   // dPhi/dh1
    float hd1b[T][HP];  // dPhi/d(tangent of h1)
    float x[T][NIN + 1];
    float u[T][NIN + 1];
    float r[T];
};

// Phi = sum_i r_i f(x_i) + u_i . grad_x f(x_i), u_i = v_i * scale (so that
// u_i . grad_x f = v_i . g_i).  The tangent pass along u (h1' = W1 u,
// a1' = silu'(h1) h1', h2' = W2 a1', y' = w3 . (silu'(h2) h2') = u . grad_x f)
// runs with the primal pass and both are differentiated in reverse.
// Lanes are atoms for the network passes and parameters for the sums.
template <int NIN>
__global__ __launch_bounds__(64) void k_mlp_grad(int n, const float *__restrict__ prm,
                                                 const float *__restrict__ norm,
                                                 const double *__restrict__ B,
                                                 const double *__restrict__ rE,
                                                 const double *__restrict__ v,
                                                 float *__restrict__ partial)
{
    using L = MlpLayout<NIN>;
    __shared__ GradLds<NIN> S;
    const int a = threadIdx.x;
    const int i = blockIdx.x * T + a;
    const bool ok = i < n;
    const int ia = ok ? i : n - 1;
    // primal and tangent of layer 1
    {
        float x[NIN], u[NIN];
#pragma unroll
        for (int k = 0; k < NIN; ++k) {
            x[k] = (float)((B[(size_t)ia * NIN + k] - (double)norm[k]) * (double)norm[NIN + k]);
            u[k] = (ok && v) ? (float)(v[(size_t)ia * NIN + k] * (double)norm[NIN + k]) : 0.0f;
            S.x[a][k] = x[k];
            S.u[a][k] = u[k];
        }
        S.r[a] = ok ? (float)rE[ia] : 0.0f;
#pragma unroll 4
        for (int j = 0; j < H; ++j) {
            float h = prm[L::B1 + j], hd = 0.0f;
#pragma unroll
            for (int k = 0; k < NIN; ++k) {
                const float w = prm[L::W1 + j * NIN + k];
                h += w * x[k];
                hd += w * u[k];
            }
            float av, s1;
            silu2(h, av, s1);
            S.a1[a][j] = av;
            S.ad1[a][j] = s1 * hd;
        }
    }
    // layer 2 and the output: dPhi/dh2, dPhi/dh2', dPhi/dw3
    {
        const float r = S.r[a];
        float a1[H], ad1[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            a1[k] = S.a1[a][k];
            ad1[k] = S.ad1[a][k];
        }
        for (int j = 0; j < H; ++j) {
            float h = prm[L::B2 + j], hd = 0.0f;
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const float w = prm[L::W2 + j * H + k];
                h += w * a1[k];
                hd += w * ad1[k];
            }
            float a2, s2, c2;
            silu3(h, a2, s2, c2);
            const float w3 = prm[L::W3 + j];
            S.d2[a][j] = r * w3 * s2 + w3 * hd * c2;
            S.t2[a][j] = w3 * s2;
            S.q3[a][j] = r * a2 + s2 * hd;
        }
    }
    // back through W2 to a1 and a1', then through layer 1
    {
        float a1b[H], ad1b[H];
#pragma unroll
        for (int k = 0; k < H; ++k) a1b[k] = ad1b[k] = 0.0f;
        for (int j = 0; j < H; ++j) {
            const float d2 = S.d2[a][j], t2 = S.t2[a][j];
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const float w = prm[L::W2 + j * H + k];
                a1b[k] += w * d2;
                ad1b[k] += w * t2;
            }
        }
        float x[NIN], u[NIN];
#pragma unroll
        for (int k = 0; k < NIN; ++k) {
            x[k] = S.x[a][k];
            u[k] = S.u[a][k];
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float h = prm[L::B1 + j], hd = 0.0f;
#pragma unroll
            for (int k = 0; k < NIN; ++k) {
                const float w = prm[L::W1 + j * NIN + k];
                h += w * x[k];
                hd += w * u[k];
            }
            float av, s1, c1;
            silu3(h, av, s1, c1);
            S.hd1b[a][j] = ad1b[j] * s1;
            S.h1b[a][j] = a1b[j] * s1 + ad1b[j] * hd * c1;
        }
    }
    __syncthreads();
    // lanes run over parameters, each summing the block's atoms in order
    const int nt = min(T, n - (int)blockIdx.x * T);
    float *out = partial + (size_t)blockIdx.x * L::NP;
    for (int p = a; p < L::NP; p += 64) {
        float s = 0.0f;
        if (p < L::B1) {
            const int j = p / NIN, k = p - j * NIN;
            for (int t = 0; t < nt; ++t) s += S.h1b[t][j] * S.x[t][k] + S.hd1b[t][j] * S.u[t][k];
        } else if (p < L::W2) {
            const int j = p - L::B1;
            for (int t = 0; t < nt; ++t) s += S.h1b[t][j];
        } else if (p < L::B2) {
            const int j = (p - L::W2) / H, k = (p - L::W2) - j * H;
            for (int t = 0; t < nt; ++t) s += S.d2[t][j] * S.a1[t][k] + S.t2[t][j] * S.ad1[t][k];
        } else if (p < L::W3) {
            const int j = p - L::B2;
            for (int t = 0; t < nt; ++t) s += S.d2[t][j];
        } else if (p < L::B3) {
            const int j = p - L::W3;
            for (int t = 0; t < nt; ++t) s += S.q3[t][j];
        } else {
            for (int t = 0; t < nt; ++t) s += S.r[t];
        }
        out[p] = s;
    }
}

// out[c] = sum over rows r in [r0, r1) of in[r][c], r ascending; blockIdx.y
// selects a chunk of kReduceChunk rows.
constexpr int kReduceChunk = 64;

__global__ __launch_bounds__(256) void k_reduce_rows(int nrows, int ncols,
                                                     const float *__restrict__ in,
                                                     float *__restrict__ out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncols) return;
    const int r0 = blockIdx.y * kReduceChunk;
    const int r1 = min(nrows, r0 + kReduceChunk);
    float s = 0.0f;
    for (int r = r0; r < r1; ++r) s += in[(size_t)r * ncols + c];
    out[(size_t)blockIdx.y * ncols + c] = s;
}

__global__ __launch_bounds__(256) void k_adam(int np, float *__restrict__ prm,
                                              float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ grad, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= np) return;
    const float gk = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    prm[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// jac[p][l][a] = dE[p][a] (FP32)
__global__ __launch_bounds__(256) void k_pack_jac(int npairs, int nb, int l,
                                                  const double *__restrict__ dE,
                                                  float *__restrict__ jac)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npairs) return;
    float *J = jac + ((size_t)p * nb + l) * 3;
    J[0] = (float)dE[3 * (size_t)p + 0];
    J[1] = (float)dE[3 * (size_t)p + 1];
    J[2] = (float)dE[3 * (size_t)p + 2];
}

// owner atom of pair p: the i with off[i] <= p < off[i+1]
__device__ __forceinline__ int pair_owner(int n, const int *__restrict__ off, int p)
{
    int lo = 0, hi = n;  // off[lo] <= p < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// dE_p = J_p^T g_{i(p)}
template <int NIN>
__global__ __launch_bounds__(256) void k_jac_force(int n, int npairs, const int *__restrict__ off,
                                                   const float *__restrict__ jac,
                                                   const double *__restrict__ g,
                                                   double *__restrict__ dE)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npairs) return;
    const int i = pair_owner(n, off, p);
    const float *J = jac + (size_t)p * NIN * 3;
    const double *gi = g + (size_t)i * NIN;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int l = 0; l < NIN; ++l) {
        const double gl = gi[l];
        s0 += gl * (double)J[3 * l + 0];
        s1 += gl * (double)J[3 * l + 1];
        s2 += gl * (double)J[3 * l + 2];
    }
    dE[3 * (size_t)p + 0] = s0;
    dE[3 * (size_t)p + 1] = s1;
    dE[3 * (size_t)p + 2] = s2;
}

// v_i = sum over pairs p = (i -> k) of J_p (lambda_i - lambda_k): with
// F_i = sum_{p of i} dE_p - sum_{p of i} dE_rev(p), dL/d(dE_p) = lambda_i - lambda_k.
template <int NIN>
__global__ __launch_bounds__(256) void k_jac_adjoint(int n, const int *__restrict__ off,
                                                     const int *__restrict__ nbr,
                                                     const float *__restrict__ jac,
                                                     const double *__restrict__ lam,
                                                     double *__restrict__ v)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double l0 = lam[3 * (size_t)i], l1 = lam[3 * (size_t)i + 1], l2 = lam[3 * (size_t)i + 2];
    double acc[NIN];
#pragma unroll
    for (int l = 0; l < NIN; ++l) acc[l] = 0.0;
    const int pe = off[i + 1];
    for (int p = off[i]; p < pe; ++p) {
        const int k = nbr[p];
        const double e0 = l0 - lam[3 * (size_t)k], e1 = l1 - lam[3 * (size_t)k + 1],
                     e2 = l2 - lam[3 * (size_t)k + 2];
        const float *J = jac + (size_t)p * NIN * 3;
#pragma unroll
        for (int l = 0; l < NIN; ++l)
            acc[l] += (double)J[3 * l] * e0 + (double)J[3 * l + 1] * e1 + (double)J[3 * l + 2] * e2;
    }
#pragma unroll
    for (int l = 0; l < NIN; ++l) v[(size_t)i * NIN + l] = acc[l];
}

// r_i = 2 wE (E_i - Eref_i), lambda_i = 2 wF (F_i - Fref_i); per block, the
// sums of (E - Eref)^2 and |F - Fref|^2 in sums[block][2].
__global__ __launch_bounds__(256) void k_residuals(int n, const double *__restrict__ E,
                                                   const double *__restrict__ Eref,
                                                   const double *__restrict__ F,
                                                   const double *__restrict__ Fref, double wE,
                                                   double wF, double *__restrict__ rE,
                                                   double *__restrict__ lam,
                                                   double *__restrict__ sums)
{
    __shared__ double se[256], sf[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0, f2 = 0.0;
    if (i < n) {
        const double de = E[i] - Eref[i];
        rE[i] = 2.0 * wE * de;
        e2 = de * de;
        for (int d = 0; d < 3; ++d) {
            const double df = F[3 * (size_t)i + d] - Fref[3 * (size_t)i + d];
            lam[3 * (size_t)i + d] = 2.0 * wF * df;
            f2 += df * df;
        }
    }
    se[threadIdx.x] = e2;
    sf[threadIdx.x] = f2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            se[threadIdx.x] += se[threadIdx.x + s];
            sf[threadIdx.x] += sf[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[2 * (size_t)blockIdx.x] = se[0];
        sums[2 * (size_t)blockIdx.x + 1] = sf[0];
    }
}

}  // namespace

bool mlp_supported(int nin) { return nin == 5 || nin == 14 || nin == 30; }

int mlp_nparams(int nin) { return H * nin + H + H * H + H + H + 1; }

size_t mlp_grad_workspace(int nin, int n)
{
    const size_t nblk = (size_t)(n + T - 1) / T;
    const size_t nchunk = (nblk + kReduceChunk - 1) / kReduceChunk;
    return (nblk + nchunk) * (size_t)mlp_nparams(nin);
}

#define SNAP_MLP_DISPATCH(nin, CALL) \
    switch (nin) {                   \
    case 5: CALL(5); break;          \
    case 14: CALL(14); break;        \
    case 30: CALL(30); break;        \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_mlp_forward(int nin, int n, const float *prm, const float *norm,
                              const float *bounds, float margin, const double *B, double *E,
                              double *g, int *flag, int *clear_flag, hipStream_t s)
{
#define CALL(K)                                                                              \
    hipLaunchKernelGGL(k_mlp_forward_w<K>, dim3((n + 63) / 64), dim3(64 * kFwdWaves), 0, s, n, \
                       prm, norm, bounds, margin, B, E, g, flag, clear_flag)
    SNAP_MLP_DISPATCH(nin, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_mlp_grad(int nin, int n, const float *prm, const float *norm, const double *B,
                           const double *rE, const double *v, float *work, float *grad,
                           hipStream_t s)
{
    const int np = mlp_nparams(nin);
    if (n == 0) {  // an empty sum: zero-fill the gradient
        hipLaunchKernelGGL(k_reduce_rows, dim3((np + 255) / 256, 1), dim3(256), 0, s, 0, np,
                           (const float *)nullptr, grad);
        return hipGetLastError();
    }
    const int nblk = (n + T - 1) / T;
#define CALL(K)                                                                               \
    hipLaunchKernelGGL(k_mlp_grad<K>, dim3(nblk), dim3(64), 0, s, n, prm, norm, B, rE, v, work)
    SNAP_MLP_DISPATCH(nin, CALL)
#undef CALL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nchunk = (nblk + kReduceChunk - 1) / kReduceChunk;
    float *mid = work + (size_t)nblk * np;
    hipLaunchKernelGGL(k_reduce_rows, dim3((np + 255) / 256, nchunk), dim3(256), 0, s, nblk, np,
                       work, mid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_rows, dim3((np + 255) / 256, 1), dim3(256), 0, s, nchunk, np, mid,
                       grad);
    return hipGetLastError();
}

hipError_t launch_adam(int np, float *prm, float *m, float *v, const float *grad, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, prm, m, v, grad, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_jac(int npairs, int nb, int l, const double *dE, float *jac, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_jac, dim3((npairs + 255) / 256), dim3(256), 0, s, npairs, nb, l, dE,
                       jac);
    return hipGetLastError();
}

hipError_t launch_jac_force(int nin, int n, int npairs, const int *off, const float *jac,
                            const double *g, double *dE, hipStream_t s)
{
#define CALL(K)                                                                              \
    hipLaunchKernelGGL(k_jac_force<K>, dim3((npairs + 255) / 256), dim3(256), 0, s, n, npairs, \
                       off, jac, g, dE)
    SNAP_MLP_DISPATCH(nin, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_jac_adjoint(int nin, int n, const int *off, const int *nbr, const float *jac,
                              const double *lam, double *v, hipStream_t s)
{
#define CALL(K)                                                                                 \
    hipLaunchKernelGGL(k_jac_adjoint<K>, dim3((n + 255) / 256), dim3(256), 0, s, n, off, nbr, jac, \
                       lam, v)
    SNAP_MLP_DISPATCH(nin, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_residuals(int n, const double *E, const double *Eref, const double *F,
                            const double *Fref, double wE, double wF, double *rE, double *lam,
                            double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(k_residuals, dim3((n + 255) / 256), dim3(256), 0, s, n, E, Eref, F, Fref,
                       wE, wF, rE, lam, sums);
    return hipGetLastError();
}

}  // namespace snapmi
