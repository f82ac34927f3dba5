// snap_misc.hip -- bispectrum (eq. (z)), energies, update_forces and workspace copies.
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// bispectrum (eq. (z)) and energy (eq. (snapatomenergy)) -- lanes are atoms
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_bispectrum(int n, int npad, const double2 *__restrict__ U,
                                                   const BTerm *__restrict__ terms,
                                                   const BItem *__restrict__ bitems,
                                                   const int *__restrict__ bl_begin, int nb,
                                                   double *__restrict__ B)
{
    const int l = blockIdx.y;
    const int atom = blockIdx.x * 64 + threadIdx.x;
    const double2 *Ua = U + atom;
    double bsum = 0.0;
    const int xe = bl_begin[l + 1];
    for (int x = bl_begin[l]; x < xe; ++x) {
        const BItem *bi = bitems + x;
        double zr = 0.0, zi = 0.0;
        const int te = bi->te;
        for (int tt = bi->tb; tt < te; ++tt) {
            const BTerm tm = terms[tt];
            const double2 u1 = Ua[(size_t)tm.f1 * npad];
            const double2 u2 = Ua[(size_t)tm.f2 * npad];
            zr += tm.cc * (u1.x * u2.x - u1.y * u2.y);
            zi += tm.cc * (u1.x * u2.y + u1.y * u2.x);
        }
        const double2 uj = Ua[(size_t)bi->f3 * npad];
        bsum += bi->w * (zr * uj.x + zi * uj.y);
    }
    if (atom < n) B[(size_t)atom * nb + l] = bsum;
}

// The same for small 2J: the U of a block of 64 atoms is staged in LDS once
// (coalesced), and the workgroup's wavefronts (one per component, up to 16)
// share the components, so every Clebsch-Gordan term reads LDS instead of
// L2 and each wavefront walks one component's terms.
constexpr int kBWaveMax = 16;

template <int NF>
__global__ __launch_bounds__(64 * kBWaveMax) void k_bispectrum_lds(int n, int npad,
                                                        const double2 *__restrict__ U,
                                                        const BTerm *__restrict__ terms,
                                                        const BItem *__restrict__ bitems,
                                                        const int *__restrict__ bl_begin, int nb,
                                                        double *__restrict__ B)
{
    __shared__ double2 Us[NF][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int atom = blockIdx.x * 64 + lane;  // < npad
    for (int f = w; f < NF; f += nw) Us[f][lane] = U[(size_t)f * npad + atom];
    __syncthreads();
    for (int l = w; l < nb; l += nw) {
        double bsum = 0.0;
        const int xe = bl_begin[l + 1];
        for (int x = bl_begin[l]; x < xe; ++x) {
            const BItem *bi = bitems + x;
            double zr = 0.0, zi = 0.0;
            const int te = bi->te;
            int tt = bi->tb;
            // eight terms per step: their (scalar) loads are issued together
            // instead of one dependent load per term
            for (; tt + 8 <= te; tt += 8) {
                BTerm tm[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) tm[k] = terms[tt + k];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const double2 u1 = Us[tm[k].f1][lane];
                    const double2 u2 = Us[tm[k].f2][lane];
                    zr += tm[k].cc * (u1.x * u2.x - u1.y * u2.y);
                    zi += tm[k].cc * (u1.x * u2.y + u1.y * u2.x);
                }
            }
            for (; tt < te; ++tt) {
                const BTerm tm = terms[tt];
                const double2 u1 = Us[tm.f1][lane];
                const double2 u2 = Us[tm.f2][lane];
                zr += tm.cc * (u1.x * u2.x - u1.y * u2.y);
                zi += tm.cc * (u1.x * u2.y + u1.y * u2.x);
            }
            const double2 uj = Us[bi->f3][lane];
            bsum += bi->w * (zr * uj.x + zi * uj.y);
        }
        if (atom < n) B[(size_t)atom * nb + l] = bsum;
    }
}

__global__ void k_energy_from_b(int n, int nb, const double *__restrict__ B,
                                const double *__restrict__ beta, int per_atom_beta,
                                double *__restrict__ energy)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *bt = per_atom_beta ? beta + (size_t)i * nb : beta;
    double e = 0.0;
    for (int l = 0; l < nb; ++l) e += bt[l] * B[(size_t)i * nb + l];
    energy[i] = e;
}

// ---------------------------------------------------------------------------
// update_forces and the energy
// ---------------------------------------------------------------------------
// kGatherLanes lanes per atom: the lanes stride over the atom's pairs
// (forces) and over the row partials of the energy, then combine with
// shuffles in a fixed order.  One pair per lane for up to 32 neighbours keeps
// the dependent rev -> dE loads of many atoms in flight at once.
constexpr int kGatherLanes = 32;

__global__ __launch_bounds__(256) void k_gather(int n, int npad, int nrows,
                                                const int *__restrict__ off,
                                                const int *__restrict__ rev,
                                                const double *__restrict__ dE,
                                                const double *__restrict__ Epart,
                                                double *__restrict__ energy,
                                                double *__restrict__ force)
{
    constexpr int L = kGatherLanes;
    // workgroup w runs on XCD w mod 8 and takes atoms of the 64-atom blocks
    // congruent to it mod 8, whose energy shares that XCD's compute_Y wrote
    constexpr int WPB = 64 / (256 / L);  // workgroups per 64-atom block
    const int wq = (int)blockIdx.x >> 3;
    const int blk = 8 * (wq / WPB) + ((int)blockIdx.x & 7);
    const int g = blk * 64 + (wq % WPB) * (256 / L) + (threadIdx.x / L);
    const int s = threadIdx.x % L;
    const int i = g < n ? g : n - 1;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    const int te = off[i + 1];
    for (int t = off[i] + s; t < te; t += L) {
        const int r = rev[t];
        fx += dE[3 * (size_t)t + 0] - dE[3 * (size_t)r + 0];
        fy += dE[3 * (size_t)t + 1] - dE[3 * (size_t)r + 1];
        fz += dE[3 * (size_t)t + 2] - dE[3 * (size_t)r + 2];
    }
    if (energy)
        for (int k = s; k < nrows; k += L) e += Epart[(size_t)k * npad + i];
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
        fx += __shfl_xor(fx, m, L);
        fy += __shfl_xor(fy, m, L);
        fz += __shfl_xor(fz, m, L);
        e += __shfl_xor(e, m, L);
    }
    if (g < n && s == 0) {
        force[3 * (size_t)g + 0] = fx;
        force[3 * (size_t)g + 1] = fy;
        force[3 * (size_t)g + 2] = fz;
        if (energy) energy[g] = e * (1.0 / 3.0);
    }
}

// ---------------------------------------------------------------------------
// virial: W = dE_total/d(strain) = sum_p dE_p (x) r_ik (lane per atom), per
// atom (optional) and per block of 256 atoms, summed in a fixed order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_virial(int n, const double *__restrict__ pos,
                                                const int *__restrict__ off,
                                                const int *__restrict__ nbr, Geom g,
                                                const double *__restrict__ dE,
                                                double *__restrict__ watom,
                                                double *__restrict__ partial)
{
    __shared__ double red[9][256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = 0.0;
    if (i < n) {
        const int pe = off[i + 1];
        for (int p = off[i]; p < pe; ++p) {
            double rv[3];
            min_image(pos, i, nbr[p], g, rv);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) w[3 * a + b] += dE[3 * (size_t)p + a] * rv[b];
        }
        if (watom)
#pragma unroll
            for (int k = 0; k < 9; ++k) watom[9 * (size_t)i + k] = w[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) red[k][threadIdx.x] = w[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 9; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 9) partial[9 * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_virial_sum(int nblk, const double *__restrict__ partial,
                             double *__restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= 9) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[9 * (size_t)b + k];
    out[k] = s;
}

// ---------------------------------------------------------------------------
// quadratic SNAP: E_i = beta . B_i + (1/2) B_i^T alpha B_i and the per-atom
// coefficients of its forces, g_i = dE_i/dB_i = beta + (1/2)(alpha + alpha^T) B_i.
// Lane per atom; the block's 64 bispectra are staged in LDS transposed
// ([component][atom]), alpha and beta are read with wavefront-uniform loads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_quadratic(int n, int nb, const double *__restrict__ B,
                                                  const double *__restrict__ beta,
                                                  const double *__restrict__ alpha,
                                                  double *__restrict__ energy,
                                                  double *__restrict__ g)
{
    extern __shared__ double qs[];  // [nb][64]
    const int lane = threadIdx.x;
    const int i0 = blockIdx.x * 64;
    const int na = min(64, n - i0);
    // the block's rows of B are one contiguous run of na * nb doubles
    for (int k = lane; k < 64 * nb; k += 64) {
        const int a = k / nb, l = k - a * nb;
        qs[l * 64 + a] = a < na ? B[(size_t)i0 * nb + k] : 0.0;
    }
    __syncthreads();
    const int i = i0 + lane;
    double e = 0.0;
    for (int l = 0; l < nb; ++l) {
        double sl = 0.0;
        for (int m = 0; m < nb; ++m)
            sl += 0.5 * (alpha[(size_t)l * nb + m] + alpha[(size_t)m * nb + l]) * qs[m * 64 + lane];
        e += (beta[l] + 0.5 * sl) * qs[l * 64 + lane];
        if (lane < na) g[(size_t)i * nb + l] = beta[l] + sl;
    }
    if (lane < na) energy[i] = e;
}

// ---------------------------------------------------------------------------
// dE/dbeta of the weighted energy sum_i g_i E_i with E_i = beta . B_i: the
// sum over atoms of g_i B_i (shared coefficients) in two passes of fixed
// order (per block of atoms, then over the blocks), or g_i B_i per atom
// ---------------------------------------------------------------------------
constexpr int kBetaGradAtoms = 256;

__global__ __launch_bounds__(64) void k_beta_grad_part(int n, int nb, const double *__restrict__ g,
                                                       const double *__restrict__ B,
                                                       double *__restrict__ part)
{
    const int i0 = blockIdx.x * kBetaGradAtoms;
    const int i1 = min(n, i0 + kBetaGradAtoms);
    for (int l = threadIdx.x; l < nb; l += 64) {
        double s = 0.0;
        for (int i = i0; i < i1; ++i) s += g[i] * B[(size_t)i * nb + l];
        part[(size_t)blockIdx.x * nb + l] = s;
    }
}

__global__ __launch_bounds__(64) void k_beta_grad_sum(int nblk, int nb,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ out)
{
    const int l = blockIdx.x * 64 + threadIdx.x;
    if (l >= nb) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * nb + l];
    out[l] = s;
}

__global__ void k_beta_grad_atom(long long total, int nb, const double *__restrict__ g,
                                 const double *__restrict__ B, double *__restrict__ out)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    out[k] = g[k / nb] * B[k];
}

// dst[e][i] = scale[e] * src[map[e] * npad + i] (map, scale optional)
__global__ void k_unscale(int n, int se, int sa, int nhalf, const double2 *__restrict__ src,
                          const int *__restrict__ map, const double *__restrict__ scale,
                          double *__restrict__ dst)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)n * nhalf) return;
    const int e = (int)(k / n), i = (int)(k - (size_t)e * n);
    const int row = map ? map[e] : e;
    const double sc = scale ? scale[e] : 1.0;
    const double2 v = src[(size_t)row * se + (size_t)i * sa];
    dst[2 * k + 0] = sc * v.x;
    dst[2 * k + 1] = sc * v.y;
}

}  // namespace

hipError_t launch_bispectrum(int n, int npad, const double2 *U, const DevTables &T, int nb,
                             double *B, const double *beta, int per_atom_beta, double *energy,
                             hipStream_t s, int nfull)
{
    const int nblk = (n + 63) / 64;
    // full elements sum_{J <= 2Jmax} (J+1)^2: 2J = 4 -> 55, 2J = 5 -> 91
    const int nw = nb < kBWaveMax ? nb : kBWaveMax;
    if (nfull == 55)
        hipLaunchKernelGGL(k_bispectrum_lds<55>, dim3(nblk), dim3(64 * nw), 0, s, n, npad, U,
                           T.bterms, T.bitems, T.bl_begin, nb, B);
    else if (nfull == 91)
        hipLaunchKernelGGL(k_bispectrum_lds<91>, dim3(nblk), dim3(64 * nw), 0, s, n, npad, U,
                           T.bterms, T.bitems, T.bl_begin, nb, B);
    else
        hipLaunchKernelGGL(k_bispectrum, dim3(nblk, nb), dim3(64), 0, s, n, npad, U, T.bterms,
                           T.bitems, T.bl_begin, nb, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !energy) return e;
    hipLaunchKernelGGL(k_energy_from_b, dim3((n + 127) / 128), dim3(128), 0, s, n, nb, B, beta,
                       per_atom_beta, energy);
    return hipGetLastError();
}

hipError_t launch_gather(int n, int npad, int nrows, const int *off, const int *rev,
                         const double *dE, const double *Epart, double *energy, double *force,
                         hipStream_t s)
{
    constexpr int apb = 256 / kGatherLanes;  // atoms per block
    // 64-atom blocks padded to a multiple of 8 (atoms past n write nothing)
    const int ngrid = ((n + 64 * 8 - 1) / (64 * 8)) * 8 * (64 / apb);
    hipLaunchKernelGGL(k_gather, dim3(ngrid), dim3(256), 0, s, n, npad, nrows, off, rev, dE, Epart,
                       energy, force);
    return hipGetLastError();
}

hipError_t launch_virial(int n, const double *pos, const int *off, const int *nbr, const Geom &g,
                         const double *dE, double *watom, double *partial, double *out,
                         hipStream_t s)
{
    const int nblk = (n + 255) / 256;
    if (nblk > 0) {
        hipLaunchKernelGGL(k_virial, dim3(nblk), dim3(256), 0, s, n, pos, off, nbr, g, dE, watom,
                           partial);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_virial_sum, dim3(1), dim3(64), 0, s, nblk, partial, out);
    return hipGetLastError();
}

hipError_t launch_quadratic(int n, int nb, const double *B, const double *beta,
                            const double *alpha, double *energy, double *g, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 64 * (size_t)nb;
    if (lds > 64 * 1024) {
        // beyond the default dynamic LDS limit (2J >= 11): raise it once
        static bool raised = false;
        if (!raised) {
            const hipError_t e = hipFuncSetAttribute((const void *)k_quadratic,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)lds);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    hipLaunchKernelGGL(k_quadratic, dim3((n + 63) / 64), dim3(64), lds, s, n, nb, B, beta, alpha,
                       energy, g);
    return hipGetLastError();
}

int beta_grad_blocks(int n) { return (n + kBetaGradAtoms - 1) / kBetaGradAtoms; }

hipError_t launch_beta_grad(int n, int nb, const double *g, const double *B, int per_atom,
                            double *part, double *out, hipStream_t s)
{
    if (per_atom) {
        const long long total = (long long)n * nb;
        if (total == 0) return hipSuccess;
        hipLaunchKernelGGL(k_beta_grad_atom, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           s, total, nb, g, B, out);
        return hipGetLastError();
    }
    const int nblk = beta_grad_blocks(n);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_beta_grad_part, dim3(nblk), dim3(64), 0, s, n, nb, g, B, part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_beta_grad_sum, dim3((nb + 63) / 64), dim3(64), 0, s, nblk, nb, part,
                       out);
    return hipGetLastError();
}

hipError_t launch_unscale(int n, int se, int sa, int nhalf, const double2 *src, const int *map,
                          const double *scale, double *dst, hipStream_t s)
{
    const size_t tot = (size_t)n * nhalf;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unscale, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, se, sa,
                       nhalf, src, map, scale, dst);
    return hipGetLastError();
}

}  // namespace snapmi
