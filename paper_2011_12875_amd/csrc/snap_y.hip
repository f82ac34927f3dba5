// snap_y.hip -- compute_Y: the adjoint of eq. (y) of arXiv 2011.12875 (see snap_device.hpp).
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_Y (adjoint of eq. (y)) -- lanes are atoms
// ---------------------------------------------------------------------------
constexpr int kYMaxQ = 8;      // J/2 + 1 for J <= 14
constexpr int kCqMax = 8 * 15; // nq * (J1 + 1) for J, J1 <= 14

constexpr int fbase_of(int J)  // first full element of rank J (blocks of (J+1)^2)
{
    int s = 0;
    for (int k = 0; k < J; ++k) s += (k + 1) * (k + 1);
    return s;
}
__device__ __forceinline__ int fbase_rt(int J)
{
    return (J * (J + 1) * (2 * J + 1)) / 6;  // sum_{k=1}^{J} k^2
}
__device__ __forceinline__ int hbase_rt(int J)
{
    // sum_{k<J} (k+1)(k/2+1), closed form per parity
    const int m = J / 2;
    // pairs (2i, 2i+1) for i < m contribute (2i+1)(i+1) + (2i+2)(i+1)
    int s = 0;
    for (int i = 0; i < m; ++i) s += (4 * i + 3) * (i + 1);
    if (J & 1) s += (2 * m + 1) * (m + 1);
    return s;
}

// Full row px of U^Jx (true values), elements f = fbase(Jx) + px (Jx+1) + q:
// one buffer descriptor for the row (scalar registers), the element offset
// in the scalar offset, the atom in the lane offset.  Entries q > Jx are
// zero, so that products with them vanish.
template <int TJ>
__device__ __forceinline__ void load_full_row(double2 (&r)[TJ + 1], int Jx, int px,
                                              const double2 *__restrict__ U, int npad,
                                              unsigned voff)
{
    const double2 *base = U + (size_t)(fbase_rt(Jx) + px * (Jx + 1)) * (size_t)npad;
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)base, (short)0, (Jx + 1) * npad * 16, 0x00020000);
#pragma unroll
    for (int q = 0; q <= TJ; ++q) {
        r[q] = make_double2(0.0, 0.0);
        if (q <= Jx) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, q * npad * 16, 0);
            r[q] = make_double2(
                __builtin_bit_cast(double, (unsigned long long)v[0] | ((unsigned long long)v[1] << 32)),
                __builtin_bit_cast(double, (unsigned long long)v[2] | ((unsigned long long)v[3] << 32)));
        }
    }
}

// One contribution (J1, J2 -> J) to row p of Y, accumulated into acc[q].
// q2 = q - q1 + D is a compile-time index into the second row.  Every
// (q, q1) with q1, q2 in [0, 2J_max] is evaluated without a test: rows are
// zero beyond J1 and J2 and the staged column coefficients beyond J1, so
// the terms outside the Clebsch-Gordan range add exact zeros (about 6 % of
// the products at 2J = 8); only the row index q < nq is tested, once per q.
// The coefficients sit at compile-time offsets cq[q (2J_max + 1) + q1].
template <int TJ, int D>
__device__ __forceinline__ void y_contrib(int J1, int J2, int p1lo, int p1hi, int cp_off, int p,
                                          int nq, const double2 *__restrict__ U, int npad,
                                          unsigned voff, const double *__restrict__ cpt,
                                          const double *cq, double f, double2 (&acc)[TJ / 2 + 1])
{
    for (int p1 = p1lo; p1 <= p1hi; ++p1) {
        const int p2 = p - p1 + D;
        // re-derive the bounds in every iteration: hoisted out of the loop,
        // the guard compares below would each hold a scalar register for the
        // whole loop and spill
        int j1 = J1, j2 = J2, qn = nq;
        asm volatile("" : "+s"(j1), "+s"(j2), "+s"(qn));
        double2 r1[TJ + 1], r2[TJ + 1];
        load_full_row<TJ>(r1, j1, p1, U, npad, voff);
        load_full_row<TJ>(r2, j2, p2, U, npad, voff);
        const double cpv = f * cpt[cp_off + (p1 - p1lo)];
#pragma unroll
        for (int q = 0; q <= TJ / 2; ++q)
            if (q < qn) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int q1 = 0; q1 <= TJ; ++q1) {
                    const int q2 = q - q1 + D;  // compile-time
                    if (q2 >= 0 && q2 <= TJ) {
                        const double c = cq[q * (TJ + 1) + q1];
                        const double2 x = r1[q1], y = r2[q2 < 0 ? 0 : (q2 > TJ ? TJ : q2)];
                        const double pr = x.x * y.x - x.y * y.y;
                        const double pi = x.x * y.y + x.y * y.x;
                        sr += c * pr;
                        si += c * pi;
                    }
                }
                acc[q].x += cpv * sr;
                acc[q].y += cpv * si;
            }
    }
}

template <int TJ, int D>
struct YDispatch {
    __device__ __forceinline__ static void run(int d, int J1, int J2, int p1lo, int p1hi,
                                               int cp_off, int p, int nq,
                                               const double2 *__restrict__ U, int npad,
                                               unsigned voff, const double *__restrict__ cpt,
                                               const double *cq, double f,
                                               double2 (&acc)[TJ / 2 + 1])
    {
        if (d == D)
            y_contrib<TJ, D>(J1, J2, p1lo, p1hi, cp_off, p, nq, U, npad, voff, cpt, cq, f, acc);
        else
            YDispatch<TJ, D + 1>::run(d, J1, J2, p1lo, p1hi, cp_off, p, nq, U, npad, voff, cpt, cq,
                                      f, acc);
    }
};
template <int TJ>
struct YDispatch<TJ, TJ + 1> {
    __device__ __forceinline__ static void run(int, int, int, int, int, int, int, int,
                                               const double2 *__restrict__, int, unsigned,
                                               const double *__restrict__, const double *, double,
                                               double2 (&)[TJ / 2 + 1])
    {
    }
};

// Workgroup = (row (J, p) of Y, block of 64 atoms); its contributions are
// split over four wavefronts and reduced in LDS.  Workgroup u runs on XCD
// u mod 8, which owns the atom blocks congruent to it mod 8 (blocks padded
// to a multiple of 8).  An XCD walks its blocks in groups of kYGroup: within
// a group row-major (the rows are sorted by decreasing cost, so the heavy
// rows of the group start first), group after group, so its L2 holds the U
// of kYGroup blocks (1.2 MB at 2J = 8) whatever the system size.  Also
// writes the row's share of the energy, (1/3) sum_q Re(Y~ conj(U~)), to
// Epart.
constexpr int kYGroup = 4;
template <int TJ>
__global__ __launch_bounds__(64 * kYWaves) __attribute__((amdgpu_waves_per_eu(2, 4))) void k_compute_y(
    int n, int npad, int nblk8, const double2 *__restrict__ U, double2 *__restrict__ Y,
    const YRowC *__restrict__ rows, const YContrib *__restrict__ contribs,
    const double *__restrict__ cpt, const double *__restrict__ cqt,
    const double *__restrict__ beta, int per_atom_beta, int nb,
    const double *__restrict__ gscale, double *__restrict__ Epart)
{
    __shared__ double2 yw[kYWaves][kYMaxQ][64];
    __shared__ double cqs[kYWaves][kCqMax];
    const int unit = blockIdx.x;
    const int nrows = (int)gridDim.x / nblk8;
    const int nbx = nblk8 >> 3;  // blocks per XCD
    const int sx = unit >> 3;    // slot within the XCD
    const int grp = sx / (kYGroup * nrows);
    const int gsz = (grp < nbx / kYGroup) ? kYGroup : nbx - grp * kYGroup;
    const int t = sx - grp * kYGroup * nrows;
    const int rix = t / gsz;
    const int blk = (grp * kYGroup + (t - rix * gsz)) * 8 + (unit & 7);
    if (blk * 64 >= n) return;  // padding block (uniform for the workgroup)
    // the wavefront index is uniform within a wavefront; say so, or every
    // value derived from it is treated as divergent (vector loads, masks)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int atom = blk * 64 + lane;
    const int asafe = atom < n ? atom : 0;
    const unsigned voff = (unsigned)atom * 16u;
    const YRowC *row = rows + rix;
    const int J = __builtin_amdgcn_readfirstlane(row->J);
    const int p = __builtin_amdgcn_readfirstlane(row->p);
    const int nq = __builtin_amdgcn_readfirstlane(row->nq);
    const double gs = gscale ? gscale[asafe] : 1.0;

    double2 y[TJ / 2 + 1];
#pragma unroll
    for (int q = 0; q <= TJ / 2; ++q) y[q] = make_double2(0.0, 0.0);
    const int cb = __builtin_amdgcn_readfirstlane(row->cb[w]);
    const int ce = __builtin_amdgcn_readfirstlane(row->cb[w + 1]);
    for (int c = cb; c < ce; ++c) {
        const YContrib *C = contribs + c;
        const int J1 = __builtin_amdgcn_readfirstlane(C->j1);
        const int J2 = __builtin_amdgcn_readfirstlane(C->j2);
        const int D = __builtin_amdgcn_readfirstlane(C->d);
        const int p1lo = __builtin_amdgcn_readfirstlane(C->p1lo);
        const int p1hi = __builtin_amdgcn_readfirstlane(C->p1hi);
        const int cp_off = __builtin_amdgcn_readfirstlane(C->cp_off);
        const int cq_off = __builtin_amdgcn_readfirstlane(C->cq_off);
        const int cl = __builtin_amdgcn_readfirstlane(C->l);
        // stage this contribution's cq table in the wavefront's LDS slice,
        // rows padded with zeros to 2J_max + 1 entries
        for (int k = lane; k < nq * (TJ + 1); k += 64) {
            const int q = k / (TJ + 1), q1 = k - q * (TJ + 1);
            cqs[w][k] = (q1 <= J1) ? cqt[cq_off + q * (J1 + 1) + q1] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the contribution's weight (multiplicity, beta, per-atom scale)
        // rides on the row coefficient, so products accumulate into y
        const double bl = per_atom_beta ? beta[(size_t)asafe * nb + cl] : beta[cl];
        const double f = C->factor * bl * gs;
        YDispatch<TJ, 0>::run(D, J1, J2, p1lo, p1hi, cp_off, p, nq, U, npad, voff, cpt, cqs[w], f,
                              y);
        // the next contribution overwrites the staged table
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int q = 0; q <= TJ / 2; ++q)
        if (q < nq) yw[w][q][lane] = y[q];
    __syncthreads();
    if (w == 0) {
        double e = 0.0;
        for (int q = 0; q < nq; ++q) {
            double2 s = yw[0][q][lane];
#pragma unroll
            for (int v = 1; v < kYWaves; ++v) {
                s.x += yw[v][q][lane].x;
                s.y += yw[v][q][lane].y;
            }
            const double sc = row->oscale[q];
            s.x *= sc;
            s.y *= sc;
            Y[(size_t)(row->ebase + q * (J + 1)) * npad + atom] = s;
            const double2 u = U[(size_t)(row->frow + q) * npad + atom];
            e += (s.x * u.x + s.y * u.y) * row->einv[q];
        }
        if (Epart && atom < n) Epart[(size_t)rix * npad + atom] = e;
    }
}

}  // namespace

#ifndef SNAP_TJ_CASES
#define SNAP_TJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

template <int TJ>
hipError_t launch_y_t(int n, int npad, const double2 *U, double2 *Y, const DevTables &T,
                      const double *beta, int per_atom_beta, int nb, const double *gscale,
                      double *Epart, hipStream_t s)
{
    const int nblk8 = (((n + 63) / 64) + 7) / 8 * 8;
    hipLaunchKernelGGL(k_compute_y<TJ>, dim3(T.nyrows * nblk8), dim3(64 * kYWaves), 0, s, n, npad,
                       nblk8, U, Y, T.yrows, T.ycontrib, T.ycp, T.ycq, beta,
                       per_atom_beta, nb, gscale, Epart);
    return hipGetLastError();
}

hipError_t launch_compute_y(int twojmax, int n, int npad, const double2 *U, double2 *Y,
                            const DevTables &T, const double *beta, int per_atom_beta, int nb,
                            const double *gscale, double *Epart, hipStream_t s)
{
    switch (twojmax) {
#define X(k) \
    case k: return launch_y_t<k>(n, npad, U, Y, T, beta, per_atom_beta, nb, gscale, Epart, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
