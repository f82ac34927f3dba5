// snap_u.hip -- compute_U: eq. (u) of arXiv 2011.12875 (see snap_device.hpp).
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_U
// ---------------------------------------------------------------------------
constexpr int kUStage = 16;  // staged elements per LDS flush (>= twojmax + 1)
constexpr int kUSlots = 32;  // pair slots per atom (two atoms per wavefront)

struct UStage {
    double2 v[kUStage][65];
    int code[kUStage];
};

// The emission order of the stored half is static: column q = 0..TJ/2, then
// level J = (q ? 2q : 0)..TJ, J+1 elements each.  Its staging schedule (slot
// of each level-column and where the LDS buffer is flushed) is therefore a
// compile-time function, so every LDS address below is an immediate.
struct StagePos {
    int slot;    // first staging slot of the level-column
    int flushed; // > 0: the buffer holding this many slots is flushed first
};
constexpr StagePos stage_pos(int TJ, int Q, int J)
{
    int nst = 0;
    for (int q = 0; q <= TJ / 2; ++q)
        for (int j = (q ? 2 * q : 0); j <= TJ; ++j) {
            int fl = 0;
            if (nst + j + 1 > kUStage) {
                fl = nst;
                nst = 0;
            }
            if (q == Q && j == J) return StagePos{nst, fl};
            nst += j + 1;
        }
    return StagePos{-1, 0};
}
constexpr int stage_end(int TJ)
{
    const StagePos last = stage_pos(TJ, TJ / 2, TJ);
    return last.slot + TJ + 1;
}

// Sum the NST staged values of both atoms over their 32 slots and add them
// to U, stored as full matrices of true values: U(p, q) = N * sum and its
// mirror U(J-p, J-q) = (-1)^(p-q) conj(U(p, q)).  The first chunk of
// neighbours starts from w_self on the diagonal (where N = 1).
template <int NST>
__device__ __forceinline__ void u_flush(UStage &st, int lane, int i0, int n, int npad, int chunk,
                                        double wself, const UInfo *__restrict__ uinfo,
                                        double2 *__restrict__ U)
{
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < 2 * NST; k0 += 64) {
        const int k = k0 + lane;
        if (k < 2 * NST) {
            const int hh = k >= NST ? 1 : 0;
            const int ss = k - hh * NST;
            double sr = 0.0, si = 0.0;
#pragma unroll 8
            for (int j = 0; j < kUSlots; ++j) {
                const double2 v = st.v[ss][hh * kUSlots + j];
                sr += v.x;
                si += v.y;
            }
            const int ia = i0 + hh;
            if (ia < n) {
                const int code = st.code[ss];
                const UInfo ui = uinfo[code & 0xffffff];
                const size_t idx = (size_t)ui.fi * npad + ia;
                double br = 0.0, bi = 0.0;
                if (chunk == 0) {
                    br = (code >> 24) ? wself : 0.0;
                } else {
                    const double2 old = U[idx];
                    br = old.x;
                    bi = old.y;
                }
                const double2 v = make_double2(br + ui.nrm * sr, bi + ui.nrm * si);
                U[idx] = v;
                if (ui.fm >= 0)
                    U[(size_t)ui.fm * npad + ia] = make_double2(ui.msign * v.x, -ui.msign * v.y);
            }
        }
    }
    __syncthreads();
}

template <int TJ, int Q, int J>
__device__ __forceinline__ void u_emit(UStage &st, int lane, double fc,
                                       const double2 (&col)[TJ + 1], int i0, int n, int npad,
                                       int chunk, double wself, const UInfo *__restrict__ uinfo,
                                       double2 *__restrict__ U)
{
    constexpr StagePos sp = stage_pos(TJ, Q, J);
    if constexpr (sp.flushed > 0)
        u_flush<sp.flushed>(st, lane, i0, n, npad, chunk, wself, uinfo, U);
    constexpr int ebase = hbase_of(J) + Q * (J + 1);
#pragma unroll
    for (int p = 0; p <= J; ++p) {
        st.v[sp.slot + p][lane] = make_double2(fc * col[p].x, fc * col[p].y);
        if (lane == 0) st.code[sp.slot + p] = (ebase + p) | ((p == Q) ? (1 << 24) : 0);
    }
}

template <int TJ, int Q, int J>
struct ULevels {
    __device__ __forceinline__ static void run(UStage &st, int lane, double fc, double2 a,
                                               double2 b, double2 (&col)[TJ + 1],
                                               double2 (&seed)[TJ + 1], int i0, int n, int npad,
                                               int chunk, double wself,
                                               const UInfo *__restrict__ uinfo,
                                               double2 *__restrict__ U)
    {
        poly_step<TJ>(J, col, a, b);
        u_emit<TJ, Q, J>(st, lane, fc, col, i0, n, npad, chunk, wself, uinfo, U);
#pragma unroll
        for (int p = 0; p <= J; ++p) pin(col[p]);
        memory_fence_compiler();
        if constexpr (J == 2 * Q + 1 && 2 * Q + 2 <= TJ) {
            mirror_seed<TJ, Q>(col, seed);
#pragma unroll
            for (int p = 0; p <= 2 * Q + 1; ++p) pin(seed[p]);
        }
        ULevels<TJ, Q, J + 1>::run(st, lane, fc, a, b, col, seed, i0, n, npad, chunk, wself, uinfo,
                                   U);
    }
};
template <int TJ, int Q>
struct ULevels<TJ, Q, TJ + 1> {
    __device__ __forceinline__ static void run(UStage &, int, double, double2, double2,
                                               double2 (&)[TJ + 1], double2 (&)[TJ + 1], int, int,
                                               int, int, double, const UInfo *__restrict__,
                                               double2 *__restrict__)
    {
    }
};

template <int TJ, int Q>
struct UColumns {
    __device__ __forceinline__ static void run(UStage &st, int lane, double fc, double2 a,
                                               double2 b, double2 (&col)[TJ + 1],
                                               double2 (&seed)[TJ + 1], int i0, int n, int npad,
                                               int chunk, double wself,
                                               const UInfo *__restrict__ uinfo,
                                               double2 *__restrict__ U)
    {
#pragma unroll
        for (int p = 0; p <= TJ; ++p)
            col[p] = (Q > 0 && p < 2 * Q) ? seed[p] : make_double2(0.0, 0.0);
        if constexpr (Q == 0) {
            col[0] = make_double2(1.0, 0.0);
            u_emit<TJ, 0, 0>(st, lane, fc, col, i0, n, npad, chunk, wself, uinfo, U);
        }
        ULevels<TJ, Q, (Q == 0 ? 1 : 2 * Q)>::run(st, lane, fc, a, b, col, seed, i0, n, npad,
                                                   chunk, wself, uinfo, U);
        UColumns<TJ, Q + 1>::run(st, lane, fc, a, b, col, seed, i0, n, npad, chunk, wself, uinfo,
                                 U);
    }
};
template <int TJ>
struct UColumns<TJ, TJ / 2 + 1> {
    __device__ __forceinline__ static void run(UStage &, int, double, double2, double2,
                                               double2 (&)[TJ + 1], double2 (&)[TJ + 1], int, int,
                                               int, int, double, const UInfo *__restrict__,
                                               double2 *__restrict__)
    {
    }
};

template <int TJ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_compute_u(int n, int npad, const double *__restrict__ pos,
                                                  const int *__restrict__ off,
                                                  const int *__restrict__ nbr, Geom g,
                                                  const UInfo *__restrict__ uinfo,
                                                  double2 *__restrict__ U,
                                                  int *__restrict__ pair_atom, int *__restrict__ flag)
{
    __shared__ UStage st;
    const int lane = threadIdx.x;
    const int h = lane >> 5, slot = lane & 31;
    const int i0 = blockIdx.x * 2;
    const int i = i0 + h;
    const int nA = (i0 < n) ? off[i0 + 1] - off[i0] : 0;
    const int nB = (i0 + 1 < n) ? off[i0 + 2] - off[i0 + 1] : 0;
    const int mx = nA > nB ? nA : nB;
    const int nchunk = mx > 0 ? (mx + kUSlots - 1) / kUSlots : 1;
    const int myn = h ? nB : nA;
    const int mybeg = (i < n) ? off[i] : 0;

    for (int c = 0; c < nchunk; ++c) {
        const int s = c * kUSlots + slot;
        const bool valid = (i < n) && (s < myn);
        const int t = mybeg + s;
        PairGeom pg;
        pg.a = make_double2(1.0, 0.0);
        pg.b = make_double2(0.0, 0.0);
        pg.fc = 0.0;
        if (valid) {
            pair_atom[t] = i;
            double rv[3];
            min_image(pos, i, nbr[t], g, rv);
            if (!pair_geometry(rv, g, pg)) flag[0] = 1;
        }
        double2 col[TJ + 1], seed[TJ + 1];
#pragma unroll
        for (int p = 0; p <= TJ; ++p) seed[p] = make_double2(0.0, 0.0);
        UColumns<TJ, 0>::run(st, lane, pg.fc, pg.a, pg.b, col, seed, i0, n, npad, c, g.wself,
                             uinfo, U);
        u_flush<stage_end(TJ)>(st, lane, i0, n, npad, c, g.wself, uinfo, U);
    }
}

template <int TJ>
hipError_t launch_u_t(int n, int npad, const double *pos, const int *off, const int *nbr,
                      const Geom &g, const UInfo *uinfo, double2 *U, int *pair_atom, int *flag,
                      hipStream_t s)
{
    const int nblk = (n + 1) / 2;
    hipLaunchKernelGGL(k_compute_u<TJ>, dim3(nblk), dim3(64), 0, s, n, npad, pos, off, nbr, g,
                       uinfo, U, pair_atom, flag);
    return hipGetLastError();
}

}  // namespace

#ifndef SNAP_TJ_CASES
#define SNAP_TJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

hipError_t launch_compute_u(int twojmax, int n, int npad, const double *pos, const int *off,
                            const int *nbr, const DevTables &T, const Geom &g, double2 *U,
                            int *pair_atom, int *flag, hipStream_t s)
{
    switch (twojmax) {
#define X(k) \
    case k: return launch_u_t<k>(n, npad, pos, off, nbr, g, T.uinfo, U, pair_atom, flag, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
