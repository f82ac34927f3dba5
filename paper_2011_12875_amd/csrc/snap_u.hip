// snap_u.hip -- compute_U: eq. (u) of arXiv 2011.12875 (see snap_device.hpp).
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_U
//
// Lanes are pairs: a workgroup is one wavefront holding two atoms of 32 pair
// slots each (neighbour lists longer than 32 run in chunks).  The stored half
// (q <= J/2) of every u_j is produced column by column by the recursion of
// eq. (hysphrecur) on the unnormalised polynomial coefficients; the start of
// column q+1 is column q at level 2q+1, mirrored.
//
// Each column has its own workgroup (one per column and pair of atoms).  The
// workgroup of column Q first reruns the short seed path -- levels 2q and
// 2q+1 of every column q < Q -- and then the levels 2Q..2J_max of column Q.
// Both parts together cost (2J_max+1)(2J_max+2)/2 elements whatever Q is (45
// at 2J = 8), so the columns are evenly loaded, and there are J_max + 1
// times more wavefronts to hide latency with than with one workgroup per
// atom pair, for 70 extra elements per pair at 2J = 8 (225 instead of 155).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int hbase_of_rt(int J)
{
    int s = 0;
    for (int k = 0; k < J; ++k) s += (k + 1) * (k / 2 + 1);
    return s;
}

constexpr int kUStage = 16;  // staged elements per LDS flush (>= twojmax + 1)
constexpr int kUSlots = 32;  // pair slots per atom (two atoms per wavefront)

// elements of column Q: levels J = (Q ? 2Q : 0)..TJ, J+1 each
constexpr int col_size(int TJ, int Q)
{
    int s = 0;
    for (int j = (Q ? 2 * Q : 0); j <= TJ; ++j) s += j + 1;
    return s;
}
// position of the first element of level J within column Q
constexpr int col_pos(int TJ, int Q, int J)
{
    int s = 0;
    for (int j = (Q ? 2 * Q : 0); j < J; ++j) s += j + 1;
    return s;
}

// LDS of one workgroup: the staged values of both atoms' slots, the
// column position of each staged slot, and the element table of the
// column (full-matrix index, mirror index, normalisation, mirror sign),
// loaded at the start of the kernel alongside the neighbour list.
template <int TJ>
struct UStage {
    double2 v[kUStage][65];
    int code[kUStage];
    const UInfo *table;
};

// The emission order of column Q is static: levels J = (Q ? 2Q : 0)..TJ,
// J+1 elements each.  Its staging schedule (slot of each level and where
// the LDS buffer is flushed) is a compile-time function, so every LDS
// address below is an immediate.
struct StagePos {
    int slot;    // first staging slot of the level
    int flushed; // > 0: the buffer holding this many slots is flushed first
};
constexpr StagePos stage_pos(int TJ, int Q, int J)
{
    int nst = 0;
    for (int j = (Q ? 2 * Q : 0); j <= TJ; ++j) {
        int fl = 0;
        if (nst + j + 1 > kUStage) {
            fl = nst;
            nst = 0;
        }
        if (j == J) return StagePos{nst, fl};
        nst += j + 1;
    }
    return StagePos{-1, 0};
}
constexpr int stage_end(int TJ, int Q)
{
    const StagePos last = stage_pos(TJ, Q, TJ);
    return last.slot + TJ + 1;
}

// Sum the NST staged values of both atoms over their 32 slots and add them
// to U, stored as full matrices of true values: U(p, q) = N * sum and its
// mirror U(J-p, J-q) = (-1)^(p-q) conj(U(p, q)).  The first chunk of
// neighbours starts from w_self on the diagonal (where N = 1).
template <int NST, int TJ>
__device__ __forceinline__ void u_flush(UStage<TJ> &st, int lane, int i0, int n, int npad,
                                        int chunk, double wself, double2 *__restrict__ U)
{
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < 2 * NST; k0 += 64) {
        const int k = k0 + lane;
        if (k < 2 * NST) {
            const int hh = k >= NST ? 1 : 0;
            const int ss = k - hh * NST;
            const int code = st.code[ss];
            const UInfo ui = st.table[code & 0xffffff];
            double sr = 0.0, si = 0.0;
#pragma unroll 8
            for (int j = 0; j < kUSlots; ++j) {
                const double2 v = st.v[ss][hh * kUSlots + j];
                sr += v.x;
                si += v.y;
            }
            const int ia = i0 + hh;
            if (ia < n) {
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
__device__ __forceinline__ void u_emit(UStage<TJ> &st, int lane, const double2 (&col)[TJ + 1],
                                       int i0, int n, int npad, int chunk, double wself,
                                       double2 *__restrict__ U)
{
    constexpr StagePos sp = stage_pos(TJ, Q, J);
    if constexpr (sp.flushed > 0) u_flush<sp.flushed, TJ>(st, lane, i0, n, npad, chunk, wself, U);
    constexpr int cpos = hbase_of(J) + Q * (J + 1);
#pragma unroll
    for (int p = 0; p <= J; ++p) {
        st.v[sp.slot + p][lane] = col[p];  // already carries f_c
        if (lane == 0) st.code[sp.slot + p] = (cpos + p) | ((p == Q) ? (1 << 24) : 0);
    }
}

// Levels J..TJ of column Q, each emitted to the staging buffer.
template <int TJ, int Q, int J>
struct ULevels {
    __device__ __forceinline__ static void run(UStage<TJ> &st, int lane, double2 a, double2 b,
                                               double2 (&col)[TJ + 1], int i0, int n, int npad,
                                               int chunk, double wself, double2 *__restrict__ U)
    {
        poly_step<TJ>(J, col, a, b);
        u_emit<TJ, Q, J>(st, lane, col, i0, n, npad, chunk, wself, U);
#pragma unroll
        for (int p = 0; p <= J; ++p) pin(col[p]);
        memory_fence_compiler();
        ULevels<TJ, Q, J + 1>::run(st, lane, a, b, col, i0, n, npad, chunk, wself, U);
    }
};
template <int TJ, int Q>
struct ULevels<TJ, Q, TJ + 1> {
    __device__ __forceinline__ static void run(UStage<TJ> &, int, double2, double2,
                                               double2 (&)[TJ + 1], int, int, int, int, double,
                                               double2 *__restrict__)
    {
    }
};

// Seed path: column q from its seed, levels up to 2q+1, mirrored into the
// seed of column q+1; for q = 0 .. Q-1.  Nothing is emitted.
template <int TJ, int q, int Q>
struct USeedPath {
    __device__ __forceinline__ static void run(double fc, double2 a, double2 b,
                                               double2 (&col)[TJ + 1], double2 (&seed)[TJ + 1])
    {
        if constexpr (q < Q) {
#pragma unroll
            for (int p = 0; p <= TJ; ++p)
                col[p] = (q > 0 && p < 2 * q) ? seed[p] : make_double2(0.0, 0.0);
            if constexpr (q == 0) col[0] = make_double2(fc, 0.0);
#pragma unroll
            for (int J = (q == 0 ? 1 : 2 * q); J <= 2 * q + 1; ++J) {
                poly_step<TJ>(J, col, a, b);
#pragma unroll
                for (int p = 0; p <= J; ++p) pin(col[p]);
            }
            mirror_seed<TJ, q>(col, seed);
#pragma unroll
            for (int p = 0; p <= 2 * q + 1; ++p) pin(seed[p]);
            USeedPath<TJ, q + 1, Q>::run(fc, a, b, col, seed);
        }
    }
};

// Column Q of one chunk of pairs: seed path, column walk, final flush.
template <int TJ, int Q>
__device__ __forceinline__ void u_column(UStage<TJ> &st, int lane, double fc, double2 a,
                                         double2 b, int i0, int n, int npad, int chunk,
                                         double wself, double2 *__restrict__ U)
{
    double2 col[TJ + 1], seed[TJ + 1];
#pragma unroll
    for (int p = 0; p <= TJ; ++p) seed[p] = make_double2(0.0, 0.0);
    USeedPath<TJ, 0, Q>::run(fc, a, b, col, seed);
#pragma unroll
    for (int p = 0; p <= TJ; ++p) col[p] = (Q > 0 && p < 2 * Q) ? seed[p] : make_double2(0.0, 0.0);
    if constexpr (Q == 0) {
        // the recursion is linear in its starting column: starting from f_c
        // instead of 1 yields f_c u directly
        col[0] = make_double2(fc, 0.0);
        u_emit<TJ, 0, 0>(st, lane, col, i0, n, npad, chunk, wself, U);
    }
    ULevels<TJ, Q, (Q == 0 ? 1 : 2 * Q)>::run(st, lane, a, b, col, i0, n, npad, chunk, wself, U);
    u_flush<stage_end(TJ, Q), TJ>(st, lane, i0, n, npad, chunk, wself, U);
}

// uniform column index -> compile-time instance
template <int TJ, int Q>
struct UColumn {
    __device__ __forceinline__ static void run(int col, UStage<TJ> &st, int lane, double fc,
                                               double2 a, double2 b, int i0, int n, int npad,
                                               int chunk, double wself, double2 *__restrict__ U)
    {
        if constexpr (Q <= TJ / 2) {
            if (col == Q)
                u_column<TJ, Q>(st, lane, fc, a, b, i0, n, npad, chunk, wself, U);
            else
                UColumn<TJ, Q + 1>::run(col, st, lane, fc, a, b, i0, n, npad, chunk, wself, U);
        }
    }
};

template <int TJ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TJ <= 10 ? 3 : 2, 8))) void k_compute_u(int n, int npad, const double *__restrict__ pos,
                                                  const int *__restrict__ off,
                                                  const int *__restrict__ nbr, Geom g,
                                                  const UInfo *__restrict__ uinfo,
                                                  double2 *__restrict__ U,
                                                  int *__restrict__ pair_atom,
                                                  int *__restrict__ flag)
{
    __shared__ UStage<TJ> st;
    constexpr int NCOL = TJ / 2 + 1;
    const int lane = threadIdx.x;
    const int colq = (int)blockIdx.x % NCOL;  // uniform
    if (lane == 0) st.table = uinfo;  // read after the first flush's barrier
    const int h = lane >> 5, slot = lane & 31;
    const int i0 = ((int)blockIdx.x / NCOL) * 2;
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
            if (colq == 0) pair_atom[t] = i;
            double rv[3];
            min_image(pos, i, nbr[t], g, rv);
            if (!pair_geometry(rv, g, pg) && colq == 0) flag[0] = 1;
        }
        UColumn<TJ, 0>::run(colq, st, lane, pg.fc, pg.a, pg.b, i0, n, npad, c, g.wself, U);
    }
}

template <int TJ>
hipError_t launch_u_t(int n, int npad, const double *pos, const int *off, const int *nbr,
                      const Geom &g, const UInfo *uinfo, double2 *U, int *pair_atom, int *flag,
                      hipStream_t s)
{
    const int nblk = ((n + 1) / 2) * (TJ / 2 + 1);
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
