// snap_dedr.hip -- compute_fused_dE: eq. (snapforce2) of arXiv 2011.12875 (see
// snap_device.hpp).  Compiled twice, for 2J <= 8 and 2J >= 9, so that the
// two halves of the template instances build in parallel.
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_fused_dE: dE_p = sum_J sum_half Re(Y~_i conj(dfc poly + fc dpoly))
// ---------------------------------------------------------------------------
template <int TJ, int ND>
struct DedrState {
    double2 col[TJ + 1], seed[TJ + 1];
    double2 dcol[ND][TJ + 1], dseed[ND][TJ + 1];
    double2 y[TJ + 1];  // Y~ of the current level, loaded one level ahead
    double S0, S[ND];
};

// Y~ elements eb .. eb + J of the atom (the level's stored elements) into y;
// Y points at the atom's row of Y~ (atom-major).
template <int TJ>
__device__ __forceinline__ void load_level(double2 (&y)[TJ + 1], int J, int eb,
                                           const double2 *__restrict__ Y, unsigned i, int npad)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) y[p] = Y[eb + p];
}

// One level: recursion for poly and its derivatives, then the dot with Y~.
// The top row p = J has no col[J] term; DZ marks a level whose input
// derivatives are all zero (the first level of column 0, from poly^0 = 1).
// The Y~ of the level is already in st.y; the loads of the next level
// (size Jn + 1 at half index ebn, Jn < 0 for none) are issued before the
// compiler fence that closes the level, so that their latency overlaps the
// next level's recursion.
// Above 2J = 10 the levels run in a loop over J (straight-line code would be
// too long); there both the look-ahead loads and the per-element pins cost
// more registers than the loop has, so the level loads its own Y~ instead.
template <int TJ>
constexpr bool kDedrStraight = TJ <= 10;

template <int TJ, int ND, bool DZ>
__device__ __forceinline__ void dedr_level(int J, int Jn, int ebn, DedrState<TJ, ND> &st,
                                           double2 a, double2 b, const double2 (&da)[ND],
                                           const double2 (&db)[ND],
                                           const double2 *__restrict__ Y, unsigned i, int npad,
                                           int eb = 0)
{
#pragma unroll
    for (int p = TJ; p >= 0; --p)
        if (p <= J) {
            double nr = 0.0, ni = 0.0;
            double dnr[ND], dni[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) dnr[d] = dni[d] = 0.0;
            // every component is one running sum of products (a single
            // multiply, then fused multiply-adds)
            if (p < J) {
                const double2 u = st.col[p];
                nr = a.x * u.x + a.y * u.y;
                ni = a.x * u.y - a.y * u.x;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    dnr[d] = da[d].x * u.x + da[d].y * u.y;
                    dni[d] = da[d].x * u.y - da[d].y * u.x;
                    if (!DZ) {
                        const double2 du = st.dcol[d][p];
                        dnr[d] = dnr[d] + a.x * du.x + a.y * du.y;
                        dni[d] = dni[d] + a.x * du.y - a.y * du.x;
                    }
                }
            }
            if (p > 0) {
                const double2 w = st.col[p - 1];
                nr = nr - b.x * w.x - b.y * w.y;
                ni = ni - b.x * w.y + b.y * w.x;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    dnr[d] = dnr[d] - db[d].x * w.x - db[d].y * w.y;
                    dni[d] = dni[d] - db[d].x * w.y + db[d].y * w.x;
                    if (!DZ) {
                        const double2 dw = st.dcol[d][p - 1];
                        dnr[d] = dnr[d] - b.x * dw.x - b.y * dw.y;
                        dni[d] = dni[d] - b.x * dw.y + b.y * dw.x;
                    }
                }
            }
            st.col[p] = make_double2(nr, ni);
#pragma unroll
            for (int d = 0; d < ND; ++d) st.dcol[d][p] = make_double2(dnr[d], dni[d]);
            if constexpr (kDedrStraight<TJ>) {
                // close each element's live range here (without, the level's
                // products are interleaved across elements and spill at 2J = 8)
                pin(st.col[p]);
#pragma unroll
                for (int d = 0; d < ND; ++d) pin(st.dcol[d][p]);
            }
        }
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) {
            double2 y;
            if constexpr (kDedrStraight<TJ>)
                y = st.y[p];
            else
                y = Y[eb + p];
            st.S0 += y.x * st.col[p].x + y.y * st.col[p].y;
#pragma unroll
            for (int d = 0; d < ND; ++d) st.S[d] += y.x * st.dcol[d][p].x + y.y * st.dcol[d][p].y;
        }
    if constexpr (kDedrStraight<TJ>)
        if (Jn >= 0) load_level<TJ>(st.y, Jn, ebn, Y, i, npad);
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) {
            pin(st.col[p]);
#pragma unroll
            for (int d = 0; d < ND; ++d) pin(st.dcol[d][p]);
        }
    pin(st.S0);
#pragma unroll
    for (int d = 0; d < ND; ++d) pin(st.S[d]);
    memory_fence_compiler();
}

template <int TJ, int ND, int Q>
__device__ __forceinline__ void dedr_column(DedrState<TJ, ND> &st, double2 a, double2 b,
                                            const double2 (&da)[ND], const double2 (&db)[ND],
                                            const double2 *__restrict__ Y, unsigned i, int npad)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p) {
        const bool fromseed = (Q > 0 && p < 2 * Q);
        st.col[p] = fromseed ? st.seed[p] : make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < ND; ++d)
            st.dcol[d][p] = fromseed ? st.dseed[d][p] : make_double2(0.0, 0.0);
    }
    if (Q == 0) st.col[0] = make_double2(1.0, 0.0);
    constexpr int J0 = (Q == 0) ? 1 : 2 * Q;
    // the level after the last one of this column: the first of the next
    constexpr int QN = Q + 1;
    constexpr int JN = (2 * QN <= TJ) ? 2 * QN : -1;
    constexpr int EBN = (JN >= 0) ? hbase_of(2 * QN) + QN * (2 * QN + 1) : 0;
    if constexpr (kDedrStraight<TJ>) {
#pragma unroll
        for (int J = J0; J <= TJ; ++J) {
            const int Jn = (J < TJ) ? J + 1 : JN;
            const int ebn = (J < TJ) ? hbase_of(J + 1) + Q * (J + 2) : EBN;
            if (Q == 0 && J == 1)
                dedr_level<TJ, ND, true>(J, Jn, ebn, st, a, b, da, db, Y, i, npad);
            else
                dedr_level<TJ, ND, false>(J, Jn, ebn, st, a, b, da, db, Y, i, npad);
            if (J == 2 * Q + 1 && 2 * Q + 2 <= TJ) {
                mirror_seed<TJ, Q>(st.col, st.seed);
#pragma unroll
                for (int d = 0; d < ND; ++d) mirror_seed<TJ, Q>(st.dcol[d], st.dseed[d]);
#pragma unroll
                for (int p = 0; p <= 2 * Q + 1; ++p) {
                    pin(st.seed[p]);
#pragma unroll
                    for (int d = 0; d < ND; ++d) pin(st.dseed[d][p]);
                }
            }
        }
    } else {
        int eb = hbase_of(J0) + Q * (J0 + 1);
#pragma unroll 1
        for (int J = J0; J <= TJ; ++J) {
            const int ebnext = eb + (J + 1) * (J / 2 + 1) + Q;  // half index of (J+1, 0, Q)
            dedr_level<TJ, ND, false>(J, -1, 0, st, a, b, da, db, Y, i, npad, eb);
            if (J == 2 * Q + 1 && 2 * Q + 2 <= TJ) {
                mirror_seed<TJ, Q>(st.col, st.seed);
#pragma unroll
                for (int d = 0; d < ND; ++d) mirror_seed<TJ, Q>(st.dcol[d], st.dseed[d]);
            }
            eb = ebnext;
        }
    }
}

template <int TJ, int ND, int Q>
struct DedrColumns {
    __device__ __forceinline__ static void run(DedrState<TJ, ND> &st, double2 a, double2 b,
                                               const double2 (&da)[ND], const double2 (&db)[ND],
                                               const double2 *__restrict__ Y, unsigned i, int npad)
    {
        dedr_column<TJ, ND, Q>(st, a, b, da, db, Y, i, npad);
        DedrColumns<TJ, ND, Q + 1>::run(st, a, b, da, db, Y, i, npad);
    }
};
template <int TJ, int ND>
struct DedrColumns<TJ, ND, TJ / 2 + 1> {
    __device__ __forceinline__ static void run(DedrState<TJ, ND> &, double2, double2,
                                               const double2 (&)[ND], const double2 (&)[ND],
                                               const double2 *__restrict__, unsigned, int)
    {
    }
};

template <int TJ, int ND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_dedr(int npairs, int nh, const double *__restrict__ pos,
                                             const int *__restrict__ nbr,
                                             const int *__restrict__ pair_atom,
                                             const double2 *__restrict__ Y, Geom g,
                                             double *__restrict__ dE)
{
    // Workgroup w runs on XCD w % 8; it takes the logical block
    // (w % 8) * per + w / 8, so each XCD works through a contiguous eighth of
    // the pairs and reads the Y~ of a contiguous eighth of the atoms into its
    // own L2.  The logical block is (pair block, direction), directions
    // innermost.
    constexpr int NDIR = 3 / ND;
    const int nblk = (npairs + 63) / 64;
    const int per = (nblk * NDIR + 7) / 8;
    const int w = (int)blockIdx.x;
    const int L = (w & 7) * per + (w >> 3);
    if (L >= nblk * NDIR) return;
    const int blk = L / NDIR;
    const int dir0 = (ND == 3) ? 0 : L - blk * NDIR;
    const int t = blk * 64 + threadIdx.x;
    const bool valid = t < npairs;
    const int tt = valid ? t : npairs - 1;
    const int i = pair_atom[tt];
    // Y~ of J = 0 and of the first level of column 0, ahead of the geometry
    const double2 *__restrict__ Yi = Y + (size_t)i * nh;  // the atom's row of Y~
    const int npad = 0;  // unused by the atom-major loads
    const double y00 = Yi[0].x;
    double rv[3];
    const int k = nbr[tt];
    min_image(pos, i, k, g, rv);
    double rc, wk;
    pair_cut(g, i, k, rc, wk);
    PairGeom pg;
    const bool ok = pair_geometry(rv, g, rc, wk, pg);

    // d a / d r_alpha, d b / d r_alpha and d f_c / d r_alpha
    double2 da[ND], db[ND];
    double dfc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int al = dir0 + d;
        const double nal = (al == 0) ? pg.n[0] : (al == 1) ? pg.n[1] : pg.n[2];
        const double dnx = ((al == 0 ? 1.0 : 0.0) - nal * pg.n[0]) / pg.r;
        const double dny = ((al == 1 ? 1.0 : 0.0) - nal * pg.n[1]) / pg.r;
        const double dnz = ((al == 2 ? 1.0 : 0.0) - nal * pg.n[2]) / pg.r;
        const double dth = pg.dth0 * nal;
        da[d] = ok ? make_double2(-pg.s0 * dth, -(pg.c0 * dth * pg.n[2] + pg.s0 * dnz))
                   : make_double2(0.0, 0.0);
        db[d] = ok ? make_double2(pg.c0 * dth * pg.n[1] + pg.s0 * dny,
                                  -(pg.c0 * dth * pg.n[0] + pg.s0 * dnx))
                   : make_double2(0.0, 0.0);
        dfc[d] = pg.dfdr * nal;
    }

    DedrState<TJ, ND> st;
#pragma unroll
    for (int d = 0; d < ND; ++d) st.S[d] = 0.0;
#pragma unroll
    for (int p = 0; p <= TJ; ++p) {
        st.seed[p] = make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < ND; ++d) st.dseed[d][p] = make_double2(0.0, 0.0);
    }
    if constexpr (TJ >= 1 && kDedrStraight<TJ>)
        load_level<TJ>(st.y, 1, hbase_of(1), Yi, (unsigned)i, npad);
    st.S0 = y00;  // J = 0: poly = 1, dpoly = 0
    DedrColumns<TJ, ND, 0>::run(st, pg.a, pg.b, da, db, Yi, (unsigned)i, npad);
    if (valid) {
#pragma unroll
        for (int d = 0; d < ND; ++d)
            dE[3 * (size_t)t + dir0 + d] = dfc[d] * st.S0 + pg.fc * st.S[d];
    }
}

template <int TJ>
hipError_t launch_dedr_t(int dirs, int npairs, int npad, const double *pos, const int *nbr,
                         const int *pair_atom, const double2 *Y, const Geom &g, double *dE,
                         hipStream_t s)
{
    // one workgroup per (64 pairs, direction group), padded to a multiple of
    // 8 for the XCD mapping in the kernel (the padding exits at once)
    const int nblk = (npairs + 63) / 64;
    const int nlog = nblk * (dirs == 3 ? 1 : 3);
    const int ngrid = ((nlog + 7) / 8) * 8;
    if (dirs == 3)
        hipLaunchKernelGGL((k_dedr<TJ, 3>), dim3(ngrid), dim3(64), 0, s, npairs, npad, pos, nbr,
                           pair_atom, Y, g, dE);
    else
        hipLaunchKernelGGL((k_dedr<TJ, 1>), dim3(ngrid), dim3(64), 0, s, npairs, npad, pos, nbr,
                           pair_atom, Y, g, dE);
    return hipGetLastError();
}

}  // namespace

#if defined(SNAP_DEDR_LOW)
#define SNAP_DEDR_FN launch_dedr_low
#define SNAP_TJ_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#else
#define SNAP_DEDR_FN launch_dedr_high
#define SNAP_TJ_CASES(X) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

hipError_t SNAP_DEDR_FN(int twojmax, int dirs, int npairs, int npad, const double *pos,
                       const int *nbr, const int *pair_atom, const double2 *Y, const DevTables &T,
                       const Geom &g, double *dE, hipStream_t s)
{
    (void)T;
    switch (twojmax) {
#define X(k) \
    case k: return launch_dedr_t<k>(dirs, npairs, npad, pos, nbr, pair_atom, Y, g, dE, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
