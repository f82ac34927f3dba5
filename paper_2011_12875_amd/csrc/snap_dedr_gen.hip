// snap_dedr_gen.hip -- compute_fused_dE (eq. (snapforce2) of arXiv 2011.12875)
// through the generators of the rotation group instead of a derivative
// recursion per direction.
//
// u_j(r) is the matrix of an SU(2) element g(r) acting on degree-2j
// polynomials.  Column q of the unnormalised coefficients (snap_device.hpp)
// is the product L1^(J-q) L2^q of the two linear forms L1 = a* x - b* y,
// L2 = b x + a y.  Differentiating the product and writing dL1, dL2 back in
// the basis {L1, L2} gives, for a displacement of r along direction alpha,
//   d poly_{.,q} = (J - 2q) al11 poly_{.,q} + (J - q) al21 poly_{.,q+1}
//                  + q al12 poly_{.,q-1},
//   al11 = a da* + b db*,  al21 = b* da* - a* db*,  al12 = a db - b da
// (da, db: derivatives of the Cayley-Klein pair along alpha; |a|^2 + |b|^2
// = 1 makes the diagonal coefficient (J - q) al11 + q al22 = (J - 2q) al11).
// The derivative of level J is tridiagonal in the column index, with integer
// weights, and the direction enters only through three complex numbers.  So
// the contraction with Y~ of eq. (snapforce2) needs, per pair, only three
// complex sums over the stored half, independent of the direction:
//   A0 = sum (J - 2q) Y~_pq conj(poly_pq)
//   Ap = sum (J - q)  Y~_pq conj(poly_p,q+1)
//   Am = sum  q       Y~_pq conj(poly_p,q-1)
// (poly_p,q+1 outside the stored half by the mirror rule), and then
//   dE_alpha = dfc_alpha S0 + f_c Re[al11* A0 + al21* Ap + al12* Am],
//   S0 = sum Re(Y~_pq conj(poly_pq)).
// One walk of the recursion per pair replaces the three derivative
// recursions of the tangent form (snap_dedr.hip): about 3.5x fewer
// floating-point operations at 2J = 8.
//
// Walking column c of level J, each element poly_pc meets Y~ of columns
// c - 1 (its Ap term), c (A0, S0) and c + 1 (Am); the column ceil(J/2) - 1
// also carries the Ap term of the last stored column, whose partner
// poly_p,q+1 is the mirror of poly_J-p,c.
//
// One lane per pair; the rows of Y~ the wavefront needs are staged in LDS
// (or, as a measured alternative, read through the texture path).
#include <algorithm>

#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

template <int TJ>
struct GenState {
    double2 col[TJ + 1], seed[TJ + 1];
    double2 A0, Ap, Am;
    double S0;
};

// Y~ of one atom: its row of the atom-major Y~ in global memory, or the copy
// of that row in LDS.
struct YRow {
    const double2 *__restrict__ p;
    __device__ __forceinline__ double2 get(int e) const { return p[e]; }
};

// Above 2J = 10 the levels of a column run in a loop (straight-line code for
// every level would not fit the instruction cache).
template <int TJ>
constexpr bool kGenStraight = TJ <= 10;

// MIR: the level may carry the mirror term (J = 2C + 1 or 2C + 2), which
// indexes the column at J - p: J must then be a compile-time constant.
template <int TJ, bool MIR, class YS>
__device__ __forceinline__ void gen_level(int C, int J, GenState<TJ> &st, double2 a, double2 b,
                                          const YS &ys)
{
    poly_step<TJ>(J, st.col, a, b);
    if (J == 2 * C + 1 && 2 * C + 2 <= TJ) {
        // seed of column C + 1: poly_{p,C+1} = (-1)^(C+1-p) conj(poly_{2C+1-p,C})
#pragma unroll
        for (int p = 0; p <= TJ; ++p)
            if (p <= 2 * C + 1) {
                const double sg = ((C + 1 - p) & 1) ? -1.0 : 1.0;
                const double2 m = st.col[2 * C + 1 - p];
                st.seed[p] = make_double2(sg * m.x, -sg * m.y);
            }
    }
    const int eb = hbase_of(J);                  // half index of (J, p = 0, q = 0)
    const bool has_m = C >= 1;                   // Ap term of column C - 1
    const bool has_p = 2 * (C + 1) <= J;         // Am term of column C + 1
    const bool mir_even = MIR && !(J & 1) && 2 * C + 2 == J;  // Ap of column J/2 (mirror partner)
    const bool mir_odd = MIR && (J & 1) && 2 * C + 1 == J;    // Ap of column (J-1)/2
    double t0r = 0.0, t0i = 0.0, tmr = 0.0, tmi = 0.0, tpr = 0.0, tpi = 0.0, trr = 0.0,
           tri = 0.0;
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) {
            const double2 u = st.col[p];
            const double2 y0 = ys.get(eb + C * (J + 1) + p);
            // Y~ conj(u), each component a running sum of fused multiply-adds
            t0r = fma(y0.x, u.x, t0r);
            t0r = fma(y0.y, u.y, t0r);
            t0i = fma(y0.y, u.x, t0i);
            t0i = fma(-y0.x, u.y, t0i);
            if (has_m) {
                const double2 ym = ys.get(eb + (C - 1) * (J + 1) + p);
                tmr = fma(ym.x, u.x, tmr);
                tmr = fma(ym.y, u.y, tmr);
                tmi = fma(ym.y, u.x, tmi);
                tmi = fma(-ym.x, u.y, tmi);
            }
            double2 yr = y0;
            if (has_p) {
                const double2 yp = ys.get(eb + (C + 1) * (J + 1) + p);
                tpr = fma(yp.x, u.x, tpr);
                tpr = fma(yp.y, u.y, tpr);
                tpi = fma(yp.y, u.x, tpi);
                tpi = fma(-yp.x, u.y, tpi);
                yr = yp;
            }
            if (MIR && (mir_even || mir_odd)) {
                // Y~_{p,q} poly_{J-p,C} (no conjugate): the mirror rule gives
                // poly_{p,q+1} = (-1)^(J-p-C) conj(poly_{J-p,C}); the sign is
                // a compile-time constant folded into the operands
                const double2 w = st.col[J - p];
                const double sg = ((J - p - C) & 1) ? -1.0 : 1.0;
                trr = fma(sg * yr.x, w.x, trr);
                trr = fma(-sg * yr.y, w.y, trr);
                tri = fma(sg * yr.x, w.y, tri);
                tri = fma(sg * yr.y, w.x, tri);
            }
            // at most two rows of Y~ reads in flight (hoisted, the reads of a
            // whole level would hold ~100 registers)
            if (kGenStraight<TJ> && (p & 1)) memory_fence_compiler();
        }
    st.S0 += t0r;
    const double w0 = (double)(J - 2 * C);
    st.A0.x += w0 * t0r;
    st.A0.y += w0 * t0i;
    if (has_m) {
        const double wm = (double)(J - C + 1);
        st.Ap.x += wm * tmr;
        st.Ap.y += wm * tmi;
    }
    if (has_p) {
        const double wp = (double)(C + 1);
        st.Am.x += wp * tpr;
        st.Am.y += wp * tpi;
    }
    if (mir_even || mir_odd) {
        const double wr = mir_even ? (double)(J / 2) : (double)(J - C);
        st.Ap.x += wr * trr;
        st.Ap.y += wr * tri;
    }
}

// Column C walked in full: levels max(1, 2C) .. TJ with their terms.
template <int TJ, int C, class YS>
__device__ __forceinline__ void walk_column(GenState<TJ> &st, double2 a, double2 b, const YS &ys)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        st.col[p] = (C > 0 && p < 2 * C) ? st.seed[p] : make_double2(0.0, 0.0);
    if (C == 0) st.col[0] = make_double2(1.0, 0.0);
    constexpr int J0 = (C == 0) ? 1 : 2 * C;
    if constexpr (kGenStraight<TJ>) {
#pragma unroll
        for (int J = J0; J <= TJ; ++J) {
            gen_level<TJ, true>(C, J, st, a, b, ys);
#pragma unroll
            for (int p = 0; p <= TJ; ++p)
                if (p <= J) pin(st.col[p]);
            memory_fence_compiler();
        }
    } else {
        // the levels with the seed and the mirror terms at compile time, the
        // rest in a loop
        constexpr int JP = (2 * C + 2 < TJ) ? 2 * C + 2 : TJ;
#pragma unroll
        for (int J = J0; J <= JP; ++J) gen_level<TJ, true>(C, J, st, a, b, ys);
#pragma unroll 1
        for (int J = JP + 1; J <= TJ; ++J) gen_level<TJ, false>(C, J, st, a, b, ys);
    }
}

// Column C on its seed path only: levels max(1, 2C) .. 2C + 1, mirrored into
// the seed of column C + 1 (no terms).
template <int TJ, int C>
__device__ __forceinline__ void seed_column(GenState<TJ> &st, double2 a, double2 b)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        st.col[p] = (C > 0 && p < 2 * C) ? st.seed[p] : make_double2(0.0, 0.0);
    if (C == 0) st.col[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int J = (C == 0 ? 1 : 2 * C); J <= 2 * C + 1; ++J) poly_step<TJ>(J, st.col, a, b);
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= 2 * C + 1) {
            const double sg = ((C + 1 - p) & 1) ? -1.0 : 1.0;
            const double2 m = st.col[2 * C + 1 - p];
            st.seed[p] = make_double2(sg * m.x, -sg * m.y);
        }
}

// Columns C .. CE - 1: those below CB on their seed path, the others walked.
template <int TJ, int C, int CB, int CE, class YS>
__device__ __forceinline__ void gen_columns(GenState<TJ> &st, double2 a, double2 b, const YS &ys)
{
    if constexpr (C < CB)
        seed_column<TJ, C>(st, a, b);
    else
        walk_column<TJ, C>(st, a, b, ys);
    if constexpr (C + 1 < CE) gen_columns<TJ, C + 1, CB, CE>(st, a, b, ys);
}

// Split of the columns over NR wavefronts: wavefront r walks the columns
// [col_begin(TJ, NR, r), col_begin(TJ, NR, r + 1)) after the seed paths of
// the columns before them.  The split minimises the largest share, an element
// of a walk costing about 2.5 times one of a seed path (three multiply-adds
// of Y~ on top of the recursion).
constexpr int col_elems(int TJ, int c)
{
    int e = 0;
    for (int J = (c == 0 ? 1 : 2 * c); J <= TJ; ++J) e += J + 1;
    return e;
}
constexpr int seed_elems(int c)
{
    int e = 0;
    for (int J = (c == 0 ? 1 : 2 * c); J <= 2 * c + 1; ++J) e += J + 1;
    return e;
}
// cost of a wavefront walking columns [b, e)
constexpr int role_cost(int TJ, int b, int e)
{
    int c0 = 0;
    for (int c = 0; c < b; ++c) c0 += 2 * seed_elems(c);
    for (int c = b; c < e; ++c) c0 += 5 * col_elems(TJ, c);
    return c0;
}
struct ColSplit {
    int b[5];
};
constexpr ColSplit col_split(int TJ, int NR)
{
    const int nc = TJ / 2 + 1;
    const int nr = NR < nc ? NR : nc;  // wavefronts with columns; the rest idle
    ColSplit best{{0, nc, nc, nc, nc}};
    if (nr <= 1) return best;
    int bc = 1 << 30;
    // boundaries 0 < b1 < b2 < b3 < nc (as many as nr - 1)
    for (int b1 = 1; b1 < nc; ++b1) {
        for (int b2 = b1 + 1; b2 <= nc; ++b2) {
            if ((nr > 2) != (b2 < nc)) continue;
            for (int b3 = b2 + 1; b3 <= nc + 1; ++b3) {
                const int c3 = b3 > nc ? nc : b3;
                if ((nr > 3) != (b3 < nc)) continue;
                const int bb[5] = {0, b1, b2 > nc ? nc : b2, c3, nc};
                int m = 0;
                for (int r = 0; r < 4; ++r)
                    if (bb[r] < bb[r + 1]) {
                        const int cst = role_cost(TJ, bb[r], bb[r + 1]);
                        m = cst > m ? cst : m;
                    }
                if (m < bc) {
                    bc = m;
                    best = ColSplit{{bb[0], bb[1], bb[2], bb[3], bb[4]}};
                }
            }
        }
    }
    return best;
}
template <int TJ, int NR, int R>
constexpr int kColB = col_split(TJ, NR).b[R];

// The sums of one pair over columns [CB, CE) (the J = 0 term with the first
// column), for the wavefront's role.
template <int TJ, int CB, int CE, class YS>
__device__ __forceinline__ void gen_sums(const PairGeom &pg, const YS &ys, GenState<TJ> &st)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p) st.seed[p] = make_double2(0.0, 0.0);
    st.A0 = st.Ap = st.Am = make_double2(0.0, 0.0);
    st.S0 = (CB == 0) ? ys.get(0).x : 0.0;  // J = 0: poly = 1
    if constexpr (TJ >= 1 && CB < CE) gen_columns<TJ, 0, CB, CE>(st, pg.a, pg.b, ys);
}

// More columns [CB, CE) for a wavefront that already walked others: their
// seed path from column 0, then their walk, added to the same sums.
template <int TJ, int CB, int CE, class YS>
__device__ __forceinline__ void gen_sums_more(const PairGeom &pg, const YS &ys, GenState<TJ> &st)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p) st.seed[p] = make_double2(0.0, 0.0);
    if constexpr (CB < CE) gen_columns<TJ, 0, CB, CE>(st, pg.a, pg.b, ys);
}

// dE for the three directions from the sums.
template <int TJ>
__device__ __forceinline__ void gen_finish(const PairGeom &pg, bool ok, const GenState<TJ> &st,
                                           double dE[3])
{
    const double2 a = pg.a, b = pg.b;
    const double ir = 1.0 / pg.r;  // one division instead of nine
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const double nal = pg.n[al];
        const double dnx = ((al == 0 ? 1.0 : 0.0) - nal * pg.n[0]) * ir;
        const double dny = ((al == 1 ? 1.0 : 0.0) - nal * pg.n[1]) * ir;
        const double dnz = ((al == 2 ? 1.0 : 0.0) - nal * pg.n[2]) * ir;
        const double dth = pg.dth0 * nal;
        const double2 da = make_double2(-pg.s0 * dth, -(pg.c0 * dth * pg.n[2] + pg.s0 * dnz));
        const double2 db = make_double2(pg.c0 * dth * pg.n[1] + pg.s0 * dny,
                                        -(pg.c0 * dth * pg.n[0] + pg.s0 * dnx));
        // al11 = a conj(da) + b conj(db)
        const double2 al11 = make_double2(a.x * da.x + a.y * da.y + b.x * db.x + b.y * db.y,
                                          a.y * da.x - a.x * da.y + b.y * db.x - b.x * db.y);
        // al12 = a db - b da; al21 = conj(b) conj(da) - conj(a) conj(db) = -conj(al12)
        const double2 al12 = make_double2(a.x * db.x - a.y * db.y - (b.x * da.x - b.y * da.y),
                                          a.x * db.y + a.y * db.x - (b.x * da.y + b.y * da.x));
        const double2 al21 = make_double2(-al12.x, al12.y);
        // Re[conj(z) w] = z.x w.x + z.y w.y
        const double S = al11.x * st.A0.x + al11.y * st.A0.y + al21.x * st.Ap.x +
                         al21.y * st.Ap.y + al12.x * st.Am.x + al12.y * st.Am.y;
        dE[al] = ok ? pg.dfdr * nal * st.S0 + pg.fc * S : 0.0;
    }
}

// Rows of Y~ staged in LDS per workgroup: as many atoms as fit in
// kStageBytes (4 .. 16); 64 consecutive pairs span ~3 atoms at 26
// neighbours.
constexpr int kStageBytes = 16 * 1024;
template <int TJ>
constexpr int kStageAtoms = (kStageBytes / (16 * hbase_of(TJ + 1)) > 16)  ? 16
                            : (kStageBytes / (16 * hbase_of(TJ + 1)) < 4) ? 4
                                                                          : kStageBytes / (16 * hbase_of(TJ + 1));

// The sums of the columns of wavefront R (compile-time bounds), dispatched
// on the wavefront's uniform index.
template <int TJ, int NR, int R, class YS>
__device__ __forceinline__ void role_sums(int role, const PairGeom &pg, const YS &ys,
                                          GenState<TJ> &st)
{
    if constexpr (R < NR) {
        if (role == R) {
            constexpr int b = kColB<TJ, NR, R>, e = kColB<TJ, NR, R + 1>;
            if constexpr (TJ == 8 && NR == 3) {
                // columns {0}, {1, 4}, {2, 3}: the longest share is 329
                // elements of the cost model instead of 358 for the best
                // contiguous split {0}, {1}, {2, 3, 4}
                if constexpr (R == 0) gen_sums<TJ, 0, 1>(pg, ys, st);
                if constexpr (R == 1) {
                    gen_sums<TJ, 1, 2>(pg, ys, st);
                    gen_sums_more<TJ, 4, 5>(pg, ys, st);
                }
                if constexpr (R == 2) gen_sums<TJ, 2, 4>(pg, ys, st);
            } else if constexpr (b < e) {
                gen_sums<TJ, b, e>(pg, ys, st);
            } else {
                // no columns for this wavefront (more wavefronts than columns)
                st.A0 = st.Ap = st.Am = make_double2(0.0, 0.0);
                st.S0 = 0.0;
            }
        } else {
            role_sums<TJ, NR, R + 1>(role, pg, ys, st);
        }
    }
}

// Workgroup = 64 consecutive pairs, one lane per pair, NR wavefronts that
// split the columns (col_split); the sums of wavefronts 1 .. NR - 1 are added
// to wavefront 0's through LDS in a fixed order.  Workgroup w runs on XCD
// w % 8 and takes logical block (w % 8) * per + w / 8, so each XCD walks a
// contiguous eighth of the pairs.  The pairs of a block belong to the atoms
// pair_atom[first] .. [last] (the list is grouped by atom); when they fit
// (STAGE), their rows of Y~, one contiguous range of the atom-major array,
// are copied to LDS and every element is read from there (about 2.5 reads
// per element of the walk; a vector load costs about three times an LDS
// read).  Otherwise the lanes read Y~ from global memory.
template <int TJ, bool STAGE, int NR>
__global__ __launch_bounds__(64 * NR) void k_dedr_gen(int npairs, int ppb, int nh,
                                                      const double *__restrict__ pos,
                                                      const int *__restrict__ nbr,
                                                      const int *__restrict__ pair_atom,
                                                      const double2 *__restrict__ Y, Geom g,
                                                      double *__restrict__ dE)
{
    constexpr int NST = STAGE ? kStageAtoms<TJ> * hbase_of(TJ + 1) : 1;
    __shared__ double2 yl[NST];
    // sums of wavefronts 1 .. NR - 1, [NR - 1][7][64]
    __shared__ double part[(NR > 1 ? (NR - 1) * 7 * 64 : 1)];
    const int nblk = (npairs + ppb - 1) / ppb;
    const int per = (nblk + 7) / 8;
    const int w = (int)blockIdx.x;
    const int L = (w & 7) * per + (w >> 3);
    if (L >= nblk) return;  // uniform for the workgroup
    const int role = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const int t = L * ppb + lane;
    const bool valid = lane < ppb && t < npairs;
    const int tt = valid ? t : min(L * ppb + ppb - 1, npairs - 1);  // a pair of the block
    const int i = pair_atom[tt];
    const int k = nbr[tt];
    double rv[3];
    min_image(pos, i, k, g, rv);
    double rc, wk;
    pair_cut(g, i, k, rc, wk);
    PairGeom pg;
    const bool ok = pair_geometry(rv, g, rc, wk, pg);
    // the geometry the last step needs waits in LDS during the walk (only the
    // Cayley-Klein pair stays in registers)
    __shared__ double keep[9][64];
    if (role == 0) {
        keep[0][lane] = pg.n[0];
        keep[1][lane] = pg.n[1];
        keep[2][lane] = pg.n[2];
        keep[3][lane] = pg.r;
        keep[4][lane] = pg.c0;
        keep[5][lane] = pg.s0;
        keep[6][lane] = pg.dth0;
        keep[7][lane] = pg.fc;
        keep[8][lane] = pg.dfdr;
    }
    memory_fence_compiler();
    GenState<TJ> st;
    bool staged = false;
    if constexpr (STAGE) {
        const int afirst = __builtin_amdgcn_readfirstlane(pair_atom[L * ppb]);
        const int alast =
            __builtin_amdgcn_readfirstlane(pair_atom[min(L * ppb + ppb - 1, npairs - 1)]);
        if (alast - afirst < kStageAtoms<TJ>) {  // uniform
            staged = true;
            const int cnt = (alast - afirst + 1) * nh;
            const double2 *src = Y + (size_t)afirst * nh;
            for (int e = (int)threadIdx.x; e < cnt; e += 64 * NR) yl[e] = src[e];
            __syncthreads();
            // (i - afirst is in range for a list grouped by atom; clamped so
            // that no other list can read outside the staged rows)
            const int ia = min(max(i - afirst, 0), alast - afirst);
            role_sums<TJ, NR, 0>(role, pg, YRow{yl + ia * nh}, st);
        }
    }
    if (!staged) role_sums<TJ, NR, 0>(role, pg, YRow{Y + (size_t)i * nh}, st);
    if constexpr (NR > 1) {
        if (role > 0) {
            double *pr = &part[(role - 1) * 7 * 64];
            pr[0 * 64 + lane] = st.S0;
            pr[1 * 64 + lane] = st.A0.x;
            pr[2 * 64 + lane] = st.A0.y;
            pr[3 * 64 + lane] = st.Ap.x;
            pr[4 * 64 + lane] = st.Ap.y;
            pr[5 * 64 + lane] = st.Am.x;
            pr[6 * 64 + lane] = st.Am.y;
        }
        __syncthreads();
        if (role > 0) return;
#pragma unroll
        for (int r = 0; r < NR - 1; ++r) {
            const double *pr = &part[r * 7 * 64];
            st.S0 += pr[0 * 64 + lane];
            st.A0.x += pr[1 * 64 + lane];
            st.A0.y += pr[2 * 64 + lane];
            st.Ap.x += pr[3 * 64 + lane];
            st.Ap.y += pr[4 * 64 + lane];
            st.Am.x += pr[5 * 64 + lane];
            st.Am.y += pr[6 * 64 + lane];
        }
    }
    memory_fence_compiler();
    pg.n[0] = keep[0][lane];
    pg.n[1] = keep[1][lane];
    pg.n[2] = keep[2][lane];
    pg.r = keep[3][lane];
    pg.c0 = keep[4][lane];
    pg.s0 = keep[5][lane];
    pg.dth0 = keep[6][lane];
    pg.fc = keep[7][lane];
    pg.dfdr = keep[8][lane];
    double d[3];
    gen_finish<TJ>(pg, ok, st, d);
    if (valid) {
        dE[3 * (size_t)t + 0] = d[0];
        dE[3 * (size_t)t + 1] = d[1];
        dE[3 * (size_t)t + 2] = d[2];
    }
}

// Wavefronts per block of 64 pairs (the columns split over them): one up to
// 2J = 4, where the walk is short, two above.
template <int TJ>
constexpr int kGenRoles = TJ >= 5 ? 2 : 1;

template <int TJ, bool STAGE, int NR>
void launch_gen_nr(int ngrid, hipStream_t s, int npairs, int ppb, int nh, const double *pos,
                   const int *nbr, const int *pair_atom, const double2 *Y, const Geom &g,
                   double *dE)
{
    hipLaunchKernelGGL((k_dedr_gen<TJ, STAGE, NR>), dim3(ngrid), dim3(64 * NR), 0, s, npairs, ppb,
                       nh, pos, nbr, pair_atom, Y, g, dE);
}

// Pairs per block: up to 64, as few as keep the blocks a multiple of the
// compute-unit count (every CU then runs the same number of blocks; 51 990
// pairs on 256 CUs: 51 per block, 4 blocks per CU, instead of 64 per block
// with 48 CUs running a fourth block while the others idle).
static int pairs_per_block(int npairs, int ncu)
{
    if (ncu <= 0) return 64;
    const long per_round = 64L * ncu;
    const long rounds = (npairs + per_round - 1) / per_round;
    const long ppb = (npairs + ncu * rounds - 1) / (ncu * rounds);
    return (int)std::max(1L, std::min(64L, ppb));
}

template <int TJ>
hipError_t launch_gen_t(int mapping, int waves, int ncu, int npairs, int nh, const double *pos,
                        const int *nbr, const int *pair_atom, const double2 *Y, const Geom &g,
                        double *dE, hipStream_t s)
{
    // one workgroup per block of pairs, padded to a multiple of 8 (the
    // padding exits)
    const int ppb = pairs_per_block(npairs, ncu);
    const int nblk = (npairs + ppb - 1) / ppb;
    const int ngrid = ((nblk + 7) / 8) * 8;
    int nr = waves > 0 ? waves : kGenRoles<TJ>;
    // At 2J = 7 and 8 the two-way column split is uneven (at 2J = 8 the
    // larger share is 430 against 358 elements of the cost model) and a
    // three-way split shortens the longest share; it pays while the blocks
    // leave room for a third wavefront per SIMD (at most four blocks per CU):
    // 2000 atoms, 2J = 8: 19.2 -> 16.5 us, 2J = 7: 15.8 -> 15.2 us, measured.
    // With more blocks the extra seed paths cost more than they save.
    if (waves == 0 && (TJ == 7 || TJ == 8) && ncu > 0 && nblk <= 4 * ncu) nr = 3;
    if (mapping == 1) {
        launch_gen_nr<TJ, false, kGenRoles<TJ>>(ngrid, s, npairs, ppb, nh, pos, nbr, pair_atom, Y,
                                                g, dE);
        return hipGetLastError();
    }
    switch (nr) {
    case 1:
        launch_gen_nr<TJ, true, 1>(ngrid, s, npairs, ppb, nh, pos, nbr, pair_atom, Y, g, dE);
        break;
    case 2:
        launch_gen_nr<TJ, true, 2>(ngrid, s, npairs, ppb, nh, pos, nbr, pair_atom, Y, g, dE);
        break;
    case 3:
        launch_gen_nr<TJ, true, 3>(ngrid, s, npairs, ppb, nh, pos, nbr, pair_atom, Y, g, dE);
        break;
    default:
        launch_gen_nr<TJ, true, 4>(ngrid, s, npairs, ppb, nh, pos, nbr, pair_atom, Y, g, dE);
        break;
    }
    return hipGetLastError();
}

}  // namespace

#ifndef SNAP_TJ_CASES
#define SNAP_TJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

hipError_t launch_dedr_gen(int twojmax, int mapping, int waves, int ncu, int npairs, int nh,
                           const double *pos, const int *nbr, const int *pair_atom,
                           const double2 *Y, const Geom &g, double *dE, hipStream_t s)
{
    switch (twojmax) {
#define X(k) \
    case k:  \
        return launch_gen_t<k>(mapping, waves, ncu, npairs, nh, pos, nbr, pair_atom, Y, g, dE, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
