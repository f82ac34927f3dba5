// snap_y.hip -- compute_Y: the adjoint of eq. (y) of arXiv 2011.12875 (see snap_device.hpp).
#include <algorithm>

#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_Y (adjoint of eq. (y)) -- lanes are atoms
// ---------------------------------------------------------------------------
// first full element of rank J (blocks of (J+1)^2)
__device__ __forceinline__ int fbase_rt(int J)
{
    return (J * (J + 1) * (2 * J + 1)) / 6;  // sum_{k=1}^{J} k^2
}
// Full row px of U^Jx (true values), elements f = fbase(Jx) + px (Jx+1) + q:
// one buffer descriptor for the row (scalar registers) whose size is the
// row's Jx + 1 elements of npad atoms (none when the row is not valid), and
// the element and atom in the lane offset.  The descriptor's range check
// (on the lane offset) returns zero for the entries q > Jx and for a row
// that is not valid, so that products with them vanish: no per-entry test,
// branch or zeroing.
template <int TJ>
__device__ __forceinline__ void load_full_row(double2 (&r)[TJ + 1], int Jx, int px, bool valid,
                                              const double2 *__restrict__ U, int npad,
                                              unsigned voff)
{
    const int pv = valid ? px : 0;
    const double2 *base = U + (size_t)(fbase_rt(Jx) + pv * (Jx + 1)) * (size_t)npad;
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)base, (short)0, valid ? (Jx + 1) * npad * 16 : 0, 0x00020000);
#pragma unroll
    for (int q = 0; q <= TJ; ++q) {
        const auto v =
            __builtin_amdgcn_raw_buffer_load_b128(rs, voff + (unsigned)(q * npad * 16), 0, 0);
        r[q] = make_double2(
            __builtin_bit_cast(double, (unsigned long long)v[0] | ((unsigned long long)v[1] << 32)),
            __builtin_bit_cast(double, (unsigned long long)v[2] | ((unsigned long long)v[3] << 32)));
    }
}

// acc[q] += cpv sum_{q1} cq[q][q1] r1[q1] r2[q - q1 + D] for q < nq.
// q2 = q - q1 + D is a compile-time index into the second row.  Every
// (q, q1) with q1, q2 in [0, 2J_max] is evaluated without a test: rows are
// zero beyond J1 and J2 and the coefficient table beyond J1, so the terms
// outside the Clebsch-Gordan range add exact zeros; only the row index
// q < nq is tested, once per q.  The coefficients are uniform over the
// wavefront and sit at compile-time offsets cq[q (2J_max + 1) + q1] of the
// global table, so they are read with scalar loads and enter the products
// as scalar operands (no LDS staging, no vector registers).
template <int TJ, int D>
__device__ __forceinline__ void row_product(const double2 (&r1)[TJ + 1],
                                            const double2 (&r2)[TJ + 1], const double *__restrict__ cq,
                                            double cpv, int nq, double2 (&acc)[TJ / 2 + 1])
{
#pragma unroll
    for (int q = 0; q <= TJ / 2; ++q)
        if (q < nq) {
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

// One contribution (J1, J2 -> J) to the rows p and p + 1 of Y, accumulated
// into acc0 and acc1.  Row p pairs U^J1 row p1 with U^J2 row p - p1 + D,
// row p + 1 pairs it with p + 1 - p1 + D: the row that row p used at
// p1 - 1.  The rows therefore form one chain, U^J2 row p + 1 - p1lo + D,
// U^J1 row p1lo, U^J2 row p - p1lo + D, U^J1 row p1lo + 1, ..., in which
// every two neighbours make one row product (alternately of row p + 1 and
// row p): each step loads one row into the slot of its rank and multiplies
// the two slots.  Rows outside [0, J2] (at the two ends of the union range)
// are zero, and so are their coefficients.
template <int TJ, int D>
__device__ __forceinline__ void y_contrib(int J1, int J2, int p1lo, int p1hi, int cp_off, int p,
                                          int nq, int two, const double2 *__restrict__ U,
                                          int npad, unsigned voff,
                                          const double *__restrict__ cpt, const double *__restrict__ cq,
                                          double f, double2 *ysum, int lane)
{
    constexpr bool kTwo = y_unit_rows(TJ) == 2;
    // the contribution's own sums: kept local, so that no accumulator is
    // live across the dispatch over D (each branch would hold its own copy)
    double2 acc0[TJ / 2 + 1], acc1[TJ / 2 + 1];
#pragma unroll
    for (int q = 0; q <= TJ / 2; ++q) {
        acc0[q] = make_double2(0.0, 0.0);
        acc1[q] = make_double2(0.0, 0.0);
    }
    double2 s1[TJ + 1], s2[TJ + 1];  // the current rows of U^J1 and U^J2
    if (kTwo && two) {
        const int p2 = p + 1 - p1lo + D;
        load_full_row<TJ>(s2, J2, p2, p2 <= J2, U, npad, voff);
    }
    for (int p1 = p1lo; p1 <= p1hi; ++p1) {
        // re-derive the bounds in every iteration: hoisted out of the loop,
        // the guard compares below would each hold a scalar register for the
        // whole loop and spill
        int j1 = J1, j2 = J2, qn = nq;
        asm volatile("" : "+s"(j1), "+s"(j2), "+s"(qn));
        const double *cp = cpt + cp_off + 2 * (p1 - p1lo);
        // the row coefficients are wavefront-uniform; at the two ends of the
        // union range one of the rows has none (zero), and its product is
        // skipped by a scalar branch
        const double c0 = cp[0], c1 = cp[1];
        load_full_row<TJ>(s1, j1, p1, true, U, npad, voff);
        if (kTwo && two && c1 != 0.0) row_product<TJ, D>(s1, s2, cq, f * c1, qn, acc1);
        const int p2 = p - p1 + D;
        load_full_row<TJ>(s2, j2, p2, p2 >= 0, U, npad, voff);
        if (c0 != 0.0) row_product<TJ, D>(s1, s2, cq, f * c0, qn, acc0);
    }
    // ysum[(r (J_max/2 + 1) + q) 64 + lane]: this lane's entries only
#pragma unroll
    for (int q = 0; q <= TJ / 2; ++q)
        if (q < nq) {
            double2 *a = ysum + q * 64 + lane;
            a->x += acc0[q].x;
            a->y += acc0[q].y;
            if constexpr (kTwo) {
                double2 *b = ysum + ((TJ / 2 + 1) + q) * 64 + lane;
                b->x += acc1[q].x;
                b->y += acc1[q].y;
            }
        }
}

template <int TJ, int D>
struct YDispatch {
    __device__ __forceinline__ static void run(int d, int J1, int J2, int p1lo, int p1hi,
                                               int cp_off, int p, int nq, int two,
                                               const double2 *__restrict__ U, int npad,
                                               unsigned voff, const double *__restrict__ cpt,
                                               const double *__restrict__ cq, double f, double2 *ysum,
                                               int lane)
    {
        if (d == D)
            y_contrib<TJ, D>(J1, J2, p1lo, p1hi, cp_off, p, nq, two, U, npad, voff, cpt, cq, f,
                             ysum, lane);
        else
            YDispatch<TJ, D + 1>::run(d, J1, J2, p1lo, p1hi, cp_off, p, nq, two, U, npad, voff,
                                      cpt, cq, f, ysum, lane);
    }
};
template <int TJ>
struct YDispatch<TJ, TJ + 1> {
    __device__ __forceinline__ static void run(int, int, int, int, int, int, int, int, int,
                                               const double2 *__restrict__, int, unsigned,
                                               const double *__restrict__, const double *, double,
                                               double2 *, int)
    {
    }
};

// Workgroup = (unit of rows p, p + 1 of J, block of 64 atoms); its
// contributions are split over four wavefronts, each of which adds its
// contributions' sums into its own LDS slice (an accumulator held in
// registers across the dispatch over D would be duplicated in every
// branch), and the slices are reduced at the end.
// Workgroup u runs on XCD u mod 8, which owns the atom blocks congruent to
// it mod 8 (blocks padded to a multiple of 8).  An XCD walks its blocks in
// groups of kYGroup: within a group unit-major (the units are sorted by
// decreasing cost, so the heavy units of the group start first), group after
// group, so its L2 holds the U of kYGroup blocks (1.2 MB at 2J = 8) whatever
// the system size.  Also writes the unit's share of the energy,
// (1/3) sum_q Re(Y~ conj(U~)) over its rows, to Epart.
constexpr int kYGroup = 4;
template <int TJ>
__global__ __launch_bounds__(64 * kYWaves) __attribute__((amdgpu_waves_per_eu(2, 4))) void k_compute_y(
    int n, int npad, int nhalf, int nblk8, const double2 *__restrict__ U, double2 *__restrict__ Y,
    const YRowC *__restrict__ rows, const YContrib *__restrict__ contribs,
    const double *__restrict__ cpt, const double *__restrict__ cqt,
    const double *__restrict__ beta, int per_atom_beta, int nb, const int *__restrict__ btype,
    int nelem, const double *__restrict__ gscale, double *__restrict__ Epart)
{
    __shared__ double2 yw[kYWaves][y_unit_rows(TJ)][TJ / 2 + 1][64];
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
    const int two = __builtin_amdgcn_readfirstlane(row->two);
    const double gs = gscale ? gscale[asafe] : 1.0;
    // coefficient row of this atom: its own (per-atom), its element's
    // (several elements; the type is clamped, a bad one is reported by
    // compute_U), or the one shared row
    int brow = per_atom_beta ? asafe : 0;
    if (btype) {
        const int t = btype[asafe];
        brow = t < 0 ? 0 : (t >= nelem ? nelem - 1 : t);
    }

    // the wave's sums of the unit's rows, in LDS
    double2 *ysum = &yw[w][0][0][0];
#pragma unroll
    for (int k = 0; k < y_unit_rows(TJ) * (TJ / 2 + 1); ++k) ysum[k * 64 + lane] = make_double2(0.0, 0.0);
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
        // the contribution's weight (multiplicity, beta, per-atom scale)
        // rides on the row coefficients, so products accumulate into y
        const double bl = beta[(size_t)brow * nb + cl];
        const double f = C->factor * bl * gs;
        YDispatch<TJ, 0>::run(D, J1, J2, p1lo, p1hi, cp_off, p, nq, two, U, npad, voff, cpt,
                              cqt + cq_off, f, ysum, lane);
    }
    __syncthreads();
    if (w == 0) {
        double e = 0.0;
        for (int r = 0; r < y_unit_rows(TJ) && r <= two; ++r)
            for (int q = 0; q < nq; ++q) {
                double2 s = yw[0][r][q][lane];
#pragma unroll
                for (int v = 1; v < kYWaves; ++v) {
                    s.x += yw[v][r][q][lane].x;
                    s.y += yw[v][r][q][lane].y;
                }
                const double sc = row->oscale[r][q];
                s.x *= sc;
                s.y *= sc;
                Y[(size_t)atom * nhalf + row->ebase + r + q * (J + 1)] = s;
                const double2 u = U[(size_t)(row->frow + r * (J + 1) + q) * npad + atom];
                e += (s.x * u.x + s.y * u.y) * row->einv[r][q];
            }
        if (Epart && atom < n) Epart[(size_t)rix * npad + atom] = e;
    }
}

// ---------------------------------------------------------------------------
// compute_Y with the U of a block of 32 atoms staged in LDS (2J <= 8)
// ---------------------------------------------------------------------------
// The U rows of compute_Y above come through the texture path, whose latency
// the wavefronts cannot hide (they wait on it a third of their time).  Here a
// workgroup first copies the full U of kYLdsAtoms atoms into LDS (146 KB at
// 2J = 8) and its kYLdsWaves wavefronts then read every row from there.
// Lanes 0..31 compute row p and lanes 32..63 row p + 1 of the unit for the
// same 32 atoms; the half of row p + 1 walks its rows of U^J1 shifted by one,
// so at each step one of the two loaded rows is common to both halves.  A
// unit's contributions are split over several wavefronts (tasks); their
// partial sums meet in LDS after the products (the U area is free by then)
// and the unit's wavefront adds them in a fixed order.
constexpr int nfull_of(int TJ) { return (TJ + 1) * (TJ + 2) * (2 * TJ + 3) / 6; }

// Row px of U^Jx of the staged block for this lane's atom: us_a = &us[0][a],
// fb = fbase(Jx) + px (Jx + 1).  All 2J_max + 1 entries are read (entries
// beyond Jx hold other finite U values, and their Clebsch-Gordan coefficients
// are zero); every index stays inside the staged block.
template <int TJ>
__device__ __forceinline__ void lds_row(double2 (&r)[TJ + 1], const double2 *us_a, int fb)
{
    const double2 *row = us_a + fb * kYLdsAtoms;
#pragma unroll
    for (int q = 0; q <= TJ; ++q) r[q] = row[q * kYLdsAtoms];
}

template <int TJ, int D>
__device__ __forceinline__ void yl_contrib(const YLContrib *C, int J1, int J2, int p, int h,
                                           int nq, const double *__restrict__ cpt,
                                           const double *__restrict__ cq, double f,
                                           const double2 *us_a, double2 (&acc)[TJ / 2 + 1])
{
    const int nsteps = __builtin_amdgcn_readfirstlane(C->nsteps);
    const int cp_off = __builtin_amdgcn_readfirstlane(C->cp_off);
    const int lo0 = __builtin_amdgcn_readfirstlane(C->lo[0]);
    const int lo1 = __builtin_amdgcn_readfirstlane(C->lo[1]);
    const int lo = h ? lo1 : lo0;
    const int fb1 = fbase_rt(J1), fb2 = fbase_rt(J2);
    double2 r1[TJ + 1], r2[TJ + 1];
    for (int k = 0; k < nsteps; ++k) {
        // a half past the end of its range reads a clamped row (zero coefficient)
        const int p1 = min(lo + k, J1);
        const int p2 = min(max(p + h - (lo + k) + D, 0), J2);
        lds_row<TJ>(r1, us_a, fb1 + p1 * (J1 + 1));
        lds_row<TJ>(r2, us_a, fb2 + p2 * (J2 + 1));
        const double c0 = cpt[cp_off + 2 * k], c1 = cpt[cp_off + 2 * k + 1];
        row_product<TJ, D>(r1, r2, cq, f * (h ? c1 : c0), nq, acc);
    }
}

template <int TJ, int D>
struct YLDispatch {
    __device__ __forceinline__ static void run(int d, const YLContrib *C, int J1, int J2, int p,
                                               int h, int nq, const double *__restrict__ cpt,
                                               const double *__restrict__ cq, double f,
                                               const double2 *us_a, double2 (&acc)[TJ / 2 + 1])
    {
        if (d == D)
            yl_contrib<TJ, D>(C, J1, J2, p, h, nq, cpt, cq, f, us_a, acc);
        else
            YLDispatch<TJ, D + 1>::run(d, C, J1, J2, p, h, nq, cpt, cq, f, us_a, acc);
    }
};
template <int TJ>
struct YLDispatch<TJ, TJ + 1> {
    __device__ __forceinline__ static void run(int, const YLContrib *, int, int, int, int, int,
                                               const double *__restrict__,
                                               const double *__restrict__, double,
                                               const double2 *, double2 (&)[TJ / 2 + 1])
    {
    }
};

// Workgroup wg runs on XCD wg mod 8, which owns the atom blocks congruent to
// it mod 8; the G workgroups (groups of units) of one block are numbered
// consecutively on that XCD, so they run together and share its L2 copy of
// the block's U.
template <int TJ>
__global__ __launch_bounds__(64 * kYLdsWaves) void k_compute_y_lds(
    int n, int npad, int nhalf, int G, const double2 *__restrict__ U, double2 *__restrict__ Y,
    const YRowC *__restrict__ rows, const YLTask *__restrict__ tasks,
    const YLGroup *__restrict__ groups, const YLContrib *__restrict__ contribs,
    const double *__restrict__ cpt, const double *__restrict__ cqt,
    const double *__restrict__ beta, int per_atom_beta, int nb, const int *__restrict__ btype,
    int nelem, const double *__restrict__ gscale, double *__restrict__ Epart)
{
    constexpr int NF = nfull_of(TJ);
    constexpr int NQ = TJ / 2 + 1;
    // the U of the block, later the partial sums of every wavefront
    constexpr int NLDS = NF * kYLdsAtoms > kYLdsWaves * NQ * 64 ? NF * kYLdsAtoms
                                                                  : kYLdsWaves * NQ * 64;
    __shared__ double2 us[NLDS];
    const int wg = blockIdx.x;
    const int slot = wg >> 3;
    const int g = slot % G;
    const int blk = (slot / G) * 8 + (wg & 7);
    const int a0 = blk * kYLdsAtoms;
    if (a0 >= n) return;  // padding workgroup (uniform)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, a = lane & 31;
    const int atom = a0 + a;  // < npad
    // stage the block's full U: element row f of 32 atoms is 512 contiguous bytes
    for (int f = threadIdx.x >> 5; f < NF; f += 2 * kYLdsWaves)
        us[f * kYLdsAtoms + a] = U[(size_t)f * npad + atom];
    __syncthreads();

    const double2 *us_a = us + a;
    double2 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = make_double2(0.0, 0.0);
    const YLTask *tk = tasks + g * kYLdsWaves + w;
    const int unit = __builtin_amdgcn_readfirstlane(tk->unit);
    if (unit >= 0) {
        const YRowC *row = rows + unit;
        const int p = __builtin_amdgcn_readfirstlane(row->p);
        const int nq = __builtin_amdgcn_readfirstlane(row->nq);
        const int asafe = atom < n ? atom : n - 1;
        const double gs = gscale ? gscale[asafe] : 1.0;
        int brow = per_atom_beta ? asafe : 0;
        if (btype) {
            const int t = btype[asafe];
            brow = t < 0 ? 0 : (t >= nelem ? nelem - 1 : t);
        }
        const int cb = __builtin_amdgcn_readfirstlane(tk->cb);
        const int ce = __builtin_amdgcn_readfirstlane(tk->ce);
        for (int c = cb; c < ce; ++c) {
            const YLContrib *C = contribs + c;
            const int J1 = __builtin_amdgcn_readfirstlane(C->j1);
            const int J2 = __builtin_amdgcn_readfirstlane(C->j2);
            const int D = __builtin_amdgcn_readfirstlane(C->d);
            const int cl = __builtin_amdgcn_readfirstlane(C->l);
            const int cq_off = __builtin_amdgcn_readfirstlane(C->cq_off);
            const double f = C->factor * beta[(size_t)brow * nb + cl] * gs;
            YLDispatch<TJ, 0>::run(D, C, J1, J2, p, h, nq, cpt, cqt + cq_off, f, us_a, acc);
        }
    }
    __syncthreads();
    // partial sums of every wavefront, [wave][q][lane], over the U area
    double2 *part = us;
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[(w * NQ + q) * 64 + lane] = acc[q];
    __syncthreads();
    const YLGroup *gr = groups + g;
    if (w < __builtin_amdgcn_readfirstlane(gr->nunits)) {
        const int u = __builtin_amdgcn_readfirstlane(gr->unit[w]);
        const YRowC *row = rows + u;
        const int J = __builtin_amdgcn_readfirstlane(row->J);
        const int nq = __builtin_amdgcn_readfirstlane(row->nq);
        const int two = __builtin_amdgcn_readfirstlane(row->two);
        const int tb = __builtin_amdgcn_readfirstlane(gr->tb[w]);
        const int te = __builtin_amdgcn_readfirstlane(gr->tb[w + 1]);
        double e = 0.0;
        if (h <= two) {
            for (int q = 0; q < nq; ++q) {
                double2 s = make_double2(0.0, 0.0);
                for (int i = tb; i < te; ++i) {
                    const int tw = __builtin_amdgcn_readfirstlane(gr->tw[i]);
                    const double2 v = part[(tw * NQ + q) * 64 + lane];
                    s.x += v.x;
                    s.y += v.y;
                }
                const double sc = row->oscale[h][q];
                s.x *= sc;
                s.y *= sc;
                Y[(size_t)atom * nhalf + row->ebase + h + q * (J + 1)] = s;
                const double2 uv = U[(size_t)(row->frow + h * (J + 1) + q) * npad + atom];
                e += (s.x * uv.x + s.y * uv.y) * row->einv[h][q];
            }
        }
        // the unit's energy share: both rows of this atom
        e += __shfl_xor(e, 32);
        if (Epart && h == 0 && atom < n) Epart[(size_t)u * npad + atom] = e;
    }
}

}  // namespace

#ifndef SNAP_TJ_CASES
#define SNAP_TJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif
#define SNAP_YLDS_CASES(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

template <int TJ>
hipError_t launch_y_t(int n, int npad, const double2 *U, double2 *Y, const DevTables &T,
                      const double *beta, int per_atom_beta, int nb, const int *btype, int nelem,
                      const double *gscale, double *Epart, hipStream_t s)
{
    const int nblk8 = (((n + 63) / 64) + 7) / 8 * 8;
    hipLaunchKernelGGL(k_compute_y<TJ>, dim3(T.nyrows * nblk8), dim3(64 * kYWaves), 0, s, n, npad,
                       T.nhalf, nblk8, U, Y, T.yrows, T.ycontrib, T.ycp, T.ycq, beta,
                       per_atom_beta, nb, btype, nelem, gscale, Epart);
    return hipGetLastError();
}

template <int TJ>
hipError_t launch_y_lds_t(int n, int npad, int gi, const double2 *U, double2 *Y,
                          const DevTables &T, const double *beta, int per_atom_beta, int nb,
                          const int *btype, int nelem, const double *gscale, double *Epart,
                          hipStream_t s)
{
    const int G = 1 << gi;
    const int nblk = (n + kYLdsAtoms - 1) / kYLdsAtoms;
    const int nblk8 = (nblk + 7) / 8 * 8;
    hipLaunchKernelGGL(k_compute_y_lds<TJ>, dim3(nblk8 * G), dim3(64 * kYLdsWaves), 0, s, n, npad,
                       T.nhalf, G, U, Y, T.yrows, T.yltask + T.yl_task_off[gi],
                       T.ylgroup + T.yl_group_off[gi], T.ylcontrib, T.ylcp, T.ycq, beta,
                       per_atom_beta, nb, btype, nelem, gscale, Epart);
    return hipGetLastError();
}

// Number of groups of units for the LDS kernel (index gi, G = 1 << gi): the
// grouping with the least estimated time, each round of workgroups costing
// the heaviest group plus the staging of a block.
static int pick_grouping(int twojmax, int n, const DevTables &T)
{
    const int nblk = (n + kYLdsAtoms - 1) / kYLdsAtoms;
    const long lds = 16L * std::max(nfull_of(twojmax) * kYLdsAtoms,
                                    kYLdsWaves * (twojmax / 2 + 1) * 64);
    const long per_cu = std::min(160L * 1024 / lds, 2L);  // 16 wavefronts per workgroup
    const long slots = 256 * per_cu;
    int best = -1;
    double bt = 0.0;
    for (int gi = 0; gi < kYLdsGroupings; ++gi) {
        if (T.yl_task_off[gi] < 0) continue;
        const long G = 1L << gi;
        const double rounds = (double)((nblk * G + slots - 1) / slots);
        const double t = rounds * ((double)T.yl_cost_total / G + 40.0 * nfull_of(twojmax));
        if (best < 0 || t < bt) {
            best = gi;
            bt = t;
        }
    }
    return best;
}

hipError_t launch_compute_y(int twojmax, int n, int npad, const double2 *U, double2 *Y,
                            const DevTables &T, const double *beta, int per_atom_beta, int nb,
                            const int *btype, int nelem, const double *gscale, double *Epart,
                            hipStream_t s)
{
    if (T.y_lds && T.y_lds_selected && twojmax >= kYLdsMinTJ && twojmax <= kYLdsMaxTJ) {
        const int gi = pick_grouping(twojmax, n, T);
        if (gi >= 0) {
            switch (twojmax) {
#define X(k) \
    case k:  \
        return launch_y_lds_t<k>(n, npad, gi, U, Y, T, beta, per_atom_beta, nb, btype, nelem, \
                                 gscale, Epart, s);
                SNAP_YLDS_CASES(X)
#undef X
            default: break;
            }
        }
    }
    switch (twojmax) {
#define X(k) \
    case k:  \
        return launch_y_t<k>(n, npad, U, Y, T, beta, per_atom_beta, nb, btype, nelem, gscale, \
                             Epart, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
