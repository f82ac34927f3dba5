// snap_u.hip -- compute_U: eq. (u) of arXiv 2011.12875 (see snap_device.hpp).
#include "snap_device.hpp"

namespace snapmi {

namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// compute_U
//
// A workgroup is one wavefront holding four atoms of 16 lanes each; every
// lane walks two pairs of its atom in lockstep (neighbours 32c + slot and
// 32c + 16 + slot of chunk c; neighbour lists longer than 32 run in chunks)
// and stages the sum of the two.  The per-atom sum over the 16 lanes then
// runs on all 64 lanes of the wavefront (4 atoms x 16 staged elements).
//
// The stored half (q <= J/2) of every u_j is produced column by column by
// the recursion of eq. (hysphrecur) on the unnormalised polynomial
// coefficients; the start of column q+1 is column q at level 2q+1,
// mirrored.  Each column has its own workgroup (one per column and group of
// four atoms).  The workgroup of column Q first reruns the short seed path
// -- levels 2q and 2q+1 of every column q < Q -- and then the levels
// 2Q..2J_max of column Q.  Both parts together cost (2J_max+1)(2J_max+2)/2
// elements whatever Q is (45 at 2J = 8), so the columns are evenly loaded,
// for 70 extra elements per pair at 2J = 8 (225 instead of 155).
// ---------------------------------------------------------------------------
#ifndef SNAP_U_STAGE
#define SNAP_U_STAGE 12
#endif
#ifndef SNAP_U_WAVES_PER_EU
#define SNAP_U_WAVES_PER_EU 3
#endif
// staged elements per LDS flush (at least a level, 2J_max + 1): twelve keep a
// workgroup's LDS under 13.3 KB, so that three wavefronts fit per SIMD
constexpr int ustage(int TJ) { return TJ + 1 > SNAP_U_STAGE ? TJ + 1 : SNAP_U_STAGE; }
constexpr int kUAtoms = 4;   // atoms per wavefront
constexpr int kUSlots = 16;  // lanes per atom
constexpr int kUChunk = 2 * kUSlots;  // pairs per atom per chunk

// Destination of the k-th element a workgroup emits: full-matrix index
// (bits 0-23), diagonal flag (bit 24), mirror sign negative (bit 25); mirror
// index (-1: none); normalisation N.  Written once per workgroup, so that a
// flush reads it from LDS instead of a table in global memory.
struct USlot {
    int code, fm;
    double nrm;
};

// Workgroups per group of atoms.  Up to 2J = 4 one walks every column in
// turn: the pair geometry (square root, two sine-cosine pairs, divisions)
// then costs more than the short columns, and the split would compute it
// once per column.  Above, one workgroup per column: with its seed path each
// costs about the same ((2J_max+1)(2J_max+2)/2 elements, 45 at 2J = 8).
template <int TJ>
constexpr int kUGroups = (TJ <= 4) ? 1 : TJ / 2 + 1;

// Elements emitted before level J of column Q (counting, when one workgroup
// walks every column, the columns before Q too).
constexpr int emit_index(int TJ, int Q, int J)
{
    int k = 0;
    if (TJ <= 4)
        for (int q = 0; q < Q; ++q)
            for (int j = (q ? 2 * q : 0); j <= TJ; ++j) k += j + 1;
    for (int j = (Q ? 2 * Q : 0); j < J; ++j) k += j + 1;
    return k;
}
// most elements one workgroup emits (column 0, or every column)
constexpr int emit_max(int TJ) { return TJ <= 4 ? emit_index(TJ, TJ / 2 + 1, 0) : emit_index(TJ, 0, TJ + 1); }

// LDS of one workgroup: staged values of the four atoms' lanes and the
// destinations of every element it emits.
template <int TJ, int NS>
struct UStage {
    double2 v[NS][65];
    USlot slot[emit_max(TJ)];
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
        if (nst + j + 1 > ustage(TJ)) {
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

// Sum the NST staged values of the four atoms over their 16 lanes and add
// them to U, stored as full matrices of true values: U(p, q) = N * sum and
// its mirror U(J-p, J-q) = (-1)^(p-q) conj(U(p, q)).  The first chunk of
// neighbours starts from w_self on the diagonal (where N = 1).
template <int TJ, int NS, int NST, int BASE>
__device__ __forceinline__ void u_flush(UStage<TJ, NS> &st, int lane, int i0, int n, int npad,
                                        int chunk, double wself, double2 *__restrict__ U)
{
    static_assert(NS <= 16 && kUAtoms * 16 == 64, "one (atom, slot) per lane");
    __syncthreads();
    // lane = (atom hh, slot ss) whatever NST is: the per-lane addresses are
    // the same for every flush (computed once, not once per flush size)
    const int hh = lane >> 4, ss = lane & 15;
    if (ss < NST) {
        const USlot ui = st.slot[BASE + ss];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < kUSlots; j0 += 4) {
            // four reads in flight at a time: all sixteen hoisted would hold
            // 64 registers on top of the recursion state
#pragma unroll
            for (int j = j0; j < j0 + 4; ++j) {
                const double2 v = st.v[ss][hh * kUSlots + j];
                sr += v.x;
                si += v.y;
            }
            pin(sr);
            pin(si);
            memory_fence_compiler();
        }
        const int ia = i0 + hh;
        if (ia < n) {
            const size_t idx = (size_t)(ui.code & 0xffffff) * npad + ia;
            double br = 0.0, bi = 0.0;
            if (chunk == 0) {
                br = ((ui.code >> 24) & 1) ? wself : 0.0;
            } else {
                const double2 old = U[idx];
                br = old.x;
                bi = old.y;
            }
            const double2 v = make_double2(br + ui.nrm * sr, bi + ui.nrm * si);
            U[idx] = v;
            if (ui.fm >= 0) {
                const double ms = (ui.code >> 25) ? -1.0 : 1.0;
                U[(size_t)ui.fm * npad + ia] = make_double2(ms * v.x, -ms * v.y);
            }
        }
    }
    __syncthreads();
}

// Fill the slot table: lane k takes the k-th element the workgroup of column
// colq emits (levels from 2 colq up, rows 0..J of each; every column in turn
// up to 2J = 4) and copies its destination from the element table.
template <int TJ, int NS>
__device__ __forceinline__ void u_init_slots(UStage<TJ, NS> &st, int lane, int colq,
                                             const UInfo *__restrict__ uinfo)
{
    const int q0 = kUGroups<TJ> == 1 ? 0 : colq;
    const int q1 = kUGroups<TJ> == 1 ? TJ / 2 : colq;
    for (int k = lane; k < emit_max(TJ); k += 64) {
        int rem = k, Q = q0, J = q0 ? 2 * q0 : 0;
        bool ok = true;
        while (rem > J) {
            rem -= J + 1;
            if (++J > TJ) {
                if (++Q > q1) {
                    ok = false;
                    break;
                }
                J = 2 * Q;
            }
        }
        if (!ok) break;
        int hb = 0;  // first half index of rank J
        for (int j = 0; j < J; ++j) hb += (j + 1) * (j / 2 + 1);
        const UInfo ui = uinfo[hb + Q * (J + 1) + rem];
        USlot sl;
        sl.code = ui.fi | ((rem == Q) ? (1 << 24) : 0) | ((ui.msign < 0.0) ? (1 << 25) : 0);
        sl.fm = ui.fm;
        sl.nrm = ui.nrm;
        st.slot[k] = sl;
    }
}

// the two pairs a lane walks: geometry and recursion state
template <int TJ>
struct UPair2 {
    double2 a0, b0, a1, b1;
    double2 c0[TJ + 1], c1[TJ + 1];  // current column of each pair
    double2 s0[TJ + 1], s1[TJ + 1];  // seed of the next column
};

template <int TJ>
__device__ __forceinline__ void step2(int J, UPair2<TJ> &w)
{
    poly_step<TJ>(J, w.c0, w.a0, w.b0);
    poly_step<TJ>(J, w.c1, w.a1, w.b1);
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) {
            pin(w.c0[p]);
            pin(w.c1[p]);
        }
}

template <int TJ, int Q, int J>
__device__ __forceinline__ void u_emit(UStage<TJ, ustage(TJ)> &st, int lane, const UPair2<TJ> &w, int i0, int n,
                                       int npad, int chunk, double wself, double2 *__restrict__ U)
{
    constexpr StagePos sp = stage_pos(TJ, Q, J);
    if constexpr (sp.flushed > 0)
        u_flush<TJ, ustage(TJ), sp.flushed, emit_index(TJ, Q, J) - sp.flushed>(st, lane, i0, n, npad,
                                                                              chunk, wself, U);
#pragma unroll
    for (int p = 0; p <= J; ++p) {
        // the two pairs' f_c u, summed
        st.v[sp.slot + p][lane] = make_double2(w.c0[p].x + w.c1[p].x, w.c0[p].y + w.c1[p].y);
    }
}

// Levels J..TJ of column Q, each emitted to the staging buffer; with SEED,
// level 2Q+1 is also mirrored into the seed of column Q+1.
template <int TJ, int Q, int J, bool SEED>
struct ULevels {
    __device__ __forceinline__ static void run(UStage<TJ, ustage(TJ)> &st, int lane, UPair2<TJ> &w, int i0, int n,
                                               int npad, int chunk, double wself,
                                               double2 *__restrict__ U)
    {
        step2<TJ>(J, w);
        u_emit<TJ, Q, J>(st, lane, w, i0, n, npad, chunk, wself, U);
        if constexpr (SEED && J == 2 * Q + 1) {
            mirror_seed<TJ, Q>(w.c0, w.s0);
            mirror_seed<TJ, Q>(w.c1, w.s1);
#pragma unroll
            for (int p = 0; p <= 2 * Q + 1; ++p) {
                pin(w.s0[p]);
                pin(w.s1[p]);
            }
        }
        memory_fence_compiler();
        ULevels<TJ, Q, J + 1, SEED>::run(st, lane, w, i0, n, npad, chunk, wself, U);
    }
};
template <int TJ, int Q, bool SEED>
struct ULevels<TJ, Q, TJ + 1, SEED> {
    __device__ __forceinline__ static void run(UStage<TJ, ustage(TJ)> &, int, UPair2<TJ> &, int, int, int, int,
                                               double, double2 *__restrict__)
    {
    }
};

// Start column q of both pairs: from the seed, or from f_c at level 0.
template <int TJ, int q>
__device__ __forceinline__ void start_column(UPair2<TJ> &w, double fc0, double fc1)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p) {
        w.c0[p] = (q > 0 && p < 2 * q) ? w.s0[p] : make_double2(0.0, 0.0);
        w.c1[p] = (q > 0 && p < 2 * q) ? w.s1[p] : make_double2(0.0, 0.0);
    }
    if constexpr (q == 0) {
        // the recursion is linear in its starting column: starting from f_c
        // instead of 1 yields f_c u directly
        w.c0[0] = make_double2(fc0, 0.0);
        w.c1[0] = make_double2(fc1, 0.0);
    }
}

// Start column q of both pairs in place: the seed of column q is already in
// the first 2q rows (mirrored there by the previous column's walk); the rows
// above it start at zero.  Column 0 starts from f_c.
template <int TJ, int q>
__device__ __forceinline__ void start_column_inplace(UPair2<TJ> &w, double fc0, double fc1)
{
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (q == 0 || p >= 2 * q) {
            w.c0[p] = make_double2(0.0, 0.0);
            w.c1[p] = make_double2(0.0, 0.0);
        }
    if constexpr (q == 0) {
        w.c0[0] = make_double2(fc0, 0.0);
        w.c1[0] = make_double2(fc1, 0.0);
    }
}

// Column q at level 2q+1 -> seed of column q+1, in place:
//   poly_{p, q+1} = (-1)^(q+1-p) conj(poly_{2q+1-p, q}),  p = 0..2q+1
template <int TJ, int Q>
__device__ __forceinline__ void mirror_inplace(double2 (&col)[TJ + 1])
{
#pragma unroll
    for (int p = 0; p < Q + 1; ++p) {
        const int m = 2 * Q + 1 - p;  // > p
        const double sp = ((Q + 1 - p) & 1) ? -1.0 : 1.0;
        const double sm = ((Q + 1 - m) & 1) ? -1.0 : 1.0;
        const double2 x = col[p], y = col[m];
        col[p] = make_double2(sp * y.x, -sp * y.y);
        col[m] = make_double2(sm * x.x, -sm * x.y);
    }
}

// Seed path of a single-column workgroup, in place: columns q = 0..Q-1 to
// level 2q+1, each mirrored into the start of the next.  Nothing is emitted.
template <int TJ, int q, int Q>
struct USeedInPlace {
    __device__ __forceinline__ static void run(UPair2<TJ> &w, double fc0, double fc1)
    {
        if constexpr (q < Q) {
            start_column_inplace<TJ, q>(w, fc0, fc1);
#pragma unroll
            for (int J = (q == 0 ? 1 : 2 * q); J <= 2 * q + 1; ++J) step2<TJ>(J, w);
            mirror_inplace<TJ, q>(w.c0);
            mirror_inplace<TJ, q>(w.c1);
#pragma unroll
            for (int p = 0; p <= 2 * q + 1; ++p) {
                pin(w.c0[p]);
                pin(w.c1[p]);
            }
            USeedInPlace<TJ, q + 1, Q>::run(w, fc0, fc1);
        }
    }
};

// Seed path: column q from its seed, levels up to 2q+1, mirrored into the
// seed of column q+1; for q = 0 .. Q-1.  Nothing is emitted.
template <int TJ, int q, int Q>
struct USeedPath {
    __device__ __forceinline__ static void run(UPair2<TJ> &w, double fc0, double fc1)
    {
        if constexpr (q < Q) {
            start_column<TJ, q>(w, fc0, fc1);
#pragma unroll
            for (int J = (q == 0 ? 1 : 2 * q); J <= 2 * q + 1; ++J) step2<TJ>(J, w);
            mirror_seed<TJ, q>(w.c0, w.s0);
            mirror_seed<TJ, q>(w.c1, w.s1);
#pragma unroll
            for (int p = 0; p <= 2 * q + 1; ++p) {
                pin(w.s0[p]);
                pin(w.s1[p]);
            }
            USeedPath<TJ, q + 1, Q>::run(w, fc0, fc1);
        }
    }
};

// Columns Q..TJ/2 walked one after another, each from the seed the previous
// walk left (CHAIN), or column Q alone (its seed path first when Q > 0).
template <int TJ, int Q, bool CHAIN>
__device__ __forceinline__ void u_walk(UStage<TJ, ustage(TJ)> &st, int lane, UPair2<TJ> &w, double fc0, double fc1,
                                       int i0, int n, int npad, int chunk, double wself,
                                       double2 *__restrict__ U)
{
    constexpr bool NEXT = CHAIN && Q < TJ / 2;
    if constexpr (CHAIN)
        start_column<TJ, Q>(w, fc0, fc1);
    else
        start_column_inplace<TJ, Q>(w, fc0, fc1);
    if constexpr (Q == 0) u_emit<TJ, 0, 0>(st, lane, w, i0, n, npad, chunk, wself, U);
    ULevels<TJ, Q, (Q == 0 ? 1 : 2 * Q), NEXT>::run(st, lane, w, i0, n, npad, chunk, wself, U);
    u_flush<TJ, ustage(TJ), stage_end(TJ, Q), emit_index(TJ, Q, TJ + 1) - stage_end(TJ, Q)>(
        st, lane, i0, n, npad, chunk, wself, U);
    if constexpr (NEXT) u_walk<TJ, Q + 1, true>(st, lane, w, fc0, fc1, i0, n, npad, chunk, wself, U);
}

// Workgroup column Q of one chunk of pairs: the seed path, then the walk.
template <int TJ, int Q, bool CHAIN>
__device__ __forceinline__ void u_column(UStage<TJ, ustage(TJ)> &st, int lane, UPair2<TJ> &w, double fc0,
                                         double fc1, int i0, int n, int npad, int chunk,
                                         double wself, double2 *__restrict__ U)
{
    if constexpr (CHAIN) {
#pragma unroll
        for (int p = 0; p <= TJ; ++p) w.s0[p] = w.s1[p] = make_double2(0.0, 0.0);
        USeedPath<TJ, 0, Q>::run(w, fc0, fc1);
    } else {
        USeedInPlace<TJ, 0, Q>::run(w, fc0, fc1);
    }
    u_walk<TJ, Q, CHAIN>(st, lane, w, fc0, fc1, i0, n, npad, chunk, wself, U);
}

// uniform workgroup column index -> compile-time instance
template <int TJ, int Q>
struct UColumn {
    __device__ __forceinline__ static void run(int col, UStage<TJ, ustage(TJ)> &st, int lane, UPair2<TJ> &w,
                                               double fc0, double fc1, int i0, int n, int npad,
                                               int chunk, double wself, double2 *__restrict__ U)
    {
        if constexpr (kUGroups<TJ> == 1) {
            (void)col;
            u_column<TJ, 0, true>(st, lane, w, fc0, fc1, i0, n, npad, chunk, wself, U);
        } else if constexpr (Q <= TJ / 2) {
            if (col == Q)
                u_column<TJ, Q, false>(st, lane, w, fc0, fc1, i0, n, npad, chunk, wself, U);
            else
                UColumn<TJ, Q + 1>::run(col, st, lane, w, fc0, fc1, i0, n, npad, chunk, wself, U);
        }
    }
};

// geometry of neighbour slot s of atom i (a = 1, b = 0, f_c = 0 when empty)
__device__ __forceinline__ void slot_geometry(bool valid, int i, int t, bool first,
                                              const double *__restrict__ pos,
                                              const int *__restrict__ nbr, const Geom &g,
                                              int *__restrict__ pair_atom, int *__restrict__ flag,
                                              PairGeom &pg)
{
    pg.a = make_double2(1.0, 0.0);
    pg.b = make_double2(0.0, 0.0);
    pg.fc = 0.0;
    if (valid) {
        if (first) pair_atom[t] = i;
        double rv[3];
        const int k = nbr[t];
        min_image(pos, i, k, g, rv);
        double rc, w;
        const bool typed = pair_cut(g, i, k, rc, w);
        if (!pair_geometry(rv, g, rc, w, pg) && first) flag[0] = 1;
        if (!typed && first) flag[0] = 2;
    }
}

template <int TJ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TJ <= 8 ? SNAP_U_WAVES_PER_EU : 2, 8))) void k_compute_u(
    int n, int npad, const double *__restrict__ pos, const int *__restrict__ off,
    const int *__restrict__ nbr, Geom g, const UInfo *__restrict__ uinfo, double2 *__restrict__ U,
    int *__restrict__ pair_atom, int *__restrict__ flag)
{
    __shared__ UStage<TJ, ustage(TJ)> st;
    constexpr int NCOL = kUGroups<TJ>;
    const int lane = threadIdx.x;
    // Workgroup w runs on XCD w mod 8 and computes the atom groups of the
    // 64-atom blocks congruent to it mod 8, block by block, all columns of a
    // group on the same XCD: the partial lines of U that the column
    // workgroups of an atom group write meet in one L2, which is also the L2
    // of the XCD whose compute_Y workgroups read that block.
    constexpr int GPB = 64 / kUAtoms;
    const int wg = (int)blockIdx.x;
    const int kk = wg >> 3;
    const int kb = kk / (GPB * NCOL), rem = kk - kb * (GPB * NCOL);
    const int colq = rem % NCOL;  // uniform
    const int i0 = (((wg & 7) + 8 * kb) * GPB + rem / NCOL) * kUAtoms;
    u_init_slots<TJ>(st, lane, colq, uinfo);  // read after the first flush's barrier
    const int h = lane / kUSlots, slot = lane % kUSlots;
    const int i = i0 + h;
    int mx = 0;
#pragma unroll
    for (int k = 0; k < kUAtoms; ++k) {
        const int cnt = (i0 + k < n) ? off[i0 + k + 1] - off[i0 + k] : 0;
        mx = cnt > mx ? cnt : mx;
    }
    const int nchunk = mx > 0 ? (mx + kUChunk - 1) / kUChunk : 1;
    const int myn = (i < n) ? off[i + 1] - off[i] : 0;
    const int mybeg = (i < n) ? off[i] : 0;

    UPair2<TJ> w;
    for (int c = 0; c < nchunk; ++c) {
        const int s0 = c * kUChunk + slot, s1 = s0 + kUSlots;
        PairGeom g0, g1;
        slot_geometry((i < n) && (s0 < myn), i, mybeg + s0, colq == 0, pos, nbr, g, pair_atom,
                      flag, g0);
        slot_geometry((i < n) && (s1 < myn), i, mybeg + s1, colq == 0, pos, nbr, g, pair_atom,
                      flag, g1);
        w.a0 = g0.a;
        w.b0 = g0.b;
        w.a1 = g1.a;
        w.b1 = g1.b;
        UColumn<TJ, 0>::run(colq, st, lane, w, g0.fc, g1.fc, i0, n, npad, c, g.wself, U);
    }
}

// ---------------------------------------------------------------------------
// compute_U, one pair per lane
//
// A workgroup is one wavefront holding two atoms of 32 lanes each; every lane
// walks one pair (neighbour 32c + slot of chunk c) through every column of
// the stored half in turn -- column 0 from f_c, column q + 1 from the mirror
// of column q at level 2q + 1 -- so the pair geometry is computed once and
// no level is computed twice.  The values are staged in LDS 32 elements at a
// time; at each flush every lane sums one (atom, element) over its atom's 32
// lanes in a fixed order and writes it, with its mirror, as a full matrix of
// true values.
// ---------------------------------------------------------------------------
constexpr int kU2Lanes = 32;  // lanes per atom
constexpr int kU2Stage = 32;  // staged elements per flush (64 lanes / 2 atoms)

struct U2Stage {
    double2 v[kU2Stage][65];  // [element slot][lane], rows padded against bank conflicts
    int code[kU2Stage];       // half index of the slot's element | diagonal flag << 24
};

__device__ __forceinline__ void u2_flush(U2Stage &st, int nst, int lane, int i0, int n, int npad,
                                         int chunk, double wself, const UInfo *__restrict__ uinfo,
                                         double2 *__restrict__ U)
{
    __syncthreads();
    const int h = lane >> 5, s = lane & 31;
    if (s < nst) {
        const int code = st.code[s];
        const UInfo ui = uinfo[code & 0xffffff];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < kU2Lanes; j0 += 8) {
            // eight reads in flight at a time (all 32 hoisted would hold 128
            // registers)
#pragma unroll
            for (int j = j0; j < j0 + 8; ++j) {
                const double2 v = st.v[s][h * kU2Lanes + j];
                sr += v.x;
                si += v.y;
            }
            memory_fence_compiler();
        }
        const int ia = i0 + h;
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
    __syncthreads();
}

// Stage element (J, p, q) (half index e) of every lane; flush when full.
__device__ __forceinline__ void u2_emit(U2Stage &st, int &nst, int lane, double2 v, int e,
                                        bool diag, int i0, int n, int npad, int chunk,
                                        double wself, const UInfo *__restrict__ uinfo,
                                        double2 *__restrict__ U)
{
    st.v[nst][lane] = v;
    if (lane == 0) st.code[nst] = e | (diag ? (1 << 24) : 0);
    if (++nst == kU2Stage) {
        u2_flush(st, nst, lane, i0, n, npad, chunk, wself, uinfo, U);
        nst = 0;
    }
}

template <int TJ>
__global__ __launch_bounds__(64) void k_compute_u2(int n, int npad, const double *__restrict__ pos,
                                                   const int *__restrict__ off,
                                                   const int *__restrict__ nbr, Geom g,
                                                   const UInfo *__restrict__ uinfo,
                                                   double2 *__restrict__ U,
                                                   int *__restrict__ pair_atom,
                                                   int *__restrict__ flag)
{
    __shared__ U2Stage st;
    const int lane = threadIdx.x;
    const int h = lane >> 5, slot = lane & 31;
    const int i0 = (int)blockIdx.x * 2;
    const int i = i0 + h;
    int mx = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int cnt = (i0 + k < n) ? off[i0 + k + 1] - off[i0 + k] : 0;
        mx = cnt > mx ? cnt : mx;
    }
    const int nchunk = mx > 0 ? (mx + kU2Lanes - 1) / kU2Lanes : 1;
    const int myn = (i < n) ? off[i + 1] - off[i] : 0;
    const int mybeg = (i < n) ? off[i] : 0;
    for (int c = 0; c < nchunk; ++c) {
        const int sn = c * kU2Lanes + slot;
        PairGeom pg;
        slot_geometry((i < n) && (sn < myn), i, mybeg + sn, true, pos, nbr, g, pair_atom, flag,
                      pg);
        double2 col[TJ + 1], seed[TJ + 1];
#pragma unroll
        for (int p = 0; p <= TJ; ++p) seed[p] = make_double2(0.0, 0.0);
        int nst = 0;
        // J = 0: f_c
        u2_emit(st, nst, lane, make_double2(pg.fc, 0.0), 0, true, i0, n, npad, c, g.wself, uinfo,
                U);
#pragma unroll
        for (int q = 0; q <= TJ / 2; ++q) {
#pragma unroll
            for (int p = 0; p <= TJ; ++p)
                col[p] = (q > 0 && p < 2 * q) ? seed[p] : make_double2(0.0, 0.0);
            if (q == 0) col[0] = make_double2(pg.fc, 0.0);
#pragma unroll
            for (int J = (q == 0 ? 1 : 2 * q); J <= TJ; ++J) {
                poly_step<TJ>(J, col, pg.a, pg.b);
                if (J == 2 * q + 1 && 2 * q + 2 <= TJ) {
                    // seed of column q + 1: (-1)^(q+1-p) conj(poly_{2q+1-p, q})
#pragma unroll
                    for (int p = 0; p <= TJ; ++p)
                        if (p <= 2 * q + 1) {
                            const double sg = ((q + 1 - p) & 1) ? -1.0 : 1.0;
                            const double2 m = col[2 * q + 1 - p];
                            seed[p] = make_double2(sg * m.x, -sg * m.y);
                        }
                }
                const int eb = hbase_of(J) + q * (J + 1);
#pragma unroll
                for (int p = 0; p <= TJ; ++p)
                    if (p <= J)
                        u2_emit(st, nst, lane, col[p], eb + p, p == q, i0, n, npad, c, g.wself,
                                uinfo, U);
            }
        }
        if (nst > 0) u2_flush(st, nst, lane, i0, n, npad, c, g.wself, uinfo, U);
    }
}

// ---------------------------------------------------------------------------
// compute_U, lanes over the elements of a level (the mapping of the paper's
// Sec. VI, kept as a measured alternative)
//
// One wavefront per atom walks its pairs one after another.  For each pair,
// level J of the recursion is computed by the lanes, one stored element
// (p, q) each (lane = q (J + 1) + p, at most 45 at 2J = 8), from level J - 1
// held in LDS as a full matrix; each lane writes its element and the mirror
// image back for level J + 1 and adds it to its running sum of that element
// over the atom's pairs (registers, one per level).  The pair geometry is
// computed by the lanes for up to 64 pairs at a time and read back from LDS
// as wavefront-uniform values.
// ---------------------------------------------------------------------------
template <int TJ>
__global__ __launch_bounds__(64) void k_compute_u3(int n, int npad, const double *__restrict__ pos,
                                                   const int *__restrict__ off,
                                                   const int *__restrict__ nbr, Geom g,
                                                   const UInfo *__restrict__ uinfo,
                                                   double2 *__restrict__ U,
                                                   int *__restrict__ pair_atom,
                                                   int *__restrict__ flag)
{
    constexpr int LW = (TJ + 1) * (TJ + 1);
    // stored elements per lane and level: (J + 1)(J/2 + 1) <= 120 at 2J = 14
    constexpr int M = ((TJ + 1) * (TJ / 2 + 1) + 63) / 64;
    __shared__ double2 lv[2][LW > 1 ? LW : 1];
    __shared__ double geo[5][64];  // a.x, a.y, b.x, b.y, f_c of 64 pairs
    const int i = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    const int beg = off[i], end = off[i + 1];
    double2 acc[TJ + 1][M];
#pragma unroll
    for (int J = 0; J <= TJ; ++J)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[J][m] = make_double2(0.0, 0.0);
    for (int c0 = beg; c0 < end; c0 += 64) {
        const int t = c0 + lane;
        PairGeom pg;
        slot_geometry(t < end, i, t, true, pos, nbr, g, pair_atom, flag, pg);
        __syncthreads();  // the previous chunk's reads of geo are done
        geo[0][lane] = pg.a.x;
        geo[1][lane] = pg.a.y;
        geo[2][lane] = pg.b.x;
        geo[3][lane] = pg.b.y;
        geo[4][lane] = pg.fc;
        __syncthreads();
        const int cnt = min(64, end - c0);
        for (int k = 0; k < cnt; ++k) {
            const double2 a = make_double2(geo[0][k], geo[1][k]);
            const double2 b = make_double2(geo[2][k], geo[3][k]);
            const double fc = geo[4][k];
            // level 0: poly = f_c (the recursion is linear in its start)
            if (lane == 0) {
                lv[0][0] = make_double2(fc, 0.0);
                acc[0][0].x += fc;
            }
            __syncthreads();
#pragma unroll
            for (int J = 1; J <= TJ; ++J) {
                const double2 *prev = lv[(J - 1) & 1];  // level J - 1: J x J, row-major
                double2 *cur = lv[J & 1];               // level J: (J+1) x (J+1)
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int e = lane + 64 * m;
                    if (e < (J + 1) * (J / 2 + 1)) {
                        const int q = e / (J + 1), p = e - q * (J + 1);
                        double nr = 0.0, ni = 0.0;
                        if (p < J) {
                            const double2 u = prev[p * J + q];
                            nr = a.x * u.x + a.y * u.y;
                            ni = a.x * u.y - a.y * u.x;
                        }
                        if (p > 0) {
                            const double2 w = prev[(p - 1) * J + q];
                            nr = nr - b.x * w.x - b.y * w.y;
                            ni = ni - b.x * w.y + b.y * w.x;
                        }
                        acc[J][m].x += nr;
                        acc[J][m].y += ni;
                        const double sg = ((p - q) & 1) ? -1.0 : 1.0;
                        cur[p * (J + 1) + q] = make_double2(nr, ni);
                        cur[(J - p) * (J + 1) + (J - q)] = make_double2(sg * nr, -sg * ni);
                    }
                }
                __syncthreads();
            }
        }
    }
    // the atom's sums, as full matrices of true values (w_self on the diagonal)
#pragma unroll
    for (int J = 0; J <= TJ; ++J)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = lane + 64 * m;
            if (e < (J + 1) * (J / 2 + 1)) {
                const int q = e / (J + 1), p = e - q * (J + 1);
                const UInfo ui = uinfo[hbase_of(J) + e];
                const double2 v = make_double2((p == q ? g.wself : 0.0) + ui.nrm * acc[J][m].x,
                                               ui.nrm * acc[J][m].y);
                U[(size_t)ui.fi * npad + i] = v;
                if (ui.fm >= 0)
                    U[(size_t)ui.fm * npad + i] = make_double2(ui.msign * v.x, -ui.msign * v.y);
            }
        }
}

template <int TJ>
hipError_t launch_u_t(int variant, int n, int npad, const double *pos, const int *off,
                      const int *nbr, const Geom &g, const UInfo *uinfo, double2 *U,
                      int *pair_atom, int *flag, hipStream_t s)
{
    if (variant == 2) {
        hipLaunchKernelGGL(k_compute_u2<TJ>, dim3((n + 1) / 2), dim3(64), 0, s, n, npad, pos, off,
                           nbr, g, uinfo, U, pair_atom, flag);
        return hipGetLastError();
    }
    if (variant == 3) {
        hipLaunchKernelGGL(k_compute_u3<TJ>, dim3(n), dim3(64), 0, s, n, npad, pos, off, nbr, g,
                           uinfo, U, pair_atom, flag);
        return hipGetLastError();
    }
    // 64-atom blocks padded to a multiple of 8 (the groups past n walk empty
    // pairs and write nothing)
    const int nblk = ((n + 64 * 8 - 1) / (64 * 8)) * 8 * (64 / kUAtoms) * kUGroups<TJ>;
    hipLaunchKernelGGL(k_compute_u<TJ>, dim3(nblk), dim3(64), 0, s, n, npad, pos, off, nbr, g,
                       uinfo, U, pair_atom, flag);
    return hipGetLastError();
}

}  // namespace

#ifndef SNAP_TJ_CASES
#define SNAP_TJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

hipError_t launch_compute_u(int twojmax, int variant, int n, int npad, const double *pos,
                            const int *off, const int *nbr, const DevTables &T, const Geom &g,
                            double2 *U, int *pair_atom, int *flag, hipStream_t s)
{
    switch (twojmax) {
#define X(k) \
    case k:  \
        return launch_u_t<k>(variant, n, npad, pos, off, nbr, g, T.uinfo, U, pair_atom, flag, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace snapmi
