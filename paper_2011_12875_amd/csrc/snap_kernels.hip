// snap_kernels.hip -- FP64 SNAP kernels for gfx950 (MI355X).
//
// Stages (arXiv 2011.12875, Sec. IV Listing 5 with the GPU refinements of
// Sec. VI):
//   k_compute_u  eq. (u): one lane per (atom, neighbour) pair runs the
//                hyperspherical-harmonic recursion eq. (hysphrecur) for the
//                stored half of every u_j (Sec. VI), column by column in
//                registers; the per-atom sum U_j is reduced through LDS in a
//                fixed order (no atomics, bit-reproducible).
//   k_compute_y  eq. (y): one lane per atom (64 consecutive atoms per
//                wavefront, like the AoSoA layout of Sec. VI), all lanes
//                running the same Clebsch-Gordan contraction program, so
//                coefficients and indices are wavefront-uniform (scalar
//                loads); rows (j, p) of Y are split over four wavefronts and
//                reduced in LDS.
//   k_bispectrum eq. (z) and eq. (snapatomenergy), on request.
//   k_dedr       eq. (snapforce2) fused with the derivative recursion
//                ("compute_fused_dE", Sec. VI): one lane per pair (and per
//                direction when split, as Sec. VI splits x, y, z), u and du
//                recomputed in registers and contracted with Y on the fly.
//   k_gather     update_forces: F_i = sum_out dE_p - sum_out dE_rev(p), a
//                deterministic gather through the reverse-pair index; also the
//                energy E_i = (1/3) Re sum_j Y_j : U_j^* (B is cubic in U).
//
// Conventions: twice-integer J, row p, column q, stored half q <= J/2.
// The recursion runs on the polynomial coefficients poly^J_{pq} = u^J_{pq}/N
// (N = sqrt(p!(J-p)!/(q!(J-q)!))), which obey
//   poly^J_{pq} = a* poly^{J-1}_{pq} - b* poly^{J-1}_{p-1,q}
// with unit weights, and the mirror rule
//   poly^J_{J-p,J-q} = (-1)^(p-q) conj(poly^J_{pq}).
// Per-atom arrays are element-major X[e * npad + atom] of double2 (re, im)
// and hold the scaled values U~ = U/N and Y~ = w N Y (w: half-sum weight).
#include <hip/hip_runtime.h>

#include "snap_kernels.hpp"

namespace snapmi {

namespace {

constexpr int hbase_of(int J)
{
    int s = 0;
    for (int k = 0; k < J; ++k) s += (k + 1) * (k / 2 + 1);
    return s;
}

struct PairGeom {
    double2 a, b;
    double fc, dfdr;
    double n[3];
    double r, c0, s0, dth0;
};

// The 3-sphere map of eq. (u): theta0 = rfac0 pi (r - rmin0)/(rcut - rmin0),
// Cayley-Klein pair a = cos theta0 - i sin theta0 n_z,
// b = sin theta0 (n_y - i n_x), switching function f_c and df_c/dr.
// Returns false for r < 1e-10 or non-finite input (the pair then contributes
// nothing: f_c = 0, a = 1, b = 0).
__device__ __forceinline__ bool pair_geometry(const double rv[3], const Geom &g, PairGeom &pg)
{
    const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    const double r = sqrt(r2);
    const bool ok = (r >= 1e-10) && (r < 1e300);  // false for NaN too
    const double rs = ok ? r : 1.0;
    pg.r = rs;
    pg.n[0] = ok ? rv[0] / rs : 0.0;
    pg.n[1] = ok ? rv[1] / rs : 0.0;
    pg.n[2] = ok ? rv[2] / rs : 1.0;
    const double span = g.rcut - g.rmin0;
    const double th0 = g.rfac0 * M_PI * (rs - g.rmin0) / span;
    double s0, c0;
    sincos(th0, &s0, &c0);
    pg.c0 = c0;
    pg.s0 = s0;
    pg.dth0 = g.rfac0 * M_PI / span;
    pg.a = ok ? make_double2(c0, -s0 * pg.n[2]) : make_double2(1.0, 0.0);
    pg.b = ok ? make_double2(s0 * pg.n[1], -s0 * pg.n[0]) : make_double2(0.0, 0.0);
    double fc = 1.0, dfdr = 0.0;
    if (g.switch_flag && rs > g.rmin0) {
        double sx, cx;
        sincos(M_PI * (rs - g.rmin0) / span, &sx, &cx);
        fc = 0.5 * (cx + 1.0);
        dfdr = -0.5 * M_PI / span * sx;
    }
    const bool inside = ok && r < g.rcut;
    pg.fc = inside ? fc : 0.0;
    pg.dfdr = inside ? dfdr : 0.0;
    return ok;
}

__device__ __forceinline__ void min_image(const double *__restrict__ pos, int i, int k,
                                          const Geom &g, double rv[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double x = pos[3 * k + d] - pos[3 * i + d];
        if (g.box[d] > 0.0) x -= g.box[d] * rint(x / g.box[d]);
        rv[d] = x;
    }
}

// Load element row `row` of an element-major per-atom array at lane offset
// voff (= atom * 16 bytes) through a buffer descriptor: the row base stays in
// scalar registers, each lane supplies one 32-bit offset, and a load past the
// row (npad atoms) returns zero instead of faulting.
__device__ __forceinline__ double2 load_row(const double2 *base, size_t row, int npad, unsigned voff)
{
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(base + row * (size_t)npad), (short)0, npad * 16, 0x00020000);
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
    return make_double2(
        __builtin_bit_cast(double, (unsigned long long)v[0] | ((unsigned long long)v[1] << 32)),
        __builtin_bit_cast(double, (unsigned long long)v[2] | ((unsigned long long)v[3] << 32)));
}

// Register pins.  The recursion is a 2-D dependency grid (row p of level J
// needs rows p and p-1 of level J-1).  Left alone, the compiler evaluates it
// row-major across all levels, which keeps every level of the previous row
// alive (and hoists every load of Y to the top), spilling at 2J >= 8.  An
// empty asm that "modifies" the live column and accumulators at each level
// boundary pins the level-major order at no instruction cost; the memory
// clobber keeps each level's loads inside its level.
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(double2 &x)
{
    asm volatile("" : "+v"(x.x), "+v"(x.y));
}
__device__ __forceinline__ void memory_fence_compiler() { asm volatile("" ::: "memory"); }

// One level of the column recursion, in place, rows p = J .. 0:
//   col[p] <- conj(a) col[p] - conj(b) col[p-1]
// The new top row p = J reads only col[J-1] (col[J] is still zero).
template <int TJ>
__device__ __forceinline__ void poly_step(int J, double2 (&col)[TJ + 1], double2 a, double2 b)
{
#pragma unroll
    for (int p = TJ; p >= 0; --p)
        if (p <= J) {
            double nr = 0.0, ni = 0.0;
            if (p < J) {
                const double2 u = col[p];
                nr = a.x * u.x + a.y * u.y;
                ni = a.x * u.y - a.y * u.x;
            }
            if (p > 0) {
                const double2 w = col[p - 1];
                nr -= b.x * w.x + b.y * w.y;
                ni -= b.x * w.y - b.y * w.x;
            }
            col[p] = make_double2(nr, ni);
        }
}

// Seed of column q+1 at level 2q+1 from column q at the same level:
//   poly_{p, q+1} = (-1)^(q+1-p) conj(poly_{2q+1-p, q})
template <int TJ, int Q>
__device__ __forceinline__ void mirror_seed(const double2 (&col)[TJ + 1], double2 (&seed)[TJ + 1])
{
#pragma unroll
    for (int p = 0; p <= 2 * Q + 1; ++p) {
        const double sg = ((Q + 1 - p) & 1) ? -1.0 : 1.0;
        const double2 m = col[2 * Q + 1 - p];
        seed[p] = make_double2(sg * m.x, -sg * m.y);
    }
}

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
// to U (the first chunk of neighbours starts from w_self on the diagonal).
template <int NST>
__device__ __forceinline__ void u_flush(UStage &st, int lane, int i0, int n, int npad, int chunk,
                                        double wself, double2 *__restrict__ U)
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
                const size_t idx = (size_t)(code & 0xffffff) * npad + ia;
                double br = 0.0, bi = 0.0;
                if (chunk == 0) {
                    br = (code >> 24) ? wself : 0.0;  // diagonal: N = 1
                } else {
                    const double2 old = U[idx];
                    br = old.x;
                    bi = old.y;
                }
                U[idx] = make_double2(br + sr, bi + si);
            }
        }
    }
    __syncthreads();
}

template <int TJ, int Q, int J>
__device__ __forceinline__ void u_emit(UStage &st, int lane, double fc,
                                       const double2 (&col)[TJ + 1], int i0, int n, int npad,
                                       int chunk, double wself, double2 *__restrict__ U)
{
    constexpr StagePos sp = stage_pos(TJ, Q, J);
    if constexpr (sp.flushed > 0) u_flush<sp.flushed>(st, lane, i0, n, npad, chunk, wself, U);
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
                                               int chunk, double wself, double2 *__restrict__ U)
    {
        poly_step<TJ>(J, col, a, b);
        u_emit<TJ, Q, J>(st, lane, fc, col, i0, n, npad, chunk, wself, U);
#pragma unroll
        for (int p = 0; p <= J; ++p) pin(col[p]);
        memory_fence_compiler();
        if constexpr (J == 2 * Q + 1 && 2 * Q + 2 <= TJ) {
            mirror_seed<TJ, Q>(col, seed);
#pragma unroll
            for (int p = 0; p <= 2 * Q + 1; ++p) pin(seed[p]);
        }
        ULevels<TJ, Q, J + 1>::run(st, lane, fc, a, b, col, seed, i0, n, npad, chunk, wself, U);
    }
};
template <int TJ, int Q>
struct ULevels<TJ, Q, TJ + 1> {
    __device__ __forceinline__ static void run(UStage &, int, double, double2, double2,
                                               double2 (&)[TJ + 1], double2 (&)[TJ + 1], int, int,
                                               int, int, double, double2 *__restrict__)
    {
    }
};

template <int TJ, int Q>
struct UColumns {
    __device__ __forceinline__ static void run(UStage &st, int lane, double fc, double2 a,
                                               double2 b, double2 (&col)[TJ + 1],
                                               double2 (&seed)[TJ + 1], int i0, int n, int npad,
                                               int chunk, double wself, double2 *__restrict__ U)
    {
#pragma unroll
        for (int p = 0; p <= TJ; ++p)
            col[p] = (Q > 0 && p < 2 * Q) ? seed[p] : make_double2(0.0, 0.0);
        if constexpr (Q == 0) {
            col[0] = make_double2(1.0, 0.0);
            u_emit<TJ, 0, 0>(st, lane, fc, col, i0, n, npad, chunk, wself, U);
        }
        ULevels<TJ, Q, (Q == 0 ? 1 : 2 * Q)>::run(st, lane, fc, a, b, col, seed, i0, n, npad,
                                                   chunk, wself, U);
        UColumns<TJ, Q + 1>::run(st, lane, fc, a, b, col, seed, i0, n, npad, chunk, wself, U);
    }
};
template <int TJ>
struct UColumns<TJ, TJ / 2 + 1> {
    __device__ __forceinline__ static void run(UStage &, int, double, double2, double2,
                                               double2 (&)[TJ + 1], double2 (&)[TJ + 1], int, int,
                                               int, int, double, double2 *__restrict__)
    {
    }
};

template <int TJ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_compute_u(int n, int npad, const double *__restrict__ pos,
                                                  const int *__restrict__ off,
                                                  const int *__restrict__ nbr, Geom g,
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
        UColumns<TJ, 0>::run(st, lane, pg.fc, pg.a, pg.b, col, seed, i0, n, npad, c, g.wself, U);
        u_flush<stage_end(TJ)>(st, lane, i0, n, npad, c, g.wself, U);
    }
}

// ---------------------------------------------------------------------------
// compute_Y (adjoint of eq. (y)) -- lanes are atoms
// ---------------------------------------------------------------------------
constexpr int kYMaxQ = 8;  // J/2 + 1 for J <= 14

__global__ __launch_bounds__(64 * kYWaves) void k_compute_y(
    int n, int npad, int nblk, const double2 *__restrict__ U, double2 *__restrict__ Y,
    const YRow *__restrict__ rows, const ZItem *__restrict__ items, const Term *__restrict__ terms,
    const double *__restrict__ beta, int per_atom_beta, int nb, const double *__restrict__ gscale)
{
    __shared__ double2 yw[kYWaves][kYMaxQ][64];
    const int unit = blockIdx.x;
    const int rix = unit / nblk, blk = unit - rix * nblk;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int atom = blk * 64 + lane;
    const int asafe = atom < n ? atom : 0;
    const YRow *row = rows + rix;
    const int nq = row->nq;
    const double gs = gscale ? gscale[asafe] : 1.0;
    for (int q = 0; q < nq; ++q) yw[w][q][lane] = make_double2(0.0, 0.0);
    const int xb = row->wb[w], xe = row->wb[w + 1];

    const double2 *Ua = U + atom;
    for (int x = xb; x < xe; ++x) {
        const ZItem *it = items + x;
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int te = it->tb[k + 1];
            for (int tt = it->tb[k]; tt < te; ++tt) {
                const Term tm = terms[tt];
                double2 u1 = Ua[(size_t)tm.i1 * npad];
                double2 u2 = Ua[(size_t)tm.i2 * npad];
                if (k & 1) u1.y = -u1.y;
                if (k & 2) u2.y = -u2.y;
                const double pr = u1.x * u2.x - u1.y * u2.y;
                const double pi = u1.x * u2.y + u1.y * u2.x;
                zr += tm.cc * pr;
                zi += tm.cc * pi;
            }
        }
        const int l = it->l;
        const double bl = per_atom_beta ? beta[(size_t)asafe * nb + l] : beta[l];
        const double f = it->factor * bl * gs;
        const int q = it->q;
        double2 acc = yw[w][q][lane];
        acc.x += f * zr;
        acc.y += f * zi;
        yw[w][q][lane] = acc;
    }
    __syncthreads();
    const int J = row->J, eb = row->ebase;
    for (int q = w; q < nq; q += kYWaves) {
        double2 s = yw[0][q][lane];
#pragma unroll
        for (int v = 1; v < kYWaves; ++v) {
            s.x += yw[v][q][lane].x;
            s.y += yw[v][q][lane].y;
        }
        Y[(size_t)(eb + q * (J + 1)) * npad + atom] = s;
    }
}

// ---------------------------------------------------------------------------
// bispectrum (eq. (z)) and energy (eq. (snapatomenergy)) -- lanes are atoms
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_bispectrum(int n, int npad, const double2 *__restrict__ U,
                                                   const ZItem *__restrict__ items,
                                                   const Term *__restrict__ terms,
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
        const ZItem *it = items + bi->item;
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int te = it->tb[k + 1];
            for (int tt = it->tb[k]; tt < te; ++tt) {
                const Term tm = terms[tt];
                double2 u1 = Ua[(size_t)tm.i1 * npad];
                double2 u2 = Ua[(size_t)tm.i2 * npad];
                if (k & 1) u1.y = -u1.y;
                if (k & 2) u2.y = -u2.y;
                zr += tm.cc * (u1.x * u2.x - u1.y * u2.y);
                zi += tm.cc * (u1.x * u2.y + u1.y * u2.x);
            }
        }
        const double2 uj = Ua[(size_t)bi->e * npad];
        bsum += zr * uj.x + zi * uj.y;
    }
    if (atom < n) B[(size_t)atom * nb + l] = bsum;
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
// compute_fused_dE: dE_p = sum_J sum_half Re(Y~_i conj(dfc poly + fc dpoly))
// ---------------------------------------------------------------------------
template <int TJ, int ND>
struct DedrState {
    double2 col[TJ + 1], seed[TJ + 1];
    double2 dcol[ND][TJ + 1], dseed[ND][TJ + 1];
    double S0, S[ND];
};

// One level: recursion for poly and its derivatives, then the dot with Y~.
// The top row p = J has no col[J] term; DZ marks a level whose input
// derivatives are all zero (the first level of column 0, from poly^0 = 1).
template <int TJ, int ND, bool DZ>
__device__ __forceinline__ void dedr_level(int J, int eb, DedrState<TJ, ND> &st, double2 a,
                                           double2 b, const double2 (&da)[ND],
                                           const double2 (&db)[ND],
                                           const double2 *__restrict__ Y, unsigned i, int npad)
{
#pragma unroll
    for (int p = TJ; p >= 0; --p)
        if (p <= J) {
            double nr = 0.0, ni = 0.0;
            double dnr[ND], dni[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) dnr[d] = dni[d] = 0.0;
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
                        dnr[d] += a.x * du.x + a.y * du.y;
                        dni[d] += a.x * du.y - a.y * du.x;
                    }
                }
            }
            if (p > 0) {
                const double2 w = st.col[p - 1];
                nr -= b.x * w.x + b.y * w.y;
                ni -= b.x * w.y - b.y * w.x;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    dnr[d] -= db[d].x * w.x + db[d].y * w.y;
                    dni[d] -= db[d].x * w.y - db[d].y * w.x;
                    if (!DZ) {
                        const double2 dw = st.dcol[d][p - 1];
                        dnr[d] -= b.x * dw.x + b.y * dw.y;
                        dni[d] -= b.x * dw.y - b.y * dw.x;
                    }
                }
            }
            st.col[p] = make_double2(nr, ni);
#pragma unroll
            for (int d = 0; d < ND; ++d) st.dcol[d][p] = make_double2(dnr[d], dni[d]);
        }
#pragma unroll
    for (int p = 0; p <= TJ; ++p)
        if (p <= J) {
            const double2 y = load_row(Y, (size_t)(eb + p), npad, i * 16u);
            st.S0 += y.x * st.col[p].x + y.y * st.col[p].y;
#pragma unroll
            for (int d = 0; d < ND; ++d) st.S[d] += y.x * st.dcol[d][p].x + y.y * st.dcol[d][p].y;
        }
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
    if (Q == 0) {
        st.col[0] = make_double2(1.0, 0.0);
        st.S0 += load_row(Y, 0, npad, i * 16u).x;  // J = 0: poly = 1, dpoly = 0
    }
    constexpr int J0 = (Q == 0) ? 1 : 2 * Q;
    constexpr bool kFull = TJ <= 10;  // straight-line code up to 2J = 10
    if constexpr (kFull) {
#pragma unroll
        for (int J = J0; J <= TJ; ++J) {
            if (Q == 0 && J == 1)
                dedr_level<TJ, ND, true>(J, hbase_of(J), st, a, b, da, db, Y, i, npad);
            else
                dedr_level<TJ, ND, false>(J, hbase_of(J) + Q * (J + 1), st, a, b, da, db, Y, i,
                                          npad);
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
            dedr_level<TJ, ND, false>(J, eb, st, a, b, da, db, Y, i, npad);
            if (J == 2 * Q + 1 && 2 * Q + 2 <= TJ) {
                mirror_seed<TJ, Q>(st.col, st.seed);
#pragma unroll
                for (int d = 0; d < ND; ++d) mirror_seed<TJ, Q>(st.dcol[d], st.dseed[d]);
            }
            eb += (J + 1) * (J / 2 + 1) + Q;  // half index of (J+1, 0, Q)
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
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_dedr(int npairs, int npad, const double *__restrict__ pos,
                                             const int *__restrict__ nbr,
                                             const int *__restrict__ pair_atom,
                                             const double2 *__restrict__ Y, Geom g,
                                             double *__restrict__ dE)
{
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int dir0 = (ND == 3) ? 0 : (int)blockIdx.y;
    const bool valid = t < npairs;
    const int tt = valid ? t : npairs - 1;
    const int i = pair_atom[tt];
    double rv[3];
    min_image(pos, i, nbr[tt], g, rv);
    PairGeom pg;
    const bool ok = pair_geometry(rv, g, pg);

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
    st.S0 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) st.S[d] = 0.0;
#pragma unroll
    for (int p = 0; p <= TJ; ++p) {
        st.seed[p] = make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < ND; ++d) st.dseed[d][p] = make_double2(0.0, 0.0);
    }
    DedrColumns<TJ, ND, 0>::run(st, pg.a, pg.b, da, db, Y, (unsigned)i, npad);
    if (valid) {
#pragma unroll
        for (int d = 0; d < ND; ++d)
            dE[3 * (size_t)t + dir0 + d] = dfc[d] * st.S0 + pg.fc * st.S[d];
    }
}

// ---------------------------------------------------------------------------
// update_forces and the energy
// ---------------------------------------------------------------------------
__global__ void k_gather(int n, int npad, int nhalf, const int *__restrict__ off,
                         const int *__restrict__ rev, const double *__restrict__ dE,
                         const double2 *__restrict__ U, const double2 *__restrict__ Y,
                         double *__restrict__ energy, double *__restrict__ force)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    const int te = off[i + 1];
    for (int t = off[i]; t < te; ++t) {
        const int r = rev[t];
        fx += dE[3 * (size_t)t + 0] - dE[3 * (size_t)r + 0];
        fy += dE[3 * (size_t)t + 1] - dE[3 * (size_t)r + 1];
        fz += dE[3 * (size_t)t + 2] - dE[3 * (size_t)r + 2];
    }
    force[3 * (size_t)i + 0] = fx;
    force[3 * (size_t)i + 1] = fy;
    force[3 * (size_t)i + 2] = fz;
    if (energy) {
        // E_i = (1/3) Re sum_full Y : conj(U) = (1/3) sum_half Re(Y~ conj(U~))
        double e = 0.0;
        for (int k = 0; k < nhalf; ++k) {
            const double2 y = Y[(size_t)k * npad + i], u = U[(size_t)k * npad + i];
            e += y.x * u.x + y.y * u.y;
        }
        energy[i] = e * (1.0 / 3.0);
    }
}

__global__ void k_unscale(int n, int npad, int nhalf, const double2 *__restrict__ src,
                          const double *__restrict__ scale, double *__restrict__ dst)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)n * nhalf) return;
    const int e = (int)(k / n), i = (int)(k - (size_t)e * n);
    const double2 v = src[(size_t)e * npad + i];
    dst[2 * k + 0] = scale[e] * v.x;
    dst[2 * k + 1] = scale[e] * v.y;
}

template <int TJ>
hipError_t launch_u_t(int n, int npad, const double *pos, const int *off, const int *nbr,
                      const Geom &g, double2 *U, int *pair_atom, int *flag, hipStream_t s)
{
    const int nblk = (n + 1) / 2;
    hipLaunchKernelGGL(k_compute_u<TJ>, dim3(nblk), dim3(64), 0, s, n, npad, pos, off, nbr, g, U,
                       pair_atom, flag);
    return hipGetLastError();
}

template <int TJ>
hipError_t launch_dedr_t(int dirs, int npairs, int npad, const double *pos, const int *nbr,
                         const int *pair_atom, const double2 *Y, const Geom &g, double *dE,
                         hipStream_t s)
{
    const int nblk = (npairs + 63) / 64;
    if (dirs == 3)
        hipLaunchKernelGGL((k_dedr<TJ, 3>), dim3(nblk, 1), dim3(64), 0, s, npairs, npad, pos, nbr,
                           pair_atom, Y, g, dE);
    else
        hipLaunchKernelGGL((k_dedr<TJ, 1>), dim3(nblk, 3), dim3(64), 0, s, npairs, npad, pos, nbr,
                           pair_atom, Y, g, dE);
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
    (void)T;
    switch (twojmax) {
#define X(k) \
    case k: return launch_u_t<k>(n, npad, pos, off, nbr, g, U, pair_atom, flag, s);
        SNAP_TJ_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dedr(int twojmax, int dirs, int npairs, int npad, const double *pos,
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

hipError_t launch_compute_y(int n, int npad, int nhalf, const double2 *U, double2 *Y,
                            const DevTables &T, const double *beta, int per_atom_beta, int nb,
                            const double *gscale, hipStream_t s)
{
    (void)nhalf;
    const int nblk = (n + 63) / 64;
    hipLaunchKernelGGL(k_compute_y, dim3(T.nrows * nblk), dim3(64 * kYWaves), 0, s, n, npad, nblk,
                       U, Y, T.rows, T.items, T.terms, beta, per_atom_beta, nb, gscale);
    return hipGetLastError();
}

hipError_t launch_bispectrum(int n, int npad, const double2 *U, const DevTables &T, int nb,
                             double *B, const double *beta, int per_atom_beta, double *energy,
                             hipStream_t s)
{
    const int nblk = (n + 63) / 64;
    hipLaunchKernelGGL(k_bispectrum, dim3(nblk, nb), dim3(64), 0, s, n, npad, U, T.items, T.terms,
                       T.bitems, T.bl_begin, nb, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !energy) return e;
    hipLaunchKernelGGL(k_energy_from_b, dim3((n + 127) / 128), dim3(128), 0, s, n, nb, B, beta,
                       per_atom_beta, energy);
    return hipGetLastError();
}

hipError_t launch_gather(int n, int npad, int nhalf, const int *off, const int *rev,
                         const double *dE, const double2 *U, const double2 *Y, double *energy,
                         double *force, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3((n + 127) / 128), dim3(128), 0, s, n, npad, nhalf, off, rev,
                       dE, U, Y, energy, force);
    return hipGetLastError();
}

hipError_t launch_unscale(int n, int npad, int nhalf, const double2 *src, const double *scale,
                          double *dst, hipStream_t s)
{
    const size_t tot = (size_t)n * nhalf;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unscale, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, npad,
                       nhalf, src, scale, dst);
    return hipGetLastError();
}

}  // namespace snapmi
