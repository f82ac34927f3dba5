// snap_device.hpp -- device helpers shared by the FP64 SNAP kernels for gfx950
// (MI355X).
//
// Stages (arXiv 2011.12875, Sec. IV Listing 5 with the GPU refinements of
// Sec. VI):
//   k_compute_u  eq. (u) (snap_u.hip): lanes walk (atom, neighbour) pairs,
//                two pairs of one atom per lane, one workgroup per column of
//                the stored half of u_j (Sec. VI) and group of four atoms;
//                the recursion eq. (hysphrecur) runs in registers and the
//                per-atom sum U_j is reduced through LDS in a fixed order (no
//                atomics, bit-reproducible).
//   k_compute_y  eq. (y) (snap_y.hip): one lane per atom (64 consecutive
//                atoms per wavefront, like the AoSoA layout of Sec. VI), all
//                lanes running the same Clebsch-Gordan contraction program,
//                so coefficients and indices are wavefront-uniform; rows
//                (j, p) of Y are split over four wavefronts and reduced in
//                LDS.
//   k_bispectrum eq. (z) and eq. (snapatomenergy), on request (snap_misc.hip;
//                U staged in LDS for small 2J).
//   k_dedr       eq. (snapforce2) fused with the derivative recursion
//                ("compute_fused_dE", Sec. VI) (snap_dedr.hip): one lane per
//                pair and direction (Sec. VI splits x, y, z too), u and du
//                recomputed in registers and contracted with Y on the fly.
//   k_gather     update_forces: F_i = sum_out dE_p - sum_out dE_rev(p), a
//                deterministic gather through the reverse-pair index; also the
//                energy E_i = (1/3) Re sum_j Y_j : U_j^* (B is cubic in U).
//   k_virial     sum_p dE_p (x) r_ik per atom and in total.
//
// Conventions: twice-integer J, row p, column q, stored half q <= J/2.
// The recursion runs on the polynomial coefficients poly^J_{pq} = u^J_{pq}/N
// (N = sqrt(p!(J-p)!/(q!(J-q)!))), which obey
//   poly^J_{pq} = a* poly^{J-1}_{pq} - b* poly^{J-1}_{p-1,q}
// with unit weights, and the mirror rule
//   poly^J_{J-p,J-q} = (-1)^(p-q) conj(poly^J_{pq}).
// Per-atom arrays are element-major X[e * npad + atom] of double2 (re, im):
// U holds full (J+1) x (J+1) matrices of true values, Y the stored half of
// the scaled Y~ = w N Y (w: half-sum weight).
#pragma once
#include <hip/hip_runtime.h>

#include "snap_kernels.hpp"

namespace snapmi {
namespace dev {

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

// Cutoff rc and density weight w of the pair (i, k): rcut and 1 for one
// element; for several, rcutfac (R_t(i) + R_t(k)) and the weight of the
// neighbour's element (the density weights eq. (u) leaves out).  A type
// outside 0..nelem-1 is clamped (no read out of range) and returns false.
__device__ __forceinline__ bool pair_cut(const Geom &g, int i, int k, double &rc, double &w)
{
    if (!g.type) {
        rc = g.rcut;
        w = 1.0;
        return true;
    }
    int ti = g.type[i], tk = g.type[k];
    const bool ok = ti >= 0 && ti < g.nelem && tk >= 0 && tk < g.nelem;
    ti = ti < 0 ? 0 : (ti >= g.nelem ? g.nelem - 1 : ti);
    tk = tk < 0 ? 0 : (tk >= g.nelem ? g.nelem - 1 : tk);
    rc = g.rcutfac * (g.erad[ti] + g.erad[tk]);
    w = g.ewt[tk];
    return ok;
}

// The 3-sphere map of eq. (u) with the pair cutoff rc:
// theta0 = rfac0 pi (r - rmin0)/(rc - rmin0), Cayley-Klein pair
// a = cos theta0 - i sin theta0 n_z, b = sin theta0 (n_y - i n_x), and the
// switching function times the pair's density weight, w f_c and w df_c/dr
// (zero from rc on).  Returns false for r < 1e-10 or non-finite input (the
// pair then contributes nothing: f_c = 0, a = 1, b = 0).
__device__ __forceinline__ bool pair_geometry(const double rv[3], const Geom &g, double rc,
                                              double w, PairGeom &pg)
{
    const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    const double r = sqrt(r2);
    const bool ok = (r >= 1e-10) && (r < 1e300);  // false for NaN too
    const double rs = ok ? r : 1.0;
    pg.r = rs;
    // two divisions per pair (1/r, 1/(rc - rmin0)); the rest are products
    const double ir = 1.0 / rs;
    pg.n[0] = ok ? rv[0] * ir : 0.0;
    pg.n[1] = ok ? rv[1] * ir : 0.0;
    pg.n[2] = ok ? rv[2] * ir : 1.0;
    const double ispan = 1.0 / (rc - g.rmin0);
    const double x = (rs - g.rmin0) * ispan;  // 0 at rmin0, 1 at the cutoff
    double s0, c0;
    sincos(g.rfac0 * M_PI * x, &s0, &c0);
    pg.c0 = c0;
    pg.s0 = s0;
    pg.dth0 = g.rfac0 * M_PI * ispan;
    pg.a = ok ? make_double2(c0, -s0 * pg.n[2]) : make_double2(1.0, 0.0);
    pg.b = ok ? make_double2(s0 * pg.n[1], -s0 * pg.n[0]) : make_double2(0.0, 0.0);
    double fc = 1.0, dfdr = 0.0;
    if (g.switch_flag && rs > g.rmin0) {
        double sx, cx;
        sincos(M_PI * x, &sx, &cx);
        fc = 0.5 * (cx + 1.0);
        dfdr = -0.5 * M_PI * ispan * sx;
    }
    const bool inside = ok && r < rc;
    pg.fc = inside ? w * fc : 0.0;
    pg.dfdr = inside ? w * dfdr : 0.0;
    return ok;
}

__device__ __forceinline__ void min_image(const double *__restrict__ pos, int i, int k,
                                          const Geom &g, double rv[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double x = pos[3 * k + d] - pos[3 * i + d];
        if (g.box[d] > 0.0) x -= g.box[d] * rint(x * g.ibox[d]);
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
            // each component is one running sum of products, so that it
            // contracts to a single multiply followed by fused multiply-adds
            double nr = 0.0, ni = 0.0;
            if (p < J) {
                const double2 u = col[p];
                nr = a.x * u.x + a.y * u.y;
                ni = a.x * u.y - a.y * u.x;
            }
            if (p > 0) {
                const double2 w = col[p - 1];
                nr = nr - b.x * w.x - b.y * w.y;
                ni = ni - b.x * w.y + b.y * w.x;
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


}  // namespace dev
}  // namespace snapmi
