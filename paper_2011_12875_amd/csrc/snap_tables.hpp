// snap_tables.hpp -- host-side index tables and contraction programs.
//
// Everything here is plain C++ run once per parameter set (snap_setup); the
// device kernels only read the flattened arrays it produces.
//
// Notation: angular momenta are twice-integers J = 2j; matrix indices
// p = j + m (row) and q = j + m' (column) run over 0..J.  Only the "half"
// elements with q <= J/2 are stored (Sec. VI of arXiv 2011.12875: u_j, U_j,
// dU_j and Y_j are determined by about half of their elements through
//   u_{J-p, J-q} = (-1)^(p-q) conj(u_{p q}) ).
#pragma once

#include <array>
#include <cstdint>
#include <vector>

namespace snapmi {

// Storage.  compute_U writes U as full (J+1)x(J+1) matrices of true values,
// element-major ("full index" f = fbase(J) + p (J+1) + q); the row loads of
// compute_Y read it directly.  Y is kept on the stored half only, scaled:
//   Y~_e = w_e N_e Y_e,
// with N_e = sqrt(p!(J-p)!/(q!(J-q)!)) the normalisation of the polynomial
// basis and w_e the half-sum weight (2 for q < J/2, 1 for q == J/2), so that
// compute_dE contracts it with plain polynomial coefficients (no square
// roots) and Re(Y : conj(dU)) over the full matrix is a plain sum over the
// stored half.

// Where compute_U puts a stored-half element e = (J, p, q): its full index
// and that of its mirror (J, J-p, J-q) (-1 when e is its own mirror), with
//   U(J-p, J-q) = (-1)^(p-q) conj(U(p, q))   and   U = N * poly-sum.
struct UInfo {
    int32_t fi, fm;
    double nrm;    // N_e
    double msign;  // (-1)^(p-q)
};

// Bispectrum program (eq. (z)): for a canonical l = (J1, J2, J),
//   B_l = sum over stored (p, q) of w Re(Z(p, q) conj(U^J(p, q))),
//   Z(p, q) = sum of terms cc U(f1) U(f2)   (full indices, true values).
#ifndef SNAP_Y_WAVES
#define SNAP_Y_WAVES 4
#endif
constexpr int kYWaves = SNAP_Y_WAVES;  // wavefronts per compute_Y workgroup
struct BTerm {
    double cc;
    int32_t f1, f2;
};
struct BItem {
    int32_t tb, te;  // terms tb .. te-1
    int32_t f3;      // full index of U^J(p, q)
    int32_t pad;
    double w;        // half-sum weight
};

// Row-blocked form of the same contraction, used by compute_Y.  One
// contribution is one input pair (J1 >= J2) of a row (J, p) of Y:
//   Z(p, q) = sum_{p1} cp[p1] sum_{q1} cq[q][q1] U^J1(p1, q1) U^J2(p2, q2),
//   p2 = p - p1 + d, q2 = q - q1 + d, d = (J1 + J2 - J)/2,
// with true (unscaled) U values; cp and cq are Clebsch-Gordan coefficients.
// A unit of compute_Y holds the rows p and p + 1 of one J (p alone for the
// last row of an even J): row p + 1 pairs U^J1 row p1 with the U^J2 row
// that row p pairs with p1 - 1, so each loaded row serves both.  The p1
// range of a contribution is the union of the two rows' ranges, and cp
// holds two values per p1 (zero where that row has no valid p2).
struct YContrib {
    int32_t j1, j2, d, l;  // input ranks, offset d, canonical component l
    double factor;         // multiplicity * (J_max + 1)/(J + 1)
    int32_t p1lo, p1hi;    // rows p1 of U^J1 used by either row (inclusive)
    int32_t cp_off;        // cp of (p1, row r) at cp_off + 2 (p1 - p1lo) + r
    int32_t cq_off;        // cq[q][q1] at cq_off + q * (2J_max + 1) + q1, q < nq (zero for q1 > j1)
    int32_t cost;          // estimated lane operations
    int32_t pad;
};

// Rows per unit: two for every supported 2J_max (the contribution's sums are
// added to LDS, so the second row costs registers only for its own sums and
// the U^J2 row it keeps); the single-row form stays for larger 2J_max.
constexpr int y_unit_rows(int twojmax) { return twojmax <= 14 ? 2 : 1; }

// A unit (rows p, p + 1 of J) of Y, split over the waves of one workgroup:
// contributions of wave w are cb[w] .. cb[w+1]-1.
struct YRowC {
    int32_t J, p, nq, ebase;  // ebase: half index of (J, p, 0)
    int32_t cb[kYWaves + 1];
    int32_t cost;             // busiest wave
    int32_t frow;             // full index of (J, p, 0)
    int32_t two;              // 1 if the unit also holds row p + 1
    double oscale[2][8];      // w N of the outputs (J, p + r, q): Y~ = w N Y
    double einv[2][8];        // 1/N of the outputs: Re(Y~ conj(U)) / N = w Re(Y conj(U))
};

// LDS-staged compute_Y (2J <= kYLdsMaxTJ).  A workgroup holds the full U of
// kYLdsAtoms atoms in LDS and computes a group of units (row pairs p, p + 1
// of one J) for them with kYLdsWaves wavefronts; lanes 0..31 take row p and
// lanes 32..63 row p + 1 of the same 32 atoms.  A unit's contributions are
// split into tasks, one per wavefront, whose partial sums are reduced in LDS.
constexpr int kYLdsAtoms = 32;
constexpr int kYLdsWaves = 16;
constexpr int kYLdsMaxTJ = 8;
constexpr int kYLdsGroupings = 4;  // programs for 1, 2, 4 and 8 groups of units
// One contribution (J1 >= J2 -> J) of a unit in the LDS kernel.  Step k of its
// loop pairs U^J1 row lo[h] + k with U^J2 row p + h - (lo[h] + k) + d for the
// half h of the wavefront (row p + h of Y): the half of row p + 1 walks its
// own range, shifted by one, so both halves run max(rows) steps instead of
// the union of their ranges.  cp[cp_off + 2k + h] is the row coefficient of
// half h at step k (zero where that half has no valid row).
struct YLContrib {
    int32_t j1, j2, d, l;
    double factor;    // multiplicity * (J_max + 1)/(J + 1)
    int32_t lo[2];    // first U^J1 row of each half
    int32_t nsteps;
    int32_t cp_off;
    int32_t cq_off;   // as YContrib
    int32_t pad;
};
// One wavefront's task: contributions cb .. ce-1 of unit `unit` (an index
// into yrows; -1 for an idle wavefront).
struct YLTask {
    int32_t unit, cb, ce, pad;
};
// The units of one group and the wavefronts (tasks) of each: slot s of group
// g is reduced by wavefront s, summing the partials of tasks tb[s] .. tb[s+1]-1.
struct YLGroup {
    int32_t nunits;
    int32_t unit[kYLdsWaves];
    int32_t tb[kYLdsWaves + 1];  // slot s: waves tw[tb[s]] .. tw[tb[s+1]-1]
    int32_t tw[kYLdsWaves];
};

struct Tables {
    int twojmax = 0;
    int nhalf = 0;
    int nb = 0;
    std::vector<int> hbase;                  // [twojmax+2] first half index of each J
    std::vector<std::array<int, 3>> helem;   // (J, p, q) per half index
    int nfullel = 0;                         // sum (J+1)^2
    std::vector<double> norm;                // N_e per half index
    std::vector<double> whalf;               // 2 or 1 per half index
    std::vector<double> unscale_y;           // 1/(w_e N_e): Y~ -> Y
    std::vector<int> half2full;              // full index of each half element
    std::vector<UInfo> uinfo;
    std::vector<std::array<int, 3>> comps;   // canonical (J1, J2, J)
    std::vector<BTerm> bterms;
    std::vector<int> bl_begin;               // [nb+1] into bitems
    std::vector<BItem> bitems;
    // row-blocked compute_Y program
    std::vector<YContrib> ycontrib;
    std::vector<YRowC> yrows;               // sorted by decreasing cost
    std::vector<double> ycp, ycq;           // Clebsch-Gordan coefficient tables
    // LDS-staged compute_Y: contributions and cp table, and for each grouping
    // gi (G = 1 << gi groups) the tasks [G][kYLdsWaves] and groups [G],
    // stored one grouping after another (offsets yl_task_off, yl_group_off)
    std::vector<YLContrib> ylcontrib;
    std::vector<double> ylcp;
    std::vector<YLTask> yltask;
    std::vector<YLGroup> ylgroup;
    int yl_task_off[kYLdsGroupings] = {0, 0, 0, 0};
    int yl_group_off[kYLdsGroupings] = {0, 0, 0, 0};
    std::vector<long> yl_cost;              // estimated cost per unit (index as yrows)
    long yterms = 0;                         // Clebsch-Gordan products per atom
    long ypartials = 0;                      // (contribution, p1, q) partial sums per atom
    std::vector<double> nfull;              // N of every full element, blocks of (J+1)^2
    // Clebsch-Gordan values actually used (for inspection and tests)
    std::vector<std::array<int, 5>> cg_keys; // J1, J2, J, M1, M2
    std::vector<double> cg_vals;

    int half_index(int J, int p, int q) const { return hbase[J] + q * (J + 1) + p; }
    int full_index(int J, int p, int q) const { return fbase[J] + p * (J + 1) + q; }
    std::vector<int> fbase;                  // [twojmax+2] first full index of each J
};

// Clebsch-Gordan coefficient <j1 m1 j2 m2 | j m>, arguments doubled,
// Condon-Shortley phase; 0 outside the coupling rules.
double clebsch_gordan(int J1, int M1, int J2, int M2, int J, int M);

// Build every table for one twojmax (0 .. 14).
void build_tables(int twojmax, Tables &t);

// Host cell-list neighbour builder; see snap_build_neighbors in snapmi.h.
// Returns 0, or -1 when cap is too small (npairs then holds the needed size).
int build_neighbors(const double *pos, int n, const double box[3], double rcut, int *off, int *nbr,
                    int *rev, int cap, int *npairs);

}  // namespace snapmi
