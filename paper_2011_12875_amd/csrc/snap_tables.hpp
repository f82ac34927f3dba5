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

// Storage scaling.  The device keeps U and Y in scaled form,
//   U~_e = U_e / N_e,   Y~_e = w_e N_e Y_e,
// with N_e = sqrt(p!(J-p)!/(q!(J-q)!)) the normalisation of the polynomial
// basis and w_e the half-sum weight (2 for q < J/2, 1 for q == J/2).  Then
// the per-pair recursion runs on plain polynomial coefficients (no square
// roots), Re(Y : conj(dU)) over the full matrix is a plain sum of
// Re(Y~ conj(dpoly)) over the stored half, and N, w fold into the
// Clebsch-Gordan coefficients of the contraction program.
//
// One term of a Clebsch-Gordan contraction:
//   Z~(p, q) += cc * X(i1) * X(i2)
// where X(i) is the stored (scaled) half element i, conjugated when the
// operand falls in the unstored half; its sign, both operand
// normalisations and the output scaling w N are folded into cc.
struct Term {
    double cc;
    int32_t i1;
    int32_t i2;
};

// One Z element Z^J_{J1 J2}(p, q) of the adjoint sum of eq. (y):
// Y^J(p, q) += factor * beta[l] * Z.  Its terms are split by conjugation
// pattern (bit 0: first operand conjugated, bit 1: second operand).
struct ZItem {
    int32_t q;        // output column (row and J come from the owning row)
    int32_t l;        // canonical component whose coefficient weights it
    double factor;    // multiplicity * (J_max + 1)/(J + 1)
    int32_t tb[5];    // terms of pattern k are tb[k] .. tb[k+1]-1
    int32_t j1, j2;   // input ranks (for inspection)
};

// A row (J, p) of Y, split over the waves of one workgroup.
constexpr int kYWaves = 4;
struct YRow {
    int32_t J, p, nq, ebase;     // ebase: half index of (J, p, 0); stride J+1 per q
    int32_t wb[kYWaves + 1];     // items of wave w: wb[w] .. wb[w+1]-1
    int32_t cost;                // terms of the busiest wave
    int32_t pad;
};

// One canonical component for the bispectrum kernel:
// B_l = sum over its items of Re(Z~ * conj(U~^J(p, q)))  (= w N Z U*/N).
struct BItem {
    int32_t item;    // index into the Z items
    int32_t e;       // half index of U^J(p, q)
};

struct Tables {
    int twojmax = 0;
    int nhalf = 0;
    int nb = 0;
    std::vector<int> hbase;                  // [twojmax+2] first half index of each J
    std::vector<std::array<int, 3>> helem;   // (J, p, q) per half index
    std::vector<double> norm;                // N_e per half index
    std::vector<double> whalf;               // 2 or 1 per half index
    std::vector<double> unscale_u, unscale_y;// N_e and 1/(w_e N_e): scaled -> true values
    std::vector<std::array<int, 3>> comps;   // canonical (J1, J2, J)
    std::vector<Term> terms;
    std::vector<ZItem> items;
    std::vector<YRow> rows;                  // sorted by decreasing cost
    std::vector<int> bl_begin;               // [nb+1] into bitems
    std::vector<BItem> bitems;
    // Clebsch-Gordan values actually used (for inspection and tests)
    std::vector<std::array<int, 5>> cg_keys; // J1, J2, J, M1, M2
    std::vector<double> cg_vals;

    int half_index(int J, int p, int q) const { return hbase[J] + q * (J + 1) + p; }
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
