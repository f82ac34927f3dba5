// snap_tables.cpp -- host tables for the SNAP kernels (see snap_tables.hpp).
#include "snap_tables.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace snapmi {

// ---------------------------------------------------------------------------
// Clebsch-Gordan coefficients (Sec. II.A, eq. (z) uses them to couple U_j1 and
// U_j2 into rank j).  Racah's closed form, evaluated with log-factorials in
// long double; Condon-Shortley phase.
// ---------------------------------------------------------------------------
static long double lfact(int n) { return std::lgamma((long double)n + 1.0L); }

double clebsch_gordan(int J1, int M1, int J2, int M2, int J, int M)
{
    if (M1 + M2 != M) return 0.0;
    if (std::abs(M1) > J1 || std::abs(M2) > J2 || std::abs(M) > J) return 0.0;
    if ((J1 + M1) % 2 || (J2 + M2) % 2 || (J + M) % 2) return 0.0;
    if (J < std::abs(J1 - J2) || J > J1 + J2 || (J1 + J2 + J) % 2) return 0.0;
    // integer arguments of the factorials
    const int s1 = (J1 + J2 - J) / 2, s2 = (J1 - J2 + J) / 2, s3 = (J2 - J1 + J) / 2;
    const int s4 = (J1 + J2 + J) / 2 + 1;
    const int a1 = (J1 + M1) / 2, b1 = (J1 - M1) / 2;
    const int a2 = (J2 + M2) / 2, b2 = (J2 - M2) / 2;
    const int a = (J + M) / 2, b = (J - M) / 2;
    const long double lpre = 0.5L * (std::log((long double)(J + 1)) + lfact(s1) + lfact(s2) +
                                     lfact(s3) - lfact(s4) + lfact(a1) + lfact(b1) + lfact(a2) +
                                     lfact(b2) + lfact(a) + lfact(b));
    const int t1 = (J - J2 + M1) / 2;  // j - j2 + m1
    const int t2 = (J - J1 - M2) / 2;  // j - j1 - m2
    const int kmin = std::max({0, -t1, -t2});
    const int kmax = std::min({s1, b1, a2});
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        const long double ld = lfact(k) + lfact(s1 - k) + lfact(b1 - k) + lfact(a2 - k) +
                               lfact(t1 + k) + lfact(t2 + k);
        const long double v = std::exp(lpre - ld);
        sum += (k % 2) ? -v : v;
    }
    return (double)sum;
}

// ---------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------
void build_tables(int tj, Tables &t)
{
    t = Tables();
    t.twojmax = tj;

    // half-matrix storage: for each J, columns q = 0..J/2, rows p = 0..J
    t.hbase.assign(tj + 2, 0);
    for (int J = 0; J <= tj; ++J) t.hbase[J + 1] = t.hbase[J] + (J + 1) * (J / 2 + 1);
    t.nhalf = t.hbase[tj + 1];
    t.helem.resize(t.nhalf);
    t.norm.assign(t.nhalf, 0.0);
    t.whalf.assign(t.nhalf, 0.0);
    t.unscale_u.assign(t.nhalf, 0.0);
    t.unscale_y.assign(t.nhalf, 0.0);
    for (int J = 0; J <= tj; ++J)
        for (int q = 0; q <= J / 2; ++q)
            for (int p = 0; p <= J; ++p) {
                const int e = t.half_index(J, p, q);
                t.helem[e] = {J, p, q};
                // u^J_{pq} = N_e poly^J_{pq}; the polynomial coefficients obey
                // eq. (hysphrecur) along a column with unit weights:
                //   poly^J_{pq} = a* poly^{J-1}_{pq} - b* poly^{J-1}_{p-1,q}
                t.norm[e] = std::sqrt(std::exp(std::lgamma(p + 1.0) + std::lgamma(J - p + 1.0) -
                                               std::lgamma(q + 1.0) - std::lgamma(J - q + 1.0)));
                t.whalf[e] = (2 * q < J) ? 2.0 : 1.0;
                t.unscale_u[e] = t.norm[e];
                t.unscale_y[e] = 1.0 / (t.whalf[e] * t.norm[e]);
            }

    // canonical components: J2 <= J1 <= J (Sec. II.A), coupling rules
    std::vector<int> cidx((tj + 1) * (tj + 1) * (tj + 1), -1);
    auto cix = [&](int a, int b, int c) -> int & { return cidx[(a * (tj + 1) + b) * (tj + 1) + c]; };
    for (int J1 = 0; J1 <= tj; ++J1)
        for (int J2 = 0; J2 <= J1; ++J2)
            for (int J = J1 - J2; J <= std::min(tj, J1 + J2); J += 2)
                if (J >= J1) {
                    cix(J1, J2, J) = (int)t.comps.size();
                    t.comps.push_back({J1, J2, J});
                }
    t.nb = (int)t.comps.size();

    // Clebsch-Gordan cache keyed by (J1, J2, J, M1, M2)
    auto cg = [&](int J1, int M1, int J2, int M2, int J) {
        return clebsch_gordan(J1, M1, J2, M2, J, M1 + M2);
    };
    for (int J1 = 0; J1 <= tj; ++J1)
        for (int J2 = 0; J2 <= J1; ++J2)
            for (int J = J1 - J2; J <= std::min(tj, J1 + J2); J += 2)
                for (int M1 = -J1; M1 <= J1; M1 += 2)
                    for (int M2 = -J2; M2 <= J2; M2 += 2)
                        if (std::abs(M1 + M2) <= J) {
                            t.cg_keys.push_back({J1, J2, J, M1, M2});
                            t.cg_vals.push_back(cg(J1, M1, J2, M2, J));
                        }

    // Operand of a product: the full element (Jx, px, qx) of U (or Y) read
    // from the stored half; elements with qx > Jx/2 come from the mirror
    // (Jx-px, Jx-qx) conjugated, with sign (-1)^(qx-px).
    // The operand's scale N_e (U = N U~) is folded into its sign.
    struct Operand { int e; bool conj; double sign; };
    auto operand = [&](int Jx, int px, int qx) -> Operand {
        if (2 * qx <= Jx) {
            const int e = t.half_index(Jx, px, qx);
            return {e, false, t.norm[e]};
        }
        const int sgn = ((qx - px) % 2 == 0) ? 1 : -1;
        const int e = t.half_index(Jx, Jx - px, Jx - qx);
        return {e, true, (double)sgn * t.norm[e]};
    };

    // The adjoint of eq. (y).  For a canonical l = (J1, J2, J) the derivative
    // of B_l = Z^J_{J1J2} : conj(U^J) with respect to each of its three
    // matrix factors is Re[X : conj(dU)] with X = Z^J_{J1J2} for U^J,
    // (J+1)/(J1+1) Z^{J1}_{J J2} for U^J1 and (J+1)/(J2+1) Z^{J2}_{J J1} for
    // U^J2 (Clebsch-Gordan symmetry).  So a stored product Z^c_{ab} (a >= b)
    // enters Y^c with beta_l times (number of factors of rank c in l) times
    // (J_max+1)/(c+1), where l is the sorted triple {a, b, c}.
    struct PendingRow { YRow row; std::vector<int> order; std::vector<ZItem> items; std::vector<std::vector<Term>> terms; };
    std::vector<PendingRow> pend;

    for (int J = 0; J <= tj; ++J)
        for (int p = 0; p <= J; ++p) {
            PendingRow pr;
            pr.row.J = J;
            pr.row.p = p;
            pr.row.nq = J / 2 + 1;
            pr.row.ebase = t.half_index(J, p, 0);
            for (int a = 0; a <= tj; ++a)
                for (int b = 0; b <= a; ++b) {
                    if (J < a - b || J > a + b || (a + b + J) % 2) continue;
                    int s[3] = {a, b, J};
                    std::sort(s, s + 3);
                    const int l = cix(s[1], s[0], s[2]);
                    const int mult = (a == J) + (b == J) + 1;
                    const double factor = (double)mult * (double)(s[2] + 1) / (double)(J + 1);
                    const int M = 2 * p - J;
                    for (int q = 0; q <= J / 2; ++q) {
                        const int Mq = 2 * q - J;
                        const int eo = t.half_index(J, p, q);
                        const double oscale = t.whalf[eo] * t.norm[eo];  // Y~ = w N Y
                        std::vector<Term> pat[4];
                        for (int p1 = 0; p1 <= a; ++p1) {
                            const int M1 = 2 * p1 - a, M2 = M - M1;
                            if (std::abs(M2) > b) continue;
                            const int p2 = (M2 + b) / 2;
                            const double cp = cg(a, M1, b, M2, J);
                            if (std::fabs(cp) < 1e-15) continue;
                            for (int q1 = 0; q1 <= a; ++q1) {
                                const int N1 = 2 * q1 - a, N2 = Mq - N1;
                                if (std::abs(N2) > b) continue;
                                const int q2 = (N2 + b) / 2;
                                const double cq = cg(a, N1, b, N2, J);
                                if (std::fabs(cq) < 1e-15) continue;
                                const Operand o1 = operand(a, p1, q1), o2 = operand(b, p2, q2);
                                const int k = (o1.conj ? 1 : 0) | (o2.conj ? 2 : 0);
                                pat[k].push_back({cp * cq * o1.sign * o2.sign * oscale, o1.e, o2.e});
                            }
                        }
                        ZItem it{};
                        it.q = q;
                        it.l = l;
                        it.factor = factor;
                        it.j1 = a;
                        it.j2 = b;
                        std::vector<Term> flat;
                        it.tb[0] = 0;
                        for (int k = 0; k < 4; ++k) {
                            flat.insert(flat.end(), pat[k].begin(), pat[k].end());
                            it.tb[k + 1] = (int)flat.size();
                        }
                        pr.items.push_back(it);
                        pr.terms.push_back(std::move(flat));
                    }
                }
            // longest-processing-time assignment of items to the waves
            std::vector<int> ord(pr.items.size());
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
                return pr.terms[x].size() > pr.terms[y].size();
            });
            std::vector<int> load(kYWaves, 0);
            std::vector<std::vector<int>> wav(kYWaves);
            for (int x : ord) {
                const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                wav[w].push_back(x);
                load[w] += (int)pr.terms[x].size() + 8;
            }
            for (int w = 0; w < kYWaves; ++w)
                for (int x : wav[w]) pr.order.push_back(x);
            int acc = 0;
            for (int w = 0; w < kYWaves; ++w) {
                pr.row.wb[w] = acc;
                acc += (int)wav[w].size();
            }
            pr.row.wb[kYWaves] = acc;
            pr.row.cost = *std::max_element(load.begin(), load.end());
            pend.push_back(std::move(pr));
        }

    // rows in decreasing cost so the heaviest start first
    std::stable_sort(pend.begin(), pend.end(),
                     [](const PendingRow &x, const PendingRow &y) { return x.row.cost > y.row.cost; });
    for (auto &pr : pend) {
        const int ib = (int)t.items.size();
        for (int w = 0; w <= kYWaves; ++w) pr.row.wb[w] += ib;
        for (int x : pr.order) {
            ZItem it = pr.items[x];
            const int tb0 = (int)t.terms.size();
            for (int k = 0; k <= 4; ++k) it.tb[k] += tb0;
            t.terms.insert(t.terms.end(), pr.terms[x].begin(), pr.terms[x].end());
            t.items.push_back(it);
        }
        t.rows.push_back(pr.row);
    }

    // bispectrum program: for each canonical (J1, J2, J), the items of
    // Z^J_{J1 J2} over all stored (p, q), with the half-sum weight
    std::vector<std::vector<BItem>> per_l(t.nb);
    for (const auto &row : t.rows)
        for (int x = row.wb[0]; x < row.wb[kYWaves]; ++x) {
            const ZItem &it = t.items[x];
            if (it.j1 > row.J || it.j2 > it.j1) continue;  // canonical: J >= J1 >= J2
            const int l = cix(it.j1, it.j2, row.J);
            if (l < 0) continue;
            const int e = t.half_index(row.J, row.p, it.q);
            per_l[l].push_back({x, e});
        }
    t.bl_begin.assign(t.nb + 1, 0);
    for (int l = 0; l < t.nb; ++l) {
        t.bl_begin[l + 1] = t.bl_begin[l] + (int)per_l[l].size();
        t.bitems.insert(t.bitems.end(), per_l[l].begin(), per_l[l].end());
    }
}

// ---------------------------------------------------------------------------
// Cell-list neighbour builder (full list, minimum image, r < rcut)
// ---------------------------------------------------------------------------
int build_neighbors(const double *pos, int n, const double box[3], double rcut, int *off, int *nbr,
                    int *rev, int cap, int *npairs)
{
    const double rc2 = rcut * rcut;
    double lo[3], ext[3];
    int nc[3];
    bool per[3];
    for (int d = 0; d < 3; ++d) {
        per[d] = box[d] > 0.0;
        if (per[d]) {
            lo[d] = 0.0;
            ext[d] = box[d];
            nc[d] = std::max(1, (int)std::floor(box[d] / rcut));
        } else {
            double mn = 0.0, mx = 0.0;
            for (int i = 0; i < n; ++i) {
                const double x = pos[3 * i + d];
                if (i == 0 || x < mn) mn = x;
                if (i == 0 || x > mx) mx = x;
            }
            lo[d] = mn;
            ext[d] = mx - mn;
            nc[d] = std::max(1, (int)std::floor(ext[d] / rcut) + 1);
        }
        nc[d] = std::min(nc[d], 1024);
    }
    const long ncell = (long)nc[0] * nc[1] * nc[2];
    std::vector<int> cell_of(n), head(ncell + 1, 0), list(n);
    for (int i = 0; i < n; ++i) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            double x = pos[3 * i + d] - lo[d];
            if (per[d]) x -= box[d] * std::floor(x / box[d]);
            const double w = ext[d] > 0.0 ? ext[d] / nc[d] : 1.0;
            int ci = (int)std::floor(x / w);
            c[d] = std::min(std::max(ci, 0), nc[d] - 1);
        }
        cell_of[i] = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
        head[cell_of[i] + 1]++;
    }
    for (long c = 0; c < ncell; ++c) head[c + 1] += head[c];
    {
        std::vector<int> fill(head.begin(), head.end() - 1);
        for (int i = 0; i < n; ++i) list[fill[cell_of[i]]++] = i;
    }
    // distinct neighbour cell offsets per dimension
    auto offsets = [&](int d, int ci) {
        std::vector<int> out;
        for (int s = -1; s <= 1; ++s) {
            int cj = ci + s;
            if (per[d]) cj = ((cj % nc[d]) + nc[d]) % nc[d];
            else if (cj < 0 || cj >= nc[d]) continue;
            if (std::find(out.begin(), out.end(), cj) == out.end()) out.push_back(cj);
        }
        return out;
    };
    long np = 0;
    std::vector<int> tmp;
    for (int i = 0; i < n; ++i) {
        const int c = cell_of[i];
        const int cz = c % nc[2], cy = (c / nc[2]) % nc[1], cx = c / (nc[1] * nc[2]);
        tmp.clear();
        for (int x : offsets(0, cx))
            for (int y : offsets(1, cy))
                for (int z : offsets(2, cz)) {
                    const int cc = (x * nc[1] + y) * nc[2] + z;
                    for (int s = head[cc]; s < head[cc + 1]; ++s) {
                        const int k = list[s];
                        if (k == i) continue;
                        double r2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double dx = pos[3 * k + d] - pos[3 * i + d];
                            if (per[d]) dx -= box[d] * std::nearbyint(dx / box[d]);
                            r2 += dx * dx;
                        }
                        if (r2 < rc2) tmp.push_back(k);
                    }
                }
        std::sort(tmp.begin(), tmp.end());
        off[i] = (int)std::min<long>(np, (long)cap);
        for (int k : tmp) {
            if (np < cap) nbr[np] = k;
            ++np;
        }
    }
    off[n] = (int)std::min<long>(np, (long)cap);
    *npairs = (int)np;
    if (np > cap) return -1;
    // reverse index: the position of i inside the (sorted) list of k
    for (int i = 0; i < n; ++i)
        for (int p = off[i]; p < off[i + 1]; ++p) {
            const int k = nbr[p];
            const int *b = nbr + off[k], *e = nbr + off[k + 1];
            const int *f = std::lower_bound(b, e, i);
            rev[p] = (f != e && *f == i) ? (int)(f - nbr) : -1;
        }
    return 0;
}

}  // namespace snapmi
