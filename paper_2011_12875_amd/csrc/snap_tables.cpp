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
// The LDS-staged compute_Y program (see YLContrib, YLTask, YLGroup)
// ---------------------------------------------------------------------------
// (q, q1) pairs the kernel's row product evaluates for offset d: q < nq and
// q1, q2 = q - q1 + d inside 0..2J_max (the compile-time loops).
static int row_product_pairs(int tj, int d, int nq)
{
    int k = 0;
    for (int q = 0; q < nq; ++q)
        for (int q1 = 0; q1 <= tj; ++q1) {
            const int q2 = q - q1 + d;
            if (q2 >= 0 && q2 <= tj) ++k;
        }
    return k;
}

template <class CG>
static void build_lds_program(Tables &t, CG cg)
{
    const int tj = t.twojmax;
    const int nunits = (int)t.yrows.size();
    // the Clebsch-Gordan column table of (J1, J2, J), shared with YContrib
    std::vector<int> cq_at((tj + 1) * (tj + 1) * (tj + 1), -1);
    for (const YRowC &r : t.yrows)
        for (int c = r.cb[0]; c < r.cb[kYWaves]; ++c) {
            const YContrib &yc = t.ycontrib[c];
            cq_at[(yc.j1 * (tj + 1) + yc.j2) * (tj + 1) + r.J] = yc.cq_off;
        }
    std::vector<std::vector<YLContrib>> ucs(nunits);
    std::vector<std::vector<long>> ucost(nunits);
    t.yl_cost.assign(nunits, 0);
    for (int u = 0; u < nunits; ++u) {
        const YRowC &r = t.yrows[u];
        const int J = r.J, p = r.p, two = r.two, nq = r.nq;
        for (int a = 0; a <= tj; ++a)
            for (int b = 0; b <= a; ++b) {
                if (J < a - b || J > a + b || (a + b + J) % 2) continue;
                YLContrib c{};
                c.j1 = a;
                c.j2 = b;
                c.d = (a + b - J) / 2;
                int s3[3] = {a, b, J};
                std::sort(s3, s3 + 3);
                c.l = -1;
                for (int l = 0; l < t.nb; ++l)
                    if (t.comps[l][0] == s3[1] && t.comps[l][1] == s3[0] && t.comps[l][2] == s3[2])
                        c.l = l;
                c.factor = (double)((a == J) + (b == J) + 1) * (double)(s3[2] + 1) / (double)(J + 1);
                // rows of half h: p1 in [p + h + d - b, p + h + d] within [0, a]
                int lo[2], hi[2];
                bool any = false;
                for (int h = 0; h < 2; ++h) {
                    lo[h] = std::max(0, p + h + c.d - b);
                    hi[h] = std::min(a, p + h + c.d);
                    if (h > two) hi[h] = lo[h] - 1;
                    any = any || lo[h] <= hi[h];
                }
                if (!any) continue;
                c.nsteps = std::max(hi[0] - lo[0] + 1, hi[1] - lo[1] + 1);
                for (int h = 0; h < 2; ++h) c.lo[h] = lo[h] <= hi[h] ? lo[h] : lo[1 - h];
                c.cp_off = (int)t.ylcp.size();
                for (int k = 0; k < c.nsteps; ++k)
                    for (int h = 0; h < 2; ++h) {
                        const int p1 = c.lo[h] + k;
                        const bool ok = lo[h] <= hi[h] && p1 <= hi[h];
                        t.ylcp.push_back(ok ? cg(a, 2 * p1 - a, b, 2 * (p + h) - J - (2 * p1 - a), J)
                                            : 0.0);
                    }
                c.cq_off = cq_at[(a * (tj + 1) + b) * (tj + 1) + J];
                const long cost =
                    (long)c.nsteps * (6 * row_product_pairs(tj, c.d, nq) + 4 * nq + a + b + 6) + 20;
                ucs[u].push_back(c);
                ucost[u].push_back(cost);
                t.yl_cost[u] += cost;
            }
    }
    // contributions stored unit by unit, heaviest first inside a unit
    std::vector<int> ubase(nunits + 1, 0);
    for (int u = 0; u < nunits; ++u) {
        std::vector<int> ord(ucs[u].size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return ucost[u][x] > ucost[u][y]; });
        std::vector<YLContrib> cs;
        std::vector<long> cc;
        for (int k : ord) {
            cs.push_back(ucs[u][k]);
            cc.push_back(ucost[u][k]);
        }
        ucs[u] = cs;
        ucost[u] = cc;
    }
    for (int gi = 0; gi < kYLdsGroupings; ++gi) {
        const int G = 1 << gi;
        t.yl_task_off[gi] = -1;
        t.yl_group_off[gi] = -1;
        // units to groups, longest processing time first
        std::vector<int> uord(nunits);
        std::iota(uord.begin(), uord.end(), 0);
        std::stable_sort(uord.begin(), uord.end(),
                         [&](int x, int y) { return t.yl_cost[x] > t.yl_cost[y]; });
        std::vector<long> gl(G, 0);
        std::vector<std::vector<int>> gu(G);
        for (int u : uord) {
            const int g = (int)(std::min_element(gl.begin(), gl.end()) - gl.begin());
            gu[g].push_back(u);
            gl[g] += t.yl_cost[u];
        }
        bool fits = true;
        for (int g = 0; g < G; ++g) fits = fits && (int)gu[g].size() <= kYLdsWaves;
        if (!fits) continue;  // every unit needs a wavefront of its own
        const int task0 = (int)t.yltask.size(), group0 = (int)t.ylgroup.size();
        t.yl_task_off[gi] = task0;
        t.yl_group_off[gi] = group0;
        for (int g = 0; g < G; ++g) {
            const std::vector<int> &us = gu[g];
            const int nu = (int)us.size();
            // wavefronts per unit, in proportion to its cost (at least one)
            std::vector<int> k(nu, 1);
            for (int extra = kYLdsWaves - nu; extra > 0 && nu > 0; --extra) {
                int best = 0;
                double bv = -1.0;
                for (int i = 0; i < nu; ++i) {
                    const double v = (double)t.yl_cost[us[i]] / k[i];
                    if (v > bv) {
                        bv = v;
                        best = i;
                    }
                }
                ++k[best];
            }
            // split each unit's contributions over its wavefronts (LPT)
            struct TaskB { int unit; std::vector<int> cs; long load; };
            std::vector<TaskB> tasks;
            std::vector<int> tslot;  // unit slot of each task
            for (int i = 0; i < nu; ++i) {
                const int u = us[i];
                std::vector<TaskB> tt(k[i]);
                for (auto &x : tt) {
                    x.unit = u;
                    x.load = 0;
                }
                for (int c = 0; c < (int)ucs[u].size(); ++c) {
                    auto it = std::min_element(tt.begin(), tt.end(), [](const TaskB &x, const TaskB &y) {
                        return x.load < y.load;
                    });
                    it->cs.push_back(c);
                    it->load += ucost[u][c];
                }
                for (auto &x : tt) {
                    tasks.push_back(x);
                    tslot.push_back(i);
                }
            }
            while ((int)tasks.size() < kYLdsWaves) {
                tasks.push_back(TaskB{-1, {}, 0});
                tslot.push_back(-1);
            }
            // wavefront w runs on SIMD w % 4: balance the SIMDs' sums (LPT)
            std::vector<int> tord(kYLdsWaves);
            std::iota(tord.begin(), tord.end(), 0);
            std::stable_sort(tord.begin(), tord.end(),
                             [&](int x, int y) { return tasks[x].load > tasks[y].load; });
            long simd[4] = {0, 0, 0, 0};
            int fill[4] = {0, 0, 0, 0};
            std::vector<int> wave_of(kYLdsWaves, -1);
            for (int x : tord) {
                int sbest = -1;
                for (int q = 0; q < 4; ++q)
                    if (fill[q] < kYLdsWaves / 4 && (sbest < 0 || simd[q] < simd[sbest])) sbest = q;
                wave_of[x] = 4 * fill[sbest] + sbest;
                ++fill[sbest];
                simd[sbest] += tasks[x].load;
            }
            std::vector<YLTask> wt(kYLdsWaves);
            for (int x = 0; x < kYLdsWaves; ++x) {
                YLTask yt{};
                yt.unit = tasks[x].unit;
                const int u = tasks[x].unit;
                yt.cb = yt.ce = 0;
                if (u >= 0) {
                    // this task's contributions, stored contiguously
                    yt.cb = (int)t.ylcontrib.size();
                    for (int c : tasks[x].cs) t.ylcontrib.push_back(ucs[u][c]);
                    yt.ce = (int)t.ylcontrib.size();
                }
                wt[wave_of[x]] = yt;
            }
            t.yltask.insert(t.yltask.end(), wt.begin(), wt.end());
            YLGroup gr{};
            gr.nunits = nu;
            int nt = 0;
            for (int i = 0; i < nu; ++i) {
                gr.unit[i] = us[i];
                gr.tb[i] = nt;
                for (int x = 0; x < kYLdsWaves; ++x)
                    if (tslot[x] == i) gr.tw[nt++] = wave_of[x];
            }
            gr.tb[nu] = nt;
            t.ylgroup.push_back(gr);
        }
    }
}

// ---------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------
void build_tables(int tj, Tables &t)
{
    t = Tables();
    t.twojmax = tj;
    auto nrm = [](int J, int p, int q) {
        // N = sqrt(p!(J-p)!/(q!(J-q)!)): u^J = N * (polynomial coefficient)
        return std::sqrt(std::exp(std::lgamma(p + 1.0) + std::lgamma(J - p + 1.0) -
                                  std::lgamma(q + 1.0) - std::lgamma(J - q + 1.0)));
    };

    // half-matrix storage: for each J, columns q = 0..J/2, rows p = 0..J;
    // full storage: for each J, rows p, columns q = 0..J
    t.hbase.assign(tj + 2, 0);
    t.fbase.assign(tj + 2, 0);
    for (int J = 0; J <= tj; ++J) {
        t.hbase[J + 1] = t.hbase[J] + (J + 1) * (J / 2 + 1);
        t.fbase[J + 1] = t.fbase[J] + (J + 1) * (J + 1);
    }
    t.nhalf = t.hbase[tj + 1];
    t.nfullel = t.fbase[tj + 1];
    t.helem.resize(t.nhalf);
    t.norm.assign(t.nhalf, 0.0);
    t.whalf.assign(t.nhalf, 0.0);
    t.unscale_y.assign(t.nhalf, 0.0);
    t.half2full.assign(t.nhalf, 0);
    t.uinfo.resize(t.nhalf);
    for (int J = 0; J <= tj; ++J)
        for (int q = 0; q <= J / 2; ++q)
            for (int p = 0; p <= J; ++p) {
                const int e = t.half_index(J, p, q);
                t.helem[e] = {J, p, q};
                t.norm[e] = nrm(J, p, q);
                t.whalf[e] = (2 * q < J) ? 2.0 : 1.0;
                t.unscale_y[e] = 1.0 / (t.whalf[e] * t.norm[e]);
                t.half2full[e] = t.full_index(J, p, q);
                UInfo ui;
                ui.fi = t.full_index(J, p, q);
                ui.fm = (J - p == p && J - q == q) ? -1 : t.full_index(J, J - p, J - q);
                ui.nrm = t.norm[e];
                ui.msign = ((p - q) % 2 == 0) ? 1.0 : -1.0;
                t.uinfo[e] = ui;
            }
    for (int J = 0; J <= tj; ++J)
        for (int p = 0; p <= J; ++p)
            for (int q = 0; q <= J; ++q) t.nfull.push_back(nrm(J, p, q));

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

    // Clebsch-Gordan values keyed by (J1, J2, J, M1, M2)
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

    // The adjoint of eq. (y).  For a canonical l = (J1, J2, J) the derivative
    // of B_l = Z^J_{J1J2} : conj(U^J) with respect to each of its three
    // matrix factors is Re[X : conj(dU)] with X = Z^J_{J1J2} for U^J,
    // (J+1)/(J1+1) Z^{J1}_{J J2} for U^J1 and (J+1)/(J2+1) Z^{J2}_{J J1} for
    // U^J2 (Clebsch-Gordan symmetry).  So a product Z^c_{ab} (a >= b) enters
    // Y^c with beta_l times (number of factors of rank c in l) times
    // (J_max+1)/(c+1), where l is the sorted triple {a, b, c}.
    {
        struct PendingC { YRowC row; std::vector<YContrib> cs; };
        std::vector<PendingC> rows;
        std::vector<int> cq_at((tj + 1) * (tj + 1) * (tj + 1), -1);
        auto cqix = [&](int a, int b, int c) -> int & { return cq_at[(a * (tj + 1) + b) * (tj + 1) + c]; };
        for (int J = 0; J <= tj; ++J)
            for (int p = 0; p <= J; p += y_unit_rows(tj)) {
                const int two = y_unit_rows(tj) == 2 && p + 1 <= J;
                PendingC pr;
                pr.row.J = J;
                pr.row.p = p;
                pr.row.nq = J / 2 + 1;
                pr.row.ebase = t.half_index(J, p, 0);
                pr.row.frow = t.full_index(J, p, 0);
                pr.row.two = two;
                for (int r = 0; r < 2; ++r)
                    for (int q = 0; q < 8; ++q) {
                        if (q < pr.row.nq && r <= two) {
                            const int e = t.half_index(J, p + r, q);
                            pr.row.oscale[r][q] = t.whalf[e] * t.norm[e];
                            pr.row.einv[r][q] = 1.0 / t.norm[e];
                        } else {
                            pr.row.oscale[r][q] = pr.row.einv[r][q] = 0.0;
                        }
                    }
                for (int a = 0; a <= tj; ++a)
                    for (int b = 0; b <= a; ++b) {
                        if (J < a - b || J > a + b || (a + b + J) % 2) continue;
                        int s3[3] = {a, b, J};
                        std::sort(s3, s3 + 3);
                        YContrib c{};
                        c.j1 = a;
                        c.j2 = b;
                        c.d = (a + b - J) / 2;
                        c.l = cix(s3[1], s3[0], s3[2]);
                        c.factor = (double)((a == J) + (b == J) + 1) * (double)(s3[2] + 1) / (double)(J + 1);
                        // valid rows of row p + r: p2 = p + r - p1 + d in [0, b]
                        c.p1lo = std::max(0, p + c.d - b);
                        c.p1hi = std::min(a, p + two + c.d);
                        if (c.p1lo > c.p1hi) continue;
                        c.cp_off = (int)t.ycp.size();
                        for (int p1 = c.p1lo; p1 <= c.p1hi; ++p1)
                            for (int r = 0; r < 2; ++r) {
                                const int p2 = p + r - p1 + c.d;
                                const bool ok = r <= two && p2 >= 0 && p2 <= b;
                                t.ycp.push_back(ok ? cg(a, 2 * p1 - a, b, 2 * (p + r) - J - (2 * p1 - a), J) : 0.0);
                            }
                        if (cqix(a, b, J) < 0) {
                            cqix(a, b, J) = (int)t.ycq.size();
                            for (int q = 0; q <= J / 2; ++q)
                                for (int q1 = 0; q1 <= tj; ++q1) {
                                    const int N1 = 2 * q1 - a, N2 = (2 * q - J) - N1;
                                    t.ycq.push_back(q1 <= a && std::abs(N2) <= b ? cg(a, N1, b, N2, J) : 0.0);
                                }
                        }
                        c.cq_off = cqix(a, b, J);
                        int terms = 0;
                        for (int q = 0; q <= J / 2; ++q)
                            for (int q1 = 0; q1 <= a; ++q1) {
                                const int q2 = q - q1 + c.d;
                                if (q2 >= 0 && q2 <= b) ++terms;
                            }
                        // the algorithmic work counts each row's own p1 range
                        for (int r = 0; r <= two; ++r) {
                            const int lo = std::max(0, p + r + c.d - b), hi = std::min(a, p + r + c.d);
                            if (lo > hi) continue;
                            t.yterms += (long)(hi - lo + 1) * terms;
                            t.ypartials += (long)(hi - lo + 1) * (J / 2 + 1);
                        }
                        const int rowsn = c.p1hi - c.p1lo + 1;
                        c.cost = rowsn * ((1 + two) * (6 * terms + 4 * (J / 2 + 1)) + 2 * (a + b + 2)) + 16;
                        pr.cs.push_back(c);
                    }
                // longest-processing-time assignment to the waves
                std::stable_sort(pr.cs.begin(), pr.cs.end(),
                                 [](const YContrib &x, const YContrib &y) { return x.cost > y.cost; });
                std::vector<int> load(kYWaves, 0);
                std::vector<std::vector<YContrib>> wav(kYWaves);
                for (const auto &c : pr.cs) {
                    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                    wav[w].push_back(c);
                    load[w] += c.cost;
                }
                pr.cs.clear();
                for (int w = 0; w < kYWaves; ++w) {
                    pr.row.cb[w] = (int)pr.cs.size();
                    pr.cs.insert(pr.cs.end(), wav[w].begin(), wav[w].end());
                }
                pr.row.cb[kYWaves] = (int)pr.cs.size();
                pr.row.cost = *std::max_element(load.begin(), load.end());
                rows.push_back(std::move(pr));
            }
        std::stable_sort(rows.begin(), rows.end(),
                         [](const PendingC &x, const PendingC &y) { return x.row.cost > y.row.cost; });
        for (auto &pr : rows) {
            const int base = (int)t.ycontrib.size();
            for (int w = 0; w <= kYWaves; ++w) pr.row.cb[w] += base;
            t.ycontrib.insert(t.ycontrib.end(), pr.cs.begin(), pr.cs.end());
            t.yrows.push_back(pr.row);
        }
    }

    if (tj <= kYLdsMaxTJ) build_lds_program(t, cg);

    // bispectrum program (eq. (z)): for each canonical (J1, J2, J) and each
    // stored (p, q) of rank J, the Clebsch-Gordan terms of Z(p, q)
    t.bl_begin.assign(t.nb + 1, 0);
    for (int l = 0; l < t.nb; ++l) {
        const int J1 = t.comps[l][0], J2 = t.comps[l][1], J = t.comps[l][2];
        for (int q = 0; q <= J / 2; ++q)
            for (int p = 0; p <= J; ++p) {
                BItem bi{};
                bi.tb = (int)t.bterms.size();
                const int M = 2 * p - J, Mq = 2 * q - J;
                for (int p1 = 0; p1 <= J1; ++p1) {
                    const int M1 = 2 * p1 - J1, M2 = M - M1;
                    if (std::abs(M2) > J2) continue;
                    const double cp = cg(J1, M1, J2, M2, J);
                    if (std::fabs(cp) < 1e-15) continue;
                    for (int q1 = 0; q1 <= J1; ++q1) {
                        const int N1 = 2 * q1 - J1, N2 = Mq - N1;
                        if (std::abs(N2) > J2) continue;
                        const double cq = cg(J1, N1, J2, N2, J);
                        if (std::fabs(cq) < 1e-15) continue;
                        t.bterms.push_back({cp * cq, t.full_index(J1, p1, q1),
                                            t.full_index(J2, (M2 + J2) / 2, (N2 + J2) / 2)});
                    }
                }
                bi.te = (int)t.bterms.size();
                bi.f3 = t.full_index(J, p, q);
                bi.w = (2 * q < J) ? 2.0 : 1.0;
                t.bitems.push_back(bi);
            }
        t.bl_begin[l + 1] = (int)t.bitems.size();
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
            // cells at least rcut wide, as on a periodic axis, so that the
            // +-1 neighbouring cells hold every partner within rcut
            nc[d] = std::max(1, (int)std::floor(ext[d] / rcut));
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
