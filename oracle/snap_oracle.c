/*
 * snap_oracle.c -- plain FP64 CPU reference for SNAP energies and forces.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (Gayatri et al., "Rapid Exploration of Optimization
 * Strategies on Advanced Architectures using TestSNAP and LAMMPS",
 * arXiv 2011.12875), written as the plain definitions, with no adjoint and no
 * symmetry shortcut:
 *
 *   Sec. II.A, eq. (u):  U_j = sum over neighbours inside Rcut of
 *                        f_c(r_ik) u_j(theta0, theta, phi), plus the
 *                        self-contribution w_self * identity that the paper
 *                        says it omits for brevity.
 *   Sec. II.A, eq. (z):  B_{j1 j2 j} = (U_j1 (x)^j_{j1 j2} U_j2) : U_j^*, the
 *                        Clebsch-Gordan product contracted with conj(U_j).
 *   Sec. II.A, eq. (snapatomenergy):  E_i = sum_l beta_l B_l.
 *   Sec. II.A, eq. (snapforce1) with eq. (dbidrk):  forces from the analytic
 *                        derivative of each B_l, taken by the literal product
 *                        rule on the trilinear form (three partial matrices),
 *                        i.e. the pre-adjoint route of Listing 1.
 *
 * Conventions the paper leaves open (its Sec. II.A defers them to the SNAP
 * reference it cites) and that this oracle fixes:
 *   - angular momenta are twice-integers J = 2j; matrix indices p = j + m,
 *     q = j + m' run over 0..J;
 *   - 3-sphere map: theta0 = rfac0*pi*(r - rmin0)/(rcut - rmin0); the
 *     Cayley-Klein pair is a = cos(theta0) - i sin(theta0) n_z,
 *     b = sin(theta0) (n_y - i n_x), n = r_ik / r;
 *   - u^J is the matrix of the SU(2) element on homogeneous degree-J
 *     polynomials in the basis x^p y^(J-p)/sqrt(p!(J-p)!), with
 *     x -> a x + b y, y -> -b* x + a* y (explicit, non-recursive formula);
 *   - switching: f_c = (cos(pi (r-rmin0)/(rcut-rmin0)) + 1)/2 inside
 *     (rmin0, rcut), 1 below rmin0, or 1 everywhere when switching is off;
 *   - Clebsch-Gordan coefficients in the Condon-Shortley convention, from
 *     Racah's closed formula;
 *   - components: J2 <= J1 <= J <= twojmax, |J1-J2| <= J <= J1+J2 and
 *     J1+J2+J even, ordered J1 ascending, then J2 ascending, then J
 *     ascending;
 *   - the pair derivative dE_p = dE_i/dr_ik for p = (i -> k); the force on
 *     i gains +dE_p and the force on k gains -dE_p;
 *   - several elements (the density weights Sec. II.A leaves out): element
 *     e has a radius R_e and a weight w_e; the pair (i, k) has the cutoff
 *     R_ik = rcutfac (R_t(i) + R_t(k)), used in the 3-sphere map and f_c of
 *     that pair, and enters U_i with the weight of the neighbour's element,
 *     w_t(k) f_c u; pairs with r_ik >= R_ik contribute nothing; E_i uses
 *     the coefficients of the centre's element.
 *
 * Parallelism: OpenMP over central atoms, one private force array per
 * thread, reduced in thread order.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_MAXJ 24

/* ------------------------------------------------------------------------ */
/* factorials and binomials (long double keeps the Racah sum accurate)       */
/* ------------------------------------------------------------------------ */

static long double factl(int n)
{
    long double f = 1.0L;
    for (int k = 2; k <= n; ++k) f *= (long double)k;
    return f;
}

static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double c = 1.0;
    for (int t = 1; t <= k; ++t) c = c * (double)(n - k + t) / (double)t;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Clebsch-Gordan coefficient <j1 m1 j2 m2 | j m>, all arguments doubled.    */
/* Racah's closed formula (Condon-Shortley phase).                           */
/* ------------------------------------------------------------------------ */

double oracle_cg(int J1, int M1, int J2, int M2, int J, int M)
{
    if (M1 + M2 != M) return 0.0;
    if (abs(M1) > J1 || abs(M2) > J2 || abs(M) > J) return 0.0;
    if (((J1 + M1) & 1) || ((J2 + M2) & 1) || ((J + M) & 1)) return 0.0;
    if (J < abs(J1 - J2) || J > J1 + J2 || ((J1 + J2 + J) & 1)) return 0.0;

    const int a = (J1 + J2 - J) / 2; /* j1+j2-j  */
    const int b = (J1 - J2 + J) / 2; /* j1-j2+j  */
    const int c = (-J1 + J2 + J) / 2;/* -j1+j2+j */
    const int s = (J1 + J2 + J) / 2 + 1;
    const int j1pm1 = (J1 + M1) / 2, j1mm1 = (J1 - M1) / 2;
    const int j2pm2 = (J2 + M2) / 2, j2mm2 = (J2 - M2) / 2;
    const int jpm = (J + M) / 2, jmm = (J - M) / 2;

    long double pre = (long double)(J + 1) * factl(a) * factl(b) * factl(c) / factl(s);
    pre *= factl(j1pm1) * factl(j1mm1) * factl(j2pm2) * factl(j2mm2) * factl(jpm) * factl(jmm);

    /* sum over k with every factorial argument non-negative */
    const int d1 = (J - J2 + M1) / 2; /* j - j2 + m1 */
    const int d2 = (J - J1 - M2) / 2; /* j - j1 - m2 */
    int kmin = 0;
    if (-d1 > kmin) kmin = -d1;
    if (-d2 > kmin) kmin = -d2;
    int kmax = a;
    if (j1mm1 < kmax) kmax = j1mm1;
    if (j2pm2 < kmax) kmax = j2pm2;
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        long double den = factl(k) * factl(a - k) * factl(j1mm1 - k) * factl(j2pm2 - k) *
                          factl(d1 + k) * factl(d2 + k);
        sum += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    return (double)(sqrtl(pre) * sum);
}

/* ------------------------------------------------------------------------ */
/* Components (the enumeration of Sec. II.A plus the coupling rules).        */
/* ------------------------------------------------------------------------ */

int oracle_components(int twojmax, int *triples)
{
    int n = 0;
    for (int J1 = 0; J1 <= twojmax; ++J1)
        for (int J2 = 0; J2 <= J1; ++J2)
            for (int J = J1 - J2; J <= J1 + J2 && J <= twojmax; J += 2)
                if (J >= J1) {
                    if (triples) {
                        triples[3 * n + 0] = J1;
                        triples[3 * n + 1] = J2;
                        triples[3 * n + 2] = J;
                    }
                    ++n;
                }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Cayley-Klein parameters of a neighbour vector and their derivatives.      */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rcut, rfac0, rmin0, wself;
    int switch_flag;
} oparams;

typedef struct {
    cplx a, b;
    cplx da[3], db[3]; /* d a / d r_alpha, d b / d r_alpha */
    double fc, dfc[3]; /* switching value and its gradient */
} ogeom;

static void geometry(const double rv[3], const oparams *P, ogeom *g)
{
    const double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    const double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    const double span = P->rcut - P->rmin0;
    const double th0 = P->rfac0 * M_PI * (r - P->rmin0) / span;
    const double dth0 = P->rfac0 * M_PI / span; /* d theta0 / d r */
    const double c0 = cos(th0), s0 = sin(th0);

    g->a = c0 - I * s0 * n[2];
    g->b = s0 * n[1] - I * s0 * n[0];

    for (int al = 0; al < 3; ++al) {
        /* d n_beta / d r_alpha = (delta_ab - n_a n_b) / r */
        const double dnx = ((al == 0) - n[al] * n[0]) / r;
        const double dny = ((al == 1) - n[al] * n[1]) / r;
        const double dnz = ((al == 2) - n[al] * n[2]) / r;
        const double dth = dth0 * n[al];
        g->da[al] = -s0 * dth - I * (c0 * dth * n[2] + s0 * dnz);
        g->db[al] = c0 * dth * (n[1] - I * n[0]) + s0 * (dny - I * dnx);
    }

    double fc = 1.0, dfdr = 0.0;
    if (P->switch_flag && r > P->rmin0) {
        const double x = M_PI * (r - P->rmin0) / span;
        fc = 0.5 * (cos(x) + 1.0);
        dfdr = -0.5 * M_PI / span * sin(x);
    }
    g->fc = fc;
    for (int al = 0; al < 3; ++al) g->dfc[al] = dfdr * n[al];
}

/* ------------------------------------------------------------------------ */
/* Explicit u^J (no recursion) and its derivative through (a, a*, b, b*).    */
/*   u_pq = sqrt(p!(J-p)!/(q!(J-q)!)) sum_s C(q,s) C(J-q,p-s)               */
/*          a^s b^(q-s) (-b*)^(p-s) (a*)^(J-q-p+s)                           */
/* Row-major: u[p*(J+1)+q].                                                  */
/* ------------------------------------------------------------------------ */

static void wigner(int J, cplx a, cplx b, cplx *u, const cplx *da, const cplx *db, cplx *du)
{
    cplx pa[ORACLE_MAXJ + 1], pb[ORACLE_MAXJ + 1], pm[ORACLE_MAXJ + 1], pc[ORACLE_MAXJ + 1];
    const cplx mbc = -conj(b), ac = conj(a);
    pa[0] = pb[0] = pm[0] = pc[0] = 1.0;
    for (int s = 1; s <= J; ++s) {
        pa[s] = pa[s - 1] * a;
        pb[s] = pb[s - 1] * b;
        pm[s] = pm[s - 1] * mbc;
        pc[s] = pc[s - 1] * ac;
    }
    for (int p = 0; p <= J; ++p)
        for (int q = 0; q <= J; ++q) {
            const double norm = sqrt((double)(factl(p) * factl(J - p) / (factl(q) * factl(J - q))));
            cplx val = 0.0, ga = 0.0, gac = 0.0, gb = 0.0, gbc = 0.0;
            int smin = p + q - J;
            if (smin < 0) smin = 0;
            const int smax = (q < p) ? q : p;
            for (int s = smin; s <= smax; ++s) {
                const int eb = q - s, em = p - s, ec = J - q - p + s;
                const double w = binom(q, s) * binom(J - q, p - s);
                val += w * pa[s] * pb[eb] * pm[em] * pc[ec];
                if (du) {
                    if (s > 0) ga += w * (double)s * pa[s - 1] * pb[eb] * pm[em] * pc[ec];
                    if (eb > 0) gb += w * (double)eb * pa[s] * pb[eb - 1] * pm[em] * pc[ec];
                    /* d/d(b*) of (-b*)^em = -em (-b*)^(em-1) */
                    if (em > 0) gbc -= w * (double)em * pa[s] * pb[eb] * pm[em - 1] * pc[ec];
                    if (ec > 0) gac += w * (double)ec * pa[s] * pb[eb] * pm[em] * pc[ec - 1];
                }
            }
            u[p * (J + 1) + q] = norm * val;
            if (du)
                for (int al = 0; al < 3; ++al)
                    du[al * (J + 1) * (J + 1) + p * (J + 1) + q] =
                        norm * (ga * da[al] + gac * conj(da[al]) + gb * db[al] + gbc * conj(db[al]));
        }
}

/* exported for the pins: u^J of a given (a, b), row-major, interleaved re/im */
void oracle_wigner(int J, double ar, double ai, double br, double bi, double *out)
{
    cplx u[(ORACLE_MAXJ + 1) * (ORACLE_MAXJ + 1)];
    wigner(J, ar + I * ai, br + I * bi, u, NULL, NULL, NULL);
    for (int k = 0; k < (J + 1) * (J + 1); ++k) {
        out[2 * k] = creal(u[k]);
        out[2 * k + 1] = cimag(u[k]);
    }
}

/* exported for the pins: Cayley-Klein a, b, their gradients and f_c */
void oracle_geometry(const double rv[3], double rcut, double rfac0, double rmin0, int switch_flag,
                     double *out /* 2+2 + 3*4 + 1 + 3 = 20 doubles */)
{
    oparams P = {rcut, rfac0, rmin0, 1.0, switch_flag};
    ogeom g;
    geometry(rv, &P, &g);
    out[0] = creal(g.a); out[1] = cimag(g.a);
    out[2] = creal(g.b); out[3] = cimag(g.b);
    for (int al = 0; al < 3; ++al) {
        out[4 + 4 * al + 0] = creal(g.da[al]);
        out[4 + 4 * al + 1] = cimag(g.da[al]);
        out[4 + 4 * al + 2] = creal(g.db[al]);
        out[4 + 4 * al + 3] = cimag(g.db[al]);
    }
    out[16] = g.fc;
    out[17] = g.dfc[0]; out[18] = g.dfc[1]; out[19] = g.dfc[2];
}

/* ------------------------------------------------------------------------ */
/* Brute-force minimum-image neighbour search (full list, r < rcut).         */
/* box[d] <= 0 means dimension d is not periodic.                            */
/* Returns the number of pairs, or -1 if cap is too small.                   */
/* ------------------------------------------------------------------------ */

static void min_image(const double *xi, const double *xk, const double box[3], double rv[3])
{
    for (int d = 0; d < 3; ++d) {
        double x = xk[d] - xi[d];
        if (box[d] > 0.0) x -= box[d] * nearbyint(x / box[d]);
        rv[d] = x;
    }
}

int oracle_neighbors(int n, const double *pos, const double box[3], double rcut, int *off, int *nbr,
                     int cap)
{
    int np = 0;
    const double rc2 = rcut * rcut;
    for (int i = 0; i < n; ++i) {
        off[i] = np;
        for (int k = 0; k < n; ++k) {
            if (k == i) continue;
            double rv[3];
            min_image(pos + 3 * i, pos + 3 * k, box, rv);
            const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
            if (r2 < rc2) {
                if (np >= cap) return -1;
                nbr[np++] = k;
            }
        }
    }
    off[n] = np;
    return np;
}

/* ------------------------------------------------------------------------ */
/* The full evaluation.                                                      */
/* ------------------------------------------------------------------------ */

/* offset of block J inside a flat list of full (J+1)x(J+1) matrices */
static int ublock(int J)
{
    int o = 0;
    for (int k = 0; k < J; ++k) o += (k + 1) * (k + 1);
    return o;
}

/*
 * oracle_snap: energies, forces, bispectra, Utot and per-pair derivatives.
 *
 *  pos[n][3], box[3]; neighbours are found here by brute force (off/nbr are
 *  outputs, sized n+1 and pair_cap).
 *  beta: [N_B] (per_atom_beta == 0) or [n][N_B].
 *  centers: list of ncenter central atoms to evaluate (NULL -> all atoms).
 *  Outputs (any may be NULL except off/nbr):
 *    E[n]            energy of each evaluated centre
 *    F[n][3]         forces accumulated from the evaluated centres only
 *    B[n][N_B]       bispectrum of each evaluated centre
 *    Utot[n][sum (J+1)^2][2]  full matrices, row-major per block, re/im
 *    dE[pair_cap][3] dE_i/dr_ik for the pairs of evaluated centres
 *  Returns the number of pairs, -1 on bad arguments, -2 if pair_cap is too
 *  small, -3 on coincident atoms.
 */
/* element description (NULL: one element, the cutoff rcut, unit weights) */
typedef struct {
    int nelem;
    const int *type;       /* [n], 0 .. nelem-1 */
    const double *radius;  /* [nelem] */
    const double *weight;  /* [nelem] */
    double rcutfac;
} oelem;

/* cutoff and density weight of the pair (i, k) */
static void pair_cut(const oelem *el, double rcut, int i, int k, double *rc, double *w)
{
    if (!el) {
        *rc = rcut;
        *w = 1.0;
        return;
    }
    *rc = el->rcutfac * (el->radius[el->type[i]] + el->radius[el->type[k]]);
    *w = el->weight[el->type[k]];
}

/* given_list: off/nbr already hold a full neighbour list of off[n] pairs
 * (the brute-force one of oracle_neighbors, built beforehand); otherwise it
 * is built here. */
static int snap_eval(int n, const double *pos, const double box[3], int twojmax, double rcut,
                     double rfac0, double rmin0, int switch_flag, double wself, const oelem *el,
                     const double *beta, int per_atom_beta, int ncenter, const int *centers,
                     int nthreads, int given_list, int *off, int *nbr, int pair_cap, double *E,
                     double *F, double *B, double *Utot, double *dE)
{
    if (n < 0 || twojmax < 0 || twojmax > ORACLE_MAXJ || rcut <= 0.0) return -1;
    const int np = given_list ? off[n] : oracle_neighbors(n, pos, box, rcut, off, nbr, pair_cap);
    if (np < 0) return -2;

    oparams P = {rcut, rfac0, rmin0, wself, switch_flag};
    const int nb = oracle_components(twojmax, NULL);
    int *tri = (int *)malloc(sizeof(int) * 3 * (nb > 0 ? nb : 1));
    oracle_components(twojmax, tri);
    const int ufull = ublock(twojmax + 1);

    /* Clebsch-Gordan table cg[J1][J2][J][p1][p2], p = (J + M)/2 */
    const int D = twojmax + 1;
    double *cgt = (double *)calloc((size_t)D * D * D * D * D, sizeof(double));
#define CGT(J1, J2, J, p1, p2) cgt[((((size_t)(J1) * D + (J2)) * D + (J)) * D + (p1)) * D + (p2)]
    for (int J1 = 0; J1 <= twojmax; ++J1)
        for (int J2 = 0; J2 <= twojmax; ++J2)
            for (int J = 0; J <= twojmax; ++J)
                for (int p1 = 0; p1 <= J1; ++p1)
                    for (int p2 = 0; p2 <= J2; ++p2) {
                        const int M1 = 2 * p1 - J1, M2 = 2 * p2 - J2, M = M1 + M2;
                        CGT(J1, J2, J, p1, p2) = oracle_cg(J1, M1, J2, M2, J, M);
                    }

    const int ncent = centers ? ncenter : n;
    /* thread count of this call only (a num_threads clause, no change to
     * the process-wide default) */
    int nthr = 1;
#ifdef _OPENMP
    nthr = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)nthreads;
    double *Fthr = NULL;
    if (F) {
        Fthr = (double *)calloc((size_t)nthr * n * 3, sizeof(double));
        memset(F, 0, sizeof(double) * 3 * (size_t)n);
    }
    int status = np;

#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *U = (cplx *)malloc(sizeof(cplx) * ufull);
        cplx *Z = (cplx *)malloc(sizeof(cplx) * D * D);
        cplx *G1 = (cplx *)malloc(sizeof(cplx) * (size_t)nb * D * D);
        cplx *G2 = (cplx *)malloc(sizeof(cplx) * (size_t)nb * D * D);
        cplx *G3 = (cplx *)malloc(sizeof(cplx) * (size_t)nb * D * D);
        cplx *u = (cplx *)malloc(sizeof(cplx) * ufull);
        cplx *du = (cplx *)malloc(sizeof(cplx) * 3 * ufull);
        double *Bi = (double *)malloc(sizeof(double) * (nb > 0 ? nb : 1));
        double *Ft = Fthr ? Fthr + (size_t)tid * n * 3 : NULL;

#pragma omp for schedule(static)
        for (int ci = 0; ci < ncent; ++ci) {
            const int i = centers ? centers[ci] : ci;
            if (i < 0 || i >= n) continue;
            const double *bet = el ? beta + (size_t)el->type[i] * nb
                                   : per_atom_beta ? beta + (size_t)i * nb : beta;

            /* eq. (u): Utot_i = w_self I + sum_k f_c u(r_ik) */
            for (int J = 0; J <= twojmax; ++J) {
                cplx *UJ = U + ublock(J);
                for (int p = 0; p <= J; ++p)
                    for (int q = 0; q <= J; ++q) UJ[p * (J + 1) + q] = (p == q) ? wself : 0.0;
            }
            int bad = 0;
            for (int t = off[i]; t < off[i + 1]; ++t) {
                double rv[3];
                min_image(pos + 3 * i, pos + 3 * nbr[t], box, rv);
                const double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                if (r < 1e-10) { bad = 1; continue; }
                double rc, w;
                pair_cut(el, rcut, i, nbr[t], &rc, &w);
                if (r >= rc) continue;
                oparams Pp = P;
                Pp.rcut = rc;
                ogeom g;
                geometry(rv, &Pp, &g);
                for (int J = 0; J <= twojmax; ++J) {
                    wigner(J, g.a, g.b, u + ublock(J), NULL, NULL, NULL);
                    cplx *UJ = U + ublock(J);
                    for (int e = 0; e < (J + 1) * (J + 1); ++e) UJ[e] += w * g.fc * u[ublock(J) + e];
                }
            }
            if (bad) {
#pragma omp atomic write
                status = -3;
            }
            if (Utot)
                for (int e = 0; e < ufull; ++e) {
                    Utot[((size_t)i * ufull + e) * 2 + 0] = creal(U[e]);
                    Utot[((size_t)i * ufull + e) * 2 + 1] = cimag(U[e]);
                }

            /* eq. (z) for every component, together with the two other
             * partial matrices of the trilinear form
             *   B_l = sum CG CG U^J1(m1,m1') U^J2(m2,m2') conj(U^J(m,m')).    */
            double Ei = 0.0;
            for (int l = 0; l < nb; ++l) {
                const int J1 = tri[3 * l], J2 = tri[3 * l + 1], J = tri[3 * l + 2];
                const cplx *U1 = U + ublock(J1), *U2 = U + ublock(J2), *U3 = U + ublock(J);
                cplx *g1 = G1 + (size_t)l * D * D, *g2 = G2 + (size_t)l * D * D,
                     *g3 = G3 + (size_t)l * D * D;
                for (int e = 0; e < D * D; ++e) g1[e] = g2[e] = g3[e] = 0.0;
                for (int p1 = 0; p1 <= J1; ++p1)
                    for (int p2 = 0; p2 <= J2; ++p2) {
                        const int M = (2 * p1 - J1) + (2 * p2 - J2);
                        if (abs(M) > J) continue;
                        const int p = (J + M) / 2;
                        const double c = CGT(J1, J2, J, p1, p2);
                        if (c == 0.0) continue;
                        for (int q1 = 0; q1 <= J1; ++q1)
                            for (int q2 = 0; q2 <= J2; ++q2) {
                                const int Mp = (2 * q1 - J1) + (2 * q2 - J2);
                                if (abs(Mp) > J) continue;
                                const int q = (J + Mp) / 2;
                                const double cc = c * CGT(J1, J2, J, q1, q2);
                                if (cc == 0.0) continue;
                                const cplx a1 = U1[p1 * (J1 + 1) + q1];
                                const cplx a2 = U2[p2 * (J2 + 1) + q2];
                                const cplx a3c = conj(U3[p * (J + 1) + q]);
                                g3[p * (J + 1) + q] += cc * a1 * a2;   /* Z^J_{J1J2} */
                                g1[p1 * (J1 + 1) + q1] += cc * a2 * a3c;
                                g2[p2 * (J2 + 1) + q2] += cc * a1 * a3c;
                            }
                    }
                cplx bl = 0.0;
                for (int p = 0; p <= J; ++p)
                    for (int q = 0; q <= J; ++q) bl += g3[p * (J + 1) + q] * conj(U3[p * (J + 1) + q]);
                Bi[l] = creal(bl);
                Ei += bet[l] * Bi[l];
            }
            if (E) E[i] = Ei;
            if (B)
                for (int l = 0; l < nb; ++l) B[(size_t)i * nb + l] = Bi[l];

            /* eq. (snapforce1) with eq. (dbidrk): per neighbour and
             * direction, dB_l/dr = Re[G3 : conj(dU^J) + G1 : dU^J1 + G2 : dU^J2] */
            if (F || dE) {
                for (int t = off[i]; t < off[i + 1]; ++t) {
                    const int k = nbr[t];
                    double rv[3];
                    min_image(pos + 3 * i, pos + 3 * k, box, rv);
                    const double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                    double de[3] = {0.0, 0.0, 0.0};
                    double rc, w;
                    pair_cut(el, rcut, i, k, &rc, &w);
                    if (r >= 1e-10 && r < rc) {
                        oparams Pp = P;
                        Pp.rcut = rc;
                        ogeom g;
                        geometry(rv, &Pp, &g);
                        for (int J = 0; J <= twojmax; ++J) {
                            const int o = ublock(J), sz = (J + 1) * (J + 1);
                            cplx dtmp[3 * (ORACLE_MAXJ + 1) * (ORACLE_MAXJ + 1)];
                            wigner(J, g.a, g.b, u + o, g.da, g.db, dtmp);
                            /* d(f_c u)/dr_alpha = grad f_c u + f_c du/dr_alpha */
                            for (int al = 0; al < 3; ++al)
                                for (int e = 0; e < sz; ++e)
                                    du[al * ufull + o + e] =
                                        w * (g.dfc[al] * u[o + e] + g.fc * dtmp[al * sz + e]);
                        }
                        for (int l = 0; l < nb; ++l) {
                            const int J1 = tri[3 * l], J2 = tri[3 * l + 1], J = tri[3 * l + 2];
                            const cplx *g1 = G1 + (size_t)l * D * D, *g2 = G2 + (size_t)l * D * D,
                                       *g3 = G3 + (size_t)l * D * D;
                            for (int al = 0; al < 3; ++al) {
                                const cplx *d1 = du + al * ufull + ublock(J1);
                                const cplx *d2 = du + al * ufull + ublock(J2);
                                const cplx *d3 = du + al * ufull + ublock(J);
                                cplx s = 0.0;
                                for (int e = 0; e < (J + 1) * (J + 1); ++e) s += g3[e] * conj(d3[e]);
                                for (int e = 0; e < (J1 + 1) * (J1 + 1); ++e) s += g1[e] * d1[e];
                                for (int e = 0; e < (J2 + 1) * (J2 + 1); ++e) s += g2[e] * d2[e];
                                de[al] += bet[l] * creal(s);
                            }
                        }
                    }
                    if (dE)
                        for (int al = 0; al < 3; ++al) dE[3 * (size_t)t + al] = de[al];
                    if (Ft)
                        for (int al = 0; al < 3; ++al) {
                            Ft[3 * (size_t)i + al] += de[al];
                            Ft[3 * (size_t)k + al] -= de[al];
                        }
                }
            }
        }
        free(U); free(Z); free(G1); free(G2); free(G3); free(u); free(du); free(Bi);
    }

    if (F)
        for (int t = 0; t < nthr; ++t)
            for (size_t e = 0; e < (size_t)n * 3; ++e) F[e] += Fthr[(size_t)t * n * 3 + e];
    free(Fthr);
    free(cgt);
    free(tri);
#undef CGT
    return status;
}

int oracle_snap(int n, const double *pos, const double box[3], int twojmax, double rcut,
                double rfac0, double rmin0, int switch_flag, double wself, const double *beta,
                int per_atom_beta, int ncenter, const int *centers, int nthreads, int *off,
                int *nbr, int pair_cap, double *E, double *F, double *B, double *Utot, double *dE)
{
    return snap_eval(n, pos, box, twojmax, rcut, rfac0, rmin0, switch_flag, wself, NULL, beta,
                     per_atom_beta, ncenter, centers, nthreads, 0, off, nbr, pair_cap, E, F, B,
                     Utot, dE);
}

/*
 * oracle_snap_list: oracle_snap on a neighbour list built beforehand by
 * oracle_neighbors with the same rcut (off[n+1], nbr[off[n]], inputs here),
 * so that the evaluation can be timed apart from the brute-force search.
 */
int oracle_snap_list(int n, const double *pos, const double box[3], int twojmax, double rcut,
                     double rfac0, double rmin0, int switch_flag, double wself, const double *beta,
                     int per_atom_beta, int ncenter, const int *centers, int nthreads,
                     const int *off, const int *nbr, double *E, double *F, double *B, double *dE)
{
    return snap_eval(n, pos, box, twojmax, rcut, rfac0, rmin0, switch_flag, wself, NULL, beta,
                     per_atom_beta, ncenter, centers, nthreads, 1, (int *)off, (int *)nbr,
                     off[n], E, F, B, NULL, dE);
}

/*
 * oracle_snap_elements: as oracle_snap for several elements (see the header
 * of this file): type[n] in 0..nelem-1, radius[nelem], weight[nelem],
 * rcutfac; beta[nelem][N_B], the coefficients of each centre element.
 * Neighbours are searched to rcutfac * 2 max(radius); pairs beyond their own
 * cutoff stay in the list with zero contribution.  Returns as oracle_snap,
 * -1 also for a type out of range.
 */
int oracle_snap_elements(int n, const double *pos, const double box[3], int twojmax, double rfac0,
                         double rmin0, int switch_flag, double wself, int nelem, const int *type,
                         const double *radius, const double *weight, double rcutfac,
                         const double *beta, int nthreads, int *off, int *nbr, int pair_cap,
                         double *E, double *F, double *B, double *Utot, double *dE)
{
    if (nelem < 1 || !type || !radius || !weight || !(rcutfac > 0.0)) return -1;
    double rmax = 0.0;
    for (int e = 0; e < nelem; ++e) {
        if (!(radius[e] > 0.0)) return -1;
        if (radius[e] > rmax) rmax = radius[e];
    }
    for (int i = 0; i < n; ++i)
        if (type[i] < 0 || type[i] >= nelem) return -1;
    const oelem el = {nelem, type, radius, weight, rcutfac};
    return snap_eval(n, pos, box, twojmax, 2.0 * rcutfac * rmax, rfac0, rmin0, switch_flag, wself,
                     &el, beta, 0, 0, NULL, nthreads, 0, off, nbr, pair_cap, E, F, B, Utot, dE);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
