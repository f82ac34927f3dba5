// snap_abi.cpp -- the C ABI of snapmi.h: contexts, device tables, workspace,
// argument checks and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/snapmi.h"
#include "snap_kernels.hpp"
#include "snap_tables.hpp"

using namespace snapmi;

// elements a context may describe (snap_set_elements)
constexpr int kMaxElements = 64;

struct snap_ctx {
    snap_params prm;
    // several elements: radius, density weight per element, pair cutoff
    // factor; device copies uploaded on the next call after a change
    int nelem = 0;
    std::vector<double> erad, ewt;
    double rcutfac = 0.0;
    bool elem_dirty = false;
    double *d_erad = nullptr, *d_ewt = nullptr;
    Tables tab;
    DevTables dev;
    bool dev_ready = false;
    int device = -1;
    Work work;
    int cap_atoms = 0;   // npad the per-atom workspace holds
    int cap_pairs = 0;   // pairs the dE / pair_atom workspace holds
    // The U_j and pair->atom map of the last forward-type call (snap_compute,
    // snap_forward, snap_jacobian) serve snap_backward and
    // snap_copy_workspace: their sizes, and the workspace generation they
    // were written in (every reallocation of U or pair_atom starts a new
    // generation, whose contents no call has written yet).
    int last_n = 0;
    int last_npairs = 0;
    unsigned long long gen = 0, last_gen = ~0ull;
    // per-block partial sums of snap_virial and snap_beta_grad (their own
    // buffer: growing it never touches U)
    double *part = nullptr;
    size_t cap_part = 0;
    // quadratic SNAP: bispectra and per-atom coefficients, [cap_quad][N_B] each
    double *qB = nullptr, *qG = nullptr;
    int cap_quad = 0;
    // stage timing (snap_profile): event pairs recorded per stage
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
};

static hipEvent_t take_event(snap_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records the start of a stage on the stream when profiling; finish() the end.
struct StageTimer {
    snap_ctx *c;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageTimer(snap_ctx *c_, int stage_, hipStream_t s_) : c(c_), stage(stage_), s(s_)
    {
        if (c->profiling && (a = take_event(c))) (void)hipEventRecord(a, s);
    }
    void finish()
    {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->ev_used.push_back({stage, {a, b}});
        a = nullptr;
    }
};

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? SNAP_ENOMEM : SNAP_EDEV, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

template <class T>
static hipError_t upload(T *&dst, const std::vector<T> &src)
{
    const size_t bytes = sizeof(T) * (src.empty() ? 1 : src.size());
    hipError_t e = hipMalloc((void **)&dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return e;
}

static void free_dev(snap_ctx *c)
{
    DevTables &d = c->dev;
    (void)hipFree(d.unscale_y);
    (void)hipFree(d.half2full);
    (void)hipFree(d.uinfo);
    (void)hipFree(d.bterms);
    (void)hipFree(d.bitems);
    (void)hipFree(d.bl_begin);
    (void)hipFree(d.ycontrib);
    (void)hipFree(d.yrows);
    (void)hipFree(d.ycp);
    (void)hipFree(d.ycq);
    (void)hipFree(d.nfull);
    (void)hipFree(d.onehot);
    (void)hipFree(d.ylcontrib);
    (void)hipFree(d.ylcp);
    (void)hipFree(d.yltask);
    (void)hipFree(d.ylgroup);
    d = DevTables();
    Work &w = c->work;
    (void)hipFree(w.U);
    (void)hipFree(w.Y);
    (void)hipFree(w.Epart);
    (void)hipFree(w.dE);
    (void)hipFree(w.pair_atom);
    (void)hipFree(w.flag);
    w = Work();
    (void)hipFree(c->d_erad);
    (void)hipFree(c->d_ewt);
    c->d_erad = c->d_ewt = nullptr;
    (void)hipFree(c->part);
    c->part = nullptr;
    c->cap_part = 0;
    (void)hipFree(c->qB);
    (void)hipFree(c->qG);
    c->qB = c->qG = nullptr;
    c->cap_quad = 0;
    c->elem_dirty = c->nelem > 0;
    c->dev_ready = false;
    c->cap_atoms = c->cap_pairs = 0;
}

static int ensure_device(snap_ctx *c)
{
    if (c->dev_ready) return SNAP_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SNAP_EDEV, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    const Tables &t = c->tab;
    DevTables &d = c->dev;
    HIP_TRY(upload(d.unscale_y, t.unscale_y), "upload unscale_y");
    HIP_TRY(upload(d.half2full, t.half2full), "upload half2full");
    HIP_TRY(upload(d.uinfo, t.uinfo), "upload uinfo");
    HIP_TRY(upload(d.bterms, t.bterms), "upload bterms");
    HIP_TRY(upload(d.bitems, t.bitems), "upload bitems");
    HIP_TRY(upload(d.bl_begin, t.bl_begin), "upload bl_begin");
    HIP_TRY(upload(d.ycontrib, t.ycontrib), "upload ycontrib");
    HIP_TRY(upload(d.yrows, t.yrows), "upload yrows");
    HIP_TRY(upload(d.ycp, t.ycp), "upload ycp");
    HIP_TRY(upload(d.ycq, t.ycq), "upload ycq");
    HIP_TRY(upload(d.nfull, t.nfull), "upload nfull");
    {
        std::vector<double> eye((size_t)t.nb * t.nb, 0.0);
        for (int l = 0; l < t.nb; ++l) eye[(size_t)l * t.nb + l] = 1.0;
        HIP_TRY(upload(d.onehot, eye), "upload unit coefficient vectors");
    }
    d.nyrows = (int)t.yrows.size();
    d.nhalf = t.nhalf;
    d.ncu = prop.multiProcessorCount;
    if (!t.ylcontrib.empty() && c->prm.y_kernel != 1) {
        HIP_TRY(upload(d.ylcontrib, t.ylcontrib), "upload ylcontrib");
        HIP_TRY(upload(d.ylcp, t.ylcp), "upload ylcp");
        HIP_TRY(upload(d.yltask, t.yltask), "upload yltask");
        HIP_TRY(upload(d.ylgroup, t.ylgroup), "upload ylgroup");
        for (int gi = 0; gi < kYLdsGroupings; ++gi) {
            d.yl_task_off[gi] = t.yl_task_off[gi];
            d.yl_group_off[gi] = t.yl_group_off[gi];
        }
        d.yl_cost_total = 0;
        for (long x : t.yl_cost) d.yl_cost_total += x;
        d.y_lds = true;
        d.y_lds_selected = c->prm.y_kernel == 2;
    }
    HIP_TRY(hipMalloc((void **)&c->work.flag, sizeof(int)), "alloc flag");
    HIP_TRY(hipMemset(c->work.flag, 0, sizeof(int)), "clear flag");
    c->device = dev;
    c->dev_ready = true;
    return SNAP_OK;
}

// Grow the workspace to n atoms and np pairs.  Growing waits for the stream
// (the old buffers may still be in use) and clears the new per-atom arrays so
// that padding lanes always read finite values.
static int ensure_work(snap_ctx *c, int n, int np, hipStream_t s)
{
    const int npad = ((n + 63) / 64) * 64;
    Work &w = c->work;
    const size_t nh = (size_t)c->tab.nhalf;
    if (npad > c->cap_atoms) {
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        (void)hipFree(w.U);
        (void)hipFree(w.Y);
        (void)hipFree(w.Epart);
        w.U = w.Y = nullptr;
        w.Epart = nullptr;
        c->cap_atoms = 0;
        ++c->gen;
        HIP_TRY(hipMalloc((void **)&w.U, sizeof(double2) * (size_t)c->tab.nfullel * npad),
                "alloc U");
        HIP_TRY(hipMalloc((void **)&w.Y, sizeof(double2) * nh * npad), "alloc Y");
        HIP_TRY(hipMalloc((void **)&w.Epart, sizeof(double) * c->tab.yrows.size() * npad),
                "alloc Epart");
        HIP_TRY(hipMemset(w.U, 0, sizeof(double2) * (size_t)c->tab.nfullel * npad), "clear U");
        HIP_TRY(hipMemset(w.Y, 0, sizeof(double2) * nh * npad), "clear Y");
        c->cap_atoms = npad;
    }
    if (np > c->cap_pairs) {
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        (void)hipFree(w.dE);
        (void)hipFree(w.pair_atom);
        w.dE = nullptr;
        w.pair_atom = nullptr;
        c->cap_pairs = 0;
        ++c->gen;
        HIP_TRY(hipMalloc((void **)&w.dE, sizeof(double) * 3 * (size_t)np), "alloc dE");
        HIP_TRY(hipMalloc((void **)&w.pair_atom, sizeof(int) * (size_t)np), "alloc pair_atom");
        c->cap_pairs = np;
    }
    // element-major arrays use the capacity as their stride
    w.npad = c->cap_atoms;
    return SNAP_OK;
}

// Grow the partial-sum buffer to at least `doubles` entries (waits for the
// stream first: earlier calls may still read it).
static int ensure_part(snap_ctx *c, size_t doubles, hipStream_t s)
{
    if (doubles <= c->cap_part) return SNAP_OK;
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    (void)hipFree(c->part);
    c->part = nullptr;
    c->cap_part = 0;
    HIP_TRY(hipMalloc((void **)&c->part, sizeof(double) * doubles), "alloc partial sums");
    c->cap_part = doubles;
    return SNAP_OK;
}

// Grow the quadratic-SNAP buffers to n atoms.
static int ensure_quad(snap_ctx *c, int n, hipStream_t s)
{
    if (n <= c->cap_quad) return SNAP_OK;
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    (void)hipFree(c->qB);
    (void)hipFree(c->qG);
    c->qB = c->qG = nullptr;
    c->cap_quad = 0;
    const size_t bytes = sizeof(double) * (size_t)n * c->tab.nb;
    HIP_TRY(hipMalloc((void **)&c->qB, bytes), "alloc quadratic bispectra");
    HIP_TRY(hipMalloc((void **)&c->qG, bytes), "alloc quadratic coefficients");
    c->cap_quad = n;
    return SNAP_OK;
}

// A forward-type call wrote U_j and the pair->atom map for (n, npairs).
static void record_forward(snap_ctx *c, int n, int npairs)
{
    c->last_n = n;
    c->last_npairs = npairs;
    c->last_gen = c->gen;
}

static int check_params(const snap_params *p)
{
    if (!p) return fail(SNAP_EINVAL, "NULL parameters");
    if (p->twojmax < 0 || p->twojmax > SNAP_MAX_TWOJMAX)
        return fail(SNAP_EINVAL, "twojmax %d outside 0..%d", p->twojmax, SNAP_MAX_TWOJMAX);
    if (!(p->rcut > 0.0) || !std::isfinite(p->rcut)) return fail(SNAP_EINVAL, "rcut must be > 0");
    if (!(p->rfac0 > 0.0 && p->rfac0 <= 1.0)) return fail(SNAP_EINVAL, "rfac0 must be in (0, 1]");
    if (!(p->rmin0 >= 0.0 && p->rmin0 < p->rcut))
        return fail(SNAP_EINVAL, "rmin0 must be in [0, rcut)");
    if (p->switch_flag != 0 && p->switch_flag != 1)
        return fail(SNAP_EINVAL, "switch_flag must be 0 or 1");
    if (!std::isfinite(p->wself)) return fail(SNAP_EINVAL, "wself must be finite");
    if (p->dedr_dirs != 0 && p->dedr_dirs != 1 && p->dedr_dirs != 3)
        return fail(SNAP_EINVAL, "dedr_dirs must be 0, 1 or 3");
    if (p->y_kernel < 0 || p->y_kernel > 2) return fail(SNAP_EINVAL, "y_kernel must be 0, 1 or 2");
    if (p->dedr_kernel < 0 || p->dedr_kernel > 4)
        return fail(SNAP_EINVAL, "dedr_kernel must be 0 .. 4");
    if (p->dedr_waves < 0 || p->dedr_waves > 4) return fail(SNAP_EINVAL, "dedr_waves must be 0 .. 4");
    if (p->u_kernel < 0 || p->u_kernel > 3) return fail(SNAP_EINVAL, "u_kernel must be 0 .. 3");
    return SNAP_OK;
}

static int check_box(const double box[3], double rcut)
{
    if (!box) return fail(SNAP_EINVAL, "NULL box");
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(box[d])) return fail(SNAP_EINVAL, "box[%d] is not finite", d);
        if (box[d] > 0.0 && box[d] < 2.0 * rcut)
            return fail(SNAP_EBOX, "periodic box edge %d (%g) shorter than 2*rcut (%g)", d, box[d],
                        2.0 * rcut);
    }
    return SNAP_OK;
}

static Geom make_geom(const snap_ctx *c, const double box[3])
{
    Geom g;
    g.rcut = c->prm.rcut;
    g.rfac0 = c->prm.rfac0;
    g.rmin0 = c->prm.rmin0;
    g.wself = c->prm.wself;
    g.switch_flag = c->prm.switch_flag;
    for (int d = 0; d < 3; ++d) {
        g.box[d] = box[d] > 0.0 ? box[d] : 0.0;
        g.ibox[d] = box[d] > 0.0 ? 1.0 / box[d] : 0.0;
    }
    return g;
}

// Directions per compute_dE lane: three (u and the pair geometry once per
// pair) up to 2J = 6, where they fit in registers; one above (measured on
// 2000 atoms: 2J = 4 13.4 -> 10.7 us, 2J = 6 22.3 -> 21.7 us, 2J = 7
// 28.3 -> 30.6 us).
static int dedr_dirs(const snap_ctx *c)
{
    if (c->prm.dedr_dirs) return c->prm.dedr_dirs;
    return c->prm.twojmax <= 6 ? 3 : 1;
}

// compute_dE: the generator form (one walk of the recursion per pair, three
// direction-independent sums) unless the tangent form is asked for.
static hipError_t run_dedr(const snap_ctx *c, int n, int npairs, int, const double *pos,
                           const int *off, const int *nbr, const int *pair_atom,
                           const double2 *Y, const Geom &g, double *dE, hipStream_t s)
{
    const int k = c->prm.dedr_kernel ? c->prm.dedr_kernel : 2;
    if (k == 1)
        return launch_dedr(c->prm.twojmax, dedr_dirs(c), npairs, c->tab.nhalf, pos, nbr,
                           pair_atom, Y, c->dev, g, dE, s);
    return launch_dedr_gen(c->prm.twojmax, k == 3 ? 1 : 0, k == 4 ? 1 : c->prm.dedr_waves,
                           c->dev.ncu, npairs, c->tab.nhalf, pos, nbr, pair_atom, Y, g, dE, s);
}

extern "C" {

const char *snap_last_error(void) { return g_err.c_str(); }

int snap_setup_ex(const snap_params *p, snap_ctx **out)
{
    if (!out) return fail(SNAP_EINVAL, "NULL output pointer");
    *out = nullptr;
    int st = check_params(p);
    if (st) return st;
    snap_ctx *c = new (std::nothrow) snap_ctx();
    if (!c) return fail(SNAP_ENOMEM, "host allocation failed");
    c->prm = *p;
    try {
        build_tables(p->twojmax, c->tab);
    } catch (const std::bad_alloc &) {
        delete c;
        return fail(SNAP_ENOMEM, "host allocation failed while building tables");
    }
    *out = c;
    g_err.clear();
    return SNAP_OK;
}

int snap_setup(int twojmax, double rcut, double rfac0, double rmin0, int switch_flag, snap_ctx **out)
{
    snap_params p;
    p.twojmax = twojmax;
    p.rcut = rcut;
    p.rfac0 = rfac0;
    p.rmin0 = rmin0;
    p.switch_flag = switch_flag;
    p.wself = 1.0;
    p.dedr_dirs = 0;
    p.y_kernel = 0;
    p.dedr_kernel = 0;
    p.dedr_waves = 0;
    p.u_kernel = 0;
    return snap_setup_ex(&p, out);
}

int snap_destroy(snap_ctx *c)
{
    if (!c) return SNAP_OK;
    for (auto &u : c->ev_used) {
        (void)hipEventSynchronize(u.second.second);
        c->ev_pool.push_back(u.second.first);
        c->ev_pool.push_back(u.second.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->dev_ready) free_dev(c);
    delete c;
    return SNAP_OK;
}

int snap_ncoeff(const snap_ctx *c)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    return c->tab.nb;
}

int snap_nhalf(const snap_ctx *c)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    return c->tab.nhalf;
}

int snap_table(const snap_ctx *c, int which, void *buf, int cap)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    const Tables &t = c->tab;
    auto put_int3 = [&](const std::vector<std::array<int, 3>> &v) {
        int *o = (int *)buf;
        for (size_t k = 0; k < v.size() && o && (int)(3 * k + 2) < cap; ++k)
            for (int d = 0; d < 3; ++d) o[3 * k + d] = v[k][d];
        return (int)(3 * v.size());
    };
    switch (which) {
    case 0: return put_int3(t.comps);
    case 1: return put_int3(t.helem);
    case 2: {
        double *o = (double *)buf;
        for (size_t k = 0; k < t.cg_vals.size() && o && (int)k < cap; ++k) o[k] = t.cg_vals[k];
        return (int)t.cg_vals.size();
    }
    case 3: {
        int *o = (int *)buf;
        for (size_t k = 0; k < t.cg_keys.size() && o && (int)(5 * k + 4) < cap; ++k)
            for (int d = 0; d < 5; ++d) o[5 * k + d] = t.cg_keys[k][d];
        return (int)(5 * t.cg_keys.size());
    }
    case 4: {
        const int v[4] = {(int)t.yterms, (int)t.ypartials, (int)t.ycontrib.size(),
                          (int)t.yrows.size()};
        int *o = (int *)buf;
        for (int k = 0; k < 4 && o && k < cap; ++k) o[k] = v[k];
        return 4;
    }
    default: return fail(SNAP_EINVAL, "unknown table %d", which);
    }
}

int snap_build_neighbors(const double *pos_host, int n, const double box[3], double rcut, int *off,
                         int *nbr, int *rev, int cap, int *npairs)
{
    if (n < 0 || !off || !npairs || (n > 0 && !pos_host) || cap < 0 || (cap > 0 && (!nbr || !rev)))
        return fail(SNAP_EINVAL, "bad arguments to snap_build_neighbors");
    if (!(rcut > 0.0)) return fail(SNAP_EINVAL, "rcut must be > 0");
    int st = check_box(box, rcut);
    if (st) return st;
    for (long k = 0; k < 3L * n; ++k)
        if (!std::isfinite(pos_host[k])) return fail(SNAP_EGEOM, "non-finite position");
    try {
        if (build_neighbors(pos_host, n, box, rcut, off, nbr, rev, cap, npairs) != 0)
            return fail(SNAP_ENOMEM, "neighbour capacity %d too small (%d pairs)", cap, *npairs);
    } catch (const std::bad_alloc &) {
        return fail(SNAP_ENOMEM, "host allocation failed in the neighbour builder");
    }
    return SNAP_OK;
}

int snap_check_neighbors(int n, const int *off, const int *nbr, const int *rev, int npairs)
{
    if (n < 0 || npairs < 0 || !off) return fail(SNAP_EINVAL, "bad arguments");
    if (off[0] != 0 || off[n] != npairs) return fail(SNAP_ENBR, "off[0] must be 0 and off[n] == npairs");
    for (int i = 0; i < n; ++i) {
        if (off[i + 1] < off[i]) return fail(SNAP_ENBR, "off decreases at atom %d", i);
        for (int p = off[i]; p < off[i + 1]; ++p) {
            const int k = nbr[p];
            if (k < 0 || k >= n) return fail(SNAP_ENBR, "neighbour index %d out of range", k);
            if (k == i) return fail(SNAP_ENBR, "atom %d lists itself", i);
            const int r = rev[p];
            if (r < 0 || r >= npairs) return fail(SNAP_ENBR, "rev[%d] = %d out of range", p, r);
            if (nbr[r] != i || r < off[k] || r >= off[k + 1] || rev[r] != p)
                return fail(SNAP_ENBR, "rev[%d] does not point at the reverse pair", p);
        }
    }
    return SNAP_OK;
}

static int common_checks(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                         const int *off, const int *nbr, const int *rev, const double *beta,
                         bool need_beta = true)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    if (n < 0 || npairs < 0) return fail(SNAP_EINVAL, "negative size");
    if (n > (1 << 24) || npairs > (1 << 30)) return fail(SNAP_EINVAL, "size too large");
    // compute_Y addresses a row of U_J (J + 1 elements of npad atoms, 16 bytes
    // each) through one buffer descriptor with 32-bit byte counts
    const long long npad = ((long long)n + 63) / 64 * 64;
    if ((long long)(c->prm.twojmax + 1) * npad * 16 >= (1ll << 31))
        return fail(SNAP_EINVAL, "n = %d too large for twojmax %d (limit %lld atoms)", n,
                    c->prm.twojmax, (long long)(((1ll << 31) - 1) / (16 * (c->prm.twojmax + 1))) / 64 * 64);
    int st = check_box(box, c->prm.rcut);
    if (st) return st;
    if (n > 0 && (!pos || !off || (need_beta && !beta)))
        return fail(SNAP_EINVAL, "NULL input pointer");
    if (npairs > 0 && (!nbr || !rev)) return fail(SNAP_EINVAL, "NULL neighbour pointer");
    return SNAP_OK;
}

// compute_U (+ pair->atom map) for the current call
static int run_u(snap_ctx *c, int n, int npairs, const double *pos, const Geom &g, const int *off,
                 const int *nbr, hipStream_t s)
{
    (void)npairs;
    HIP_TRY(launch_compute_u(c->prm.twojmax, c->prm.u_kernel ? c->prm.u_kernel : 1, n,
                             c->work.npad, pos, off, nbr, c->dev, g, c->work.U,
                             c->work.pair_atom, c->work.flag, s),
            "compute_U launch");
    return SNAP_OK;
}

// Upload the element arrays after snap_set_elements changed them.
static int ensure_elements(snap_ctx *c)
{
    if (!c->elem_dirty) return SNAP_OK;
    // earlier calls may still read the old arrays
    if (c->d_erad || c->d_ewt) HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    (void)hipFree(c->d_erad);
    (void)hipFree(c->d_ewt);
    c->d_erad = c->d_ewt = nullptr;
    HIP_TRY(upload(c->d_erad, c->erad), "upload element radii");
    HIP_TRY(upload(c->d_ewt, c->ewt), "upload element weights");
    c->elem_dirty = false;
    return SNAP_OK;
}

// snap_compute and snap_compute_elements (type != NULL: beta per element)
static int compute_impl(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                        const int *off, const int *nbr, const int *rev, const int *type,
                        const double *beta, int per_atom_beta, double *energy, double *force,
                        double *bispec, double *dE_pair, void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, beta);
    if (st) return st;
    if (n > 0 && (!energy || !force)) return fail(SNAP_EINVAL, "NULL output pointer");
    if (type && c->nelem < 1) return fail(SNAP_EINVAL, "no elements set (snap_set_elements)");
    if ((st = ensure_device(c))) return st;
    if (type && (st = ensure_elements(c))) return st;
    if (n == 0) return SNAP_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_work(c, n, npairs > 0 ? npairs : 1, s))) return st;
    Geom g = make_geom(c, box);
    if (type) {
        g.type = type;
        g.erad = c->d_erad;
        g.ewt = c->d_ewt;
        g.rcutfac = c->rcutfac;
        g.nelem = c->nelem;
    }
    Work &w = c->work;
    const int nb = c->tab.nb;
    double *dE = dE_pair ? dE_pair : w.dE;
    {
        StageTimer tm(c, 0, s);
        if ((st = run_u(c, n, npairs, pos, g, off, nbr, s))) return st;
        tm.finish();
    }
    {
        StageTimer tm(c, 1, s);
        HIP_TRY(launch_compute_y(c->prm.twojmax, n, w.npad, w.U, w.Y, c->dev, beta, per_atom_beta,
                                 nb, type, c->nelem, nullptr, w.Epart, s),
                "compute_Y launch");
        tm.finish();
    }
    if (npairs > 0) {
        StageTimer tm(c, 2, s);
        HIP_TRY(run_dedr(c, n, npairs, w.npad, pos, off, nbr, w.pair_atom, w.Y, g, dE, s),
                "compute_dE launch");
        tm.finish();
    }
    {
        StageTimer tm(c, 3, s);
        HIP_TRY(launch_gather(n, w.npad, c->dev.nyrows, off, rev, dE, w.Epart, energy, force, s),
                "update_forces launch");
        tm.finish();
    }
    if (bispec) {
        StageTimer tm(c, 4, s);
        HIP_TRY(launch_bispectrum(n, w.npad, w.U, c->dev, nb, bispec, beta, per_atom_beta, nullptr,
                                  s, c->tab.nfullel),
                "bispectrum launch");
        tm.finish();
    }
    record_forward(c, n, npairs);
    return SNAP_OK;
}

int snap_compute(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                 const int *off, const int *nbr, const int *rev, const double *beta,
                 int per_atom_beta, double *energy, double *force, double *bispec,
                 double *dE_pair, void *stream)
{
    return compute_impl(c, n, npairs, pos, box, off, nbr, rev, nullptr, beta, per_atom_beta,
                        energy, force, bispec, dE_pair, stream);
}

int snap_compute_noalloc(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                         const int *off, const int *nbr, const int *rev, const double *beta,
                         int per_atom_beta, double *energy, double *force, double *bispec,
                         double *dE_pair, void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, beta);
    if (st) return st;
    if (n > 0 && (!energy || !force)) return fail(SNAP_EINVAL, "NULL output pointer");
    if (!c->dev_ready)
        return fail(SNAP_EINVAL,
                    "the context's tables are not on the device yet: one allocating call "
                    "(snap_compute or snap_forward) on this context must come first");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != c->device)
        return fail(SNAP_EDEV, "context tables are on device %d, current device is %d", c->device,
                    dev);
    if (n == 0) return SNAP_OK;
    // the workspace carved from the static array: U (element-major, full
    // matrices), Y (atom-major half), Epart, dE (unless the caller takes it),
    // pair->atom map, each 256-byte aligned
    const int npad = (n + 63) / 64 * 64;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t bU = al(sizeof(double2) * (size_t)c->tab.nfullel * npad);
    const size_t bY = al(sizeof(double2) * (size_t)c->tab.nhalf * npad);
    const size_t bE = al(sizeof(double) * c->tab.yrows.size() * npad);
    const size_t bD = dE_pair ? 0 : al(sizeof(double) * 3 * (size_t)(npairs > 0 ? npairs : 1));
    const size_t bP = al(sizeof(int) * (size_t)(npairs > 0 ? npairs : 1));
    const size_t need = bU + bY + bE + bD + bP;
    if (need > static_scratch_bytes())
        return fail(SNAP_EINVAL,
                    "n = %d, %d pairs at twojmax %d need %zu bytes of workspace; the static "
                    "workspace holds %zu",
                    n, npairs, c->prm.twojmax, need, static_scratch_bytes());
    void *base = nullptr;
    HIP_TRY(static_scratch(&base), "hipGetSymbolAddress of the static workspace");
    unsigned char *b = (unsigned char *)base;
    Work w;
    w.U = (double2 *)b;
    w.Y = (double2 *)(b + bU);
    w.Epart = (double *)(b + bU + bY);
    w.dE = dE_pair ? dE_pair : (double *)(b + bU + bY + bE);
    w.pair_atom = (int *)(b + bU + bY + bE + bD);
    w.flag = c->work.flag;
    w.npad = npad;
    hipStream_t s = (hipStream_t)stream;
    Geom g = make_geom(c, box);
    const int nb = c->tab.nb;
    // the array keeps the previous call's contents: the padding atoms, which
    // the kernels read but never write, start from zero
    HIP_TRY(launch_zero_padding(w.U, c->tab.nfullel, w.Y, c->tab.nhalf, n, npad, s),
            "workspace padding");
    HIP_TRY(launch_compute_u(c->prm.twojmax, c->prm.u_kernel ? c->prm.u_kernel : 1, n, npad, pos,
                             off, nbr, c->dev, g, w.U, w.pair_atom, w.flag, s),
            "compute_U launch");
    HIP_TRY(launch_compute_y(c->prm.twojmax, n, npad, w.U, w.Y, c->dev, beta, per_atom_beta, nb,
                             nullptr, 0, nullptr, w.Epart, s),
            "compute_Y launch");
    if (npairs > 0)
        HIP_TRY(run_dedr(c, n, npairs, npad, pos, off, nbr, w.pair_atom, w.Y, g, w.dE, s),
                "compute_dE launch");
    HIP_TRY(launch_gather(n, npad, c->dev.nyrows, off, rev, w.dE, w.Epart, energy, force, s),
            "update_forces launch");
    if (bispec)
        HIP_TRY(launch_bispectrum(n, npad, w.U, c->dev, nb, bispec, beta, per_atom_beta, nullptr,
                                  s, c->tab.nfullel),
                "bispectrum launch");
    return SNAP_OK;
}

int snap_compute_quadratic(snap_ctx *c, int n, int npairs, const double *pos,
                           const double box[3], const int *off, const int *nbr, const int *rev,
                           const double *beta, const double *alpha, double *energy,
                           double *force, double *bispec, double *dE_pair, void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, beta);
    if (st) return st;
    if (n > 0 && (!energy || !force || !alpha)) return fail(SNAP_EINVAL, "NULL pointer argument");
    if ((st = ensure_device(c))) return st;
    if (n == 0) return SNAP_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_work(c, n, npairs > 0 ? npairs : 1, s))) return st;
    if ((st = ensure_quad(c, n, s))) return st;
    const Geom g = make_geom(c, box);
    Work &w = c->work;
    const int nb = c->tab.nb;
    double *B = bispec ? bispec : c->qB;
    double *dE = dE_pair ? dE_pair : w.dE;
    {
        StageTimer tm(c, 0, s);
        if ((st = run_u(c, n, npairs, pos, g, off, nbr, s))) return st;
        tm.finish();
    }
    {
        StageTimer tm(c, 4, s);
        HIP_TRY(launch_bispectrum(n, w.npad, w.U, c->dev, nb, B, nullptr, 0, nullptr, s,
                                  c->tab.nfullel),
                "bispectrum launch");
        HIP_TRY(launch_quadratic(n, nb, B, beta, alpha, energy, c->qG, s), "quadratic launch");
        tm.finish();
    }
    {
        // Y from the per-atom coefficients g_i = dE_i/dB_i (Sec. IV: the
        // adjoint takes any per-atom coefficient vector)
        StageTimer tm(c, 1, s);
        HIP_TRY(launch_compute_y(c->prm.twojmax, n, w.npad, w.U, w.Y, c->dev, c->qG, 1, nb,
                                 nullptr, 0, nullptr, nullptr, s),
                "compute_Y launch");
        tm.finish();
    }
    if (npairs > 0) {
        StageTimer tm(c, 2, s);
        HIP_TRY(run_dedr(c, n, npairs, w.npad, pos, off, nbr, w.pair_atom, w.Y, g, dE, s),
                "compute_dE launch");
        tm.finish();
    }
    {
        StageTimer tm(c, 3, s);
        HIP_TRY(launch_gather(n, w.npad, c->dev.nyrows, off, rev, dE, nullptr, nullptr, force, s),
                "update_forces launch");
        tm.finish();
    }
    record_forward(c, n, npairs);
    return SNAP_OK;
}

int snap_set_elements(snap_ctx *c, int nelem, const double *radius, const double *weight,
                      double rcutfac)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    if (nelem < 0 || nelem > kMaxElements)
        return fail(SNAP_EINVAL, "nelem %d outside 0..%d", nelem, kMaxElements);
    if (nelem == 0) {
        c->nelem = 0;
        c->erad.clear();
        c->ewt.clear();
        return SNAP_OK;
    }
    if (!radius || !weight) return fail(SNAP_EINVAL, "NULL element array");
    if (!(rcutfac > 0.0) || !std::isfinite(rcutfac)) return fail(SNAP_EINVAL, "rcutfac must be > 0");
    double rmax = 0.0;
    for (int e = 0; e < nelem; ++e) {
        if (!(radius[e] > 0.0) || !std::isfinite(radius[e]))
            return fail(SNAP_EINVAL, "radius[%d] must be > 0", e);
        if (!std::isfinite(weight[e])) return fail(SNAP_EINVAL, "weight[%d] must be finite", e);
        rmax = radius[e] > rmax ? radius[e] : rmax;
    }
    if (2.0 * rcutfac * rmax > c->prm.rcut * (1.0 + 1e-12))
        return fail(SNAP_EINVAL,
                    "largest pair cutoff %g exceeds the context's rcut %g (the neighbour "
                    "list cutoff)", 2.0 * rcutfac * rmax, c->prm.rcut);
    c->nelem = nelem;
    c->erad.assign(radius, radius + nelem);
    c->ewt.assign(weight, weight + nelem);
    c->rcutfac = rcutfac;
    c->elem_dirty = true;
    return SNAP_OK;
}

int snap_compute_elements(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                          const int *off, const int *nbr, const int *rev, const int *type,
                          const double *beta, double *energy, double *force, double *bispec,
                          double *dE_pair, void *stream)
{
    if (n > 0 && !type) return fail(SNAP_EINVAL, "NULL type pointer");
    return compute_impl(c, n, npairs, pos, box, off, nbr, rev, n > 0 ? type : nullptr, beta, 0,
                        energy, force, bispec, dE_pair, stream);
}

int snap_forward(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                 const int *off, const int *nbr, const int *rev, const double *beta,
                 int per_atom_beta, double *energy, double *bispec, void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, beta, energy != nullptr);
    if (st) return st;
    if (n > 0 && !bispec) return fail(SNAP_EINVAL, "NULL output pointer");
    if ((st = ensure_device(c))) return st;
    if (n == 0) return SNAP_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_work(c, n, npairs > 0 ? npairs : 1, s))) return st;
    const Geom g = make_geom(c, box);
    if ((st = run_u(c, n, npairs, pos, g, off, nbr, s))) return st;
    HIP_TRY(launch_bispectrum(n, c->work.npad, c->work.U, c->dev, c->tab.nb, bispec, beta,
                              per_atom_beta, energy, s, c->tab.nfullel),
            "bispectrum launch");
    record_forward(c, n, npairs);
    return SNAP_OK;
}

int snap_backward(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                  const int *off, const int *nbr, const int *rev, const double *beta,
                  int per_atom_beta, const double *grad_energy, double *force, double *dE_pair,
                  void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, beta);
    if (st) return st;
    if (n > 0 && (!grad_energy || !force)) return fail(SNAP_EINVAL, "NULL gradient pointer");
    if (n == 0) return SNAP_OK;
    // the U_j and pair->atom map of the last forward-type call are reused:
    // same sizes, and no reallocation of the workspace since
    if (!c->dev_ready || n != c->last_n || npairs != c->last_npairs || c->gen != c->last_gen)
        return fail(SNAP_EINVAL,
                    "snap_backward needs the U of a snap_forward (or snap_compute) on this "
                    "context with the same n and npairs, and no larger call in between");
    hipStream_t s = (hipStream_t)stream;
    const Geom g = make_geom(c, box);
    Work &w = c->work;
    double *dE = dE_pair ? dE_pair : w.dE;
    HIP_TRY(launch_compute_y(c->prm.twojmax, n, w.npad, w.U, w.Y, c->dev, beta, per_atom_beta,
                             c->tab.nb, nullptr, 0, grad_energy, nullptr, s),
            "compute_Y launch");
    if (npairs > 0)
        HIP_TRY(run_dedr(c, n, npairs, w.npad, pos, off, nbr, w.pair_atom, w.Y, g, dE, s),
                "compute_dE launch");
    HIP_TRY(launch_gather(n, w.npad, c->dev.nyrows, off, rev, dE, nullptr, nullptr, force, s),
            "update_forces launch");
    return SNAP_OK;
}

int snap_copy_workspace(snap_ctx *c, int which, int n, double *dst, void *stream)
{
    if (!c || !dst || (which != 0 && which != 1)) return fail(SNAP_EINVAL, "bad arguments");
    if (!c->dev_ready || c->last_n <= 0 || c->gen != c->last_gen)
        return fail(SNAP_EINVAL, "no evaluation to copy from");
    if (n != c->last_n)
        return fail(SNAP_EINVAL, "n = %d but the last evaluation had %d atoms", n, c->last_n);
    // the workspace holds scaled values (U/N and w N Y); return true ones
    const double2 *src = which == 0 ? c->work.U : c->work.Y;
    const int *map = which == 0 ? c->dev.half2full : nullptr;
    const double *scale = which == 0 ? nullptr : c->dev.unscale_y;
    const int se = which == 0 ? c->work.npad : 1, sa = which == 0 ? 1 : c->tab.nhalf;
    HIP_TRY(launch_unscale(c->last_n, se, sa, c->tab.nhalf, src, map, scale, dst,
                           (hipStream_t)stream),
            "copy workspace");
    return SNAP_OK;
}

int snap_profile(snap_ctx *c, int enable)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    c->profiling = enable != 0;
    return SNAP_OK;
}

int snap_stage_times(snap_ctx *c, double ms[5], int launches[5])
{
    if (!c || !ms || !launches) return fail(SNAP_EINVAL, "bad arguments");
    for (int k = 0; k < 5; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &u : c->ev_used) {
        HIP_TRY(hipEventSynchronize(u.second.second), "hipEventSynchronize");
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, u.second.first, u.second.second), "hipEventElapsedTime");
        ms[u.first] += (double)t;
        launches[u.first] += 1;
        c->ev_pool.push_back(u.second.first);
        c->ev_pool.push_back(u.second.second);
    }
    c->ev_used.clear();
    return SNAP_OK;
}

int snap_sync_status(snap_ctx *c, void *stream)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    if (!c->dev_ready) return SNAP_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, c->work.flag, sizeof(int), hipMemcpyDeviceToHost), "read flag");
    if (flag) {
        HIP_TRY(hipMemset(c->work.flag, 0, sizeof(int)), "clear flag");
        if (flag == 2) return fail(SNAP_EINVAL, "atom type outside 0..nelem-1");
        return fail(SNAP_EGEOM, "coincident atoms (r < 1e-10 A) or non-finite positions");
    }
    return SNAP_OK;
}


int snap_virial(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                const int *off, const int *nbr, const double *dE_pair, double *virial_atom,
                double *virial, void *stream)
{
    // no reverse index or coefficients are read: nbr stands in for rev
    int st = common_checks(c, n, npairs, pos, box, off, nbr, nbr, nullptr, false);
    if (st) return st;
    if (!virial) return fail(SNAP_EINVAL, "NULL virial pointer");
    if (npairs > 0 && !dE_pair) return fail(SNAP_EINVAL, "NULL dE_pair pointer");
    if ((st = ensure_device(c))) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_part(c, 9 * ((size_t)n / 256 + 1), s))) return st;
    const Geom g = make_geom(c, box);
    HIP_TRY(launch_virial(n, pos, off, nbr, g, dE_pair, n > 0 ? virial_atom : nullptr, c->part,
                          virial, s),
            "virial launch");
    return SNAP_OK;
}

int snap_beta_grad(snap_ctx *c, int n, const double *grad_energy, const double *bispec,
                   int per_atom, double *grad_beta, void *stream)
{
    if (!c) return fail(SNAP_EINVAL, "NULL context");
    if (n < 0 || n > (1 << 24)) return fail(SNAP_EINVAL, "n out of range");
    if (per_atom != 0 && per_atom != 1) return fail(SNAP_EINVAL, "per_atom must be 0 or 1");
    if (!grad_beta || (n > 0 && (!grad_energy || !bispec)))
        return fail(SNAP_EINVAL, "NULL pointer argument");
    int st = ensure_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!per_atom && (st = ensure_part(c, (size_t)beta_grad_blocks(n) * c->tab.nb + 1, s)))
        return st;
    HIP_TRY(launch_beta_grad(n, c->tab.nb, grad_energy, bispec, per_atom, c->part, grad_beta, s),
            "coefficient gradient launch");
    return SNAP_OK;
}

// ---------------------------------------------------------------------------
// learned surrogate
// ---------------------------------------------------------------------------

int snap_jacobian(snap_ctx *c, int n, int npairs, const double *pos, const double box[3],
                  const int *off, const int *nbr, const int *rev, double *bispec, float *jac,
                  void *stream)
{
    int st = common_checks(c, n, npairs, pos, box, off, nbr, rev, nullptr, false);
    if (st) return st;
    if (npairs > 0 && !jac) return fail(SNAP_EINVAL, "NULL Jacobian pointer");
    if ((st = ensure_device(c))) return st;
    if (n == 0) return SNAP_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_work(c, n, npairs > 0 ? npairs : 1, s))) return st;
    const Geom g = make_geom(c, box);
    Work &w = c->work;
    const int nb = c->tab.nb;
    if ((st = run_u(c, n, npairs, pos, g, off, nbr, s))) return st;
    if (bispec)
        HIP_TRY(launch_bispectrum(n, w.npad, w.U, c->dev, nb, bispec, nullptr, 0, nullptr, s,
                                  c->tab.nfullel),
                "bispectrum launch");
    record_forward(c, n, npairs);
    if (npairs == 0) return SNAP_OK;
    for (int l = 0; l < nb; ++l) {
        const double *el = c->dev.onehot + (size_t)l * nb;
        HIP_TRY(launch_compute_y(c->prm.twojmax, n, w.npad, w.U, w.Y, c->dev, el, 0, nb, nullptr, 0,
                                 nullptr, nullptr, s),
                "compute_Y launch");
        HIP_TRY(run_dedr(c, n, npairs, w.npad, pos, off, nbr, w.pair_atom, w.Y, g, w.dE, s),
                "compute_dE launch");
        HIP_TRY(launch_pack_jac(npairs, nb, l, w.dE, jac, s), "Jacobian store");
    }
    return SNAP_OK;
}

// Checks shared by the context-free entry points: a usable gfx950 device.
static int check_free_call(int nin)
{
    if (nin >= 0 && !mlp_supported(nin)) return fail(SNAP_EINVAL, "nin %d not supported (5, 14, 30)", nin);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    static thread_local int checked_dev = -1;
    if (checked_dev != dev) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(SNAP_EDEV, "device %d is %s; this library is built for gfx950", dev,
                        prop.gcnArchName);
        checked_dev = dev;
    }
    return SNAP_OK;
}

int snap_mlp_nparams(int nin)
{
    if (!mlp_supported(nin)) return fail(SNAP_EINVAL, "nin %d not supported (5, 14, 30)", nin);
    return mlp_nparams(nin);
}

long long snap_mlp_workspace(int nin, int n)
{
    if (!mlp_supported(nin)) return fail(SNAP_EINVAL, "nin %d not supported (5, 14, 30)", nin);
    if (n < 0 || n > (1 << 24)) return fail(SNAP_EINVAL, "n out of range");
    return (long long)mlp_grad_workspace(nin, n);
}

int snap_mlp_forward(int nin, int n, const float *params, const float *norm,
                     const float *bounds, float margin, const double *bispec, double *energy,
                     double *grad_b, int *ood_flag, int *clear_flag, void *stream)
{
    if (clear_flag && clear_flag == ood_flag)
        return fail(SNAP_EINVAL, "clear_flag must differ from ood_flag");
    if (n < 0 || n > (1 << 24)) return fail(SNAP_EINVAL, "n out of range");
    if (!std::isfinite(margin) || margin < 0.0f) return fail(SNAP_EINVAL, "margin must be >= 0");
    int st = check_free_call(nin);
    if (st) return st;
    if (n == 0) return SNAP_OK;
    if (!params || !norm || !bispec || !energy || !grad_b)
        return fail(SNAP_EINVAL, "NULL pointer argument");
    HIP_TRY(launch_mlp_forward(nin, n, params, norm, bounds, margin, bispec, energy, grad_b,
                               ood_flag, clear_flag, (hipStream_t)stream),
            "network forward launch");
    return SNAP_OK;
}

int snap_mlp_grad(int nin, int n, const float *params, const float *norm, const double *bispec,
                  const double *dl_de, const double *dl_dg, float *work, float *grad,
                  void *stream)
{
    if (n < 0 || n > (1 << 24)) return fail(SNAP_EINVAL, "n out of range");
    int st = check_free_call(nin);
    if (st) return st;
    if (!grad) return fail(SNAP_EINVAL, "NULL gradient pointer");
    hipStream_t s = (hipStream_t)stream;
    if (n > 0 && (!params || !norm || !bispec || !dl_de || !work))
        return fail(SNAP_EINVAL, "NULL pointer argument");
    HIP_TRY(launch_mlp_grad(nin, n, params, norm, bispec, dl_de, dl_dg, work, grad, s),
            "network gradient launch");
    return SNAP_OK;
}

int snap_adam_step(int np, float *params, float *m, float *v, const float *grad, float lr,
                   float beta1, float beta2, float eps, int step, void *stream)
{
    if (np <= 0 || !params || !m || !v || !grad) return fail(SNAP_EINVAL, "bad Adam arguments");
    if (step < 1) return fail(SNAP_EINVAL, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
        !std::isfinite(lr))
        return fail(SNAP_EINVAL, "Adam hyper-parameters out of range");
    int st = check_free_call(-1);
    if (st) return st;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    HIP_TRY(launch_adam(np, params, m, v, grad, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream),
            "Adam launch");
    return SNAP_OK;
}

int snap_jacobian_forces(int nin, int n, int npairs, const int *off, const int *rev,
                         const float *jac, const double *grad_b, double *dE_pair, double *force,
                         void *stream)
{
    if (n < 0 || npairs < 0 || n > (1 << 24) || npairs > (1 << 30))
        return fail(SNAP_EINVAL, "size out of range");
    int st = check_free_call(nin);
    if (st) return st;
    if (n == 0) return SNAP_OK;
    if (!off || !grad_b || !force || (npairs > 0 && (!rev || !jac || !dE_pair)))
        return fail(SNAP_EINVAL, "NULL pointer argument");
    hipStream_t s = (hipStream_t)stream;
    if (npairs > 0)
        HIP_TRY(launch_jac_force(nin, n, npairs, off, jac, grad_b, dE_pair, s),
                "Jacobian force launch");
    HIP_TRY(launch_gather(n, 0, 0, off, rev, dE_pair, nullptr, nullptr, force, s),
            "update_forces launch");
    return SNAP_OK;
}

int snap_jacobian_adjoint(int nin, int n, int npairs, const int *off, const int *nbr,
                          const float *jac, const double *dl_dforce, double *dl_dg, void *stream)
{
    if (n < 0 || npairs < 0 || n > (1 << 24) || npairs > (1 << 30))
        return fail(SNAP_EINVAL, "size out of range");
    int st = check_free_call(nin);
    if (st) return st;
    if (n == 0) return SNAP_OK;
    if (!off || !dl_dforce || !dl_dg || (npairs > 0 && (!nbr || !jac)))
        return fail(SNAP_EINVAL, "NULL pointer argument");
    HIP_TRY(launch_jac_adjoint(nin, n, off, nbr, jac, dl_dforce, dl_dg, (hipStream_t)stream),
            "Jacobian adjoint launch");
    return SNAP_OK;
}

int snap_fit_residuals(int n, const double *energy, const double *energy_ref,
                       const double *force, const double *force_ref, double w_energy,
                       double w_force, double *dl_de, double *dl_dforce, double *sums,
                       void *stream)
{
    if (n < 0 || n > (1 << 24)) return fail(SNAP_EINVAL, "n out of range");
    if (!std::isfinite(w_energy) || !std::isfinite(w_force))
        return fail(SNAP_EINVAL, "loss weights must be finite");
    int st = check_free_call(-1);
    if (st) return st;
    if (n == 0) return SNAP_OK;
    if (!energy || !energy_ref || !force || !force_ref || !dl_de || !dl_dforce || !sums)
        return fail(SNAP_EINVAL, "NULL pointer argument");
    HIP_TRY(launch_residuals(n, energy, energy_ref, force, force_ref, w_energy, w_force, dl_de,
                             dl_dforce, sums, (hipStream_t)stream),
            "residual launch");
    return SNAP_OK;
}

}  // extern "C"
