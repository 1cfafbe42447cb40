// C ABI of libapic (declared in include/apic.h): host-side validation,
// workspace layout, binning state and dispatch to the gfx950 kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <type_traits>
#include <vector>

#include "apic.h"
#include "apic_kernels.h"

namespace {

using namespace apic;

thread_local std::string g_last_error;

apic_status fail(apic_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
apic_status fail(apic_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

constexpr size_t kAlign = 256;
// Shadow planes are a whole number of 64-particle blocks apart, so that every
// plane starts on a 256-byte boundary like the first: the transfers read and
// write runs of 64 particles aligned to the planes and cover whole cache
// lines only when every plane shares that alignment.
constexpr int64_t kPlaneAlign = 64;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int slab_nodes(int dim, int degree) {
    const int re = (dim == 3 ? 4 : 8) + degree;
    return dim == 3 ? re * re * re : re * re;
}

// ---------------------------------------------------------------------------
// Workspace layout for a grid and a particle capacity `cap`.
// ---------------------------------------------------------------------------
struct ListOff {
    size_t tile_gen, slot, rec_count, nfull, nsparse, rec_list, rec_tile, tot, rpre, bpre, ctr;
};

struct TabOff {
    size_t kcount, kmov, kprefix, maxc, tcount, off, lvl_off, lvl_mask;
};

struct Layout {
    GridDims d;
    size_t elem;
    bool comp;
    int64_t cap;    // particle capacity
    int64_t sst;    // plane stride of the shadow state: cap rounded up to kPlaneAlign
    int64_t rc;     // record (slab) capacity: min(tiles, cap)
    int64_t rcap;   // list capacity per bucket: ceil(tiles / kBuckets)
    int64_t slab_stride;
    size_t o_vt, o_uref, o_flags, o_vmax, o_cfl, o_dt, o_diag_out, o_diag_part, o_key_count, o_scount,
        o_head;
    ListOff lists[2];
    TabOff tabs[2];
    size_t o_slabs;
    size_t fixed_end;
    size_t o_pkey, o_prank, o_next, o_pord, o_sh_cell, o_sh_id, o_sh_f;
    size_t total;
};

Layout make_layout(const apic_grid_desc *g, int64_t cap) {
    Layout L{};
    L.d.dim = g->dim;
    L.d.deg = g->degree;
    const int te = g->dim == 3 ? 4 : 8;
    L.d.tiles = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < g->dim) {
            L.d.n[a] = g->cells[a];
            L.d.N[a] = g->cells[a] + 1;
            L.d.TN[a] = (L.d.N[a] + te - 1) / te;
            L.d.tiles *= L.d.TN[a];
        } else {
            L.d.n[a] = 0;
            L.d.N[a] = 1;
            L.d.TN[a] = 1;
        }
    }
    L.d.G = L.d.tiles * 64;
    L.elem = g->precision == APIC_F64 ? 8 : 4;
    L.comp = (g->options & APIC_OPT_COMPENSATED) != 0;
    L.cap = cap < 1 ? 1 : cap;
    L.sst = (L.cap + kPlaneAlign - 1) / kPlaneAlign * kPlaneAlign;
    L.rc = L.d.tiles < L.cap ? L.d.tiles : L.cap;
    L.rcap = (L.d.tiles + kBuckets - 1) / kBuckets;
    const size_t TT = (size_t)L.d.tiles, G = (size_t)L.d.G, dim = (size_t)g->dim, e = L.elem;
    const size_t RC = (size_t)L.rc, cp = (size_t)L.cap, LB = (size_t)kBuckets * (size_t)L.rcap;
    L.slab_stride = (int64_t)((1 + dim) * slab_nodes(g->dim, g->degree) * (L.comp ? 2 : 1));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.o_vt = take(dim * G * e);
    L.o_uref = take(dim * TT * e);
    L.o_flags = take(64);
    L.o_vmax = take((size_t)kVmaxSlots * 4);
    L.o_cfl = take((size_t)kVmaxSlots * 8);
    L.o_dt = take(2 * sizeof(double));
    L.o_diag_out = take(8 * sizeof(double));
    L.o_diag_part = take((size_t)kDiagBlocks * 8 * sizeof(double));
    L.o_key_count = take(G * 4);
    L.o_scount = take(G * 4);
    L.o_head = take(G * 4);
    for (int k = 0; k < 2; ++k) {
        ListOff &l = L.lists[k];
        l.tile_gen = take(TT * 4);
        l.slot = take(TT * 4);
        l.rec_count = take((size_t)kBuckets * 4);
        l.nfull = take((size_t)kBuckets * 4);
        l.nsparse = take((size_t)kBuckets * 4);
        l.rec_list = take(LB * 4);
        l.rec_tile = take(RC * 4);
        l.tot = take((size_t)kBuckets * 4);
        l.rpre = take((size_t)(kBuckets + 1) * 4);
        l.bpre = take((size_t)(kBuckets + 1) * 4);
        l.ctr = take((size_t)kCtrCount * 4);
    }
    for (int k = 0; k < 2; ++k) {
        TabOff &t = L.tabs[k];
        t.kcount = take(TT * 64 * 4);
        t.kmov = take(TT * 64 * 4);
        t.kprefix = take(TT * 64 * 4);
        t.maxc = take(TT * 4);
        t.tcount = take(TT * 4);
        t.off = take(TT * 4);
        t.lvl_off = take(TT * (size_t)kMaxLevels * 4);
        t.lvl_mask = take(TT * (size_t)kMaxLevels * 8);
    }
    L.o_slabs = take(RC * (size_t)L.slab_stride * e);
    L.fixed_end = o;
    L.o_pkey = take(cp * 4);
    L.o_prank = take(cp * 4);
    L.o_next = take(cp * 4);
    L.o_pord = take(cp * 8);
    L.o_sh_cell = take(cp * 4);
    L.o_sh_id = take(cp * 4);
    L.o_sh_f = take((2 * dim + 2 * dim * dim + 1) * (size_t)L.sst * e);
    L.total = o;
    return L;
}

// Largest particle capacity whose layout fits in `bytes` (0 if none).
int64_t capacity_for(const apic_grid_desc *g, size_t bytes) {
    if (make_layout(g, 1).total > bytes) return 0;
    int64_t lo = 1, hi = 2;
    while (hi < ((int64_t)1 << 31) && make_layout(g, hi).total <= bytes) {
        lo = hi;
        hi *= 2;
    }
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(g, mid).total <= bytes)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
apic_status check_grid(const apic_grid_desc *g) {
    if (!g) return fail(APIC_E_INVAL, "grid descriptor is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(APIC_E_INVAL, "dim must be 2 or 3 (got %d)", g->dim);
    if (g->degree != APIC_MULTILINEAR && g->degree != APIC_QUADRATIC && g->degree != APIC_CUBIC)
        return fail(APIC_E_INVAL, "degree must be 1 (multilinear), 2 (quadratic) or 3 (cubic) (got %d)", g->degree);
    if (g->precision != APIC_F32 && g->precision != APIC_F64)
        return fail(APIC_E_INVAL, "precision must be APIC_F32 or APIC_F64 (got %d)", g->precision);
    if (g->options & ~(APIC_OPT_COMPENSATED | APIC_OPT_FUSED_TRANSFER | APIC_OPT_ADAPTIVE_DT |
                       APIC_OPT_ABSOLUTE_POSITIONS | APIC_OPT_BATCH_GRAPH))
        return fail(APIC_E_INVAL, "unknown option bits 0x%x", g->options);
    if (g->options & APIC_OPT_ABSOLUTE_POSITIONS) {
        if (g->precision != APIC_F32 || g->degree == APIC_MULTILINEAR)
            return fail(APIC_E_UNSUPPORTED, "absolute positions need binary32 and quadratic or cubic weights");
        if (g->options & APIC_OPT_ADAPTIVE_DT)
            return fail(APIC_E_UNSUPPORTED, "absolute positions are not offered with adaptive steps");
    }
    const int maxc = g->dim == 3 ? 1024 : 65535;
    for (int a = 0; a < g->dim; ++a)
        if (g->cells[a] < g->degree + 1 || g->cells[a] > maxc)
            return fail(APIC_E_INVAL, "cells[%d] = %d outside [%d, %d]", a, g->cells[a], g->degree + 1, maxc);
    if (!(g->dx > 0.0) || !isfinite(g->dx)) return fail(APIC_E_INVAL, "dx must be positive and finite");
    const Layout L = make_layout(g, 1);
    if (L.d.G >= (int64_t)0xFFFFFFFFu) return fail(APIC_E_INVAL, "grid too large");
    return APIC_OK;
}

// Grid, particle planes and parameters (not the workspace).
apic_status check_fields(const apic_scene *s) {
    if (!s) return fail(APIC_E_INVAL, "scene is NULL");
    apic_status rc = check_grid(&s->grid);
    if (rc != APIC_OK) return rc;
    const apic_particles &p = s->p;
    if (p.n < 0) return fail(APIC_E_INVAL, "particle count n = %lld is negative", (long long)p.n);
    const int64_t elem = s->grid.precision == APIC_F64 ? 8 : 4;
    if (p.n * elem >= ((int64_t)1 << 32))
        return fail(APIC_E_INVAL, "particle count %lld too large: n * element size must stay below 2^32 bytes",
                    (long long)p.n);
    if (p.n > 0) {
        if (p.stride < p.n) return fail(APIC_E_INVAL, "stride %lld < n %lld", (long long)p.stride, (long long)p.n);
        if (!p.cell || !p.off || !p.v || !p.B || !p.F || !p.mass)
            return fail(APIC_E_INVAL, "a particle plane pointer is NULL");
    }
    const apic_params &q = s->prm;
    if (!(q.dt >= 0.0) || !isfinite(q.dt)) return fail(APIC_E_INVAL, "dt must be finite and >= 0");
    for (int a = 0; a < 3; ++a)
        if (!isfinite(q.gravity[a])) return fail(APIC_E_INVAL, "gravity must be finite");
    if (q.model != APIC_MODEL_NONE && q.model != APIC_MODEL_NEO_HOOKEAN)
        return fail(APIC_E_INVAL, "unknown model %d", q.model);
    if (q.model == APIC_MODEL_NEO_HOOKEAN) {
        if (!(q.mu >= 0.0) || !isfinite(q.mu) || !isfinite(q.lambda))
            return fail(APIC_E_INVAL, "neo-Hookean mu must be >= 0 and lambda finite");
        if (!(q.rho0 > 0.0) || !isfinite(q.rho0)) return fail(APIC_E_INVAL, "rho0 must be positive");
    }
    for (int k = 0; k < 6; ++k)
        if (q.band[k] < 0) return fail(APIC_E_INVAL, "band widths must be >= 0");
    if (q.transfer != APIC_TRANSFER_APIC && q.transfer != APIC_TRANSFER_RPIC && q.transfer != APIC_TRANSFER_PIC)
        return fail(APIC_E_INVAL, "unknown transfer %d", q.transfer);
    if (s->grid.degree == APIC_MULTILINEAR && q.transfer != APIC_TRANSFER_APIC)
        return fail(APIC_E_UNSUPPORTED, "the multilinear kernel carries the lagged C of APIC only");
    if ((s->grid.options & APIC_OPT_ADAPTIVE_DT) && !(q.cfl > 0.0 && q.cfl <= 1.0))
        return fail(APIC_E_INVAL, "adaptive steps need a CFL number 0 < cfl <= 1");
    return APIC_OK;
}

apic_status check_scene(const apic_scene *s, int64_t *cap_out) {
    apic_status rc = check_fields(s);
    if (rc != APIC_OK) return rc;
    const apic_particles &p = s->p;
    if (!s->workspace) return fail(APIC_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)s->workspace) % kAlign) return fail(APIC_E_WORKSPACE, "workspace must be 256-byte aligned");
    const int64_t cap = capacity_for(&s->grid, s->workspace_bytes);
    if (cap < p.n || cap < 1)
        return fail(APIC_E_WORKSPACE, "workspace of %zu bytes holds %lld particles, %lld given (need %zu bytes)",
                    s->workspace_bytes, (long long)cap, (long long)p.n,
                    make_layout(&s->grid, p.n > 0 ? p.n : 1).total);
    *cap_out = cap;
    return APIC_OK;
}

// ---------------------------------------------------------------------------
// Host-side binning state per workspace.
// ---------------------------------------------------------------------------
struct SceneState {
    apic_grid_desc grid;
    size_t wbytes = 0;
    bool binned = false;     // the user's particle buffers follow layout `cur`
    int cur = 0;             // layout (list parity) of the particles
    int grid_meta = -1;      // layout the slabs (last apic_p2g) belong to
    bool vt_valid = false;   // grid velocities of layout grid_meta are current
    uint32_t gen[2] = {0u, 0u};  // generation of the last build per parity
    int64_t n = -1;
    void *cell = nullptr;
    int64_t stride = 0;
};

std::mutex g_mu;
std::unordered_map<void *, SceneState> g_states;

bool same_grid(const apic_grid_desc &a, const apic_grid_desc &b) { return memcmp(&a, &b, sizeof a) == 0; }

// c of the CFL quantity |v_p| + c |B_p|_F (Sec. 4.3): 6 sqrt(d) / dx for
// quadratic and cubic weights; sqrt(d) dx for the lagged C_p of the
// multilinear kernel, whose grid velocities v_p + C_p (x_i - x_p) have
// |x_i - x_p| <= sqrt(d) dx.
double cfl_factor(const apic_grid_desc &g) {
    const double sd = sqrt((double)g.dim);
    return g.degree == APIC_MULTILINEAR ? sd * g.dx : 6.0 * sd / g.dx;
}

apic_status hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(APIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return APIC_OK;
}

// ---------------------------------------------------------------------------
// Optional phase timing (apic_timing_enable / apic_timing_read)
// ---------------------------------------------------------------------------
struct Timing {
    std::mutex mu;
    bool enabled = false;
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Timing g_timing;

// Set while apic_step_noalloc runs on this thread: no timing events (their
// creation is left out of a call that promises no allocation).
thread_local bool g_untimed = false;

// Runs `launch` bracketed by timing events when timing is enabled.
template <typename F>
void timed(int phase, hipStream_t st, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        if (g_timing.enabled && !g_untimed) {
            a = g_timing.take();
            b = g_timing.take();
        }
    }
    if (a && b) (void)hipEventRecord(a, st);
    launch();
    if (a && b) {
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lock(g_timing.mu);
        g_timing.recs.push_back({phase, a, b});
    }
}

// Like timed(), for a launcher that takes the events itself and has the
// kernel dispatch stamp them (its start and end, not the stream's
// surroundings): launch(a, b), a and b null when timing is off.
template <typename F>
void timed_kernel(int phase, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        if (g_timing.enabled && !g_untimed) {
            a = g_timing.take();
            b = g_timing.take();
            if (!a || !b) a = b = nullptr;
        }
    }
    launch(a, b);
    if (a && b) {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        g_timing.recs.push_back({phase, a, b});
    }
}

// Drops the last `count` timing records of `phase` (launches that did no
// work), returning their events to the pool.
void untime_last(int phase, int count) {
    if (count <= 0) return;
    std::lock_guard<std::mutex> lock(g_timing.mu);
    auto &recs = g_timing.recs;
    for (size_t i = recs.size(); i > 0 && count > 0; --i) {
        if (recs[i - 1].phase != phase) continue;
        g_timing.pool.push_back(recs[i - 1].a);
        g_timing.pool.push_back(recs[i - 1].b);
        recs.erase(recs.begin() + (i - 1));
        --count;
    }
}

// ---------------------------------------------------------------------------
// Typed views of one scene
// ---------------------------------------------------------------------------
template <typename T>
struct View {
    Layout L;
    Parts<T> user, shadow;
    BinLists lists[2];
    TileTables tab[2];
    BinScratch sc;
    Slabs<T> slabs;
    GridState<T> g;
    StepParams<T> prm;
    double *diag_part, *diag_out;
};

template <typename T>
View<T> make_view(const apic_scene *s, int64_t cap, const SceneState &ss) {
    View<T> v;
    v.L = make_layout(&s->grid, cap);
    const Layout &L = v.L;
    char *w = (char *)s->workspace;
    v.user.cell = s->p.cell;
    v.user.off = (T *)s->p.off;
    v.user.v = (T *)s->p.v;
    v.user.B = (T *)s->p.B;
    v.user.F = (T *)s->p.F;
    v.user.m = (T *)s->p.mass;
    v.user.id = s->p.id;
    v.user.n = s->p.n;
    v.user.s = s->p.stride;
    const int64_t dim = L.d.dim, cp = L.sst;
    v.shadow.cell = (uint32_t *)(w + L.o_sh_cell);
    v.shadow.id = s->p.id ? (int32_t *)(w + L.o_sh_id) : nullptr;
    T *f = (T *)(w + L.o_sh_f);
    v.shadow.off = f;
    v.shadow.v = f + dim * cp;
    v.shadow.B = f + 2 * dim * cp;
    v.shadow.F = f + (2 * dim + dim * dim) * cp;
    v.shadow.m = f + (2 * dim + 2 * dim * dim) * cp;
    v.shadow.n = s->p.n;
    v.shadow.s = cp;
    for (int k = 0; k < 2; ++k) {
        const ListOff &o = L.lists[k];
        BinLists &b = v.lists[k];
        b.gen = ss.gen[k];
        b.tile_gen = (uint32_t *)(w + o.tile_gen);
        b.slot = (uint32_t *)(w + o.slot);
        b.rec_count = (uint32_t *)(w + o.rec_count);
        b.nfull = (uint32_t *)(w + o.nfull);
        b.nsparse = (uint32_t *)(w + o.nsparse);
        b.rec_list = (uint32_t *)(w + o.rec_list);
        b.rec_tile = (uint32_t *)(w + o.rec_tile);
        b.tot = (uint32_t *)(w + o.tot);
        b.rpre = (uint32_t *)(w + o.rpre);
        b.bpre = (uint32_t *)(w + o.bpre);
        b.ctr = (uint32_t *)(w + o.ctr);
        b.rcap = L.rcap;
    }
    for (int k = 0; k < 2; ++k) {
        const TabOff &o = L.tabs[k];
        TileTables &t = v.tab[k];
        t.kcount = (uint32_t *)(w + o.kcount);
        t.kmov = (uint32_t *)(w + o.kmov);
        t.kprefix = (uint32_t *)(w + o.kprefix);
        t.maxc = (uint32_t *)(w + o.maxc);
        t.tcount = (uint32_t *)(w + o.tcount);
        t.off = (uint32_t *)(w + o.off);
        t.lvl_off = (uint32_t *)(w + o.lvl_off);
        t.lvl_mask = (uint64_t *)(w + o.lvl_mask);
    }
    v.sc.key_count = (uint32_t *)(w + L.o_key_count);
    v.sc.scount = (uint32_t *)(w + L.o_scount);
    v.sc.pkey = (uint32_t *)(w + L.o_pkey);
    v.sc.prank = (uint32_t *)(w + L.o_prank);
    v.sc.next = (uint32_t *)(w + L.o_next);
    v.sc.pord = (uint64_t *)(w + L.o_pord);
    v.sc.head = (uint32_t *)(w + L.o_head);
    v.slabs.v = (T *)(w + L.o_slabs);
    v.slabs.stride = L.slab_stride;
    v.g.vt = (T *)(w + L.o_vt);
    v.g.uref = (T *)(w + L.o_uref);
    v.g.flags = (uint32_t *)(w + L.o_flags);
    v.g.vmax = (uint32_t *)(w + L.o_vmax);
    v.g.cfl = nullptr;
    v.g.cfl_c = cfl_factor(s->grid);
    v.g.d = L.d;
    v.g.dx = (T)s->grid.dx;
    v.g.inv_dx = (T)(1.0 / s->grid.dx);
    v.prm.dt = (T)s->prm.dt;
    for (int a = 0; a < 3; ++a) v.prm.g[a] = (T)s->prm.gravity[a];
    v.prm.model = s->prm.model;
    v.prm.transfer = s->prm.transfer;
    for (int k = 0; k < 6; ++k) v.prm.band[k] = s->prm.band[k];
    v.prm.mu = (T)s->prm.mu;
    v.prm.lam = (T)s->prm.lambda;
    v.prm.inv_rho0 = s->prm.rho0 > 0.0 ? (T)(1.0 / s->prm.rho0) : T(0);
    v.prm.dt_dev = nullptr;
    v.diag_part = (double *)(w + L.o_diag_part);
    v.diag_out = (double *)(w + L.o_diag_out);
    return v;
}

// Next generation of list parity `k` before a layout is built in it.  On
// wrap-around the parity's tags are cleared so no stale tag can match.
template <typename T>
void begin_build(View<T> &v, SceneState &ss, int k, hipStream_t st) {
    if (ss.gen[k] == 0xFFFFFFFFu) {
        launch_fill<uint32_t>(v.lists[k].tile_gen, v.L.d.tiles, 0u, st);
        ss.gen[k] = 0u;
    }
    ss.gen[k] += 1u;
    v.lists[k].gen = ss.gen[k];
}

// Device part of a reset: zero the fixed region (counters, tags, tables).
void device_reset(const apic_scene *s, int64_t cap, hipStream_t st) {
    const Layout L = make_layout(&s->grid, cap);
    launch_fill<uint32_t>((uint32_t *)s->workspace, (int64_t)(L.fixed_end / 4), 0u, st);
}

// Registry entry of the scene, created (and the workspace reset) on first
// use or when the grid or workspace size changed; `binned` is dropped when
// the particle buffers are not the ones last binned.
SceneState &state_of(const apic_scene *s, int64_t cap, hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_states.find(s->workspace);
    if (it == g_states.end() || !same_grid(it->second.grid, s->grid) || it->second.wbytes != s->workspace_bytes) {
        SceneState fresh;
        fresh.grid = s->grid;
        fresh.wbytes = s->workspace_bytes;
        g_states[s->workspace] = fresh;
        device_reset(s, cap, st);
        it = g_states.find(s->workspace);
    }
    SceneState &ss = it->second;
    if (ss.n != s->p.n || ss.cell != (void *)s->p.cell || ss.stride != s->p.stride) {
        ss.binned = false;
        ss.n = s->p.n;
        ss.cell = (void *)s->p.cell;
        ss.stride = s->p.stride;
    }
    return ss;
}

// ---------------------------------------------------------------------------
// Typed operations
// ---------------------------------------------------------------------------
enum class Op { Sort, P2G, GridUpdate, G2P, Export, DiagParticles, DiagEnergy, DiagGrid, Cfl, Pack, Unpack };

struct OpArgs {
    void *ptr;
    int which;
};

// Bins the particles of `src` (at their current positions) into list
// parity `nxt` and writes them, in the new order, to `dst`.
template <typename T, int DIM, int DEG, bool ABS = false>
void bin_static(View<T> &v, SceneState &ss, const Parts<T> &src, const Parts<T> &dst, int nxt, hipStream_t st) {
    begin_build(v, ss, nxt, st);
    launch_bin_reset(v.lists[nxt], st);
    launch_bin_keys_static<T, DIM, DEG, ABS>(src, v.L.d, v.lists[nxt], v.sc, v.g.flags, v.g.inv_dx, st);
    launch_bin_records<DIM>(v.L.d, v.lists[nxt], v.tab[nxt], v.sc, v.L.rc, st);
    launch_bin_finalize(v.lists[nxt], v.L.rc, st);
    launch_bin_scatter_copy<T, DIM>(src, dst, v.lists[nxt], v.tab[nxt], v.sc, st);
}

// One G2P from `src` (layout `cur`) into `dst` (layout 1 - cur).  The
// counters of the new layout were zeroed by the preceding P2G; `reset`
// zeroes them again (calls outside a whole step).
template <typename T, int DIM, int DEG, bool ABS = false>
void g2p_rebin(View<T> &v, SceneState &ss, const Parts<T> &src, const Parts<T> &dst, int cur, bool reset,
               hipStream_t st) {
    const int nxt = 1 - cur;
    begin_build(v, ss, nxt, st);
    timed(APIC_PHASE_BIN, st, [&] {
        if (reset) launch_bin_reset(v.lists[nxt], st);
        launch_bin_keys_moved<T, DIM, DEG, ABS>(src, v.lists[cur], v.tab[cur], v.g, v.prm, v.lists[nxt], v.sc,
                                                v.L.rc, st);
        launch_bin_records<DIM>(v.L.d, v.lists[nxt], v.tab[nxt], v.sc, v.L.rc, st);
        launch_bin_finalize(v.lists[nxt], v.L.rc, st);
    });
    timed(APIC_PHASE_G2P, st, [&] {
        launch_g2p<T, DIM, DEG, ABS>(src, dst, v.lists[cur], v.tab[cur], v.lists[nxt], v.tab[nxt], v.sc, v.g, v.prm,
                                     v.L.rc, st);
    });
}

// G2P fused with the next step's P2G: binary32 quadratic 3D, where a lane
// holds every node sum of its key in registers.
template <typename T, int DIM, int DEG>
constexpr bool fused_step() {
    return std::is_same<T, float>::value && DIM == 3 && DEG == 2;
}

// As g2p_rebin, then the slabs of the new layout for the next step: the
// particles that kept their key in the fused pass, the others after it.
template <typename T, int DIM, int DEG, bool COMP>
void g2p2g_rebin(View<T> &v, SceneState &ss, const Parts<T> &src, const Parts<T> &dst, int cur, hipStream_t st) {
    const int nxt = 1 - cur;
    begin_build(v, ss, nxt, st);
    timed(APIC_PHASE_BIN, st, [&] {
        launch_bin_keys_moved<T, DIM, DEG>(src, v.lists[cur], v.tab[cur], v.g, v.prm, v.lists[nxt], v.sc, v.L.rc,
                                           st);
        launch_bin_records<DIM>(v.L.d, v.lists[nxt], v.tab[nxt], v.sc, v.L.rc, st);
        launch_bin_finalize(v.lists[nxt], v.L.rc, st);
    });
    if constexpr (fused_step<T, DIM, DEG>()) {
        timed(APIC_PHASE_G2P, st, [&] {
            launch_g2p2g<T, DEG, COMP>(src, dst, v.lists[cur], v.tab[cur], v.lists[nxt], v.tab[nxt], v.sc, v.slabs,
                                       v.g, v.prm, v.L.rc, st);
        });
        timed(APIC_PHASE_P2G, st, [&] {
            launch_p2g_movers<T, DEG, COMP>(dst, v.lists[cur], v.lists[nxt], v.tab[nxt], v.slabs, v.g, v.prm,
                                            v.L.rc, st);
        });
    }
}

template <typename T, int DIM, int DEG, bool COMP, bool ABS>
apic_status run(Op op, const apic_scene *s, int64_t cap, hipStream_t st, const OpArgs &a) {
    SceneState &ss = state_of(s, cap, st);
    View<T> v = make_view<T>(s, cap, ss);
    switch (op) {
        case Op::Sort: {
            const int nxt = 1 - ss.cur;
            bin_static<T, DIM, DEG, ABS>(v, ss, v.user, v.shadow, nxt, st);
            launch_copy_state<T, DIM>(v.shadow, v.user, st);
            ss.cur = nxt;
            ss.binned = true;
            if (ss.grid_meta == nxt) ss.grid_meta = -1;
            ss.vt_valid = false;
            break;
        }
        case Op::P2G: {
            if (!ss.binned) {
                apic_status rc = run<T, DIM, DEG, COMP, ABS>(Op::Sort, s, cap, st, a);
                if (rc != APIC_OK) return rc;
                v = make_view<T>(s, cap, ss);
            }
            launch_keep_affine<T, DIM>(v.user, s->prm.transfer, st);
            launch_p2g<T, DIM, DEG, COMP, ABS>(v.user, v.lists[ss.cur], v.lists[1 - ss.cur], v.tab[ss.cur], v.slabs, v.g,
                                          v.prm, v.L.rc, st);
            ss.grid_meta = ss.cur;
            ss.vt_valid = false;
            break;
        }
        case Op::GridUpdate:
            if (ss.grid_meta < 0 || ss.grid_meta != ss.cur || !ss.binned)
                return fail(APIC_E_INVAL, "apic_grid_update needs a preceding apic_p2g on the current particles");
            launch_grid_update<T, DIM, DEG, COMP>(v.lists[ss.grid_meta], v.slabs, v.g, v.prm, v.L.rc, st);
            ss.vt_valid = true;
            break;
        case Op::G2P:
            if (!ss.vt_valid || !ss.binned || ss.grid_meta != ss.cur)
                return fail(APIC_E_INVAL, "apic_g2p needs apic_p2g and apic_grid_update on the current particles");
            g2p_rebin<T, DIM, DEG, ABS>(v, ss, v.user, v.shadow, ss.cur, true, st);
            launch_copy_state<T, DIM>(v.shadow, v.user, st);
            ss.cur = 1 - ss.cur;
            ss.vt_valid = false;
            break;
        case Op::Export:
            if (ss.grid_meta < 0) return fail(APIC_E_INVAL, "no grid yet: call apic_p2g first");
            launch_grid_export<T, DIM, DEG, COMP>(v.lists[ss.grid_meta], v.slabs, v.g, a.which, (T *)a.ptr, st);
            break;
        case Op::DiagParticles:
            launch_diag_particles<T, DIM>(v.user, s->grid.dx, s->grid.degree != APIC_MULTILINEAR, v.diag_part,
                                          v.diag_out, st, ABS);
            break;
        case Op::DiagEnergy:
            launch_diag_energy<T, DIM>(v.user, s->prm.model, s->prm.mu, s->prm.lambda, s->prm.rho0, v.diag_part,
                                       v.diag_out, st);
            break;
        case Op::Cfl:
            launch_cfl_bound<T, DIM>(v.user, cfl_factor(s->grid), v.diag_part, v.diag_out, st);
            break;
        case Op::DiagGrid:
            if (ss.grid_meta < 0) return fail(APIC_E_INVAL, "no grid yet: call apic_p2g first");
            launch_diag_grid<T, DIM, DEG, COMP>(v.lists[ss.grid_meta], v.slabs, v.g, a.which, s->prm.dt, v.diag_part,
                                                v.diag_out, st);
            break;
        case Op::Pack:
            launch_pack_positions<T, DIM>(v.user, (const double *)a.ptr, s->grid.dx, st, ABS);
            ss.binned = false;
            break;
        case Op::Unpack:
            launch_unpack_positions<T, DIM>(v.user, (double *)a.ptr, s->grid.dx, st, ABS);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APIC_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return APIC_OK;
}

// Whole steps for one scene with the particle state alternating between the
// caller's buffers and the workspace shadow; ends in the caller's buffers.
template <typename T, int DIM, int DEG, bool COMP, bool ABS>
apic_status run_steps(apic_scene *s, int64_t cap, int32_t n_steps, int32_t sort_every, hipStream_t st) {
    SceneState &ss = state_of(s, cap, st);
    View<T> v = make_view<T>(s, cap, ss);
    Parts<T> bufs[2] = {v.user, v.shadow};
    int where = 0;
    if (!ss.binned) {
        timed(APIC_PHASE_SORT, st, [&] { bin_static<T, DIM, DEG, ABS>(v, ss, v.user, v.shadow, 1 - ss.cur, st); });
        ss.cur = 1 - ss.cur;
        where = 1;
    }
    // adaptive steps: dt chosen on the device before each step's P2G from the
    // bound of the state it starts from (a pass over the particles for the
    // first step, the bound the previous transfer to particles folded in
    // for the others)
    const bool adaptive = (s->grid.options & APIC_OPT_ADAPTIVE_DT) != 0;
    char *w = (char *)s->workspace;
    unsigned long long *cfl_slots = (unsigned long long *)(w + v.L.o_cfl);
    double *dt_state = (double *)(w + v.L.o_dt);
    if (adaptive) {
        v.g.cfl = cfl_slots;
        v.prm.dt_dev = dt_state;
    }
    const double nu_dx = s->prm.cfl * s->grid.dx;
    launch_keep_affine<T, DIM>(bufs[where], s->prm.transfer, st);
    bool slabs_ready = false;  // the slabs already hold this step's P2G
    for (int32_t k = 0; k < n_steps; ++k) {
        if (sort_every > 0 && k > 0 && k % sort_every == 0) {
            timed(APIC_PHASE_SORT, st,
                  [&] { bin_static<T, DIM, DEG, ABS>(v, ss, bufs[where], bufs[1 - where], 1 - ss.cur, st); });
            ss.cur = 1 - ss.cur;
            where = 1 - where;
            slabs_ready = false;
        }
        if (adaptive) {
            if (k == 0) {
                const int nb = launch_cfl_partials<T, DIM>(bufs[where], cfl_factor(s->grid), v.diag_part, st);
                launch_adapt_dt(v.diag_part, nb, cfl_slots, s->prm.dt, nu_dx, dt_state, st);
            } else {
                launch_adapt_dt((const double *)cfl_slots, kVmaxSlots, cfl_slots, s->prm.dt, nu_dx, dt_state, st);
            }
        }
        if (!slabs_ready) {
            timed(APIC_PHASE_P2G, st, [&] {
                launch_p2g<T, DIM, DEG, COMP, ABS>(bufs[where], v.lists[ss.cur], v.lists[1 - ss.cur], v.tab[ss.cur],
                                              v.slabs, v.g, v.prm, v.L.rc, st);
            });
        }
        timed(APIC_PHASE_GRID_UPDATE, st, [&] {
            launch_grid_update<T, DIM, DEG, COMP>(v.lists[ss.cur], v.slabs, v.g, v.prm, v.L.rc, st);
        });
        ss.grid_meta = ss.cur;
        // the last step of the call leaves the slabs of the step it made
        const bool fuse = fused_step<T, DIM, DEG>() && !ABS && (s->grid.options & APIC_OPT_FUSED_TRANSFER) && !adaptive &&
                          k + 1 < n_steps && !(sort_every > 0 && (k + 1) % sort_every == 0);
        if (fuse)
            g2p2g_rebin<T, DIM, DEG, COMP>(v, ss, bufs[where], bufs[1 - where], ss.cur, st);
        else
            g2p_rebin<T, DIM, DEG, ABS>(v, ss, bufs[where], bufs[1 - where], ss.cur, false, st);
        slabs_ready = fuse;
        ss.cur = 1 - ss.cur;
        where = 1 - where;
    }
    if (where == 1) launch_copy_state<T, DIM>(v.shadow, v.user, st);
    ss.binned = true;
    ss.vt_valid = false;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APIC_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return APIC_OK;
}

// Absolute binary32 positions exist for binary32 quadratic and cubic weights
// (checked on the host before any launch).
template <typename T, int DEG>
constexpr bool abs_supported() {
    return std::is_same<T, float>::value && DEG >= 2;
}

template <typename T, int DIM, int DEG>
apic_status run_c(Op op, const apic_scene *s, int64_t cap, hipStream_t st, const OpArgs &a) {
    const bool comp = (s->grid.options & APIC_OPT_COMPENSATED) != 0;
    if (s->grid.options & APIC_OPT_ABSOLUTE_POSITIONS) {
        if constexpr (abs_supported<T, DEG>())
            return comp ? run<T, DIM, DEG, true, true>(op, s, cap, st, a) : run<T, DIM, DEG, false, true>(op, s, cap, st, a);
        return fail(APIC_E_UNSUPPORTED, "absolute positions need binary32 and quadratic or cubic weights");
    }
    return comp ? run<T, DIM, DEG, true, false>(op, s, cap, st, a) : run<T, DIM, DEG, false, false>(op, s, cap, st, a);
}
// f(std::integral_constant<int, DEG>) for the grid's B-spline degree.
template <typename F>
apic_status by_degree(int degree, F &&f) {
    switch (degree) {
        case APIC_MULTILINEAR: return f(std::integral_constant<int, 1>{});
        case APIC_CUBIC: return f(std::integral_constant<int, 3>{});
        default: return f(std::integral_constant<int, 2>{});
    }
}

template <typename T, int DIM>
apic_status run_k(Op op, const apic_scene *s, int64_t cap, hipStream_t st, const OpArgs &a) {
    return by_degree(s->grid.degree, [&](auto d) { return run_c<T, DIM, decltype(d)::value>(op, s, cap, st, a); });
}
template <typename T>
apic_status run_d(Op op, const apic_scene *s, int64_t cap, hipStream_t st, const OpArgs &a) {
    if (s->grid.dim == 3) return run_k<T, 3>(op, s, cap, st, a);
    return run_k<T, 2>(op, s, cap, st, a);
}

apic_status dispatch(Op op, const apic_scene *s, void *stream, const OpArgs &a = OpArgs{nullptr, 0}) {
    int64_t cap = 0;
    apic_status rc = check_scene(s, &cap);
    if (rc != APIC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (s->grid.precision == APIC_F64) return run_d<double>(op, s, cap, st, a);
    return run_d<float>(op, s, cap, st, a);
}

template <typename T, int DIM, int DEG>
apic_status steps_c(apic_scene *s, int64_t cap, int32_t n, int32_t k, hipStream_t st) {
    const bool comp = (s->grid.options & APIC_OPT_COMPENSATED) != 0;
    if (s->grid.options & APIC_OPT_ABSOLUTE_POSITIONS) {
        if constexpr (abs_supported<T, DEG>())
            return comp ? run_steps<T, DIM, DEG, true, true>(s, cap, n, k, st)
                        : run_steps<T, DIM, DEG, false, true>(s, cap, n, k, st);
        return fail(APIC_E_UNSUPPORTED, "absolute positions need binary32 and quadratic or cubic weights");
    }
    return comp ? run_steps<T, DIM, DEG, true, false>(s, cap, n, k, st)
                : run_steps<T, DIM, DEG, false, false>(s, cap, n, k, st);
}

template <typename T, int DIM>
apic_status steps_k(apic_scene *s, int64_t cap, int32_t n, int32_t k, hipStream_t st) {
    return by_degree(s->grid.degree,
                     [&](auto d) { return steps_c<T, DIM, decltype(d)::value>(s, cap, n, k, st); });
}

apic_status dispatch_steps(apic_scene *s, int64_t cap, int32_t n, int32_t k, hipStream_t st) {
    const bool f64 = s->grid.precision == APIC_F64, d3 = s->grid.dim == 3;
    if (f64) return d3 ? steps_k<double, 3>(s, cap, n, k, st) : steps_k<double, 2>(s, cap, n, k, st);
    return d3 ? steps_k<float, 3>(s, cap, n, k, st) : steps_k<float, 2>(s, cap, n, k, st);
}

// ---------------------------------------------------------------------------
// Batched steps (apic_step_batch)
// ---------------------------------------------------------------------------
constexpr size_t kDescBytes = (sizeof(SceneDesc<double>) + 15) / 16 * 16;

// The scene table (descriptors, then the per-kind item starts), then the
// queue counter of persistent launches.
size_t batch_table_bytes(int32_t n) {
    return align_up((size_t)n * kDescBytes) + align_up((size_t)BK_COUNT * (size_t)(n + 1) * 4);
}

size_t batch_bytes(int32_t n) { return batch_table_bytes(n) + align_up(sizeof(uint32_t)); }

// Host staging of the scene table, per batch workspace; `done` guards reuse.
struct BatchHost {
    void *pinned = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
std::unordered_map<void *, BatchHost> g_batch;
std::mutex g_batch_mu;

// --- launch plans ---------------------------------------------------------------
struct BatchPlan {
    int32_t per_block;      // particles per block of a scene's share
    int32_t blocks_per_cu;  // 0: one block per item; else a persistent launch of this many blocks per CU
};
constexpr BatchPlan kBatchPlans[] = {{1024, 0}, {512, 0}, {2048, 0}, {1024, 4}, {512, 8}};
constexpr int kBatchPlanCount = (int)(sizeof(kBatchPlans) / sizeof(kBatchPlans[0]));
constexpr int kTuneRounds = 2;
int g_forced_plan = -1;

// Blocks of one scene's share of a batched launch, by particle count (the
// kernels stride over any remainder).
int share_blocks(int64_t n, int per_block, int cap) {
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

int octave(int64_t v) {
    int o = 0;
    while (v > 1) {
        v >>= 1;
        ++o;
    }
    return o;
}

// Tuning state per (precision, dim, degree, options, scene-count octave,
// particle-count octave).
using TuneKey = std::tuple<int, int, int, int, int, int>;
struct TuneState {
    double best_ns[kBatchPlanCount];
    int rounds[kBatchPlanCount] = {};
    int chosen = -1;
    bool pending = false;  // a timed call whose events are not read yet
    int plan = 0;
    double updates = 0.0;  // particle-steps of the timed call
    hipEvent_t a = nullptr, b = nullptr;
    TuneState() {
        for (double &v : best_ns) v = INFINITY;
    }
};
std::map<TuneKey, TuneState> g_tune;

TuneKey tune_key(const apic_scene *s, int32_t n) {
    int64_t np = 0;
    for (int32_t i = 0; i < n; ++i) np += s[i].p.n;
    const apic_grid_desc &g = s[0].grid;
    return TuneKey{g.precision, g.dim, g.degree, g.options & ~APIC_OPT_BATCH_GRAPH, octave(n), octave(np)};
}

// Reads a finished measurement into the state.
apic_status tune_collect(TuneState &ts) {
    if (!ts.pending) return APIC_OK;
    apic_status rc = hip_check(hipEventSynchronize(ts.b), "apic_step_batch tuning");
    float ms = 0.f;
    if (rc == APIC_OK) rc = hip_check(hipEventElapsedTime(&ms, ts.a, ts.b), "apic_step_batch tuning");
    ts.pending = false;
    if (rc != APIC_OK) return rc;
    const double ns = ts.updates > 0.0 ? (double)ms * 1e6 / ts.updates : INFINITY;
    ts.best_ns[ts.plan] = std::min(ts.best_ns[ts.plan], ns);
    ts.rounds[ts.plan] += 1;
    return APIC_OK;
}

// Plan of the next call: the tuned one, else the next plan to time.
int tune_next(TuneState &ts) {
    if (ts.chosen >= 0) return ts.chosen;
    for (int r = 0; r < kTuneRounds; ++r)
        for (int p = 0; p < kBatchPlanCount; ++p)
            if (ts.rounds[p] <= r) return p;
    int best = 0;
    for (int p = 1; p < kBatchPlanCount; ++p)
        if (ts.best_ns[p] < ts.best_ns[best]) best = p;
    ts.chosen = best;
    return best;
}

int device_cus() {
    static std::mutex mu;
    static std::unordered_map<int, int> cus;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev] = c;
    return c;
}

// --- graphs of batched calls ------------------------------------------------------
struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
std::unordered_map<std::string, BatchGraph> g_graphs;
constexpr size_t kMaxGraphs = 64;

// Stream the launch sequences are captured on (one per device, default
// priority; the graphs are launched on the caller's stream).
hipStream_t capture_stream() {
    static std::mutex mu;
    static std::unordered_map<int, hipStream_t> streams;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = s;
    return s;
}

void drop_graphs() {
    for (auto &kv : g_graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
}

template <typename V>
void key_put(std::string &k, const V &v) {
    k.append((const char *)&v, sizeof v);
}

template <typename T, int DIM, int DEG, bool COMP>
apic_status run_batch(apic_scene *scenes, int32_t n, int32_t n_steps, void *bws, hipStream_t st) {
    const bool adaptive = (scenes[0].grid.options & APIC_OPT_ADAPTIVE_DT) != 0;
    const TuneKey tkey = tune_key(scenes, n);
    TuneState &ts = g_tune[tkey];
    apic_status rc0 = tune_collect(ts);
    if (rc0 != APIC_OK) return rc0;
    const bool tuning = g_forced_plan < 0 && ts.chosen < 0 && n_steps > 0;
    const int plan_id = g_forced_plan >= 0 ? g_forced_plan : tune_next(ts);
    const BatchPlan plan = kBatchPlans[plan_id];
    std::vector<SceneDesc<T>> descs((size_t)n);
    std::vector<int32_t> starts((size_t)BK_COUNT * (size_t)(n + 1));
    std::vector<SceneState *> states((size_t)n);
    int32_t total[BK_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    double updates = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t cap = 0;
        (void)check_scene(&scenes[i], &cap);
        SceneState &ss = state_of(&scenes[i], cap, st);
        // generations of both parities must not wrap within the call
        for (int p = 0; p < 2; ++p)
            if (ss.gen[p] > 0xFFFFFFFFu - (uint32_t)n_steps - 2u) {
                View<T> v = make_view<T>(&scenes[i], cap, ss);
                launch_fill<uint32_t>(v.lists[p].tile_gen, v.L.d.tiles, 0u, st);
                ss.gen[p] = 0u;
                if (p == ss.cur) ss.binned = false;   // its tags are gone: bin again
                if (p == ss.grid_meta) ss.grid_meta = -1;
            }
        View<T> v = make_view<T>(&scenes[i], cap, ss);
        int where = 0;
        if (!ss.binned) {
            timed(APIC_PHASE_SORT, st, [&] { bin_static<T, DIM, DEG>(v, ss, v.user, v.shadow, 1 - ss.cur, st); });
            ss.cur = 1 - ss.cur;
            ss.binned = true;
            where = 1;
        }
        launch_keep_affine<T, DIM>(where ? v.shadow : v.user, scenes[i].prm.transfer, st);
        SceneDesc<T> &d = descs[(size_t)i];
        d.bufs[0] = v.user;
        d.bufs[1] = v.shadow;
        if (!v.user.id || !v.shadow.id) d.bufs[0].id = d.bufs[1].id = nullptr;
        for (int p = 0; p < 2; ++p) {
            d.lists[p] = v.lists[p];
            d.lists[p].gen = ss.gen[p];
            d.tab[p] = v.tab[p];
        }
        d.sc = v.sc;
        d.slabs = v.slabs;
        d.g = v.g;
        d.prm = v.prm;
        d.rc = v.L.rc;
        d.cur0 = ss.cur;
        d.where0 = where;
        d.dt_cap = scenes[i].prm.dt;
        d.nu_dx = scenes[i].prm.cfl * scenes[i].grid.dx;
        if (adaptive) {
            char *w = (char *)scenes[i].workspace;
            d.g.cfl = (unsigned long long *)(w + v.L.o_cfl);
            d.prm.dt_dev = (const double *)(w + v.L.o_dt);
        }
        states[(size_t)i] = &ss;
        const int64_t np = scenes[i].p.n;
        updates += (double)np * (double)n_steps;
        const int pb = plan.per_block;
        const int share[BK_COUNT] = {share_blocks(np, pb, 4096), share_blocks(np, pb, 8192), share_blocks(np, pb, 2048),
                                     share_blocks(np, pb, 1024), share_blocks(np, pb, 4096), share_blocks(np, 1024, 4096),
                                     // finalize: one block per ~65k particles (a few hundred records)
                                     share_blocks(np, 65536, 128)};
        for (int k = 0; k < BK_COUNT; ++k) {
            starts[(size_t)k * (n + 1) + i] = total[k];
            total[k] += share[k];
        }
    }
    for (int k = 0; k < BK_COUNT; ++k) starts[(size_t)k * (n + 1) + n] = total[k];

    // scene table: host staging (pinned, reused once its last copy is done)
    BatchHost &bh = g_batch[bws];
    const size_t need = batch_bytes(n);
    if (bh.pending) {
        apic_status rc = hip_check(hipEventSynchronize(bh.done), "apic_step_batch staging");
        if (rc != APIC_OK) return rc;
        bh.pending = false;
    }
    if (bh.bytes < need) {
        if (bh.pinned) (void)hipHostFree(bh.pinned);
        bh.pinned = nullptr;
        bh.bytes = 0;
        apic_status rc = hip_check(hipHostMalloc(&bh.pinned, need, hipHostMallocDefault), "apic_step_batch staging");
        if (rc != APIC_OK) return rc;
        bh.bytes = need;
    }
    if (!bh.done) {
        apic_status rc = hip_check(hipEventCreateWithFlags(&bh.done, hipEventDisableTiming), "apic_step_batch event");
        if (rc != APIC_OK) return rc;
    }
    char *host = (char *)bh.pinned;
    memcpy(host, descs.data(), (size_t)n * sizeof(SceneDesc<T>));
    const size_t o_start = align_up((size_t)n * kDescBytes);
    memcpy(host + o_start, starts.data(), starts.size() * 4);
    // descriptors are packed at sizeof(SceneDesc<T>) (<= kDescBytes per entry)
    apic_status rc = hip_check(hipMemcpyAsync(bws, host, batch_table_bytes(n), hipMemcpyHostToDevice, st),
                               "apic_step_batch table");
    if (rc != APIC_OK) return rc;
    rc = hip_check(hipEventRecord(bh.done, st), "apic_step_batch event");
    if (rc != APIC_OK) return rc;
    bh.pending = true;

    const SceneDesc<T> *dd = (const SceneDesc<T> *)bws;
    const int32_t *ds = (const int32_t *)((const char *)bws + o_start);
    uint32_t *ctr = (uint32_t *)((char *)bws + batch_table_bytes(n));
    auto start_of = [&](int k) { return ds + (size_t)k * (n + 1); };
    const int qblocks = plan.blocks_per_cu * device_cus();
    // the launches of the call's steps on stream s
    auto emit = [&](hipStream_t s) {
        uint32_t base = 0;
        // how the blocks of a launch of kind `kind` take its items
        auto queue_of = [&](int kind, int &blocks) {
            BatchQueue q{nullptr, 0u, (uint32_t)total[kind]};
            blocks = total[kind];
            if (plan.blocks_per_cu > 0) {
                blocks = std::min(total[kind], qblocks);
                q.ctr = ctr;
                q.base = base;
                base += (uint32_t)total[kind] + (uint32_t)blocks;
            }
            return q;
        };
        if (plan.blocks_per_cu > 0 && n_steps > 0) launch_fill<uint32_t>(ctr, 1, 0u, s);
        for (int32_t k = 0; k < n_steps; ++k) {
            int nb = 0;
            if (adaptive) launch_adapt_dt_batch<T, DIM>(dd, start_of(BK_COPY), n, total[BK_COPY], k == 0, s);
            BatchQueue q = queue_of(BK_P2G, nb);
            timed(APIC_PHASE_P2G, s, [&] { launch_p2g_batch<T, DIM, DEG, COMP>(dd, start_of(BK_P2G), n, k, q, nb, s); });
            q = queue_of(BK_GRID, nb);
            timed(APIC_PHASE_GRID_UPDATE, s,
                  [&] { launch_grid_update_batch<T, DIM, DEG, COMP>(dd, start_of(BK_GRID), n, k, q, nb, s); });
            timed(APIC_PHASE_BIN, s, [&] {
                int nk = 0, nr = 0;
                const BatchQueue qk = queue_of(BK_KEYS, nk);
                launch_bin_keys_moved_batch<T, DIM, DEG>(dd, start_of(BK_KEYS), n, k, qk, nk, s);
                const BatchQueue qr = queue_of(BK_RECORDS, nr);
                launch_bin_records_batch<T, DIM>(dd, start_of(BK_RECORDS), n, k, qr, nr, s);
                launch_bin_finalize_batch<T>(dd, start_of(BK_FINAL), n, k, total[BK_FINAL], s);
            });
            q = queue_of(BK_G2P, nb);
            timed(APIC_PHASE_G2P, s,
                  [&] { launch_g2p_batch<T, DIM, DEG>(dd, start_of(BK_G2P), n, k, q, nb, adaptive, s); });
        }
        launch_copy_back_batch<T, DIM>(dd, start_of(BK_COPY), n, n_steps, total[BK_COPY], s);
    };

    if (tuning) {
        if (!ts.a) rc = hip_check(hipEventCreate(&ts.a), "apic_step_batch tuning");
        if (rc == APIC_OK && !ts.b) rc = hip_check(hipEventCreate(&ts.b), "apic_step_batch tuning");
        if (rc == APIC_OK) rc = hip_check(hipEventRecord(ts.a, st), "apic_step_batch tuning");
        if (rc != APIC_OK) return rc;
    }
    bool timing = false;
    {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        timing = g_timing.enabled;
    }
    if ((scenes[0].grid.options & APIC_OPT_BATCH_GRAPH) && !timing && n_steps > 0) {
        // the graph of this scene set, step count and plan: every kernel
        // argument is fixed by them (the table behind `bws` is written above)
        std::string key;
        int dev = 0;
        (void)hipGetDevice(&dev);
        key_put(key, dev);
        key_put(key, bws);
        key_put(key, n);
        key_put(key, n_steps);
        key_put(key, plan_id);
        key_put(key, (int)sizeof(T));
        key_put(key, DIM * 100 + DEG * 10 + (COMP ? 1 : 0));
        key_put(key, (int)adaptive);
        key_put(key, qblocks);
        key.append((const char *)starts.data(), starts.size() * 4);
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            if (g_graphs.size() >= kMaxGraphs) drop_graphs();
            hipStream_t cs = capture_stream();
            if (!cs) return fail(APIC_E_HIP, "apic_step_batch: no capture stream");
            BatchGraph bg;
            rc = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "apic_step_batch capture");
            if (rc != APIC_OK) return rc;
            emit(cs);
            rc = hip_check(hipStreamEndCapture(cs, &bg.graph), "apic_step_batch capture");
            if (rc == APIC_OK) rc = hip_check(hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0),
                                              "apic_step_batch graph");
            if (rc != APIC_OK) {
                if (bg.graph) (void)hipGraphDestroy(bg.graph);
                return rc;
            }
            it = g_graphs.emplace(key, bg).first;
        }
        rc = hip_check(hipGraphLaunch(it->second.exec, st), "apic_step_batch graph launch");
        if (rc != APIC_OK) return rc;
    } else {
        emit(st);
    }
    if (tuning) {
        rc = hip_check(hipEventRecord(ts.b, st), "apic_step_batch tuning");
        if (rc != APIC_OK) return rc;
        ts.pending = true;
        ts.plan = plan_id;
        ts.updates = updates;
    }
    for (int32_t i = 0; i < n; ++i) {
        SceneState &ss = *states[(size_t)i];
        const int cur0 = ss.cur;
        // builds of this call: step k builds parity (cur0 + 1 + k) & 1
        ss.gen[(cur0 + 1) & 1] += (uint32_t)((n_steps + 1) / 2);
        ss.gen[cur0] += (uint32_t)(n_steps / 2);
        ss.cur = (cur0 + n_steps) & 1;
        if (n_steps > 0) ss.grid_meta = (cur0 + n_steps - 1) & 1;
        ss.binned = true;
        ss.vt_valid = false;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APIC_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return APIC_OK;
}

template <typename T, int DIM, int DEG>
apic_status batch_c(apic_scene *s, int32_t n, int32_t k, void *bws, hipStream_t st) {
    if (s[0].grid.options & APIC_OPT_COMPENSATED) return run_batch<T, DIM, DEG, true>(s, n, k, bws, st);
    return run_batch<T, DIM, DEG, false>(s, n, k, bws, st);
}

template <typename T, int DIM>
apic_status batch_k(apic_scene *s, int32_t n, int32_t k, void *bws, hipStream_t st) {
    return by_degree(s[0].grid.degree, [&](auto d) { return batch_c<T, DIM, decltype(d)::value>(s, n, k, bws, st); });
}

apic_status dispatch_batch(apic_scene *s, int32_t n, int32_t k, void *bws, hipStream_t st) {
    const bool f64 = s[0].grid.precision == APIC_F64, d3 = s[0].grid.dim == 3;
    if (f64) return d3 ? batch_k<double, 3>(s, n, k, bws, st) : batch_k<double, 2>(s, n, k, bws, st);
    return d3 ? batch_k<float, 3>(s, n, k, bws, st) : batch_k<float, 2>(s, n, k, bws, st);
}

}  // namespace

extern "C" {

apic_status apic_workspace_bytes(const apic_grid_desc *grid, int64_t max_particles, size_t *bytes) {
    apic_status rc = check_grid(grid);
    if (rc != APIC_OK) return rc;
    if (!bytes) return fail(APIC_E_INVAL, "bytes is NULL");
    if (max_particles < 0) return fail(APIC_E_INVAL, "max_particles is negative");
    *bytes = make_layout(grid, max_particles > 0 ? max_particles : 1).total;
    return APIC_OK;
}

apic_status apic_reset(apic_scene *scene, void *stream) {
    int64_t cap = 0;
    apic_status rc = check_scene(scene, &cap);
    if (rc != APIC_OK) return rc;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_states.erase(scene->workspace);
    }
    (void)state_of(scene, cap, (hipStream_t)stream);  // fresh entry, device reset
    return hip_check(hipGetLastError(), "apic_reset");
}

apic_status apic_sort(apic_scene *scene, void *stream) { return dispatch(Op::Sort, scene, stream); }

apic_status apic_p2g(apic_scene *scene, void *stream) { return dispatch(Op::P2G, scene, stream); }

apic_status apic_grid_update(apic_scene *scene, void *stream) { return dispatch(Op::GridUpdate, scene, stream); }

apic_status apic_g2p(apic_scene *scene, void *stream) { return dispatch(Op::G2P, scene, stream); }

apic_status apic_step(apic_scene *scenes, int32_t n_scenes, int32_t n_steps, int32_t sort_every, void *stream) {
    if (n_scenes < 0 || n_steps < 0 || sort_every < 0)
        return fail(APIC_E_INVAL, "n_scenes, n_steps and sort_every must be >= 0");
    if (n_scenes > 0 && !scenes) return fail(APIC_E_INVAL, "scenes is NULL");
    int64_t caps[1];
    for (int32_t k = 0; k < n_scenes; ++k) {
        apic_status rc = check_scene(&scenes[k], caps);
        if (rc != APIC_OK) return rc;
        for (int32_t j = 0; j < k; ++j)
            if (scenes[j].workspace == scenes[k].workspace)
                return fail(APIC_E_INVAL, "scenes %d and %d share a workspace", j, k);
    }
    for (int32_t k = 0; k < n_scenes; ++k) {
        int64_t cap = 0;
        (void)check_scene(&scenes[k], &cap);
        apic_status rc = dispatch_steps(&scenes[k], cap, n_steps, sort_every, (hipStream_t)stream);
        if (rc != APIC_OK) return rc;
    }
    return APIC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Steps without a caller workspace (apic_step_noalloc): the workspace is a
// file-scope device array of fixed size, one per GPU, whose address is taken
// once per device with hipGetSymbolAddress (in host code the array's name is
// not a device address).
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;            // also serializes the calls' host work
void *g_scratch_ptr[kMaxDevices] = {};

apic_status scratch_address(void **out) {
    int dev = 0;
    apic_status rc = hip_check(hipGetDevice(&dev), "apic_step_noalloc: hipGetDevice");
    if (rc != APIC_OK) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(APIC_E_UNSUPPORTED, "device index %d above %d", dev, kMaxDevices);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "apic_step_noalloc: hipGetSymbolAddress");
        if (rc != APIC_OK) return rc;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return APIC_OK;
}

}  // namespace

extern "C" {

apic_status apic_noalloc_max_bytes(size_t *bytes) {
    if (!bytes) return fail(APIC_E_INVAL, "bytes is NULL");
    *bytes = kNoAllocBytes;
    return APIC_OK;
}

apic_status apic_step_noalloc(apic_scene *scene, int32_t n_steps, void *stream) {
    if (n_steps < 0) return fail(APIC_E_INVAL, "n_steps must be >= 0");
    apic_status rc = check_fields(scene);
    if (rc != APIC_OK) return rc;
    const int64_t n = scene->p.n > 0 ? scene->p.n : 1;
    const size_t need = make_layout(&scene->grid, n).total;
    if (need > kNoAllocBytes)
        return fail(APIC_E_WORKSPACE,
                    "apic_step_noalloc: this grid and %lld particles need %zu bytes of workspace, above the %zu "
                    "the library holds for calls without one",
                    (long long)scene->p.n, need, kNoAllocBytes);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    void *ptr = nullptr;
    rc = scratch_address(&ptr);
    if (rc != APIC_OK) return rc;
    apic_scene s = *scene;
    s.workspace = ptr;
    s.workspace_bytes = kNoAllocBytes;
    int64_t cap = 0;
    rc = check_scene(&s, &cap);
    if (rc != APIC_OK) return rc;
    {
        // the array holds whatever the last call left: start from a cleared
        // workspace (its counters, tags and tables; a fill kernel, no memset)
        std::lock_guard<std::mutex> lk(g_mu);
        g_states.erase(ptr);
    }
    g_untimed = true;
    rc = dispatch_steps(&s, cap, n_steps, 0, (hipStream_t)stream);
    g_untimed = false;
    {
        // the next call starts from a cleared array too
        std::lock_guard<std::mutex> lk(g_mu);
        g_states.erase(ptr);
    }
    return rc;
}

apic_status apic_batch_plan_count(int32_t *count) {
    if (!count) return fail(APIC_E_INVAL, "count is NULL");
    *count = kBatchPlanCount;
    return APIC_OK;
}

apic_status apic_batch_plan_info(int32_t plan, int32_t *particles_per_block, int32_t *blocks_per_cu) {
    if (plan < 0 || plan >= kBatchPlanCount) return fail(APIC_E_INVAL, "plan %d outside [0, %d)", plan, kBatchPlanCount);
    if (!particles_per_block || !blocks_per_cu) return fail(APIC_E_INVAL, "output pointer is NULL");
    *particles_per_block = kBatchPlans[plan].per_block;
    *blocks_per_cu = kBatchPlans[plan].blocks_per_cu;
    return APIC_OK;
}

apic_status apic_batch_set_plan(int32_t plan) {
    if (plan < -1 || plan >= kBatchPlanCount)
        return fail(APIC_E_INVAL, "plan %d outside [-1, %d)", plan, kBatchPlanCount);
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_forced_plan = plan;
    return APIC_OK;
}

apic_status apic_batch_tuning(const apic_scene *scenes, int32_t n_scenes, int32_t *plan, double *ns) {
    if (!scenes || n_scenes <= 0) return fail(APIC_E_INVAL, "scenes is NULL or n_scenes <= 0");
    if (!plan || !ns) return fail(APIC_E_INVAL, "output pointer is NULL");
    std::lock_guard<std::mutex> lock(g_batch_mu);
    auto it = g_tune.find(tune_key(scenes, n_scenes));
    *plan = -1;
    for (int p = 0; p < kBatchPlanCount; ++p) ns[p] = INFINITY;
    if (it == g_tune.end()) return APIC_OK;
    apic_status rc = tune_collect(it->second);
    if (rc != APIC_OK) return rc;
    if (it->second.chosen < 0) (void)tune_next(it->second);  // chooses once every plan is timed
    *plan = it->second.chosen;
    for (int p = 0; p < kBatchPlanCount; ++p) ns[p] = it->second.best_ns[p];
    return APIC_OK;
}

apic_status apic_batch_workspace_bytes(int32_t n_scenes, size_t *bytes) {
    if (n_scenes < 0) return fail(APIC_E_INVAL, "n_scenes must be >= 0");
    if (!bytes) return fail(APIC_E_INVAL, "bytes is NULL");
    *bytes = batch_bytes(n_scenes);
    return APIC_OK;
}

apic_status apic_step_batch(apic_scene *scenes, int32_t n_scenes, int32_t n_steps, void *batch_ws,
                            size_t batch_ws_bytes, void *stream) {
    if (n_scenes < 0 || n_steps < 0) return fail(APIC_E_INVAL, "n_scenes and n_steps must be >= 0");
    if (n_scenes == 0) return APIC_OK;
    if (!scenes) return fail(APIC_E_INVAL, "scenes is NULL");
    if (!batch_ws) return fail(APIC_E_WORKSPACE, "batch workspace is NULL");
    if (((uintptr_t)batch_ws) % kAlign) return fail(APIC_E_WORKSPACE, "batch workspace must be 256-byte aligned");
    if (batch_ws_bytes < batch_bytes(n_scenes))
        return fail(APIC_E_WORKSPACE, "batch workspace of %zu bytes, %zu needed for %d scenes", batch_ws_bytes,
                    batch_bytes(n_scenes), n_scenes);
    for (int32_t k = 0; k < n_scenes; ++k) {
        int64_t cap = 0;
        apic_status rc = check_scene(&scenes[k], &cap);
        if (rc != APIC_OK) return rc;
        const apic_grid_desc &a = scenes[0].grid, &b = scenes[k].grid;
        if (a.dim != b.dim || a.degree != b.degree || a.precision != b.precision || a.options != b.options)
            return fail(APIC_E_INVAL, "scene %d differs from scene 0 in dim, degree, precision or options", k);
        if (b.options & APIC_OPT_ABSOLUTE_POSITIONS)
            return fail(APIC_E_UNSUPPORTED, "apic_step_batch does not take absolute positions");
    }
    {
        std::unordered_map<void *, int32_t> seen;
        for (int32_t k = 0; k < n_scenes; ++k)
            if (!seen.emplace(scenes[k].workspace, k).second)
                return fail(APIC_E_INVAL, "scenes %d and %d share a workspace", seen[scenes[k].workspace], k);
    }
    std::lock_guard<std::mutex> lock(g_batch_mu);
    return dispatch_batch(scenes, n_scenes, n_steps, batch_ws, (hipStream_t)stream);
}

apic_status apic_grid_export(const apic_scene *scene, int32_t field, void *out, void *stream) {
    if (field != APIC_GRID_MASS && field != APIC_GRID_MOMENTUM && field != APIC_GRID_VELOCITY)
        return fail(APIC_E_INVAL, "unknown grid field %d", field);
    if (!out) return fail(APIC_E_INVAL, "out is NULL");
    return dispatch(Op::Export, scene, stream, OpArgs{out, field});
}

apic_status apic_diagnostics(const apic_scene *scene, int32_t which, double *out, void *stream) {
    if (!out) return fail(APIC_E_INVAL, "out is NULL");
    apic_status rc;
    if (which == APIC_DIAG_PARTICLES)
        rc = dispatch(Op::DiagParticles, scene, stream);
    else if (which == APIC_DIAG_ENERGY)
        rc = dispatch(Op::DiagEnergy, scene, stream);
    else if (which == APIC_DIAG_GRID || which == APIC_DIAG_GRID_NEW)
        rc = dispatch(Op::DiagGrid, scene, stream, OpArgs{nullptr, which});
    else
        return fail(APIC_E_INVAL, "unknown diagnostics kind %d", which);
    if (rc != APIC_OK) return rc;
    int64_t cap = 0;
    (void)check_scene(scene, &cap);
    const Layout L = make_layout(&scene->grid, cap);
    hipStream_t st = (hipStream_t)stream;
    rc = hip_check(hipMemcpyAsync(out, (char *)scene->workspace + L.o_diag_out, 8 * sizeof(double),
                                  hipMemcpyDeviceToHost, st),
                   "apic_diagnostics copy");
    if (rc != APIC_OK) return rc;
    return hip_check(hipStreamSynchronize(st), "apic_diagnostics sync");
}

apic_status apic_cfl_dt(const apic_scene *scene, double nu, double *dt_out, void *stream) {
    if (!dt_out) return fail(APIC_E_INVAL, "dt_out is NULL");
    if (!(nu > 0.0) || !isfinite(nu)) return fail(APIC_E_INVAL, "nu must be positive and finite");
    apic_status rc = dispatch(Op::Cfl, scene, stream);
    if (rc != APIC_OK) return rc;
    int64_t cap = 0;
    (void)check_scene(scene, &cap);
    const Layout L = make_layout(&scene->grid, cap);
    hipStream_t st = (hipStream_t)stream;
    double worst = 0.0;
    rc = hip_check(hipMemcpyAsync(&worst, (char *)scene->workspace + L.o_diag_out, sizeof(double),
                                  hipMemcpyDeviceToHost, st),
                   "apic_cfl_dt copy");
    if (rc != APIC_OK) return rc;
    rc = hip_check(hipStreamSynchronize(st), "apic_cfl_dt sync");
    if (rc != APIC_OK) return rc;
    *dt_out = worst == 0.0 ? INFINITY : nu * scene->grid.dx / worst;
    return APIC_OK;
}

apic_status apic_step_time(const apic_scene *scene, double *dt_last, double *t_out, void *stream) {
    if (!dt_last || !t_out) return fail(APIC_E_INVAL, "dt_last or t_out is NULL");
    int64_t cap = 0;
    apic_status rc = check_scene(scene, &cap);
    if (rc != APIC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    (void)state_of(scene, cap, st);
    const Layout L = make_layout(&scene->grid, cap);
    double h[2] = {0.0, 0.0};
    rc = hip_check(hipMemcpyAsync(h, (char *)scene->workspace + L.o_dt, sizeof h, hipMemcpyDeviceToHost, st),
                   "apic_step_time copy");
    if (rc != APIC_OK) return rc;
    rc = hip_check(hipStreamSynchronize(st), "apic_step_time sync");
    if (rc != APIC_OK) return rc;
    *dt_last = h[0];
    *t_out = h[1];
    return APIC_OK;
}

apic_status apic_get_flags(const apic_scene *scene, uint32_t *flags, void *stream) {
    if (!flags) return fail(APIC_E_INVAL, "flags is NULL");
    int64_t cap = 0;
    apic_status rc = check_scene(scene, &cap);
    if (rc != APIC_OK) return rc;
    (void)state_of(scene, cap, (hipStream_t)stream);
    const Layout L = make_layout(&scene->grid, cap);
    hipStream_t st = (hipStream_t)stream;
    rc = hip_check(hipMemcpyAsync(flags, (char *)scene->workspace + L.o_flags, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, st),
                   "apic_get_flags copy");
    if (rc != APIC_OK) return rc;
    return hip_check(hipStreamSynchronize(st), "apic_get_flags sync");
}

apic_status apic_clear_flags(apic_scene *scene, void *stream) {
    int64_t cap = 0;
    apic_status rc = check_scene(scene, &cap);
    if (rc != APIC_OK) return rc;
    (void)state_of(scene, cap, (hipStream_t)stream);
    const Layout L = make_layout(&scene->grid, cap);
    launch_fill<uint32_t>((uint32_t *)((char *)scene->workspace + L.o_flags), 16, 0u, (hipStream_t)stream);
    return hip_check(hipGetLastError(), "apic_clear_flags");
}

apic_status apic_positions_from_absolute(apic_scene *scene, const double *x, void *stream) {
    if (!x && scene && scene->p.n > 0) return fail(APIC_E_INVAL, "x is NULL");
    return dispatch(Op::Pack, scene, stream, OpArgs{(void *)x, 0});
}

apic_status apic_positions_to_absolute(const apic_scene *scene, double *x, void *stream) {
    if (!x && scene && scene->p.n > 0) return fail(APIC_E_INVAL, "x is NULL");
    return dispatch(Op::Unpack, scene, stream, OpArgs{(void *)x, 0});
}

apic_status apic_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> lock(g_timing.mu);
    g_timing.enabled = enable != 0;
    return APIC_OK;
}

apic_status apic_timing_read(int64_t *counts, double *mean_ms) {
    if (!counts || !mean_ms) return fail(APIC_E_INVAL, "counts and mean_ms must not be NULL");
    std::vector<Timing::Rec> recs;
    {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        recs.swap(g_timing.recs);
    }
    double sum[APIC_PHASE_COUNT] = {0};
    int64_t cnt[APIC_PHASE_COUNT] = {0};
    apic_status rc = APIC_OK;
    for (const auto &r : recs) {
        if (rc == APIC_OK) rc = hip_check(hipEventSynchronize(r.b), "apic_timing_read");
        float ms = 0.f;
        if (rc == APIC_OK) rc = hip_check(hipEventElapsedTime(&ms, r.a, r.b), "apic_timing_read");
        if (rc == APIC_OK && r.phase >= 0 && r.phase < APIC_PHASE_COUNT) {
            sum[r.phase] += ms;
            cnt[r.phase] += 1;
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_timing.mu);
        for (const auto &r : recs) {
            g_timing.pool.push_back(r.a);
            g_timing.pool.push_back(r.b);
        }
    }
    for (int k = 0; k < APIC_PHASE_COUNT; ++k) {
        counts[k] = cnt[k];
        mean_ms[k] = cnt[k] ? sum[k] / (double)cnt[k] : 0.0;
    }
    return rc;
}

const char *apic_last_error(void) { return g_last_error.c_str(); }

const char *apic_version(void) { return "libapic 0.2 (gfx950)"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Implicit midpoint step (Sec. 3.3 at lambda = 1/2; Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
namespace {

// sticky bands do not change the workspace layout
constexpr int32_t kNoBand[6] = {0, 0, 0, 0, 0, 0};

struct MidLayout {
    size_t mf, gv, dv, dvt, r, rc, pv, s, delta, part, part2, epart, out, flags, tflags, counts, cg;
    size_t key, perm, count, cursor, start, bsum, klist, nlist, slot, slab, scell, soff, sF, sm, smv, sM, sid, total;
    MidGrid g;
};

MidLayout mid_layout(const apic_grid_desc &gd, const int32_t *band, int64_t n) {
    MidLayout L{};
    L.g = mid_grid(gd.dim, gd.cells, band, gd.dx);
    const MidGrid &g = L.g;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(o + bytes);
        return o;
    };
    const size_t vb = (size_t)g.nodes * gd.dim * sizeof(double);
    const size_t np = (size_t)std::max<int64_t>(n, 1);
    // a key tile is listed only when it holds a particle
    const size_t maxk = (size_t)std::min<int64_t>(g.tiles, std::max<int64_t>(n, 1));
    L.mf = take((size_t)g.nodes * sizeof(double));
    L.gv = take(vb);
    L.dv = take(vb);
    L.dvt = take(vb);
    L.r = take(vb);
    L.rc = take(vb);
    L.pv = take(vb);
    L.s = take(vb);
    L.delta = take(vb);
    L.part = take((size_t)mid_node_blocks(g.tiles) * 2 * sizeof(double));
    L.part2 = take((size_t)mid_node_blocks(g.tiles) * sizeof(double));
    L.epart = take(maxk * sizeof(double));
    L.out = take(4 * sizeof(double));
    L.flags = take(sizeof(uint32_t));
    L.tflags = take(sizeof(uint32_t));
    L.counts = take(2 * sizeof(int32_t));
    L.cg = take(sizeof(MidCg));
    L.key = take(np * 4);
    L.perm = take(np * 4);
    // counting sort: one bucket per node slot, then one for the particles outside the grid
    L.count = take((size_t)(g.nodes + 1) * 4);
    L.cursor = take((size_t)(g.nodes + 1) * 4);
    L.start = take((size_t)(g.nodes + 2) * 4);
    L.bsum = take((size_t)mid_scan_blocks(g.nodes + 1) * 4);
    L.klist = take((size_t)g.tiles * 4);
    L.nlist = take((size_t)g.tiles * 4);
    L.slot = take((size_t)g.tiles * 4);
    L.slab = take(maxk * (size_t)(1 + gd.dim) * mid_region_nodes(gd.dim, gd.degree) * sizeof(double));
    L.scell = take(np * 4);
    L.soff = take(np * gd.dim * sizeof(double));
    L.sF = take(np * gd.dim * gd.dim * sizeof(double));
    L.sm = take(np * sizeof(double));
    L.smv = take(np * gd.dim * sizeof(double));
    L.sM = take(np * (gd.dim * gd.dim + 1) * sizeof(double));
    L.sid = take(np * 4);
    L.total = off;
    return L;
}

struct MidOpts {
    double newton_tol, cg_tol;
    int max_newton, max_cg;
};

// CG iterations launched before the first look at the device's stop flag
// (later looks come after the iterations the convergence rate says are left).
constexpr int kCgPoll = 8;

template <int DIM, int DEG>
apic_status mid_run(apic_scene *s, int32_t n_steps, const MidOpts &o, apic_midpoint_stats *stats, hipStream_t st) {
    const MidLayout L = mid_layout(s->grid, s->prm.band, s->p.n);
    const MidGrid &g = L.g;
    char *ws = (char *)s->workspace;
    double *mf = (double *)(ws + L.mf), *gv = (double *)(ws + L.gv);
    double *dv = (double *)(ws + L.dv), *dvt = (double *)(ws + L.dvt);
    double *r = (double *)(ws + L.r), *rc = (double *)(ws + L.rc), *pv = (double *)(ws + L.pv);
    double *sv = (double *)(ws + L.s), *delta = (double *)(ws + L.delta), *part = (double *)(ws + L.part);
    double *part2 = (double *)(ws + L.part2);
    double *epart = (double *)(ws + L.epart), *out = (double *)(ws + L.out);
    uint32_t *flags = (uint32_t *)(ws + L.flags);
    uint32_t *tflags = (uint32_t *)(ws + L.tflags);  // flags of the iterate being tried
    int32_t *counts = (int32_t *)(ws + L.counts);
    MidCg *cg = (MidCg *)(ws + L.cg);

    const MidMaterial mat{s->prm.mu, s->prm.lambda, s->prm.rho0};
    Parts<double> P{};
    P.cell = s->p.cell;
    P.off = (double *)s->p.off;
    P.v = (double *)s->p.v;
    P.B = (double *)s->p.B;
    P.F = (double *)s->p.F;
    P.m = (double *)s->p.mass;
    P.id = s->p.id;
    P.n = s->p.n;
    P.s = s->p.stride;
    MidSorted S{};
    S.perm = (uint32_t *)(ws + L.perm);
    S.start = (const uint32_t *)(ws + L.start);
    S.cell = (uint32_t *)(ws + L.scell);
    S.off = (double *)(ws + L.soff);
    S.F = (double *)(ws + L.sF);
    S.m = (double *)(ws + L.sm);
    S.mv = (double *)(ws + L.smv);
    S.M = (double *)(ws + L.sM);
    S.id = P.id ? (uint32_t *)(ws + L.sid) : nullptr;
    S.n = std::max<int64_t>(P.n, 1);
    S.dx = s->grid.dx;
    MidTiles tl{};
    tl.klist = (int32_t *)(ws + L.klist);
    tl.nlist = (int32_t *)(ws + L.nlist);
    tl.slot = (int32_t *)(ws + L.slot);
    tl.slab = (double *)(ws + L.slab);
    uint32_t *key = (uint32_t *)(ws + L.key), *count = (uint32_t *)(ws + L.count);
    uint32_t *cursor = (uint32_t *)(ws + L.cursor), *bsum = (uint32_t *)(ws + L.bsum);
    const double dt = s->prm.dt;
    const double *grav = s->prm.gravity;
    const bool elastic = s->prm.model == APIC_MODEL_NEO_HOOKEAN && P.n > 0;
    apic_status rc0 = APIC_OK;
    auto fetch = [&](void *dst, const void *src, size_t bytes) {
        if (rc0 != APIC_OK) return;
        rc0 = hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st), "apic_step_midpoint");
        if (rc0 == APIC_OK) rc0 = hip_check(hipStreamSynchronize(st), "apic_step_midpoint");
    };
    // E(dv) and |r|_M with r written to `r` (Sec. 4.1); an inverted element
    // makes E infinite and raises its flag in tflags
    auto eval = [&](const double *dvx, double &E, double &res) {
        double host[2] = {0.0, 0.0};
        launch_fill<uint32_t>(tflags, 1, 0u, st);
        if (elastic)
            timed_kernel(APIC_PHASE_MID_FORCE, [&](hipEvent_t a, hipEvent_t b) {
                launch_mid_force_tiles<DIM, DEG>(S, g, tl, mat, gv, dvx, dt, epart, tflags, st, a, b);
            });
        launch_mid_force_nodes<DIM, DEG>(g, tl, elastic, dvx, dt, grav, mf, r, epart, part, out, st);
        fetch(host, out, sizeof host);
        res = sqrt(host[0]);
        E = host[1];
    };

    launch_fill<uint32_t>(flags, 1, 0u, st);
    launch_fill<uint32_t>((uint32_t *)cg, sizeof(MidCg) / sizeof(uint32_t), 0u, st);
    *stats = apic_midpoint_stats{};
    stats->converged = 1;
    const double tol2 = o.cg_tol * o.cg_tol;
    uint32_t cg_seen = 0;  // CG iterations counted on the device at the last look
    for (int32_t step = 0; step < n_steps && rc0 == APIC_OK; ++step) {
        launch_mid_sort<DIM, DEG>(P, g, S, tl, key, count, cursor, bsum, counts, flags, st);
        int32_t nkn[2] = {0, 0};
        fetch(nkn, counts, sizeof nkn);
        tl.nk = nkn[0];
        tl.nn = nkn[1];
        stats->res0 = 0.0;
        stats->res = 0.0;
        if (tl.nk == 0 || rc0 != APIC_OK) continue;  // no particle inside the grid: nothing moves
        launch_mid_sort_state<DIM, DEG>(P, S, tl, g.nodes, st);
        launch_mid_p2g<DIM, DEG>(S, g, tl, mf, gv, st);
        launch_mid_axpy<DIM>(g, tl, nullptr, 0.0, gv, dv, st);  // dv = 0
        double E = 0.0, res = 0.0;
        eval(dv, E, res);
        launch_mid_flags_accept(flags, tflags, st);
        const double res0 = res;
        int it = 0;
        for (; it < o.max_newton && rc0 == APIC_OK; ++it) {
            if (res0 == 0.0 || res <= o.newton_tol * res0) break;
            // conjugate gradient in the mass inner product (Sec. 4.2) on
            // (I - dt^2/4 M^{-1} df/dx) delta = -r, its scalars on the device
            launch_mid_cg_init<DIM>(g, tl, mf, r, delta, rc, pv, part, cg, tol2, (uint32_t)o.max_cg, st);
            int chunk = kCgPoll;
            for (int k = 0; k < o.max_cg && rc0 == APIC_OK;) {
                chunk = std::min(chunk, o.max_cg - k);
                for (int j = 0; j < chunk; ++j, ++k) {
                    if (elastic)
                        timed_kernel(APIC_PHASE_MID_APPLY, [&](hipEvent_t a, hipEvent_t b) {
                            launch_mid_apply_tiles<DIM, DEG>(S, g, tl, mat, pv, cg, st, a, b);
                        });
                    launch_mid_apply_nodes<DIM, DEG>(g, tl, elastic, pv, mf, dt, sv, part, cg, st);
                    launch_mid_cg_step<DIM>(g, tl, mf, r, pv, sv, delta, rc, part, part2, cg, k, st);
                    launch_mid_cg_dir<DIM>(g, tl, rc, pv, part2, cg, k, st);
                }
                MidCg now{};
                fetch(&now, cg, sizeof now);
                // launches after the stop did no work: out of the timing records
                if (elastic) untime_last(APIC_PHASE_MID_APPLY, chunk - (int)(now.iters - cg_seen));
                cg_seen = now.iters;
                if (now.done) break;
                // next look after the iterations the rate so far says are left
                // (launches past the stop cost a few microseconds each, a look
                // a synchronization)
                const double gam = now.gamma[k & 1];
                chunk = kCgPoll;
                if (gam > 0.0 && gam < now.gamma0 && now.tol2 > 0.0) {
                    const double per = std::log(gam / now.gamma0) / k;
                    const double left = std::log(now.tol2 * now.gamma0 / gam) / per;
                    chunk = (int)std::min(32.0, std::max(1.0, std::ceil(left)));
                }
            }
            // backtracking line search: E must not increase, or |r|_M must
            // fall (near the minimum E is flat to within its rounding); a
            // trial that inverts an element has E = +inf and is halved
            double stepl = 1.0, En = 0.0, resn = 0.0;
            for (int k = 0; k < 30 && rc0 == APIC_OK; ++k) {
                launch_mid_axpy<DIM>(g, tl, dv, stepl, delta, dvt, st);
                eval(dvt, En, resn);
                if ((std::isfinite(En) && (En <= E || resn < res)) || k == 29) break;
                stepl *= 0.5;
                stats->halvings += 1;
            }
            launch_mid_flags_accept(flags, tflags, st);
            std::swap(dv, dvt);
            E = En;
            res = resn;
        }
        stats->newton_iters += it;
        stats->res0 = res0;
        stats->res = res;
        if (!(res0 == 0.0 || res <= o.newton_tol * res0)) stats->converged = 0;
        launch_mid_finish<DIM>(g, tl, mf, gv, dv, dt, rc, sv, st);
        launch_mid_g2p<DIM, DEG>(P, S, g, tl, rc, sv, st);
    }
    if (rc0 != APIC_OK) return rc0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APIC_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    uint32_t fl = 0;
    MidCg cgh{};
    fetch(&fl, flags, sizeof fl);
    fetch(&cgh, cg, sizeof cgh);
    stats->flags = fl;
    stats->cg_iters = (int32_t)cgh.iters;
    return rc0;
}

}  // namespace

extern "C" {

apic_status apic_midpoint_workspace_bytes(const apic_grid_desc *grid, int64_t max_particles, size_t *bytes) {
    apic_status rc = check_grid(grid);
    if (rc != APIC_OK) return rc;
    if (!bytes) return fail(APIC_E_INVAL, "bytes is NULL");
    if (max_particles < 0) return fail(APIC_E_INVAL, "max_particles must be >= 0");
    *bytes = mid_layout(*grid, kNoBand, max_particles).total;
    return APIC_OK;
}

apic_status apic_step_midpoint(apic_scene *s, int32_t n_steps, const apic_midpoint_opts *opts,
                               apic_midpoint_stats *stats, void *stream) {
    apic_status rc = check_fields(s);
    if (rc != APIC_OK) return rc;
    if (!stats) return fail(APIC_E_INVAL, "stats is NULL");
    if (n_steps < 0) return fail(APIC_E_INVAL, "n_steps must be >= 0");
    if (s->grid.precision != APIC_F64) return fail(APIC_E_UNSUPPORTED, "the midpoint step runs in binary64 only");
    if (s->grid.degree != APIC_QUADRATIC && s->grid.degree != APIC_CUBIC)
        return fail(APIC_E_UNSUPPORTED, "the midpoint step takes quadratic or cubic weights");
    if (s->prm.transfer != APIC_TRANSFER_APIC)
        return fail(APIC_E_UNSUPPORTED, "the midpoint step uses the APIC transfers only");
    if (s->grid.options & APIC_OPT_ADAPTIVE_DT)
        return fail(APIC_E_UNSUPPORTED, "adaptive steps are not available with the midpoint step");
    MidOpts o{1e-10, 1e-8, 20, 500};
    if (opts) {
        if (!(opts->newton_tol >= 0.0) || !(opts->cg_tol >= 0.0) || !isfinite(opts->newton_tol) ||
            !isfinite(opts->cg_tol) || opts->max_newton < 0 || opts->max_cg < 0)
            return fail(APIC_E_INVAL, "midpoint options: tolerances must be finite and >= 0, limits >= 0");
        if (opts->newton_tol > 0.0) o.newton_tol = opts->newton_tol;
        if (opts->cg_tol > 0.0) o.cg_tol = opts->cg_tol;
        if (opts->max_newton > 0) o.max_newton = opts->max_newton;
        if (opts->max_cg > 0) o.max_cg = opts->max_cg;
    }
    if (!s->workspace) return fail(APIC_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)s->workspace) % kAlign) return fail(APIC_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t need = mid_layout(s->grid, s->prm.band, s->p.n).total;
    if (s->workspace_bytes < need)
        return fail(APIC_E_WORKSPACE, "workspace of %zu bytes is below the %zu the midpoint step needs",
                    s->workspace_bytes, need);
    {
        // the workspace no longer holds the explicit path's binning or grid
        std::lock_guard<std::mutex> lock(g_mu);
        g_states.erase(s->workspace);
    }
    hipStream_t st = (hipStream_t)stream;
    const int key = s->grid.dim * 10 + s->grid.degree;
    switch (key) {
        case 22: return mid_run<2, 2>(s, n_steps, o, stats, st);
        case 23: return mid_run<2, 3>(s, n_steps, o, stats, st);
        case 32: return mid_run<3, 2>(s, n_steps, o, stats, st);
        default: return mid_run<3, 3>(s, n_steps, o, stats, st);
    }
}

}  // extern "C"
