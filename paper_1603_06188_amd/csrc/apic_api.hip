// C ABI of libapic (declared in include/apic.h): host-side validation,
// workspace layout and dispatch to the gfx950 kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

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
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout.  The fixed part (grid planes, flags, reduction buffers)
// persists between calls; the transient part (sort buffers, shadow particle
// state) is sized by the particle count of the call and reused freely.
struct Layout {
    GridDims d;
    size_t elem;
    bool comp;
    size_t o_m, o_mv, o_vt, o_cm, o_cmv, o_flags, o_diag_out, o_diag_part, fixed_end;
    size_t o_keys, o_perm, o_counts, o_cursor, o_sums, o_sh_cell, o_sh_id, o_sh_f, total;
    int64_t n;
};

Layout make_layout(const apic_grid_desc *g, int64_t n) {
    Layout L{};
    L.d.dim = g->dim;
    L.d.deg = g->degree;
    const int tile_edge = g->dim == 3 ? 4 : 8;
    L.d.tiles = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < g->dim) {
            L.d.n[a] = g->cells[a];
            L.d.N[a] = g->cells[a] + 1;
            L.d.TN[a] = (L.d.N[a] + tile_edge - 1) / tile_edge;
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
    L.n = n;
    const size_t G = (size_t)L.d.G, dim = (size_t)g->dim, e = L.elem;
    size_t o = 0;
    L.o_m = o;
    o = align_up(o + G * e);
    L.o_mv = o;
    o = align_up(o + dim * G * e);
    L.o_vt = o;
    o = align_up(o + dim * G * e);
    L.o_cm = o;
    o = align_up(o + (L.comp ? G * e : 0));
    L.o_cmv = o;
    o = align_up(o + (L.comp ? dim * G * e : 0));
    L.o_flags = o;
    o = align_up(o + 64);
    L.o_diag_out = o;
    o = align_up(o + 8 * sizeof(double));
    L.o_diag_part = o;
    o = align_up(o + (size_t)kDiagBlocks * 8 * sizeof(double));
    L.fixed_end = o;
    const size_t nn = (size_t)(n > 0 ? n : 0);
    const size_t nkeys = G + 2;
    L.o_keys = o;
    o = align_up(o + nn * 4);
    L.o_perm = o;
    o = align_up(o + nn * 4);
    L.o_counts = o;
    o = align_up(o + nkeys * 4);
    L.o_cursor = o;
    o = align_up(o + nkeys * 4);
    L.o_sums = o;
    o = align_up(o + ((nkeys + 1023) / 1024 + 1) * 4);
    L.o_sh_cell = o;
    o = align_up(o + nn * 4);
    L.o_sh_id = o;
    o = align_up(o + nn * 4);
    L.o_sh_f = o;
    o = align_up(o + (size_t)(2 + 2 * dim + 2 * dim * dim) * nn * e);
    L.total = o;
    return L;
}

apic_status check_grid(const apic_grid_desc *g) {
    if (!g) return fail(APIC_E_INVAL, "grid descriptor is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(APIC_E_INVAL, "dim must be 2 or 3 (got %d)", g->dim);
    if (g->degree != APIC_QUADRATIC && g->degree != APIC_CUBIC)
        return fail(APIC_E_INVAL, "degree must be 2 (quadratic) or 3 (cubic) (got %d)", g->degree);
    if (g->precision != APIC_F32 && g->precision != APIC_F64)
        return fail(APIC_E_INVAL, "precision must be APIC_F32 or APIC_F64 (got %d)", g->precision);
    if (g->options & ~APIC_OPT_COMPENSATED) return fail(APIC_E_INVAL, "unknown option bits 0x%x", g->options);
    const int maxc = g->dim == 3 ? 1024 : 65535;
    for (int a = 0; a < g->dim; ++a)
        if (g->cells[a] < g->degree + 1 || g->cells[a] > maxc)
            return fail(APIC_E_INVAL, "cells[%d] = %d outside [%d, %d]", a, g->cells[a], g->degree + 1, maxc);
    if (!(g->dx > 0.0) || !isfinite(g->dx)) return fail(APIC_E_INVAL, "dx must be positive and finite");
    const Layout L = make_layout(g, 0);
    if (L.d.G + 2 > (int64_t)0xFFFFFFFFu) return fail(APIC_E_INVAL, "grid too large");
    return APIC_OK;
}

apic_status check_scene(const apic_scene *s) {
    if (!s) return fail(APIC_E_INVAL, "scene is NULL");
    apic_status rc = check_grid(&s->grid);
    if (rc != APIC_OK) return rc;
    const apic_particles &p = s->p;
    if (p.n < 0) return fail(APIC_E_INVAL, "particle count n = %lld is negative", (long long)p.n);
    if (p.n > (int64_t)0x7FFFFFFF) return fail(APIC_E_INVAL, "particle count above 2^31 - 1");
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
    if (!s->workspace) return fail(APIC_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)s->workspace) % kAlign) return fail(APIC_E_WORKSPACE, "workspace must be 256-byte aligned");
    const Layout L = make_layout(&s->grid, p.n);
    if (s->workspace_bytes < L.total)
        return fail(APIC_E_WORKSPACE, "workspace has %zu bytes, %zu needed", s->workspace_bytes, L.total);
    return APIC_OK;
}

template <typename T>
Parts<T> parts_of(const apic_scene *s) {
    Parts<T> P;
    P.cell = s->p.cell;
    P.off = (T *)s->p.off;
    P.v = (T *)s->p.v;
    P.B = (T *)s->p.B;
    P.F = (T *)s->p.F;
    P.m = (T *)s->p.mass;
    P.id = s->p.id;
    P.n = s->p.n;
    P.s = s->p.stride;
    return P;
}

template <typename T>
Parts<T> shadow_of(const apic_scene *s, const Layout &L) {
    char *w = (char *)s->workspace;
    const int64_t n = L.n, dim = L.d.dim;
    Parts<T> P;
    P.cell = (uint32_t *)(w + L.o_sh_cell);
    P.id = (int32_t *)(w + L.o_sh_id);
    T *f = (T *)(w + L.o_sh_f);
    P.off = f;
    P.v = f + dim * n;
    P.B = f + 2 * dim * n;
    P.F = f + (2 * dim + dim * dim) * n;
    P.m = f + (2 * dim + 2 * dim * dim) * n;
    P.n = n;
    P.s = n;
    return P;
}

template <typename T>
GridPlanes<T> planes_of(const apic_scene *s, const Layout &L) {
    char *w = (char *)s->workspace;
    GridPlanes<T> g;
    g.m = (T *)(w + L.o_m);
    g.mv = (T *)(w + L.o_mv);
    g.vt = (T *)(w + L.o_vt);
    g.cm = (T *)(w + L.o_cm);
    g.cmv = (T *)(w + L.o_cmv);
    g.flags = (uint32_t *)(w + L.o_flags);
    g.d = L.d;
    g.dx = (T)s->grid.dx;
    g.inv_dx = (T)(1.0 / s->grid.dx);
    return g;
}

template <typename T>
StepParams<T> params_of(const apic_scene *s) {
    StepParams<T> q;
    q.dt = (T)s->prm.dt;
    for (int a = 0; a < 3; ++a) q.g[a] = (T)s->prm.gravity[a];
    q.model = s->prm.model;
    for (int k = 0; k < 6; ++k) q.band[k] = s->prm.band[k];
    q.mu = (T)s->prm.mu;
    q.lam = (T)s->prm.lambda;
    q.inv_rho0 = s->prm.rho0 > 0.0 ? (T)(1.0 / s->prm.rho0) : T(0);
    return q;
}

enum class Op { Sort, P2G, GridUpdate, G2P, Export, DiagParticles, DiagGrid, Pack, Unpack };

struct OpArgs {
    void *ptr;    // export destination / positions / diag host out
    int which;    // export field / diag kind
};

template <typename T, int DIM, int DEG, bool COMP>
apic_status run(Op op, const apic_scene *s, hipStream_t st, const OpArgs &a) {
    const Layout L = make_layout(&s->grid, s->p.n);
    const Parts<T> P = parts_of<T>(s);
    const GridPlanes<T> g = planes_of<T>(s, L);
    const StepParams<T> q = params_of<T>(s);
    char *w = (char *)s->workspace;
    switch (op) {
        case Op::Sort: {
            SortBuffers sb;
            sb.keys = (uint32_t *)(w + L.o_keys);
            sb.perm = (uint32_t *)(w + L.o_perm);
            sb.counts = (uint32_t *)(w + L.o_counts);
            sb.cursor = (uint32_t *)(w + L.o_cursor);
            sb.sums = (uint32_t *)(w + L.o_sums);
            launch_sort<T, DIM, DEG>(P, shadow_of<T>(s, L), L.d, sb, st);
            break;
        }
        case Op::P2G:
            launch_p2g<T, DIM, DEG, COMP>(P, g, q, st);
            break;
        case Op::GridUpdate:
            launch_grid_update<T, DIM, COMP>(g, q, st);
            break;
        case Op::G2P:
            launch_g2p<T, DIM, DEG>(P, g, q, st);
            break;
        case Op::Export:
            launch_grid_export<T, DIM, COMP>(g, a.which, (T *)a.ptr, st);
            break;
        case Op::DiagParticles:
            launch_diag_particles<T, DIM>(P, s->grid.dx, (double *)(w + L.o_diag_part), (double *)(w + L.o_diag_out),
                                          st);
            break;
        case Op::DiagGrid:
            launch_diag_grid<T, DIM, COMP>(g, a.which, s->prm.dt, (double *)(w + L.o_diag_part),
                                           (double *)(w + L.o_diag_out), st);
            break;
        case Op::Pack:
            launch_pack_positions<T, DIM>(P, (const double *)a.ptr, s->grid.dx, st);
            break;
        case Op::Unpack:
            launch_unpack_positions<T, DIM>(P, (double *)a.ptr, s->grid.dx, st);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APIC_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return APIC_OK;
}

template <typename T, int DIM, int DEG>
apic_status run_c(Op op, const apic_scene *s, hipStream_t st, const OpArgs &a) {
    if (s->grid.options & APIC_OPT_COMPENSATED) return run<T, DIM, DEG, true>(op, s, st, a);
    return run<T, DIM, DEG, false>(op, s, st, a);
}

template <typename T, int DIM>
apic_status run_k(Op op, const apic_scene *s, hipStream_t st, const OpArgs &a) {
    if (s->grid.degree == APIC_CUBIC) return run_c<T, DIM, 3>(op, s, st, a);
    return run_c<T, DIM, 2>(op, s, st, a);
}

template <typename T>
apic_status run_d(Op op, const apic_scene *s, hipStream_t st, const OpArgs &a) {
    if (s->grid.dim == 3) return run_k<T, 3>(op, s, st, a);
    return run_k<T, 2>(op, s, st, a);
}

apic_status dispatch(Op op, const apic_scene *s, void *stream, const OpArgs &a = OpArgs{nullptr, 0}) {
    apic_status rc = check_scene(s);
    if (rc != APIC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (s->grid.precision == APIC_F64) return run_d<double>(op, s, st, a);
    return run_d<float>(op, s, st, a);
}

apic_status hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(APIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return APIC_OK;
}

}  // namespace

extern "C" {

apic_status apic_workspace_bytes(const apic_grid_desc *grid, int64_t max_particles, size_t *bytes) {
    apic_status rc = check_grid(grid);
    if (rc != APIC_OK) return rc;
    if (!bytes) return fail(APIC_E_INVAL, "bytes is NULL");
    if (max_particles < 0) return fail(APIC_E_INVAL, "max_particles is negative");
    *bytes = make_layout(grid, max_particles).total;
    return APIC_OK;
}

apic_status apic_reset(apic_scene *scene, void *stream) {
    apic_status rc = check_scene(scene);
    if (rc != APIC_OK) return rc;
    const Layout L = make_layout(&scene->grid, scene->p.n);
    launch_fill<uint32_t>((uint32_t *)scene->workspace, (int64_t)(L.fixed_end / 4), 0u, (hipStream_t)stream);
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
    for (int32_t k = 0; k < n_scenes; ++k) {
        apic_status rc = check_scene(&scenes[k]);
        if (rc != APIC_OK) return rc;
    }
    for (int32_t step = 0; step < n_steps; ++step) {
        for (int32_t k = 0; k < n_scenes; ++k) {
            apic_status rc = APIC_OK;
            if (sort_every > 0 && step % sort_every == 0) rc = dispatch(Op::Sort, &scenes[k], stream);
            if (rc == APIC_OK) rc = dispatch(Op::P2G, &scenes[k], stream);
            if (rc == APIC_OK) rc = dispatch(Op::GridUpdate, &scenes[k], stream);
            if (rc == APIC_OK) rc = dispatch(Op::G2P, &scenes[k], stream);
            if (rc != APIC_OK) return rc;
        }
    }
    return APIC_OK;
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
    else if (which == APIC_DIAG_GRID || which == APIC_DIAG_GRID_NEW)
        rc = dispatch(Op::DiagGrid, scene, stream, OpArgs{nullptr, which});
    else
        return fail(APIC_E_INVAL, "unknown diagnostics kind %d", which);
    if (rc != APIC_OK) return rc;
    const Layout L = make_layout(&scene->grid, scene->p.n);
    hipStream_t st = (hipStream_t)stream;
    rc = hip_check(hipMemcpyAsync(out, (char *)scene->workspace + L.o_diag_out, 8 * sizeof(double),
                                  hipMemcpyDeviceToHost, st),
                   "apic_diagnostics copy");
    if (rc != APIC_OK) return rc;
    return hip_check(hipStreamSynchronize(st), "apic_diagnostics sync");
}

apic_status apic_get_flags(const apic_scene *scene, uint32_t *flags, void *stream) {
    if (!flags) return fail(APIC_E_INVAL, "flags is NULL");
    apic_status rc = check_scene(scene);
    if (rc != APIC_OK) return rc;
    const Layout L = make_layout(&scene->grid, scene->p.n);
    hipStream_t st = (hipStream_t)stream;
    rc = hip_check(hipMemcpyAsync(flags, (char *)scene->workspace + L.o_flags, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, st),
                   "apic_get_flags copy");
    if (rc != APIC_OK) return rc;
    return hip_check(hipStreamSynchronize(st), "apic_get_flags sync");
}

apic_status apic_clear_flags(apic_scene *scene, void *stream) {
    apic_status rc = check_scene(scene);
    if (rc != APIC_OK) return rc;
    const Layout L = make_layout(&scene->grid, scene->p.n);
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

const char *apic_last_error(void) { return g_last_error.c_str(); }

const char *apic_version(void) { return "libapic 0.1 (gfx950)"; }

}  // extern "C"
