// plan.hip -- a prepared renderer for fixed shapes and fixed device buffers (the batched path):
// it owns its workspace, holds the launch tuning (given by the caller, or chosen by timing the
// candidate launch shapes on the caller's data), and captures the forward and the backward launch
// sequences once each as HIP graphs that later calls replay.
//
// The graphs hold kernel nodes only (every clear in the sequence is a fill kernel), so replays
// are self-contained. An instance-capacity overflow is detected by digs_plan_check, which then
// grows the workspace and drops the graphs; the next call re-captures them.
#include <string.h>

#include <algorithm>
#include <new>

#include "kernels.h"

struct digs_plan {
    digs_geom geom;
    digs_grid grid;
    int n = 0, T = 0;
    digs_tuning tuning;
    digs_plan_buffers b;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraph_t gf = nullptr, gb = nullptr, gv = nullptr;
    hipGraphExec_t ef = nullptr, eb = nullptr, ev = nullptr;
    bool canonical = false;   // the workspace holds the per-Gaussian stage of the buffers' Gaussians
    float tune_ms[DIGS_TUNE_CANDIDATES][2];
};

static int hip_rc(hipError_t e) { return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e); }

static void drop_graphs(digs_plan *p)
{
    if (p->ef) (void)hipGraphExecDestroy(p->ef);
    if (p->eb) (void)hipGraphExecDestroy(p->eb);
    if (p->ev) (void)hipGraphExecDestroy(p->ev);
    if (p->gf) (void)hipGraphDestroy(p->gf);
    if (p->gb) (void)hipGraphDestroy(p->gb);
    if (p->gv) (void)hipGraphDestroy(p->gv);
    p->ef = p->eb = p->ev = nullptr;
    p->gf = p->gb = p->gv = nullptr;
    p->canonical = false;
}

static int plan_alloc(digs_plan *p)
{
    const size_t need = digs_workspace_size(&p->geom, &p->grid, p->n, p->T, &p->tuning);
    if (need == 0) return DIGS_EINVAL;
    if (p->ws && p->ws_bytes >= need) return DIGS_OK;
    drop_graphs(p);
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
    if (hipMalloc(&p->ws, need) != hipSuccess) {
        (void)hipGetLastError();
        p->ws = nullptr;
        return DIGS_ENOMEM;
    }
    p->ws_bytes = need;
    return digs_reset_diagnostics(p->ws, p->cap);
}

static int run_fwd(digs_plan *p, hipStream_t s, bool views_only = false)
{
    const digs_plan_buffers &b = p->b;
    return project_fwd_impl(&p->geom, &p->grid, b.coef, p->n, b.mu, b.scale, b.quat, b.rho,
                            p->T, b.angles, b.w, b.proj, p->ws, p->ws_bytes, &p->tuning,
                            views_only, s);
}

static int run_bwd(digs_plan *p, hipStream_t s)
{
    const digs_plan_buffers &b = p->b;
    return digs_project_bwd(&p->geom, &p->grid, b.coef, p->n, b.mu, b.scale, b.quat, b.rho,
                            p->T, b.angles, b.w, b.grad_proj, b.g_mu, b.g_scale, b.g_quat,
                            b.g_rho, b.g_coef, b.g_w, p->ws, p->ws_bytes, &p->tuning,
                            DIGS_BWD_REUSE_FWD, s);
}

// Record one launch sequence on the plan's own stream as a graph (stage timing is switched off
// while recording so that no event nodes enter the graph). which: 0 forward, 1 backward,
// 2 forward of the per-view stages only.
static int capture(digs_plan *p, int which)
{
    const int prof = digs_profile_enable(-1);
    digs_profile_enable(0);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    int rc = hip_rc(e);
    if (rc == DIGS_OK) {
        rc = which == 0 ? run_fwd(p, p->cap) : which == 2 ? run_fwd(p, p->cap, true)
                                                          : run_bwd(p, p->cap);
        e = hipStreamEndCapture(p->cap, &g);
        if (rc == DIGS_OK) rc = hip_rc(e);
    }
    digs_profile_enable(prof);
    if (rc != DIGS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return digs_set_hip_error(e);
    }
    if (which == 0) {
        p->gf = g;
        p->ef = x;
    } else if (which == 2) {
        p->gv = g;
        p->ev = x;
    } else {
        p->gb = g;
        p->eb = x;
    }
    return DIGS_OK;
}

static int read_diag(digs_plan *p, digs_diag *d) { return digs_read_diagnostics(p->ws, d, p->cap); }

static int64_t capacity_for(uint64_t instances)
{
    return (int64_t)(instances + instances / 4 + 4096);
}

// Time fwd (+ bwd) of one tuning on the plan's stream: one warm-up, then the median of three.
static int time_tuning(digs_plan *p, float *fwd_ms, float *bwd_ms)
{
    hipEvent_t ev[3];
    for (int i = 0; i < 3; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) return digs_set_hip_error(hipGetLastError());
    const bool bwd = p->b.grad_proj != nullptr;
    float f[3], b[3];
    int rc = DIGS_OK;
    for (int rep = 0; rep < 4 && rc == DIGS_OK; ++rep) {
        rc = hip_rc(hipEventRecord(ev[0], p->cap));
        if (rc == DIGS_OK) rc = run_fwd(p, p->cap);
        if (rc == DIGS_OK) rc = hip_rc(hipEventRecord(ev[1], p->cap));
        if (rc == DIGS_OK && bwd) rc = run_bwd(p, p->cap);
        if (rc == DIGS_OK) rc = hip_rc(hipEventRecord(ev[2], p->cap));
        if (rc == DIGS_OK) rc = hip_rc(hipEventSynchronize(ev[2]));
        if (rc == DIGS_OK && rep > 0) {
            (void)hipEventElapsedTime(&f[rep - 1], ev[0], ev[1]);
            b[rep - 1] = 0.0f;
            if (bwd) (void)hipEventElapsedTime(&b[rep - 1], ev[1], ev[2]);
        }
    }
    for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
    if (rc != DIGS_OK) return rc;
    std::sort(f, f + 3);
    std::sort(b, b + 3);
    *fwd_ms = f[1];
    *bwd_ms = b[1];
    return DIGS_OK;
}

// Tile shapes the autotuner tries (pixels), the default first, and the launch shapes it times for
// each: forward splat waves per tile x persistent or one-workgroup-per-item splats. Candidate c is
// shape c / 4, launch shape c % 4.
static const int kTileW[DIGS_TUNE_CANDIDATES / 4] = {16, 32, 8};
static const int kTileH[DIGS_TUNE_CANDIDATES / 4] = {16, 8, 8};
static const int kWaves[4] = {4, 4, 1, 1};
static const int kPersist[4] = {0, 1, 0, 1};

// Drop the workspace and allocate one sized for the current tuning.
static int plan_realloc(digs_plan *p)
{
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
    return plan_alloc(p);
}

// The autotuner. For each tile shape the call's detector allows: size the instance capacity from a
// measured forward, then time the four launch shapes on the caller's data. Launch shapes of one
// tile shape compute bitwise-identical results; tile shapes add the same terms in different
// orders, so a shape other than the default is kept only when it is faster by more than 3% (a
// near tie does not flip between runs). The list slices follow from each shape's item count.
static int autotune(digs_plan *p)
{
    const int nshapes = DIGS_TUNE_CANDIDATES / 4;
    bool shape_ok[DIGS_TUNE_CANDIDATES / 4];
    int64_t shape_cap[DIGS_TUNE_CANDIDATES / 4];
    int shape_slices[DIGS_TUNE_CANDIDATES / 4];
    int best = -1;
    float best_ms = 0.0f, default_ms = 0.0f;
    int rc = DIGS_OK;
    for (int sh = 0; sh < nshapes; ++sh) {
        memset(&p->tuning, 0, sizeof(p->tuning));
        p->tuning.tile_w = kTileW[sh];
        p->tuning.tile_h = kTileH[sh];
        WsLayout L;
        shape_ok[sh] = ws_layout(&p->geom, &p->grid, p->n, p->T, &p->tuning, &L);
        if (!shape_ok[sh]) continue;   // too many tiles of this shape for the detector
        p->tuning.slices = L.slices;
        shape_slices[sh] = L.slices;
        shape_cap[sh] = 0;
        if ((rc = plan_realloc(p)) != DIGS_OK) return rc;
        if (p->n == 0 || p->T == 0) {
            if (sh == 0) return DIGS_OK;
            continue;
        }
        rc = run_fwd(p, p->cap);
        digs_diag d;
        if (rc == DIGS_OK) rc = read_diag(p, &d);
        if (rc != DIGS_OK) return rc;
        p->tuning.capacity = capacity_for(d.instances);
        shape_cap[sh] = p->tuning.capacity;
        if ((rc = plan_realloc(p)) != DIGS_OK) return rc;
        float shape_best = 0.0f;
        for (int v = 0; v < 4; ++v) {
            const int c = 4 * sh + v;
            p->tuning.splat_waves = kWaves[v];
            p->tuning.persistent = kPersist[v];
            rc = time_tuning(p, &p->tune_ms[c][0], &p->tune_ms[c][1]);
            if (rc != DIGS_OK) return rc;
            const float ms = p->tune_ms[c][0] + p->tune_ms[c][1];
            if (v == 0 || ms < shape_best) shape_best = ms;
            if (sh == 0) default_ms = shape_best;
            const bool better = sh == 0 ? (best < 0 || ms < best_ms)
                                        : (ms < best_ms && ms < 0.97f * default_ms);
            if (better) {
                best = c;
                best_ms = ms;
            }
        }
    }
    memset(&p->tuning, 0, sizeof(p->tuning));
    const int sh = best < 0 ? 0 : best / 4, v = best < 0 ? 0 : best % 4;
    p->tuning.tile_w = kTileW[sh];
    p->tuning.tile_h = kTileH[sh];
    p->tuning.slices = shape_slices[sh];
    p->tuning.capacity = shape_cap[sh];
    p->tuning.splat_waves = kWaves[v];
    p->tuning.persistent = kPersist[v];
    if ((rc = plan_realloc(p)) != DIGS_OK) return rc;
    return digs_reset_diagnostics(p->ws, p->cap);
}

extern "C" int digs_plan_create(const digs_geom *geom, const digs_grid *grid, int n, int T,
                                const digs_tuning *tuning, const digs_plan_buffers *bufs,
                                digs_plan **out)
{
    if (!out || !geom || !grid || !bufs) return DIGS_EINVAL;
    *out = nullptr;
    if (digs_workspace_size(geom, grid, n, T, tuning) == 0) return DIGS_EINVAL;
    const digs_plan_buffers &b = *bufs;
    if (T > 0 && (!b.proj || !b.g_w || !b.g_coef)) return DIGS_EINVAL;
    if (T > 0 && n > 0 &&
        (!b.coef || !b.mu || !b.scale || !b.quat || !b.rho || !b.angles || !b.w || !b.g_mu ||
         !b.g_scale || !b.g_quat || !b.g_rho))
        return DIGS_EINVAL;
    digs_plan *p = new (std::nothrow) digs_plan;
    if (!p) return DIGS_ENOMEM;
    p->geom = *geom;
    p->grid = *grid;
    p->n = n;
    p->T = T;
    p->b = b;
    memset(p->tune_ms, 0, sizeof(p->tune_ms));
    render_prepare_launch_shapes();
    int rc = hip_rc(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    if (rc == DIGS_OK) {
        if (tuning) {
            p->tuning = *tuning;
            rc = plan_alloc(p);
        } else {
            rc = autotune(p);
        }
    }
    if (rc == DIGS_OK) rc = hip_rc(hipStreamSynchronize(p->cap));
    if (rc != DIGS_OK) {
        digs_plan_destroy(p);
        return rc;
    }
    *out = p;
    return DIGS_OK;
}

// The caller's stream waits for everything the plan's own stream has queued before a replay.
static int order_after_plan_stream(digs_plan *p, hipStream_t s)
{
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return digs_set_hip_error(hipGetLastError());
    hipError_t e = hipEventRecord(ev, p->cap);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    (void)hipEventDestroy(ev);
    return hip_rc(e);
}

extern "C" int digs_plan_fwd(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0) return DIGS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!p->ef) {
        int rc = capture(p, 0);
        if (rc == DIGS_OK) rc = order_after_plan_stream(p, s);
        if (rc != DIGS_OK) return rc;
    }
    const int rc = hip_rc(hipGraphLaunch(p->ef, s));
    if (rc == DIGS_OK) p->canonical = true;
    return rc;
}

extern "C" int digs_plan_fwd_views(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0) return DIGS_OK;
    if (!p->canonical) return DIGS_EINVAL;   // no digs_plan_fwd on this workspace yet
    hipStream_t s = (hipStream_t)stream;
    if (!p->ev) {
        int rc = capture(p, 2);
        if (rc == DIGS_OK) rc = order_after_plan_stream(p, s);
        if (rc != DIGS_OK) return rc;
    }
    return hip_rc(hipGraphLaunch(p->ev, s));
}

extern "C" int digs_plan_bwd(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0 && p->n == 0) return DIGS_OK;
    if (!p->b.grad_proj && p->n > 0 && p->T > 0) return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!p->eb) {
        int rc = capture(p, 1);
        if (rc == DIGS_OK) rc = order_after_plan_stream(p, s);
        if (rc != DIGS_OK) return rc;
    }
    return hip_rc(hipGraphLaunch(p->eb, s));
}

extern "C" int digs_plan_check(digs_plan *p, digs_diag *out, int *resized, void *stream)
{
    if (!p || !out) return DIGS_EINVAL;
    if (resized) *resized = 0;
    int rc = hip_rc(hipStreamSynchronize((hipStream_t)stream));
    if (rc == DIGS_OK) rc = read_diag(p, out);
    if (rc != DIGS_OK || !out->overflow) return rc;
    // grow the capacity past the largest need of the calls since the last check (an earlier call
    // may have needed more than the last one), never below the current capacity; the graphs are
    // re-captured on the next call
    const uint64_t need = out->max_instances > out->instances ? out->max_instances : out->instances;
    p->tuning.capacity = std::max<int64_t>(p->tuning.capacity, capacity_for(need));
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
    rc = plan_alloc(p);
    if (rc == DIGS_OK) rc = hip_rc(hipStreamSynchronize(p->cap));
    if (rc == DIGS_OK && resized) *resized = 1;
    return rc;
}

extern "C" int digs_plan_get_tuning(const digs_plan *p, digs_tuning *out, float *tune_ms)
{
    if (!p || !out) return DIGS_EINVAL;
    *out = p->tuning;
    if (tune_ms) memcpy(tune_ms, p->tune_ms, sizeof(p->tune_ms));
    return DIGS_OK;
}

extern "C" int digs_plan_destroy(digs_plan *p)
{
    if (!p) return DIGS_OK;
    if (p->cap) (void)hipStreamSynchronize(p->cap);
    drop_graphs(p);
    if (p->ws) (void)hipFree(p->ws);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
    return DIGS_OK;
}
