// plan.hip -- a prepared renderer for fixed shapes and fixed device buffers (the batched path):
// it owns its workspace, holds the launch tuning (given by the caller, or chosen by timing the
// candidate launch shapes on the caller's data), and captures the forward and the backward launch
// sequences once each as HIP graphs that later calls replay. When a sequence is first called the
// plan times its graph replay against launching the same kernels directly on the stream and keeps
// the faster (a graph replay costs a few microseconds more than direct launches for short
// sequences such as one view's forward); both give the same bits.
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
    int replay = DIGS_REPLAY_TIMED;
    int chosen[3] = {0, 0, 0};   // per sequence (0 forward, 1 backward, 2 per-view forward):
                                 // DIGS_REPLAY_GRAPH or _DIRECT, 0 before its first call
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
    p->chosen[0] = p->chosen[1] = p->chosen[2] = 0;
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
    hipGraph_t &gs = which == 0 ? p->gf : which == 2 ? p->gv : p->gb;
    hipGraphExec_t &xs = which == 0 ? p->ef : which == 2 ? p->ev : p->eb;
    if (xs) (void)hipGraphExecDestroy(xs);   // (one recorded earlier whose timing failed)
    if (gs) (void)hipGraphDestroy(gs);
    gs = g;
    xs = x;
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

// One stream waits for everything another has queued so far.
static int order_after(hipStream_t waiter, hipStream_t s)
{
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return digs_set_hip_error(hipGetLastError());
    hipError_t e = hipEventRecord(ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
    (void)hipEventDestroy(ev);
    return hip_rc(e);
}

static int run_direct(digs_plan *p, int which, hipStream_t s)
{
    return which == 0 ? run_fwd(p, s) : which == 2 ? run_fwd(p, s, true) : run_bwd(p, s);
}

static hipGraphExec_t graph_of(const digs_plan *p, int which)
{
    return which == 0 ? p->ef : which == 2 ? p->ev : p->eb;
}

// Median of three timed runs of sequence `which` on the plan's stream, after one untimed run;
// graph: as a replay, else as direct launches.
static int time_sequence(digs_plan *p, int which, bool graph, float *ms)
{
    hipEvent_t e[4];
    for (int k = 0; k < 4; ++k)
        if (hipEventCreate(&e[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(e[j]);
            return digs_set_hip_error(hipGetLastError());
        }
    int rc = DIGS_OK;
    for (int k = 0; k < 4 && rc == DIGS_OK; ++k) {
        rc = graph ? hip_rc(hipGraphLaunch(graph_of(p, which), p->cap))
                   : run_direct(p, which, p->cap);
        if (rc == DIGS_OK) rc = hip_rc(hipEventRecord(e[k], p->cap));
    }
    if (rc == DIGS_OK) rc = hip_rc(hipEventSynchronize(e[3]));
    float t[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3 && rc == DIGS_OK; ++k)
        rc = hip_rc(hipEventElapsedTime(&t[k], e[k], e[k + 1]));
    for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]);
    std::sort(t, t + 3);
    *ms = t[1];
    return rc;
}

// Before the first call of sequence `which` (or the first after the graphs were dropped): record
// its graph unless the replay is fixed to direct launches, and under DIGS_REPLAY_TIMED time the
// replay against direct launches on the plan's stream (after the work queued on `s`; `s` then
// waits for the timing runs, which compute what the call itself computes) and keep the faster.
static int prepare_sequence(digs_plan *p, int which, hipStream_t s)
{
    if (p->chosen[which] != 0) return DIGS_OK;
    if (p->replay == DIGS_REPLAY_DIRECT) {
        p->chosen[which] = DIGS_REPLAY_DIRECT;
        return DIGS_OK;
    }
    int rc = capture(p, which);
    if (rc != DIGS_OK) return rc;
    if (p->replay == DIGS_REPLAY_GRAPH) {
        p->chosen[which] = DIGS_REPLAY_GRAPH;
        return order_after(s, p->cap);
    }
    const int prof = digs_profile_enable(-1);
    digs_profile_enable(0);
    float tg = 0.0f, td = 0.0f;
    rc = order_after(p->cap, s);
    if (rc == DIGS_OK) rc = time_sequence(p, which, true, &tg);
    if (rc == DIGS_OK) rc = time_sequence(p, which, false, &td);
    digs_profile_enable(prof);
    if (rc == DIGS_OK) rc = order_after(s, p->cap);
    if (rc != DIGS_OK) return rc;
    p->chosen[which] = tg <= td ? DIGS_REPLAY_GRAPH : DIGS_REPLAY_DIRECT;
    return DIGS_OK;
}

static int launch_sequence(digs_plan *p, int which, hipStream_t s)
{
    const int rc = prepare_sequence(p, which, s);
    if (rc != DIGS_OK) return rc;
    return p->chosen[which] == DIGS_REPLAY_DIRECT ? run_direct(p, which, s)
                                                  : hip_rc(hipGraphLaunch(graph_of(p, which), s));
}

extern "C" int digs_plan_fwd(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0) return DIGS_OK;
    const int rc = launch_sequence(p, 0, (hipStream_t)stream);
    if (rc == DIGS_OK) p->canonical = true;
    return rc;
}

extern "C" int digs_plan_fwd_views(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0) return DIGS_OK;
    if (!p->canonical) return DIGS_EINVAL;   // no digs_plan_fwd on this workspace yet
    return launch_sequence(p, 2, (hipStream_t)stream);
}

extern "C" int digs_plan_bwd(digs_plan *p, void *stream)
{
    if (!p) return DIGS_EINVAL;
    if (p->T == 0 && p->n == 0) return DIGS_OK;
    if (!p->b.grad_proj && p->n > 0 && p->T > 0) return DIGS_EINVAL;
    return launch_sequence(p, 1, (hipStream_t)stream);
}

extern "C" int digs_plan_set_replay(digs_plan *p, int mode)
{
    if (!p || mode < DIGS_REPLAY_TIMED || mode > DIGS_REPLAY_DIRECT) return DIGS_EINVAL;
    // (replays may still be running on the callers' streams: the device is synchronised before
    // their graphs are destroyed)
    const int rc = hip_rc(hipDeviceSynchronize());
    if (rc != DIGS_OK) return rc;
    const bool canonical = p->canonical;   // the workspace keeps its contents
    drop_graphs(p);
    p->canonical = canonical;
    p->replay = mode;
    return DIGS_OK;
}

extern "C" int digs_plan_get_replay(const digs_plan *p, int *modes)
{
    if (!p || !modes) return DIGS_EINVAL;
    modes[0] = p->chosen[0];
    modes[1] = p->chosen[2];
    modes[2] = p->chosen[1];
    return DIGS_OK;
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
