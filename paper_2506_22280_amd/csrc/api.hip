// api.hip -- the extern "C" entry points of libdigs (declared in include/digs.h).
#include <math.h>
#include <algorithm>
#include <string.h>

#include "kernels.h"

static thread_local int g_last_hip_error = 0;

int digs_set_hip_error(hipError_t e)
{
    g_last_hip_error = (int)e;
    return DIGS_EHIP;
}

static int check(hipError_t e) { return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e); }

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static bool grid_ok(const digs_grid *g)
{
    return g && g->R >= 1 && g->R <= DIGS_MAX_RANK && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 &&
           g->spacing[0] > 0.0f && g->spacing[1] > 0.0f && g->spacing[2] > 0.0f &&
           isfinite(g->origin[0]) && isfinite(g->origin[1]) && isfinite(g->origin[2]) &&
           (size_t)(g->nx + 4) * (g->ny + 4) * (g->nz + 4) < (1u << 30);
}

static bool geom_ok(const digs_geom *g)
{
    if (!g || !(g->sid > 0.0f) || !(g->sdd > g->sid) || g->nu <= 0 || g->nv <= 0 ||
        !(g->pitch_u > 0.0f) || !(g->pitch_v > 0.0f) || !isfinite(g->off_u) ||
        !isfinite(g->off_v) || g->nu > 65535 || g->nv > 65535 ||
        (g->model != DIGS_MODEL_EXACT && g->model != DIGS_MODEL_EWA))
        return false;
    return true;
}

// The tile shape a tuning asks for (16 x 16 by default); false if it is not one of the shapes
// of one, two or four 8x8 blocks with edges of 8, 16 or 32 pixels.
static bool tile_shape(const digs_tuning *t, int *tw, int *th)
{
    *tw = DIGS_TILE;
    *th = DIGS_TILE;
    if (!t || (t->tile_w == 0 && t->tile_h == 0)) return true;
    auto edge = [](int e) { return e == 8 || e == 16 || e == 32; };
    if (!edge(t->tile_w) || !edge(t->tile_h) || t->tile_w * t->tile_h > DIGS_TILE_PX) return false;
    *tw = t->tile_w;
    *th = t->tile_h;
    return true;
}

static int log2_edge(int e) { return e == 8 ? 3 : (e == 16 ? 4 : 5); }

DevGeom make_dev_geom(const digs_geom *g, int tw, int th)
{
    DevGeom d;
    d.sid = g->sid;
    d.sdd = g->sdd;
    d.nu = g->nu;
    d.nv = g->nv;
    d.pitch_u = g->pitch_u;
    d.pitch_v = g->pitch_v;
    d.off_u = g->off_u;
    d.off_v = g->off_v;
    d.tile_w = tw;
    d.tile_h = th;
    d.tile_lw = log2_edge(tw);
    d.tile_lh = log2_edge(th);
    d.tile_bx = tw / 8;
    d.tile_nb = (tw / 8) * (th / 8);
    d.tiles_x = (g->nu + tw - 1) / tw;
    d.tiles_y = (g->nv + th - 1) / th;
    d.ntiles = d.tiles_x * d.tiles_y;
    d.ewa = g->model == DIGS_MODEL_EWA ? 1 : 0;
    return d;
}

DevGrid make_dev_grid(const digs_grid *g)
{
    DevGrid d;
    d.R = g->R;
    d.nx = g->nx;
    d.ny = g->ny;
    d.nz = g->nz;
    d.ox = g->origin[0];
    d.oy = g->origin[1];
    d.oz = g->origin[2];
    d.hx = g->spacing[0];
    d.hy = g->spacing[1];
    d.hz = g->spacing[2];
    return d;
}

// 16 instances per (view, Gaussian) at 16x16 tiles, in proportion for smaller tiles
static int64_t default_capacity(int n, int T, int tile_px)
{
    return (int64_t)16 * (DIGS_TILE_PX / tile_px) * n * T + 4096;
}

// Workgroups per tile list when the caller leaves it open: a launch with few (view, tile) items
// (one view, a small detector) leaves most SIMDs with one wave, so its lists are cut into slices
// until there are about 4096 workgroups, at most DIGS_MAX_SLICES per list (one 256x256 view of
// 50k Gaussians: forward 0.28 ms with one slice, 0.19 with 8, 0.17 with 16).
static int default_slices(int64_t items)
{
    if (items >= 2048 || items <= 0) return 1;
    const int64_t s = (4096 + items - 1) / items;
    return (int)(s < DIGS_MAX_SLICES ? s : DIGS_MAX_SLICES);
}

bool ws_layout(const digs_geom *geom, const digs_grid *grid, int n, int T,
               const digs_tuning *tuning, WsLayout *L, bool fwd_only)
{
    if (!geom_ok(geom) || !grid_ok(grid) || n < 0 || T < 0 || n > DIGS_MAX_GAUSSIANS) return false;
    if (tuning && (tuning->slices < 0 || tuning->slices > DIGS_MAX_SLICES)) return false;
    int tw, th;
    if (!tile_shape(tuning, &tw, &th)) return false;
    memset(L, 0, sizeof(*L));
    const DevGeom G = make_dev_geom(geom, tw, th);
    if ((int64_t)G.tiles_x * G.tiles_y > DIGS_MAX_TILES) return false;
    L->n = n;
    L->T = T;
    L->R = grid->R;
    L->slices = (tuning && tuning->slices > 0) ? tuning->slices
                                               : default_slices((int64_t)T * G.ntiles);
    // tile binning: smaller workgroups when the launch would have fewer than ~1024 of them
    {
        const int64_t full = (int64_t)(T > 0 ? T : 1) * ((n + DIGS_BIN_ITEMS - 1) / DIGS_BIN_ITEMS);
        L->bin_items = full < 1024 ? DIGS_BIN_ITEMS_SMALL : DIGS_BIN_ITEMS;
    }
    L->nblk = (n + L->bin_items - 1) / L->bin_items;
    L->ntiles = G.ntiles;
    L->ncells = (grid->nx + 4) * (grid->ny + 4) * (grid->nz + 4);
    L->gq_stride = 6 + 12 * grid->R;
    // the per-Gaussian adjoint runs one thread per (Gaussian, chunk of views): enough chunks for
    // about 256k threads (at this kernel's register use one round of the chip holds ~130k, so the
    // last round's tail stays short), a function of n and T alone so that the sums' order is fixed
    {
        const int Tp = T > 0 ? T : 1;
        const int want = (int)std::min<int64_t>(Tp, std::max<int64_t>(1, (262144 + (int64_t)n - 1) /
                                                                           std::max(n, 1)));
        L->tpc = (Tp + want - 1) / want;
        L->tchunks = (Tp + L->tpc - 1) / L->tpc;
    }
    int64_t cap = (tuning && tuning->capacity > 0) ? tuning->capacity
                                                   : default_capacity(n, T, tw * th);
    if (cap > 0xFFFFFF00ll) cap = 0xFFFFFF00ll;   // list positions are 32-bit
    L->cap = (size_t)cap;
    const size_t N = (size_t)(n > 0 ? n : 1), TN = (size_t)(T > 0 ? T : 1) * N;
    const size_t cnt_elems = (size_t)(T > 0 ? T : 1) * G.ntiles * (L->nblk > 0 ? L->nblk : 1) + 1;
    const int nblk_r = (int)((N + DIGS_BIN_ITEMS - 1) / DIGS_BIN_ITEMS);
    size_t sc = scan_scratch_elems(cnt_elems);
    size_t s2 = scan_scratch_elems(TN), s3 = scan_scratch_elems((size_t)256 * nblk_r);
    if (s2 > sc) sc = s2;
    if (s3 > sc) sc = s3;
    L->scratch_elems = sc;
    const int nparts = (int)((N + 255) / 256) * 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L->diag = take(sizeof(DiagBlock));
    L->queue = take(8 * sizeof(uint32_t));
    L->uv = take(sizeof(float) * 12 * grid->R * N);
    L->gsort = take(sizeof(float) * 11 * N);
    L->rec = take(sizeof(float) * DIGS_REC_FLOATS * TN);
    L->rect = take(sizeof(int) * 4 * TN);
    L->gcount = take(sizeof(uint32_t) * TN);
    L->cnt = take(sizeof(uint32_t) * 2 * cnt_elems);   // counts, then the waves' offsets
    L->scratch = take(sizeof(uint32_t) * sc);
    L->list = take(sizeof(uint32_t) * L->cap);
    const size_t bwd = fwd_only ? 0 : 1;   // the backward's arrays
    L->goff = take(bwd * sizeof(uint32_t) * TN);
    L->part = take(bwd * sizeof(float) * DIGS_PART_FLOATS * L->cap);
    L->gwpart = take(bwd * sizeof(float) * (size_t)(T > 0 ? T : 1) * grid->R * nparts);
    L->keys_a = take(sizeof(uint32_t) * N);
    L->vals_a = take(sizeof(uint32_t) * N);
    L->keys_b = take(sizeof(uint32_t) * N);
    L->vals_b = take(sizeof(uint32_t) * N);
    L->rhist = take(sizeof(uint32_t) * 2 * 256 * (size_t)nblk_r);
    L->cell_start = take(sizeof(uint32_t) * ((size_t)L->ncells + 1));
    L->tacc = take(bwd * sizeof(float) * (13 + 12 * (size_t)grid->R) * L->tchunks * N);
    L->order = take(sizeof(uint32_t) * N);
    L->gq = take(bwd * sizeof(float) * L->gq_stride * N);
    L->spart = take(L->slices > 1 ? sizeof(float) * L->slices * (size_t)(T > 0 ? T : 1) *
                                        G.ntiles * (size_t)(tw * th)
                                  : 0);
    L->total = off;
    return true;
}

extern "C" size_t digs_workspace_size(const digs_geom *geom, const digs_grid *grid, int n, int T,
                                      const digs_tuning *tuning)
{
    WsLayout L;
    if (!ws_layout(geom, grid, n, T, tuning, &L)) return 0;
    return L.total;
}

extern "C" int digs_ffd_eval(const digs_grid *grid, const float *coef, int n, const float *x,
                             int T, const float *w, float *disp, float *jac, void *stream)
{
    if (!grid_ok(grid) || n < 0) return DIGS_EINVAL;
    if (n == 0) return DIGS_OK;
    if (!coef || !x || !disp || (w && T <= 0)) return DIGS_EINVAL;
    return check(launch_ffd_eval(make_dev_grid(grid), coef, n, x, w ? T : 0, w, disp, jac,
                                 (hipStream_t)stream));
}

extern "C" int digs_deform_gaussians(const digs_grid *grid, const float *coef, int n,
                                     const float *mu, const float *scale, const float *quat,
                                     int T, const float *w, float *mu_t, float *cov_t,
                                     void *stream)
{
    if (!grid_ok(grid) || n < 0 || T < 0) return DIGS_EINVAL;
    if (n == 0 || T == 0) return DIGS_OK;
    if (!coef || !mu || !scale || !quat || !w || !mu_t || !cov_t) return DIGS_EINVAL;
    return check(launch_deform(make_dev_grid(grid), coef, n, mu, scale, quat, T, w, mu_t, cov_t,
                               (hipStream_t)stream));
}

static bool temporal_ok(int Ct, int R, float t0, float dt, int T)
{
    return Ct >= 1 && R >= 1 && R <= DIGS_MAX_RANK && T >= 0 && isfinite(t0) && dt > 0.0f &&
           isfinite(dt) && (int64_t)Ct * R < (1ll << 30) && (int64_t)T * R < (1ll << 30);
}

extern "C" int digs_temporal_weights(int Ct, int R, const float *ctrl, float t0, float dt, int T,
                                     const float *times, float *w, void *stream)
{
    if (!temporal_ok(Ct, R, t0, dt, T)) return DIGS_EINVAL;
    if (T == 0) return DIGS_OK;
    if (!ctrl || !times || !w) return DIGS_EINVAL;
    return check(launch_temporal_fwd(Ct, R, ctrl, t0, dt, T, times, w, (hipStream_t)stream));
}

extern "C" int digs_temporal_weights_bwd(int Ct, int R, float t0, float dt, int T,
                                         const float *times, const float *g_w, float *g_ctrl,
                                         void *stream)
{
    if (!temporal_ok(Ct, R, t0, dt, T)) return DIGS_EINVAL;
    if (!g_ctrl || (T > 0 && (!times || !g_w))) return DIGS_EINVAL;
    if (T == 0) return check(render_zero(g_ctrl, (size_t)Ct * R, (hipStream_t)stream));
    return check(launch_temporal_bwd(Ct, R, t0, dt, T, times, g_w, g_ctrl, (hipStream_t)stream));
}

int render_prepare(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                   const float *mu, const float *scale, const float *quat, const float *rho,
                   int T, const float *angles, const float *w, void *ws, size_t ws_bytes,
                   const digs_tuning *tuning, bool fwd_only, RenderArgs *a)
{
    if (!geom_ok(geom) || !grid_ok(grid) || n < 0 || T < 0 || n > DIGS_MAX_GAUSSIANS)
        return DIGS_EINVAL;
    if (tuning && (tuning->capacity < 0 || !(tuning->cull_radius >= 0.0f) ||
                   (tuning->splat_waves != 0 && tuning->splat_waves != 1 &&
                    tuning->splat_waves != 4) ||
                   tuning->slices < 0 || tuning->slices > DIGS_MAX_SLICES ||
                   tuning->persistent < 0 || tuning->persistent > 1))
        return DIGS_EINVAL;
    if (T > 0 && n > 0 && (!coef || !mu || !scale || !quat || !rho || !angles || !w))
        return DIGS_EINVAL;
    if (!ws_layout(geom, grid, n, T, tuning, &a->L, fwd_only)) return DIGS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < a->L.total) return DIGS_ENOWS;
    int tw, th;
    (void)tile_shape(tuning, &tw, &th);   // checked by ws_layout
    a->geom = make_dev_geom(geom, tw, th);
    a->grid = make_dev_grid(grid);
    a->coef = coef;
    a->basis = nullptr;
    a->mu = mu;
    a->scale = scale;
    a->quat = quat;
    a->rho = rho;
    a->angles = angles;
    a->w = w;
    a->n = n;
    a->T = T;
    a->cull = (tuning && tuning->cull_radius > 0.0f) ? tuning->cull_radius : 5.0f;
    a->splat_waves = (tuning && tuning->splat_waves) ? tuning->splat_waves : 4;
    a->persistent = tuning ? tuning->persistent : 0;
    a->ws = (char *)ws;
    return DIGS_OK;
}

int project_fwd_impl(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                     const float *mu, const float *scale, const float *quat, const float *rho,
                     int T, const float *angles, const float *w, float *proj, void *ws,
                     size_t ws_bytes, const digs_tuning *tuning, bool views_only, void *stream)
{
    RenderArgs a;
    int rc = render_prepare(geom, grid, coef, n, mu, scale, quat, rho, T, angles, w, ws,
                            ws_bytes, tuning, false, &a);
    if (rc) return rc;
    if (T == 0) return DIGS_OK;
    if (!proj) return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return check(render_zero(proj, (size_t)T * geom->nu * geom->nv, s));
    hipError_t e = views_only ? render_forward_views(a, s) : render_forward_setup(a, s);
    if (e == hipSuccess) e = render_forward_splat(a, proj, s);
    return check(e);
}

extern "C" int digs_project_fwd(const digs_geom *geom, const digs_grid *grid, const float *coef,
                                int n, const float *mu, const float *scale, const float *quat,
                                const float *rho, int T, const float *angles, const float *w,
                                float *proj, void *ws, size_t ws_bytes,
                                const digs_tuning *tuning, void *stream)
{
    return project_fwd_impl(geom, grid, coef, n, mu, scale, quat, rho, T, angles, w, proj, ws,
                            ws_bytes, tuning, false, stream);
}

extern "C" int digs_project_bwd(const digs_geom *geom, const digs_grid *grid, const float *coef,
                                int n, const float *mu, const float *scale, const float *quat,
                                const float *rho, int T, const float *angles, const float *w,
                                const float *grad_proj, float *g_mu, float *g_scale,
                                float *g_quat, float *g_rho, float *g_coef, float *g_w, void *ws,
                                size_t ws_bytes, const digs_tuning *tuning, int flags,
                                void *stream)
{
    RenderArgs a;
    int rc = render_prepare(geom, grid, coef, n, mu, scale, quat, rho, T, angles, w, ws,
                            ws_bytes, tuning, false, &a);
    if (rc) return rc;
    if (!g_coef || (n > 0 && (!g_mu || !g_scale || !g_quat || !g_rho)) ||
        (T > 0 && (!g_w || (n > 0 && !grad_proj))))
        return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t ncoef = (size_t)grid->R * grid->nx * grid->ny * grid->nz * 3;
    hipError_t e = hipSuccess;
    if (n == 0 || T == 0) {
        e = render_zero(g_coef, ncoef, s);
        if (e == hipSuccess && T > 0) e = render_zero(g_w, (size_t)T * grid->R, s);
        if (e == hipSuccess && n > 0) {
            e = render_zero(g_mu, (size_t)3 * n, s);
            if (e == hipSuccess) e = render_zero(g_scale, (size_t)3 * n, s);
            if (e == hipSuccess) e = render_zero(g_quat, (size_t)4 * n, s);
            if (e == hipSuccess) e = render_zero(g_rho, (size_t)n, s);
        }
        return check(e);
    }
    if (!(flags & DIGS_BWD_REUSE_FWD)) e = render_forward_setup(a, s);
    if (e == hipSuccess)
        e = render_backward(a, grad_proj, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    return check(e);
}

// The second ablation's motion model (per-Gaussian basis instead of the lattice): the same
// forward and adjoint with U, V gathered from `basis` and no lattice terms.
extern "C" int digs_project_basis_fwd(const digs_geom *geom, const digs_grid *grid,
                                      const float *basis, int n, const float *mu,
                                      const float *scale, const float *quat, const float *rho,
                                      int T, const float *angles, const float *w, float *proj,
                                      void *ws, size_t ws_bytes, const digs_tuning *tuning,
                                      void *stream)
{
    RenderArgs a;
    int rc = render_prepare(geom, grid, basis, n, mu, scale, quat, rho, T, angles, w, ws,
                            ws_bytes, tuning, false, &a);
    if (rc) return rc;
    a.basis = basis;
    if (T == 0) return DIGS_OK;
    if (!proj) return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return check(render_zero(proj, (size_t)T * geom->nu * geom->nv, s));
    hipError_t e = render_forward_setup(a, s);
    if (e == hipSuccess) e = render_forward_splat(a, proj, s);
    return check(e);
}

extern "C" int digs_project_basis_bwd(const digs_geom *geom, const digs_grid *grid,
                                      const float *basis, int n, const float *mu,
                                      const float *scale, const float *quat, const float *rho,
                                      int T, const float *angles, const float *w,
                                      const float *grad_proj, float *g_mu, float *g_scale,
                                      float *g_quat, float *g_rho, float *g_basis, float *g_w,
                                      void *ws, size_t ws_bytes, const digs_tuning *tuning,
                                      int flags, void *stream)
{
    RenderArgs a;
    int rc = render_prepare(geom, grid, basis, n, mu, scale, quat, rho, T, angles, w, ws,
                            ws_bytes, tuning, false, &a);
    if (rc) return rc;
    a.basis = basis;
    if ((n > 0 && (!g_mu || !g_scale || !g_quat || !g_rho || !g_basis)) ||
        (T > 0 && (!g_w || (n > 0 && !grad_proj))))
        return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (n == 0 || T == 0) {
        if (T > 0) e = render_zero(g_w, (size_t)T * grid->R, s);
        if (e == hipSuccess && n > 0) {
            e = render_zero(g_mu, (size_t)3 * n, s);
            if (e == hipSuccess) e = render_zero(g_scale, (size_t)3 * n, s);
            if (e == hipSuccess) e = render_zero(g_quat, (size_t)4 * n, s);
            if (e == hipSuccess) e = render_zero(g_rho, (size_t)n, s);
            if (e == hipSuccess) e = render_zero(g_basis, (size_t)12 * grid->R * n, s);
        }
        return check(e);
    }
    if (!(flags & DIGS_BWD_REUSE_FWD)) e = render_forward_setup(a, s);
    if (e == hipSuccess)
        e = render_backward(a, grad_proj, g_mu, g_scale, g_quat, g_rho, g_basis, g_w, s);
    return check(e);
}

extern "C" int digs_count_pairs(const digs_geom *geom, const digs_grid *grid, int n, int T,
                                void *ws, size_t ws_bytes, const digs_tuning *tuning,
                                uint64_t *out, void *stream)
{
    RenderArgs a;
    if (!out) return DIGS_EINVAL;
    const float dummy = 0.0f;
    int rc = render_prepare(geom, grid, &dummy, n, &dummy, &dummy, &dummy, &dummy, T, &dummy,
                            &dummy, ws, ws_bytes, tuning, false, &a);
    if (rc) return rc;
    out[0] = out[1] = out[2] = 0;
    if (n == 0 || T == 0) return DIGS_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = render_count_pairs(a, s);
    DiagBlock d;
    if (e == hipSuccess) e = hipMemcpyAsync(&d, ws, sizeof(d), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return digs_set_hip_error(e);
    out[0] = d.stat[0];
    out[1] = d.stat[1];
    out[2] = d.stat[2];
    return DIGS_OK;
}

extern "C" int digs_read_diagnostics(const void *ws, digs_diag *out, void *stream)
{
    if (!ws || !out) return DIGS_EINVAL;
    DiagBlock d;
    hipError_t e = hipMemcpyAsync(&d, ws, sizeof(d), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return digs_set_hip_error(e);
    memset(out, 0, sizeof(*out));
    if (d.stamp != DIAG_STAMP) return DIGS_OK;   // no call has run on this workspace yet
    out->instances = d.instances;
    out->capacity = d.capacity;
    out->overflow = d.overflow;
    out->nonfinite = d.nonfinite;
    out->folded = d.folded;
    out->behind_source = d.behind_source;
    out->wide = d.wide;
    out->max_instances = d.max_instances;
    return DIGS_OK;
}

__global__ void k_diag_reset(DiagBlock *d) { diag_clear(d); }

extern "C" int digs_reset_diagnostics(void *ws, void *stream)
{
    if (!ws) return DIGS_EINVAL;
    hipLaunchKernelGGL(k_diag_reset, dim3(1), dim3(1), 0, (hipStream_t)stream, (DiagBlock *)ws);
    return check(hipGetLastError());
}

extern "C" const char *digs_strerror(int code)
{
    switch (code) {
    case DIGS_OK: return "ok";
    case DIGS_EINVAL: return "invalid argument";
    case DIGS_ENOWS: return "workspace missing, misaligned or too small";
    case DIGS_EHIP: return "HIP runtime error";
    case DIGS_ECAPACITY: return "instance capacity exceeded";
    case DIGS_ENOMEM: return "out of device memory";
    case DIGS_ESCRATCH: return "problem too large for the fixed device array of the no-allocation call";
    default: return "unknown error";
    }
}

extern "C" int digs_last_hip_error(void) { return g_last_hip_error; }
