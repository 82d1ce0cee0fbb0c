// kernels.h -- internal interface between the libdigs entry points and their kernels.
#pragma once

#include "common.h"

// ------------------------------------------------------------------------------------------
// Workspace layout of digs_project_fwd / digs_project_bwd (byte offsets, 256-byte aligned).
struct WsLayout {
    size_t diag;       // DiagBlock
    size_t queue;      // [8] u32 work-queue counters of the persistent splats
    size_t uv;         // [3R + 9R][N] f32: per-rank u_r(mu), grad u_r(mu) at the canonical means
    size_t gsort;      // [11][N] f32: mu, scale, quat, rho of the Gaussians in cell order
    size_t rec;        // [T][N][16] f32 projected records
    size_t rect;       // [T][N] int4 tile rectangle (tx0 | tx1 << 16, ty0 | ty1 << 16) and instance mask
    size_t gcount;     // [T][N] u32 instances per (t,n) (the forward's set-up)
    size_t goff;       // [T][N] u32 instance offsets: exclusive scan of gcount (the backward's)
    size_t cnt;        // [T][ntiles][nblk] u32 per-block tile counts, scanned in place; then as
                       //     many words of the blocks' per-wave offsets (binning)
    size_t scratch;    // scan block sums
    size_t list;       // [cap] u32 Gaussian index of each instance, grouped by (t, tile)
    size_t part;       // [cap][12] f32 backward partial sums, instance (t,n,k) at goff[t][n]+k
    size_t gwpart;     // [T][R][4*ceil(N/256)] f32 per-wave partial sums of dL/dw
    size_t keys_a, vals_a, keys_b, vals_b;  // [N] u32 cell sort ping-pong
    size_t rhist;      // 2 x [256][ceil(N/1024)] u32 radix digit histograms, per-wave offsets
    size_t cell_start;                      // [ncells + 1] u32 first position of each cell
    size_t tacc;       // [13 + 12R][tchunks][N] f32 per-Gaussian adjoint sums over chunks of views
    size_t order;      // [N] u32 the Gaussian at each position of cell order (per-Gaussian arrays
                       //     of a call, records included, are laid out in cell order)
    size_t gq;         // [N][6 + 12R] f32 per-Gaussian coefficient-gradient sources, cell order
    size_t spart;      // [slices][T][ntiles][tile pixels] f32 forward partial images (slices > 1)
    size_t total;
    // derived sizes
    int n, T, R, nblk, ntiles, ncells, gq_stride;
    int bin_items;     // Gaussians per tile-binning workgroup (nblk = ceil(n / bin_items))
    int tpc, tchunks;  // views per chunk of the per-Gaussian adjoint, and the number of chunks
    int slices;        // workgroups per tile list in the splats (1: the whole list)
    size_t cap;
    size_t scratch_elems;
};

// fwd_only: the forward's arrays alone (the backward's partials, adjoint sums and coefficient-
// gradient sources get no space)
bool ws_layout(const digs_geom *geom, const digs_grid *grid, int n, int T,
               const digs_tuning *tuning, WsLayout *L, bool fwd_only = false);

DevGeom make_dev_geom(const digs_geom *g, int tile_w, int tile_h);
DevGrid make_dev_grid(const digs_grid *g);

// scan.hip
size_t scan_scratch_elems(size_t n);
// exclusive prefix sum of src (default: data itself) into data
hipError_t launch_exclusive_scan(uint32_t *data, size_t n, uint32_t *scratch, hipStream_t s,
                                 const uint32_t *src = nullptr);

// ffd.hip
hipError_t launch_ffd_eval(const DevGrid &g, const float *coef, int n, const float *x, int T,
                           const float *w, float *disp, float *jac, hipStream_t s);
hipError_t launch_deform(const DevGrid &g, const float *coef, int n, const float *mu,
                         const float *scale, const float *quat, int T, const float *w,
                         float *mu_t, float *cov_t, hipStream_t s);
hipError_t launch_temporal_fwd(int Ct, int R, const float *ctrl, float t0, float dt, int T,
                               const float *times, float *w, hipStream_t s);
hipError_t launch_temporal_bwd(int Ct, int R, float t0, float dt, int T, const float *times,
                               const float *g_w, float *g_ctrl, hipStream_t s);

// render.hip
struct RenderArgs {
    DevGeom geom;
    DevGrid grid;
    const float *coef, *mu, *scale, *quat, *rho, *angles, *w;
    const float *basis;   // per-Gaussian motion basis [R][12][N] instead of the FFD, or null
    int n, T;
    float cull;
    int splat_waves, persistent;
    char *ws;
    WsLayout L;
};
hipError_t render_forward_setup(const RenderArgs &a, hipStream_t s);   // a1-a4
hipError_t render_forward_canonical(const RenderArgs &a, hipStream_t s);   // a1 (per Gaussian)
hipError_t render_forward_views(const RenderArgs &a, hipStream_t s);       // a2-a4 (per view)
// digs_project_fwd; with views_only the per-Gaussian stage in ws is taken as it is (it must come
// from an earlier call on ws with the same Gaussians and lattice)
int project_fwd_impl(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                     const float *mu, const float *scale, const float *quat, const float *rho,
                     int T, const float *angles, const float *w, float *proj, void *ws,
                     size_t ws_bytes, const digs_tuning *tuning, bool views_only, void *stream);
hipError_t render_forward_splat(const RenderArgs &a, float *proj, hipStream_t s);  // a5
// g_coef: dL/dcoef, or with a.basis dL/dbasis [R][12][N]
hipError_t render_backward(const RenderArgs &a, const float *grad_proj, float *g_mu,
                           float *g_scale, float *g_quat, float *g_rho, float *g_coef,
                           float *g_w, hipStream_t s);                   // a6-a8
hipError_t render_zero(float *p, size_t count, hipStream_t s);
// Checks the arguments of a render call and fills *a (api.hip); DIGS_OK or a DIGS_E* code.
int render_prepare(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                   const float *mu, const float *scale, const float *quat, const float *rho, int T,
                   const float *angles, const float *w, void *ws, size_t ws_bytes,
                   const digs_tuning *tuning, bool fwd_only, RenderArgs *a);
hipError_t render_count_pairs(const RenderArgs &a, hipStream_t s);   // measurement only
void render_prepare_launch_shapes();
