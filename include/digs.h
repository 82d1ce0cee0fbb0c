/*
 * digs.h -- C ABI of libdigs, the gfx950 (MI355X) implementation of the deformation-informed
 * Gaussian X-ray renderer of DIGS (Huang et al., "Dynamic CBCT Reconstruction using
 * Deformation-Informed 4D Gaussian Splatting and a Low-Rank Free-Form Deformation Model").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays.   Every array argument is a DEVICE pointer to float32, C-contiguous, in the
 *           structure-of-arrays layouts given per argument. Structs (digs_geom, digs_grid,
 *           digs_tuning, digs_diag) are HOST pointers, read during the call only.
 * Ownership. The caller owns every buffer. Entry points never allocate device memory, except
 *           digs_plan_create (which owns the plan's workspace until digs_plan_destroy).
 *           Outputs are overwritten, gradients included.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null stream). Work is
 *           enqueued asynchronously; no entry point synchronises unless it says so.
 * Errors.   0 on success, a negative DIGS_E* code otherwise; nothing else crosses the ABI.
 *           Conditions that only the kernels can see (instance-list overflow, non-finite
 *           values, folded deformations, Gaussians at or behind the source) are counted in a
 *           diagnostics block inside the workspace; read it with digs_read_diagnostics after
 *           the work has run. An overflow is never silent: the results of that call are then
 *           incomplete and the call must be repeated with a larger capacity.
 * Threads.  Calls are re-entrant when their workspaces differ. Calls that share a workspace
 *           must be ordered on one stream.
 * Units.    mm, mm^-1 (densities), radians. Quaternions (w,x,y,z), unnormalised (normalised
 *           inside). Scales are linear standard deviations (mm). Activations of any learned
 *           parameterisation belong to the caller.
 *
 * Symbols used below: N Gaussians, T projections (time points) in a call, R ranks of the
 * low-rank motion model, (nx, ny, nz) control lattice, (nu, nv) detector columns and rows.
 */
#ifndef DIGS_H
#define DIGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIGS_OK 0
#define DIGS_EINVAL (-1)   /* null pointer, negative size, R outside 1..8, bad geometry       */
#define DIGS_ENOWS (-2)    /* workspace missing, misaligned or smaller than required          */
#define DIGS_EHIP (-3)     /* a HIP launch or runtime call failed (see digs_last_hip_error)    */
#define DIGS_ECAPACITY (-4) /* instance capacity exceeded (reported by diagnostics checks)     */
#define DIGS_ENOMEM (-5)   /* digs_plan_create could not allocate                             */
#define DIGS_ESCRATCH (-6) /* digs_project_fwd_noalloc: the problem does not fit the fixed array */

#define DIGS_MAX_RANK 8
#define DIGS_MAX_TILES 4096 /* detector tiles per projection, at the call's tile shape            */
#define DIGS_MAX_GAUSSIANS 16777215 /* 2^24 - 1 Gaussians per call                               */

/* Cone-beam CT geometry of a circular orbit about z (the paper's acquisition, Sec. 4.1).
 * View angle theta: source at sid*(cos, sin, 0); detector centre at (sid - sdd)*(cos, sin, 0);
 * detector axes e_u = (-sin, cos, 0), e_v = (0, 0, 1). Pixel (row j, column i) centre:
 * centre + (x_i + off_u) e_u + (y_j + off_v) e_v, x_i = (i - (nu-1)/2) pitch_u,
 * y_j = (j - (nv-1)/2) pitch_v. Projections are stored proj[t][j][i]. */
typedef struct digs_geom {
    float sid, sdd;          /* source-isocentre, source-detector distances (mm), sdd > sid > 0 */
    int nu, nv;              /* detector columns, rows (>0; at most DIGS_MAX_TILES tiles)      */
    float pitch_u, pitch_v;  /* pixel pitch (mm, >0)                                           */
    float off_u, off_v;      /* detector offset along e_u, e_v (mm)                            */
    int model;               /* projection model, DIGS_MODEL_EXACT (0) or DIGS_MODEL_EWA (1)   */
} digs_geom;

/* Projection models. EXACT: each Gaussian's line integral along the ray from the source to the
 * pixel centre, in closed form (Eq. 2 integrated along the ray of Eq. 1; what Eq. 4 approximates).
 * EWA: the 2D-Gaussian approximation of Sec. 3.1, Eq. 4: the Gaussian projected through the local
 * affine approximation of the perspective map at its mean (covariance J W Sigma' W^T J^T, top-left
 * 2x2), with density scaled so that the 2D Gaussian's peak equals the line integral along the ray
 * through the mean, rho sqrt(2 pi / (d^T Sigma'^-1 d)) for the unit direction d of that ray. */
#define DIGS_MODEL_EXACT 0
#define DIGS_MODEL_EWA 1

/* Uniform control lattice of the cubic B-spline FFD (Sec. 3.3, Eq. 10): control point (i,j,k)
 * of rank r sits at origin + (i,j,k)*spacing and stores d^r_ijk. Lattice index space is
 * 0-based; stencil indices outside the lattice are clamped to its edge. */
typedef struct digs_grid {
    int R;                   /* ranks N_r, 1..8                                                */
    int nx, ny, nz;          /* lattice size (each >= 1)                                        */
    float origin[3];         /* mm                                                             */
    float spacing[3];        /* mm, > 0                                                        */
} digs_grid;

/* Launch tuning; NULL selects the defaults. */
#define DIGS_MAX_SLICES 16
typedef struct digs_tuning {
    float cull_radius;       /* Mahalanobis cut-off of each Gaussian's footprint (default 5)   */
    int64_t capacity;        /* (Gaussian, tile) instances per call (default 16*N*T at 16x16
                                tiles, times 256 / tile pixels for smaller tiles)              */
    int splat_waves;         /* forward splat: waves per tile, 4 (one per 8x8 block, at most as
                                many as the tile has blocks) or 1 (default 4)                  */
    int slices;              /* workgroups per tile list in the splats, 1..DIGS_MAX_SLICES; 0: by
                                shape (1 when the call has >= 2048 (view, tile) items, else
                                enough for about 4096 workgroups, at most 16). Another value adds
                                the same terms in another order (results bitwise reproducible
                                for one value). With slices > 1 the splats are not persistent. */
    int persistent;          /* 1: splats run as persistent kernels over per-XCD work queues of
                                (view, tile) items; 0: one workgroup per item (default 0)      */
    int tile_w, tile_h;      /* detector tile in pixels; 0, 0: 16 x 16. A tile is one, two or
                                four blocks of 8 x 8 pixels: 16x16, 32x8, 8x32, 16x8, 8x16 or 8x8,
                                with at most DIGS_MAX_TILES tiles per projection. The tile shape
                                sets which (Gaussian, tile) instances exist and the lists' order
                                of work, so another shape adds the same terms in another order
                                (and needs another instance capacity). */
} digs_tuning;

/* Diagnostics counted by the kernels (read after the work has run). */
typedef struct digs_diag {
    uint64_t instances;      /* (Gaussian, tile) instances the last call needed               */
    uint64_t capacity;       /* capacity of the workspace                                     */
    uint32_t overflow;       /* nonzero if any call since the last reset exceeded capacity    */
    uint32_t nonfinite;      /* (t,n) with non-finite inputs or singular K, skipped           */
    uint32_t folded;         /* (t,n) with det K <= 0 (rendered, counted)                     */
    uint32_t behind_source;  /* (t,n) whose mean is not in front of the source, skipped       */
    uint32_t wide;           /* (t,n) whose footprint conic is not an ellipse: whole detector  */
    uint32_t reserved0;
    uint64_t max_instances;  /* the largest `instances` of any call since the last reset        */
    uint32_t reserved[4];
} digs_diag;

/* ---------------------------------------------------------------------------------------------
 * digs_ffd_eval -- the low-rank cubic B-spline FFD and its Jacobian (Sec. 3.3, Eq. 9-11).
 *   coef  [R][nz][ny][nx][3]   control displacements d^r (mm per unit weight)
 *   x     [3][n]               query points (mm)
 *   w     [T][R] or NULL       temporal weights
 *   disp  w == NULL: [R][3][n] per-rank u_r(x);  else [T][3][n] sum_r w[t][r] u_r(x)
 *   jac   w == NULL: [R][9][n] per-rank grad u_r(x);  else [T][9][n] sum_r w[t][r] grad u_r(x)
 *         (row-major 3x3, jac[.][3a+b][i] = d u_a / d x_b; the identity of Eq. 11 is NOT added)
 *         jac may be NULL (skipped).
 * n == 0 is a no-op. Errors: DIGS_EINVAL, DIGS_EHIP. */
int digs_ffd_eval(const digs_grid *grid, const float *coef, int n, const float *x, int T,
                  const float *w, float *disp, float *jac, void *stream);

/* digs_deform_gaussians -- the deformation-informed warp (Sec. 3.2, Eq. 7-8): for every
 * (t, n), mu' = mu + sum_r w_r(t) u_r(mu) and Sigma' = K Sigma K^T with
 * K = I + sum_r w_r(t) grad u_r(mu), Sigma = R(q) diag(s^2) R(q)^T (Sec. 3.1); rho unchanged.
 *   mu [3][n], scale [3][n], quat [4][n], w [T][R]
 *   mu_t [T][3][n];  cov_t [T][6][n] packed (xx, xy, xz, yy, yz, zz)
 * Errors: DIGS_EINVAL, DIGS_EHIP. */
int digs_deform_gaussians(const digs_grid *grid, const float *coef, int n, const float *mu,
                          const float *scale, const float *quat, int T, const float *w,
                          float *mu_t, float *cov_t, void *stream);

/* digs_temporal_weights -- the temporal weights w_r(t) of the low-rank motion model: a cubic
 * 1-D B-spline in time (Sec. 3.3, after Eq. 11; Sec. 4.2 places a control value every 4 time
 * points), with the lattice's knot convention: control value j sits at time t0 + j*dt;
 * p = (times[t] - t0)/dt, f = floor(p), u = p - f and
 *   w[t][r] = sum_{l=0..3} B_l(u) ctrl[clamp(f - 1 + l, 0, Ct - 1)][r].
 *   ctrl [Ct][R] control values, times [T] (any unit, the same as t0 and dt), w [T][R] out.
 * digs_temporal_weights_bwd: g_ctrl [Ct][R] = the adjoint applied to g_w [T][R] (overwritten).
 * Errors: DIGS_EINVAL (Ct < 1, R outside 1..8, dt <= 0, null pointers), DIGS_EHIP. */
int digs_temporal_weights(int Ct, int R, const float *ctrl, float t0, float dt, int T,
                          const float *times, float *w, void *stream);
int digs_temporal_weights_bwd(int Ct, int R, float t0, float dt, int T, const float *times,
                              const float *g_w, float *g_ctrl, void *stream);

/* Workspace bytes that digs_project_fwd / digs_project_bwd need for this problem size (one
 * workspace serves both). Returns 0 for invalid arguments. */
size_t digs_workspace_size(const digs_geom *geom, const digs_grid *grid, int n, int T,
                           const digs_tuning *tuning);

/* digs_project_fwd -- projections of the deformed Gaussians (Sec. 3.1, Eq. 1, 3, 4, 6):
 * proj[t][j][i] = sum_n of the integral of G_n(x | rho_n, mu'_{n,t}, Sigma'_{n,t}) along the
 * whole ray from the source to pixel (j,i) at angle angles[t], each Gaussian cut off beyond
 * tuning->cull_radius Mahalanobis units of its footprint.
 *   mu [3][n], scale [3][n], quat [4][n], rho [n]; angles [T]; w [T][R]; proj [T][nv][nu]
 *   ws / ws_bytes: device workspace of at least digs_workspace_size bytes, 256-byte aligned.
 * The workspace keeps what digs_project_bwd can reuse (see DIGS_BWD_REUSE_FWD).
 * n == 0 writes zeros. Errors: DIGS_EINVAL, DIGS_ENOWS, DIGS_EHIP. */
int digs_project_fwd(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                     const float *mu, const float *scale, const float *quat, const float *rho,
                     int T, const float *angles, const float *w, float *proj, void *ws,
                     size_t ws_bytes, const digs_tuning *tuning, void *stream);

#define DIGS_BWD_REUSE_FWD 1  /* ws holds the state of a digs_project_fwd with identical inputs
                                 and tuning */

/* digs_project_fwd_noalloc -- digs_project_fwd for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the forward's intermediate buffers in a device array the library owns
 * (DIGS_NOALLOC_SCRATCH_BYTES on every GPU it runs on, held until the process ends) instead of a
 * caller workspace. The call allocates nothing and takes no workspace.
 *   Arguments as digs_project_fwd; diag_out is a DEVICE pointer to one digs_diag (or NULL) that
 *   receives this call's diagnostics when its work has run (max_instances = instances; overflow
 *   means proj is incomplete and the call must be repeated with a larger tuning->capacity).
 * Limit: the forward's working set (about 84 bytes per (view, Gaussian), 4 bytes per instance of
 * capacity, 12R + 24 floats per Gaussian) must fit DIGS_NOALLOC_SCRATCH_BYTES, else DIGS_ESCRATCH
 * is returned before any device work. Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (unordered streams or threads) race; order them on one stream.
 * Errors: DIGS_EINVAL, DIGS_ESCRATCH, DIGS_EHIP. */
#define DIGS_NOALLOC_SCRATCH_BYTES (64u << 20)
int digs_project_fwd_noalloc(const digs_geom *geom, const digs_grid *grid, const float *coef,
                             int n, const float *mu, const float *scale, const float *quat,
                             const float *rho, int T, const float *angles, const float *w,
                             float *proj, digs_diag *diag_out, const digs_tuning *tuning,
                             void *stream);

/* digs_project_bwd -- the hand-written adjoint of digs_project_fwd. Given grad_proj = dL/dproj
 * [T][nv][nu], writes dL/d(each input):
 *   g_mu [3][n], g_scale [3][n], g_quat [4][n], g_rho [n], g_coef [R][nz][ny][nx][3], g_w [T][R]
 * The mean gradient includes the term through K(mu) (second derivatives of the B-spline).
 * A Gaussian whose inputs the forward rejects (non-finite mean, quaternion or density, a scale
 * that is not positive; counted in nonfinite) gets zero gradients and adds nothing to g_coef.
 * Without DIGS_BWD_REUSE_FWD in `flags` the forward set-up and binning are recomputed.
 * Reductions are fixed-order: results are bitwise reproducible run to run.
 * Errors: DIGS_EINVAL, DIGS_ENOWS, DIGS_EHIP. */
int digs_project_bwd(const digs_geom *geom, const digs_grid *grid, const float *coef, int n,
                     const float *mu, const float *scale, const float *quat, const float *rho,
                     int T, const float *angles, const float *w, const float *grad_proj,
                     float *g_mu, float *g_scale, float *g_quat, float *g_rho, float *g_coef,
                     float *g_w, void *ws, size_t ws_bytes, const digs_tuning *tuning, int flags,
                     void *stream);

/* digs_project_basis_fwd / digs_project_basis_bwd -- the same forward and adjoint with the
 * motion model of the paper's second ablation (Sec. 4.3): the spatial basis is stored per
 * Gaussian instead of being interpolated from the control lattice, so for every (t, n)
 *   mu' = mu + sum_r w_r(t) u_{n,r},  K = I + sum_r w_r(t) V_{n,r},  Sigma' = K Sigma K^T.
 *   basis [R][12][n]: rows 0..2 u_{n,r} (mm per unit weight), rows 3..11 V_{n,r} row-major.
 *   grid: R and the lattice geometry, used only to order the Gaussians by cell for memory
 *   locality (no coefficients are read). Workspace as digs_project_fwd (same size).
 *   g_basis [R][12][n] = dL/dbasis; g_mu has no lattice terms. Other arguments, layouts and
 *   errors as digs_project_fwd / digs_project_bwd. */
int digs_project_basis_fwd(const digs_geom *geom, const digs_grid *grid, const float *basis,
                           int n, const float *mu, const float *scale, const float *quat,
                           const float *rho, int T, const float *angles, const float *w,
                           float *proj, void *ws, size_t ws_bytes, const digs_tuning *tuning,
                           void *stream);
int digs_project_basis_bwd(const digs_geom *geom, const digs_grid *grid, const float *basis,
                           int n, const float *mu, const float *scale, const float *quat,
                           const float *rho, int T, const float *angles, const float *w,
                           const float *grad_proj, float *g_mu, float *g_scale, float *g_quat,
                           float *g_rho, float *g_basis, float *g_w, void *ws, size_t ws_bytes,
                           const digs_tuning *tuning, int flags, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Plans: the batched path. A plan fixes the shapes (geometry, lattice, N, T) and the device
 * buffers below; it owns its workspace and replays the forward and the backward as HIP graphs
 * (captured on first use) or as direct launches (digs_plan_set_replay). Inputs are read at replay time, so the caller updates a batch by
 * writing new contents (views' angles and weights, parameters) into the same buffers.
 *
 * digs_plan_create: tuning != NULL fixes the launch tuning; tuning == NULL runs the autotuner,
 * which renders the buffers' current contents (they must hold valid inputs, and grad_proj valid
 * dL/dproj if given). For each tile shape 16x16, 32x8 and 8x8 that the detector allows it sizes
 * the instance capacity from a measured forward (1.25 x the need + 4096) and times four launch
 * shapes (forward splat 4 or 1 waves per tile x persistent or one-workgroup-per-item splats;
 * within one tile shape all give bitwise-identical results); it keeps the fastest forward +
 * backward, a tile shape other than 16x16 only if it is more than 3% faster than the best 16x16
 * candidate (tile shapes sum in different orders, so a near tie should not flip between runs).
 * The list slices follow from the chosen shape. Synchronises its own stream; allocates the
 * workspace (hipMalloc).
 * digs_plan_fwd / digs_plan_bwd: replay on `stream` (bwd reuses the last fwd's binning).
 * digs_plan_fwd_views: the forward without its per-Gaussian stage (the cell order of the means and
 * the FFD at the canonical means, Sec. 3.3 Eq. 10-11, which do not depend on the views): it takes
 * that stage from the last digs_plan_fwd, so it is valid only while the Gaussian and lattice
 * buffers hold the values that call read (only angles and w changed since); rendering many views
 * of one model. DIGS_EINVAL if no digs_plan_fwd has run since the plan was created or resized.
 * digs_plan_check: synchronises `stream`, returns the diagnostics; if an instance overflow
 * happened in any call since the last check it grows the workspace to hold the largest need of
 * those calls (max_instances; the capacity never shrinks), sets *resized = 1, and the caller must
 * repeat the calls made since the last check.
 * digs_plan_set_replay: how the plan re-issues each of its three launch sequences (forward,
 * per-view forward, backward). DIGS_REPLAY_TIMED (the default): when a sequence is first called,
 * its HIP-graph replay and direct launches of the same kernels on the stream are each timed three
 * times (median, after one untimed run, on the plan's own stream, ordered after the work queued on
 * `stream` and before what follows on it; the timing runs compute what the call computes) and
 * the faster is kept. DIGS_REPLAY_GRAPH and DIGS_REPLAY_DIRECT fix the choice. Both give the
 * same bits. Synchronises the device and drops the recorded graphs (each sequence is recorded,
 * and timed, again at its next call); the workspace keeps its contents.
 * digs_plan_get_replay: modes[0..2] = the choice for the forward, the per-view forward and the
 * backward (DIGS_REPLAY_GRAPH or DIGS_REPLAY_DIRECT; 0 while the sequence has not been called).
 * digs_plan_get_tuning: the tuning in use and, if tune_ms != NULL, the autotuner's timings
 * tune_ms[c][0] (forward) and tune_ms[c][1] (backward) in ms per candidate c: tile shape c / 4
 * (16x16, 32x8, 8x8; zeros for a shape not tried), launch shape c % 4 (waves 4, 4, 1, 1 x
 * persistent 0, 1, 0, 1).
 * Errors: DIGS_EINVAL, DIGS_ENOMEM, DIGS_EHIP. */
#define DIGS_TUNE_CANDIDATES 12
#define DIGS_REPLAY_TIMED 0
#define DIGS_REPLAY_GRAPH 1
#define DIGS_REPLAY_DIRECT 2

typedef struct digs_plan digs_plan;

typedef struct digs_plan_buffers {
    const float *coef, *mu, *scale, *quat, *rho;   /* as digs_project_fwd                    */
    const float *angles, *w;                       /* [T], [T][R]                             */
    float *proj;                                   /* [T][nv][nu] forward output              */
    const float *grad_proj;                        /* [T][nv][nu] dL/dproj (NULL: no backward) */
    float *g_mu, *g_scale, *g_quat, *g_rho, *g_coef, *g_w;   /* backward outputs            */
} digs_plan_buffers;

int digs_plan_create(const digs_geom *geom, const digs_grid *grid, int n, int T,
                     const digs_tuning *tuning, const digs_plan_buffers *bufs, digs_plan **out);
int digs_plan_fwd(digs_plan *plan, void *stream);
int digs_plan_fwd_views(digs_plan *plan, void *stream);
int digs_plan_bwd(digs_plan *plan, void *stream);
int digs_plan_check(digs_plan *plan, digs_diag *out, int *resized, void *stream);
int digs_plan_set_replay(digs_plan *plan, int mode);
int digs_plan_get_replay(const digs_plan *plan, int *modes);
int digs_plan_get_tuning(const digs_plan *plan, digs_tuning *out, float *tune_ms);
int digs_plan_destroy(digs_plan *plan);

/* ---------------------------------------------------------------------------------------------
 * The dynamic volume at one time point (Sec. 3.2, Eq. 6; Sec. 3.3, Eq. 9), on a voxel grid whose
 * voxel (i,j,k) centre sits at origin + (i,j,k)*spacing; volumes are stored [nz][ny][nx].
 * digs_dvf_grid: dvf [3][nz][ny][nx] = sum_r w[r] u_r(x) at every voxel centre (w: device, [R]).
 * digs_phi_grid: phi [nz][ny][nx] = sum_n rho_n exp(-(x - mu'_n)^T Sigma'_n^-1 (x - mu'_n) / 2)
 *   with (mu', Sigma') the warp of Eq. 7-8 at weights w, each Gaussian cut off beyond Mahalanobis
 *   radius `cull` along each axis (0: default 5). ws of digs_phi_workspace_size bytes (256-byte
 *   aligned) with room for `capacity` (brick, Gaussian) pairs (0: 64 n + 4096); the number
 *   needed and any overflow are reported by digs_read_diagnostics(ws).
 * Errors: DIGS_EINVAL, DIGS_ENOWS, DIGS_EHIP. */
typedef struct digs_vgrid {
    int nx, ny, nz;          /* voxels per axis, 1..4096                                        */
    float origin[3];         /* centre of voxel (0,0,0), mm                                     */
    float spacing[3];        /* mm, > 0                                                         */
} digs_vgrid;

int digs_dvf_grid(const digs_grid *grid, const float *coef, const float *w, const digs_vgrid *vg,
                  float *dvf, void *stream);
size_t digs_phi_workspace_size(const digs_vgrid *vg, int n, int64_t capacity);
int digs_phi_grid(const digs_grid *grid, const float *coef, int n, const float *mu,
                  const float *scale, const float *quat, const float *rho, const float *w,
                  const digs_vgrid *vg, float cull, int64_t capacity, float *phi, void *ws,
                  size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------------------
 * The per-projection temporal-weight fit and its learned warm start. For a measured view P_t the
 * plain fit finds the weights w_t of the low-rank motion model (Sec. 3.3, Eq. 9) minimising
 * 1/2 ||I(w_t) - P_t||^2 by Levenberg-Marquardt (host loop: one batched digs_project_fwd of the
 * base weights and R raised copies per step, then digs_lm_normal_eq). The warm start predicts w_t
 * from the downsampled view and the gantry angle with a small MLP whose products run on the
 * matrix cores (digs_gemm_bf16). Device pointers, float32, row-major; asynchronous on `stream`.
 *
 * digs_lm_normal_eq: imgs [T][R+1][npix] (base image, then the base with w_r raised by h[r]),
 *   meas [T][npix], h [R] (device) -> out [T][R(R+1)/2 + R + 1]: J^T J (upper triangle, row-major),
 *   J^T res, res.res with J_r = (I_r - I_0)/h_r, res = I_0 - P. Fixed-order sums.
 * digs_gemm_bf16: C[M][N] = A . B with A [M][K] (lda; transA: stored [K][M]) and B [K][N] (ldb;
 *   transB: stored [N][K]), FP32 in memory, BF16 operands on MFMA (v_mfma_f32_32x32x16_bf16), FP32
 *   accumulate; then, in order, + C if accumulate, + bias[N] if bias, max(., 0) if relu, 0 where
 *   gate[M][N] (leading dimension ldc) is <= 0 if gate.
 * digs_colsum: out[N] = column sums of X [M][N] (ldx). digs_mse: mean of
 *   (pred - (target - mean)/std)^2 over [B][R], its gradient dpred [B][R] and (if loss) the value.
 * digs_adam: one Adam step (bias-corrected; step >= 1) on n FP32 weights with moments m, v.
 * digs_downsample: out[t][0 .. (nv/fy)(nu/fx)) = scale x the fy x fx block means of proj
 *   [T][nv][nu] (row-major), standardised per feature as (x - fmean[i]) * fistd[i] if fmean and
 *   fistd are given (both or neither), then sin and cos of angles[t] if angles (ld_out per row).
 * digs_standardize: X[i][j] = (X[i][j] - mean[j]) * istd[j] for j < N, in place.
 * Errors: DIGS_EINVAL, DIGS_EHIP. */
int digs_lm_normal_eq(int T, int R, int npix, const float *imgs, const float *meas,
                      const float *h, float *out, void *stream);
int digs_gemm_bf16(int M, int N, int K, const float *A, int lda, int transA, const float *B,
                   int ldb, int transB, float *C, int ldc, const float *bias, const float *gate,
                   int relu, int accumulate, void *stream);
int digs_colsum(int M, int N, const float *X, int ldx, float *out, void *stream);
int digs_mse(int B, int R, const float *pred, const float *target, const float *mean,
             const float *stdv, float *dpred, float *loss, void *stream);
int digs_adam(int n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2,
              float eps, int step, void *stream);
int digs_downsample(int T, int nv, int nu, int fy, int fx, const float *proj,
                    const float *angles, float scale, const float *fmean, const float *fistd,
                    float *out, int ld_out, void *stream);
int digs_standardize(int M, int N, float *X, int ldx, const float *mean, const float *istd,
                     void *stream);

/* ---------------------------------------------------------------------------------------------
 * The reconstruction loop around the renderer (Sec. 4.2: the Gaussians and the space and time
 * B-spline grids updated jointly by Adam on the L2 projection loss). Device pointers, float32;
 * asynchronous on `stream`.
 * digs_l2_residual: grad[i] = proj[i] - meas[i] for i < n (dL/dproj of L = 1/2 ||proj - meas||^2)
 *   and, if loss is not NULL (a buffer of 1 + DIGS_L2_PARTS floats), loss[0] = L; loss[1..] hold
 *   per-workgroup parts, added in a fixed order, so L is the same on every run.
 * digs_adam_mapped: one bias-corrected Adam step (step >= 1) on n unconstrained parameters raw
 *   given dL/dvalue, where value = map(raw): map 0 identity (value must equal raw), 1 exp (for
 *   scales), 2 softplus (for densities); the chain rule is applied to the gradient, then raw is
 *   updated and value rewritten from it. m, v: the moments (zero before step 1).
 * Errors: DIGS_EINVAL, DIGS_EHIP. */
#define DIGS_L2_PARTS 256
int digs_l2_residual(int64_t n, const float *proj, const float *meas, float *grad, float *loss,
                     void *stream);
int digs_adam_mapped(int n, float *raw, float *value, const float *g_value, float *m, float *v,
                     float lr, float b1, float b2, float eps, int step, int map, void *stream);

/* Diagnostics of a workspace: digs_read_diagnostics synchronises `stream` and copies the block
 * to *out (all zero if no call has run on the workspace yet); digs_reset_diagnostics clears it
 * (asynchronously, on `stream`). The block sits at the start of the workspace and carries a stamp:
 * the first call on a new workspace clears it whatever the memory held, so no reset is needed
 * before first use. Counters accumulate over calls until a reset. */
int digs_read_diagnostics(const void *ws, digs_diag *out, void *stream);
int digs_reset_diagnostics(void *ws, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Measurement support (not on the compute path).
 * digs_count_pairs: after a digs_project_fwd on `ws` (same arguments), synchronises `stream` and
 * counts, over that call's projections: out[0] the (Gaussian, pixel) pairs inside each cut-off
 * footprint and on the detector (the algorithmic work of the splat), out[1] the pairs the forward
 * splat evaluates (8x8 pixel blocks touched by a footprint box), out[2] the pairs the backward
 * splat evaluates (the same blocks). Errors: DIGS_EINVAL, DIGS_ENOWS, DIGS_EHIP.
 * digs_profile_enable / digs_profile_read: when enabled, every kernel stage launched by the
 * library is bracketed by two HIP events recorded on its launch stream (plans switch this off
 * while they record their graphs); digs_profile_enable(on) returns the previous state, and
 * on < 0 only queries it; digs_profile_read
 * waits for the recorded events and returns, per stage, the launches and summed milliseconds
 * (reset != 0 clears the sums). Single-threaded use only. Returns the number of entries. */
typedef struct digs_profile_entry {
    char name[32];
    int64_t launches;
    double total_ms;
} digs_profile_entry;

int digs_count_pairs(const digs_geom *geom, const digs_grid *grid, int n, int T, void *ws,
                     size_t ws_bytes, const digs_tuning *tuning, uint64_t *out, void *stream);
int digs_profile_enable(int on);
int digs_profile_read(digs_profile_entry *out, int max_entries, int reset);

/* Message for a DIGS_E* code; the HIP error code of the last DIGS_EHIP on this thread. */
const char *digs_strerror(int code);
int digs_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DIGS_H */
