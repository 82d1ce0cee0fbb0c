// voxel.hip -- the dynamic volume at one time point on a voxel grid: the displacement field of the
// low-rank motion model, D(x,t) - x = sum_r w_r u_r(x) (Sec. 3.3, Eq. 9-10), and the dynamic
// attenuation phi(x,t) = sum_n G_n(x | rho_n, mu'_n, Sigma'_n) of the warped Gaussians (Sec. 3.2,
// Eq. 6-8).
//
// DVF: one workgroup per 64 x 16 voxel patch of a z-slice. The tensor-product B-spline is
// applied one axis at a time through LDS (z pieces and rank weights per lattice column, then y
// pieces per voxel row, then x pieces per voxel), so a voxel costs a few FMAs and the kernel is
// bound by the 12 bytes it writes per voxel.
//
// phi: each Gaussian's cut-off box (Mahalanobis radius r_c per axis) is binned into 8x8x8-voxel
// bricks by emitting (brick, Gaussian) pairs in Gaussian order and sorting them stably by brick;
// one workgroup per brick then sums its Gaussians over its 512 voxels in that fixed order and
// writes every voxel once.
#include <math.h>
#include <string.h>

#include "bin.h"
#include "ffd_device.h"

struct DevVGrid {
    int nx, ny, nz;
    float ox, oy, oz, sx, sy, sz;
};

static DevVGrid make_dev_vgrid(const digs_vgrid *v)
{
    DevVGrid d;
    d.nx = v->nx;
    d.ny = v->ny;
    d.nz = v->nz;
    d.ox = v->origin[0];
    d.oy = v->origin[1];
    d.oz = v->origin[2];
    d.sx = v->spacing[0];
    d.sy = v->spacing[1];
    d.sz = v->spacing[2];
    return d;
}

static bool vgrid_ok(const digs_vgrid *v)
{
    return v && v->nx >= 1 && v->ny >= 1 && v->nz >= 1 && v->nx <= 4096 && v->ny <= 4096 &&
           v->nz <= 4096 && v->spacing[0] > 0.0f && v->spacing[1] > 0.0f &&
           v->spacing[2] > 0.0f && isfinite(v->origin[0]) && isfinite(v->origin[1]) &&
           isfinite(v->origin[2]);
}

static bool lattice_ok(const digs_grid *g)
{
    return g && g->R >= 1 && g->R <= DIGS_MAX_RANK && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 &&
           g->spacing[0] > 0.0f && g->spacing[1] > 0.0f && g->spacing[2] > 0.0f;
}

// floor of a lattice coordinate, clamped far enough outside the lattice that the clamped stencil
// is unchanged (keeps the int conversion defined)
__device__ __forceinline__ int lattice_floor(float q, int n)
{
    return (int)fminf(fmaxf(floorf(q), -4.0f), (float)n + 4.0f);
}

// ------------------------------------------------------------------------------------------
// One workgroup per 64 (x) x 16 (y) voxel patch of a z-slice. Stage 1 applies the z pieces (and
// the rank weights) to every lattice column (i, j) the patch needs: P[j][i] = sum_r w_r sum_n
// B_n(z) d^r[i][j][fz-1+n]; stage 2 the y pieces per voxel row: L[row][i] = sum_m B_m(y_row)
// P[fy-1+m][i]; stage 3 the x pieces per voxel. All three stages use every thread.
#define DVF_ROW 64
#define DVF_ROWS 16
#define DVF_LMAX 40
#define DVF_JMAX 12

__global__ __launch_bounds__(256) void k_dvf_rows(DevGrid g, const float *__restrict__ coef,
                                                  const float *__restrict__ w, DevVGrid v,
                                                  float *__restrict__ dvf)
{
    __shared__ float P[DVF_JMAX][DVF_LMAX][3];
    __shared__ float L[DVF_ROWS][DVF_LMAX][3];
    const int x0 = blockIdx.x * DVF_ROW, y0 = blockIdx.y * DVF_ROWS, z = blockIdx.z;
    const int xl = min(x0 + DVF_ROW, v.nx) - 1, yl = min(y0 + DVF_ROWS, v.ny) - 1;
    const int ilo = lattice_floor((v.ox + (float)x0 * v.sx - g.ox) / g.hx, g.nx) - 1;
    const int ihi = lattice_floor((v.ox + (float)xl * v.sx - g.ox) / g.hx, g.nx) + 2;
    const int jlo = lattice_floor((v.oy + (float)y0 * v.sy - g.oy) / g.hy, g.ny) - 1;
    const int jhi = lattice_floor((v.oy + (float)yl * v.sy - g.oy) / g.hy, g.ny) + 2;
    const int nL = min(ihi - ilo + 1, DVF_LMAX), nJ = min(jhi - jlo + 1, DVF_JMAX);
    const float qz = (v.oz + (float)z * v.sz - g.oz) / g.hz;
    const int fz = lattice_floor(qz, g.nz);
    float Bz[4];
    bspline4(qz - floorf(qz), Bz);
    const size_t rank_stride = (size_t)g.nz * g.ny * g.nx * 3;
    // stage 1: z pieces and rank weights, one lattice column and component per thread-step
    for (int e = threadIdx.x; e < nJ * nL * 3; e += 256) {
        const int a = e % 3, i = (e / 3) % nL, j = e / (3 * nL);
        const int ii = clampi(ilo + i, g.nx), jj = clampi(jlo + j, g.ny);
        float acc = 0.0f;
        for (int rk = 0; rk < g.R; ++rk) {
            const float *base = coef + rk * rank_stride + ((size_t)jj * g.nx + ii) * 3 + a;
            float t = 0.0f;
#pragma unroll
            for (int n = 0; n < 4; ++n)
                t = fmaf(Bz[n], base[(size_t)clampi(fz - 1 + n, g.nz) * g.ny * g.nx * 3], t);
            acc = fmaf(w[rk], t, acc);
        }
        P[j][i][a] = acc;
    }
    __syncthreads();
    // stage 2: y pieces per voxel row
    for (int e = threadIdx.x; e < DVF_ROWS * nL * 3; e += 256) {
        const int a = e % 3, i = (e / 3) % nL, r = e / (3 * nL);
        const int y = min(y0 + r, v.ny - 1);
        const float qy = (v.oy + (float)y * v.sy - g.oy) / g.hy;
        const int fy = lattice_floor(qy, g.ny);
        float By[4];
        bspline4(qy - floorf(qy), By);
        float acc = 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc = fmaf(By[m], P[min(max(fy - 1 + m - jlo, 0), nJ - 1)][i][a], acc);
        L[r][i][a] = acc;
    }
    __syncthreads();
    // stage 3: x pieces; thread = column x, rows r, r + 4, r + 8, r + 12
    const int x = x0 + (int)(threadIdx.x % DVF_ROW);
    if (x >= v.nx) return;
    const float qx = (v.ox + (float)x * v.sx - g.ox) / g.hx;
    const int fx = lattice_floor(qx, g.nx);
    float Bx[4];
    bspline4(qx - floorf(qx), Bx);
    int li[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) li[l] = min(max(fx - 1 + l - ilo, 0), nL - 1);
    const size_t plane = (size_t)v.nz * v.ny * v.nx;
#pragma unroll
    for (int k = 0; k < DVF_ROWS / 4; ++k) {
        const int r = (int)(threadIdx.x / DVF_ROW) + 4 * k, y = y0 + r;
        if (y >= v.ny) break;
        float u[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int a = 0; a < 3; ++a) u[a] = fmaf(Bx[l], L[r][li[l]][a], u[a]);
        const size_t o = ((size_t)z * v.ny + y) * v.nx + x;
        __builtin_nontemporal_store(u[0], dvf + o);   // streaming stores: written once
        __builtin_nontemporal_store(u[1], dvf + plane + o);
        __builtin_nontemporal_store(u[2], dvf + 2 * plane + o);
    }
}

// One workgroup per 64 (x) x 16 (y) x 16 (z) voxel slab, for voxels much finer than the lattice.
// Stage 0 combines the ranks once for the lattice block the slab needs, C[k][j][i] = sum_r w_r
// d^r[k][j][i] (each control point read once per slab, not once per z-slice and rank); then, per
// z-slice, stage 1 applies the z pieces to every lattice column, stage 2 the y pieces per voxel
// row and stage 3 the x pieces per voxel, whose three components are written once each
// (coalesced along x). The z, y and x piece weights are computed once per slab.
#define SLAB_Z 16
#define SLAB_CMAX 4096   // floats of the rank-combined lattice block (nz * ny * nx * 3)

__global__ __launch_bounds__(256) void k_dvf_slab(DevGrid g, const float *__restrict__ coef,
                                                  const float *__restrict__ w, DevVGrid v,
                                                  float *__restrict__ dvf)
{
    __shared__ float C[SLAB_CMAX];
    __shared__ float4 P[DVF_JMAX][DVF_LMAX];   // (x, y, z) components, w unused: one 16-byte
    __shared__ float4 L[DVF_ROWS][DVF_LMAX];   // LDS read per B-spline tap
    __shared__ float By[DVF_ROWS][4];
    __shared__ int fyr[DVF_ROWS];
    const int x0 = blockIdx.x * DVF_ROW, y0 = blockIdx.y * DVF_ROWS, z0 = blockIdx.z * SLAB_Z;
    const int xl = min(x0 + DVF_ROW, v.nx) - 1, yl = min(y0 + DVF_ROWS, v.ny) - 1;
    const int zl = min(z0 + SLAB_Z, v.nz) - 1;
    const int ilo = lattice_floor((v.ox + (float)x0 * v.sx - g.ox) / g.hx, g.nx) - 1;
    const int ihi = lattice_floor((v.ox + (float)xl * v.sx - g.ox) / g.hx, g.nx) + 2;
    const int jlo = lattice_floor((v.oy + (float)y0 * v.sy - g.oy) / g.hy, g.ny) - 1;
    const int jhi = lattice_floor((v.oy + (float)yl * v.sy - g.oy) / g.hy, g.ny) + 2;
    const int klo = lattice_floor((v.oz + (float)z0 * v.sz - g.oz) / g.hz, g.nz) - 1;
    const int khi = lattice_floor((v.oz + (float)zl * v.sz - g.oz) / g.hz, g.nz) + 2;
    // the host checks that the block fits; the clamps keep every access inside the arrays
    const int nL = min(ihi - ilo + 1, DVF_LMAX), nJ = min(jhi - jlo + 1, DVF_JMAX);
    const int nK = max(1, min(khi - klo + 1, SLAB_CMAX / (3 * nL * nJ)));
    const size_t rank_stride = (size_t)g.nz * g.ny * g.nx * 3;
    // stage 0: the ranks combined, one lattice value per thread-step (a, i fastest: contiguous
    // in the lattice's layout)
    for (int e = threadIdx.x; e < nK * nJ * nL * 3; e += 256) {
        const int a = e % 3, i = (e / 3) % nL, j = (e / (3 * nL)) % nJ, k = e / (3 * nL * nJ);
        const size_t o = (((size_t)clampi(klo + k, g.nz) * g.ny + clampi(jlo + j, g.ny)) * g.nx +
                          clampi(ilo + i, g.nx)) * 3 + a;
        float acc = 0.0f;
        for (int rk = 0; rk < g.R; ++rk) acc = fmaf(w[rk], coef[rk * rank_stride + o], acc);
        C[e] = acc;
    }
    if (threadIdx.x < DVF_ROWS) {
        const int y = min(y0 + (int)threadIdx.x, v.ny - 1);
        const float qy = (v.oy + (float)y * v.sy - g.oy) / g.hy;
        float b[4];
        bspline4(qy - floorf(qy), b);
#pragma unroll
        for (int m = 0; m < 4; ++m) By[threadIdx.x][m] = b[m];
        fyr[threadIdx.x] = lattice_floor(qy, g.ny) - 1 - jlo;
    }
    // the x pieces of this thread's column
    const int x = x0 + (int)(threadIdx.x % DVF_ROW);
    const float qx = (v.ox + (float)min(x, v.nx - 1) * v.sx - g.ox) / g.hx;
    const int fx = lattice_floor(qx, g.nx);
    float Bx[4];
    bspline4(qx - floorf(qx), Bx);
    int li[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) li[l] = min(max(fx - 1 + l - ilo, 0), nL - 1);
    const size_t plane = (size_t)v.nz * v.ny * v.nx;
    __syncthreads();
    for (int z = z0; z <= zl; ++z) {
        const float qz = (v.oz + (float)z * v.sz - g.oz) / g.hz;
        const int kz = lattice_floor(qz, g.nz) - 1 - klo;
        float Bz[4];
        bspline4(qz - floorf(qz), Bz);
        // stage 1: z pieces per lattice column (thread-step = one column's three components)
        for (int e = threadIdx.x; e < nJ * nL; e += 256) {
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const float *c = C + min(max(kz + n, 0), nK - 1) * (nJ * nL * 3) + 3 * e;
                acc.x = fmaf(Bz[n], c[0], acc.x);
                acc.y = fmaf(Bz[n], c[1], acc.y);
                acc.z = fmaf(Bz[n], c[2], acc.z);
            }
            P[e / nL][e % nL] = acc;
        }
        __syncthreads();
        // stage 2: y pieces per voxel row
        for (int e = threadIdx.x; e < DVF_ROWS * nL; e += 256) {
            const int i = e % nL, r = e / nL;
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float4 p = P[min(max(fyr[r] + m, 0), nJ - 1)][i];
                const float b = By[r][m];
                acc.x = fmaf(b, p.x, acc.x);
                acc.y = fmaf(b, p.y, acc.y);
                acc.z = fmaf(b, p.z, acc.z);
            }
            L[r][i] = acc;
        }
        __syncthreads();
        // stage 3: x pieces; thread = column x, rows r, r + 4, r + 8, r + 12
        if (x < v.nx) {
#pragma unroll
            for (int k = 0; k < DVF_ROWS / 4; ++k) {
                const int r = (int)(threadIdx.x / DVF_ROW) + 4 * k, y = y0 + r;
                if (y > yl) break;
                float u[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const float4 q = L[r][li[l]];
                    u[0] = fmaf(Bx[l], q.x, u[0]);
                    u[1] = fmaf(Bx[l], q.y, u[1]);
                    u[2] = fmaf(Bx[l], q.z, u[2]);
                }
                const size_t o = ((size_t)z * v.ny + y) * v.nx + x;
                // streaming stores: the field is written once and not read back here
                __builtin_nontemporal_store(u[0], dvf + o);
                __builtin_nontemporal_store(u[1], dvf + plane + o);
                __builtin_nontemporal_store(u[2], dvf + 2 * plane + o);
            }
        }
    }
}

// Any voxel spacing: the full 64-point stencil per voxel.
__global__ __launch_bounds__(256) void k_dvf_points(DevGrid g, const float *__restrict__ coef,
                                                    const float *__restrict__ w, DevVGrid v,
                                                    float *__restrict__ dvf)
{
    const size_t plane = (size_t)v.nz * v.ny * v.nx;
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= plane) return;
    const int x = (int)(o % v.nx), y = (int)((o / v.nx) % v.ny), z = (int)(o / ((size_t)v.nx * v.ny));
    Stencil st;
    make_stencil(g, v.ox + (float)x * v.sx, v.oy + (float)y * v.sy, v.oz + (float)z * v.sz, st,
                 false);
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int rk = 0; rk < g.R; ++rk) {
        float u[3], J[9];
        ffd_rank(g, coef, rk, st, u, J);
        for (int a = 0; a < 3; ++a) acc[a] = fmaf(w[rk], u[a], acc[a]);
    }
    __builtin_nontemporal_store(acc[0], dvf + o);   // streaming stores: written once
    __builtin_nontemporal_store(acc[1], dvf + plane + o);
    __builtin_nontemporal_store(acc[2], dvf + 2 * plane + o);
}

extern "C" int digs_dvf_grid(const digs_grid *grid, const float *coef, const float *w,
                             const digs_vgrid *vg, float *dvf, void *stream)
{
    if (!lattice_ok(grid) || !vgrid_ok(vg) || !coef || !w || !dvf) return DIGS_EINVAL;
    const DevGrid g = make_dev_grid(grid);
    const DevVGrid v = make_dev_vgrid(vg);
    hipStream_t s = (hipStream_t)stream;
    // the slab kernel's LDS holds the lattice block of a 64 x 16 x 16 voxel slab, the patch
    // kernel's the lattice columns of a 64 x 16 voxel patch
    const double nLx = (double)(DVF_ROW - 1) * v.sx / g.hx + 5.0;
    const double nJy = (double)(DVF_ROWS - 1) * v.sy / g.hy + 5.0;
    const double nKz = (double)(SLAB_Z - 1) * v.sz / g.hz + 5.0;
    if (nLx <= (double)DVF_LMAX && nJy <= (double)DVF_JMAX &&
        floor(nKz) * floor(nJy) * floor(nLx) * 3.0 <= (double)SLAB_CMAX) {
        const dim3 blocks((v.nx + DVF_ROW - 1) / DVF_ROW, (v.ny + DVF_ROWS - 1) / DVF_ROWS,
                          (v.nz + SLAB_Z - 1) / SLAB_Z);
        hipLaunchKernelGGL(k_dvf_slab, blocks, dim3(256), 0, s, g, coef, w, v, dvf);
    } else if (nLx <= (double)DVF_LMAX && nJy <= (double)DVF_JMAX) {
        const dim3 blocks((v.nx + DVF_ROW - 1) / DVF_ROW, (v.ny + DVF_ROWS - 1) / DVF_ROWS, v.nz);
        hipLaunchKernelGGL(k_dvf_rows, blocks, dim3(256), 0, s, g, coef, w, v, dvf);
    } else {
        const size_t m = (size_t)v.nx * v.ny * v.nz;
        hipLaunchKernelGGL(k_dvf_points, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, g,
                           coef, w, v, dvf);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e);
}

// ------------------------------------------------------------------------------------------
#define BRICK 8
#define PHI_REC 12   // floats per Gaussian record: centre (3, voxel index units), exp2 quadratic
                     // coefficients (6), rho, 2 unused

struct PhiLayout {
    size_t diag, rec, brange, count, scratch, ka, va, kb, vb, rhist, bstart, total;
    size_t cap, scratch_elems;
    int nbx, nby, nbz, nbricks;
};

static bool phi_layout(const digs_vgrid *vg, int n, int64_t capacity, PhiLayout *L)
{
    if (!vgrid_ok(vg) || n < 0 || n > DIGS_MAX_GAUSSIANS) return false;
    memset(L, 0, sizeof(*L));
    L->nbx = (vg->nx + BRICK - 1) / BRICK;
    L->nby = (vg->ny + BRICK - 1) / BRICK;
    L->nbz = (vg->nz + BRICK - 1) / BRICK;
    L->nbricks = L->nbx * L->nby * L->nbz;
    int64_t cap = capacity > 0 ? capacity : (int64_t)64 * n + 4096;
    if (cap > 0x7FFFFF00ll) cap = 0x7FFFFF00ll;
    L->cap = (size_t)cap;
    const size_t N = (size_t)(n > 0 ? n : 1);
    const size_t nblk = (L->cap + DIGS_BIN_ITEMS - 1) / DIGS_BIN_ITEMS;
    size_t sc = scan_scratch_elems(N + 1), s2 = scan_scratch_elems(256 * nblk);
    L->scratch_elems = sc > s2 ? sc : s2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    L->diag = take(sizeof(DiagBlock));
    L->rec = take(sizeof(float) * PHI_REC * N);
    L->brange = take(sizeof(int2) * N);
    L->count = take(sizeof(uint32_t) * (N + 1));
    L->scratch = take(sizeof(uint32_t) * L->scratch_elems);
    L->ka = take(sizeof(uint32_t) * L->cap);
    L->va = take(sizeof(uint32_t) * L->cap);
    L->kb = take(sizeof(uint32_t) * L->cap);
    L->vb = take(sizeof(uint32_t) * L->cap);
    L->rhist = take(sizeof(uint32_t) * 2 * 256 * nblk);   // counts, then the waves' offsets
    L->bstart = take(sizeof(uint32_t) * ((size_t)L->nbricks + 1));
    L->total = off;
    return true;
}

// Per Gaussian: the warp at the query weights (Eq. 7-9), the quadratic form of its deformed
// covariance in voxel-index coordinates (scaled for exp2), its cut-off box and the bricks it meets.
template <int NR>
__global__ __launch_bounds__(256) void k_phi_setup(DevGrid g, const float *__restrict__ coef,
                                                   int n, const float *__restrict__ mu,
                                                   const float *__restrict__ scale,
                                                   const float *__restrict__ quat,
                                                   const float *__restrict__ rho,
                                                   const float *__restrict__ w, DevVGrid v,
                                                   float cull, float *__restrict__ rec,
                                                   int2 *__restrict__ brange,
                                                   uint32_t *__restrict__ count,
                                                   DiagBlock *__restrict__ diag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {   // the scan's total slot
        count[n] = 0;
        return;
    }
    const float m0[3] = {mu[i], mu[n + i], mu[2 * n + i]};
    const float s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
    float q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float Rm[9];
    quat_to_rot(q[0] * qn, q[1] * qn, q[2] * qn, q[3] * qn, Rm);
    Stencil st;
    make_stencil(g, m0[0], m0[1], m0[2], st, false);
    float K[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
    float mp[3] = {m0[0], m0[1], m0[2]};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        float u[3], J[9];
        ffd_rank(g, coef, r, st, u, J);
        const float wr = w[r];
#pragma unroll
        for (int a = 0; a < 3; ++a) mp[a] = fmaf(wr, u[a], mp[a]);
#pragma unroll
        for (int k = 0; k < 9; ++k) K[k] = fmaf(wr, J[k], K[k]);
    }
    // M = K R diag(s); Sigma' = M M^T; W = M^-1 = diag(1/s) R^T K^-1; A = W^T W = Sigma'^-1
    float Ki[9];
    const float detK = inv3(K, Ki);
    float M[9], W[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            M[3 * a + b] = (K[3 * a] * Rm[b] + K[3 * a + 1] * Rm[3 + b] + K[3 * a + 2] * Rm[6 + b]) *
                           s[b];
            W[3 * a + b] = (Rm[a] * Ki[b] + Rm[3 + a] * Ki[3 + b] + Rm[6 + a] * Ki[6 + b]) / s[a];
        }
    float Sd[3], A[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) Sd[a] = M[3 * a] * M[3 * a] + M[3 * a + 1] * M[3 * a + 1] +
                                        M[3 * a + 2] * M[3 * a + 2];
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k)
        A[k] = W[ia[k]] * W[ib[k]] + W[3 + ia[k]] * W[3 + ib[k]] + W[6 + ia[k]] * W[6 + ib[k]];
    const float vs[3] = {v.sx, v.sy, v.sz}, vo[3] = {v.ox, v.oy, v.oz};
    const int vn[3] = {v.nx, v.ny, v.nz};
    bool ok = isfinite(detK) && detK != 0.0f && s[0] > 0.0f && s[1] > 0.0f && s[2] > 0.0f &&
              isfinite(qn) && isfinite(rho[i]);
    float c[3];
    int lo[3] = {1, 1, 1}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c[a] = (mp[a] - vo[a]) / vs[a];
        const float hw = cull * sqrtf(fmaxf(Sd[a], 0.0f)) / vs[a];
        ok = ok && isfinite(c[a]) && isfinite(hw);
        const float l = fminf(fmaxf(ceilf(c[a] - hw), -1.0f), (float)vn[a]);
        const float h = fminf(fmaxf(floorf(c[a] + hw), -1.0f), (float)vn[a]);
        lo[a] = max((int)l, 0);
        hi[a] = min((int)h, vn[a] - 1);
    }
    if (!ok) atomicAdd(&diag->nonfinite, 1u);
    else if (detK <= 0.0f) atomicAdd(&diag->folded, 1u);
    const bool any = ok && lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2];
    float *o = rec + (size_t)i * PHI_REC;
    // exp2 argument: -log2(e)/2 * delta^T (S A S) delta with delta in voxel units
    const float c2 = -0.72134752044448170f;
    o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
    o[3] = any ? c2 * A[0] * vs[0] * vs[0] : 0.0f;
    o[4] = any ? 2.0f * c2 * A[1] * vs[0] * vs[1] : 0.0f;
    o[5] = any ? 2.0f * c2 * A[2] * vs[0] * vs[2] : 0.0f;
    o[6] = any ? c2 * A[3] * vs[1] * vs[1] : 0.0f;
    o[7] = any ? 2.0f * c2 * A[4] * vs[1] * vs[2] : 0.0f;
    o[8] = any ? c2 * A[5] * vs[2] * vs[2] : 0.0f;
    o[9] = any ? rho[i] : 0.0f;
    o[10] = 0.0f;
    o[11] = 0.0f;
    uint32_t cnt = 0;
    int2 br = make_int2(1, 0);
    if (any) {
        const int bx0 = lo[0] / BRICK, bx1 = hi[0] / BRICK, by0 = lo[1] / BRICK,
                  by1 = hi[1] / BRICK, bz0 = lo[2] / BRICK, bz1 = hi[2] / BRICK;
        cnt = (uint32_t)((bx1 - bx0 + 1) * (by1 - by0 + 1) * (bz1 - bz0 + 1));
        br = make_int2(bx0 | (bx1 << 10) | (by0 << 20), by1 | (bz0 << 10) | (bz1 << 20));
    }
    brange[i] = br;
    count[i] = cnt;
}

// (brick, Gaussian) pairs of every Gaussian at its scanned offset, bricks in z, y, x order
__global__ __launch_bounds__(256) void k_phi_emit(int n, const int2 *__restrict__ brange,
                                                  const uint32_t *__restrict__ off, int nbx,
                                                  int nby, size_t cap, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals,
                                                  DiagBlock *__restrict__ diag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        diag->instances = off[n];
        diag->capacity = cap;
        if ((size_t)off[n] > cap) diag->overflow = 1u;
        if ((unsigned long long)off[n] > diag->max_instances) diag->max_instances = off[n];
    }
    if (i >= n) return;
    const int2 br = brange[i];
    const int bx0 = br.x & 1023, bx1 = (br.x >> 10) & 1023, by0 = (br.x >> 20) & 1023;
    const int by1 = br.y & 1023, bz0 = (br.y >> 10) & 1023, bz1 = (br.y >> 20) & 1023;
    size_t p = off[i];
    for (int bz = bz0; bz <= bz1; ++bz)
        for (int by = by0; by <= by1; ++by)
            for (int bx = bx0; bx <= bx1; ++bx, ++p) {
                if (p >= cap) return;
                keys[p] = (uint32_t)((bz * nby + by) * nbx + bx);
                vals[p] = (uint32_t)i;
            }
}

// Pairs past the emitted ones (from *total to cap) get a key past every brick, so that they sort
// last and no brick's range reaches them.
__global__ __launch_bounds__(256) void k_phi_tail_keys(const uint32_t *__restrict__ total,
                                                       size_t cap, uint32_t sentinel,
                                                       uint32_t *__restrict__ keys,
                                                       uint32_t *__restrict__ vals)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= cap || p < (size_t)*total) return;
    keys[p] = sentinel;
    vals[p] = 0u;
}

// bstart[b] = position of the first pair of brick b in sorted order (for every b in 0..nbricks)
__global__ void k_brick_start(int m, int nbricks, const uint32_t *__restrict__ keys,
                              uint32_t *__restrict__ bstart)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > m) return;
    const uint32_t hi = (p < m) ? min(keys[p], (uint32_t)nbricks) : (uint32_t)nbricks;
    const uint32_t lo = (p > 0) ? min(keys[p - 1], (uint32_t)nbricks) + 1u : 0u;
    for (uint32_t k = lo; k <= hi; ++k) bstart[k] = (uint32_t)p;
}

// One workgroup per 8x8x8 brick: thread = (x, y, z and z + 4); the brick's Gaussians in order.
__global__ __launch_bounds__(256) void k_phi_splat(DevVGrid v, int nbx, int nby,
                                                   const float *__restrict__ rec,
                                                   const uint32_t *__restrict__ vals,
                                                   const uint32_t *__restrict__ bstart,
                                                   size_t cap, float *__restrict__ phi)
{
    const int b = blockIdx.x;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tx = threadIdx.x & 7, ty = (threadIdx.x >> 3) & 7, tz = threadIdx.x >> 6;
    const int x = bx * BRICK + tx, y = by * BRICK + ty, z = bz * BRICK + tz;
    const float fx = (float)x, fy = (float)y, fz0 = (float)z, fz1 = (float)(z + 4);
    uint32_t p0 = bstart[b], p1 = bstart[b + 1];
    p0 = (uint32_t)min((size_t)p0, cap);
    p1 = (uint32_t)min((size_t)max(p1, p0), cap);
    float acc0 = 0.0f, acc1 = 0.0f;
    for (uint32_t p = p0; p < p1; ++p) {
        const uint32_t gi = uniform(vals[p]);
        const float *r = rec + (size_t)gi * PHI_REC;
        const float dx = fx - r[0], dy = fy - r[1];
        const float qxy = fmaf(dx, fmaf(r[3], dx, r[4] * dy), r[6] * dy * dy);
        const float lin = fmaf(r[5], dx, r[7] * dy);
        const float dz0 = fz0 - r[2], dz1 = fz1 - r[2];
        const float e0 = fmaf(dz0, fmaf(r[8], dz0, lin), qxy);
        const float e1 = fmaf(dz1, fmaf(r[8], dz1, lin), qxy);
        acc0 = fmaf(r[9], __builtin_amdgcn_exp2f(e0), acc0);
        acc1 = fmaf(r[9], __builtin_amdgcn_exp2f(e1), acc1);
    }
    const size_t row = (size_t)v.ny * v.nx;
    if (x < v.nx && y < v.ny) {
        if (z < v.nz) phi[(size_t)z * row + (size_t)y * v.nx + x] = acc0;
        if (z + 4 < v.nz) phi[(size_t)(z + 4) * row + (size_t)y * v.nx + x] = acc1;
    }
}

extern "C" size_t digs_phi_workspace_size(const digs_vgrid *vg, int n, int64_t capacity)
{
    PhiLayout L;
    if (capacity < 0 || !phi_layout(vg, n, capacity, &L)) return 0;
    return L.total;
}

template <int NR>
static void phi_setup_launch(const DevGrid &g, const float *coef, int n, const float *mu,
                             const float *scale, const float *quat, const float *rho,
                             const float *w, const DevVGrid &v, float cull, char *ws,
                             const PhiLayout &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_phi_setup<NR>, dim3((n + 1 + 255) / 256), dim3(256), 0, s, g, coef, n,
                       mu, scale, quat, rho, w, v, cull, (float *)(ws + L.rec),
                       (int2 *)(ws + L.brange), (uint32_t *)(ws + L.count),
                       (DiagBlock *)(ws + L.diag));
}

__global__ void k_phi_diag_begin(DiagBlock *d)
{
    if (d->stamp != DIAG_STAMP) diag_clear(d);
    d->instances = 0;
    d->overflow = 0;
    d->nonfinite = 0;
    d->folded = 0;
}

extern "C" int digs_phi_grid(const digs_grid *grid, const float *coef, int n, const float *mu,
                             const float *scale, const float *quat, const float *rho,
                             const float *w, const digs_vgrid *vg, float cull, int64_t capacity,
                             float *phi, void *ws, size_t ws_bytes, void *stream)
{
    PhiLayout L;
    if (!lattice_ok(grid) || capacity < 0 || !(cull >= 0.0f) || !phi_layout(vg, n, capacity, &L))
        return DIGS_EINVAL;
    if (!phi || (n > 0 && (!coef || !mu || !scale || !quat || !rho || !w))) return DIGS_EINVAL;
    if (L.nbx > 1024 || L.nby > 1024 || L.nbz > 1024) return DIGS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < L.total) return DIGS_ENOWS;
    hipStream_t s = (hipStream_t)stream;
    const DevGrid g = make_dev_grid(grid);
    const DevVGrid v = make_dev_vgrid(vg);
    const float r = cull > 0.0f ? cull : 5.0f;
    char *W = (char *)ws;
    DiagBlock *diag = (DiagBlock *)(W + L.diag);
    hipLaunchKernelGGL(k_phi_diag_begin, dim3(1), dim3(1), 0, s, diag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return digs_set_hip_error(e);
    if (n == 0) {
        e = render_zero(phi, (size_t)v.nx * v.ny * v.nz, s);
        return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e);
    }
    switch (g.R) {
    case 1: phi_setup_launch<1>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 2: phi_setup_launch<2>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 3: phi_setup_launch<3>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 4: phi_setup_launch<4>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 5: phi_setup_launch<5>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 6: phi_setup_launch<6>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    case 7: phi_setup_launch<7>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    default: phi_setup_launch<8>(g, coef, n, mu, scale, quat, rho, w, v, r, W, L, s); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return digs_set_hip_error(e);
    uint32_t *count = (uint32_t *)(W + L.count), *scratch = (uint32_t *)(W + L.scratch);
    if ((e = launch_exclusive_scan(count, (size_t)n + 1, scratch, s)) != hipSuccess)
        return digs_set_hip_error(e);
    uint32_t *ka = (uint32_t *)(W + L.ka), *va = (uint32_t *)(W + L.va);
    uint32_t *kb = (uint32_t *)(W + L.kb), *vb = (uint32_t *)(W + L.vb);
    hipLaunchKernelGGL(k_phi_emit, dim3((n + 255) / 256), dim3(256), 0, s, n,
                       (const int2 *)(W + L.brange), count, L.nbx, L.nby, L.cap, ka, va, diag);
    if ((e = hipGetLastError()) != hipSuccess) return digs_set_hip_error(e);
    // The pair count is known only on the device; the sort and the splat run over the capacity
    // and clamp to it (pairs past the emitted ones carry keys past every brick).
    hipLaunchKernelGGL(k_phi_tail_keys, dim3((unsigned)((L.cap + 255) / 256)), dim3(256), 0, s,
                       count + n, L.cap, (uint32_t)L.nbricks, ka, va);
    if ((e = hipGetLastError()) != hipSuccess) return digs_set_hip_error(e);
    bool swapped = false;
    e = radix_sort_pairs(ka, va, kb, vb, (int)L.cap, bits_for(L.nbricks + 1),
                         (uint32_t *)(W + L.rhist), scratch, &swapped, s);
    if (e != hipSuccess) return digs_set_hip_error(e);
    const uint32_t *keys = swapped ? kb : ka, *vals = swapped ? vb : va;
    hipLaunchKernelGGL(k_brick_start, dim3((unsigned)((L.cap + 1 + 255) / 256)), dim3(256), 0, s,
                       (int)L.cap, L.nbricks, keys, (uint32_t *)(W + L.bstart));
    if ((e = hipGetLastError()) != hipSuccess) return digs_set_hip_error(e);
    hipLaunchKernelGGL(k_phi_splat, dim3(L.nbricks), dim3(256), 0, s, v, L.nbx, L.nby,
                       (const float *)(W + L.rec), vals, (const uint32_t *)(W + L.bstart), L.cap,
                       phi);
    e = hipGetLastError();
    return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e);
}
