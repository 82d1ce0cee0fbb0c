// ffd_device.h -- device-side cubic B-spline stencil of the FFD (Sec. 3.3, Eq. 10-11).
#pragma once

#include "common.h"

// The 4x4x4 neighbourhood of a point: clamped lattice indices and the B-spline pieces of the
// fractional coordinate per axis, with first (and optionally second) derivatives already
// converted to world units (divided by the spacing, squared spacing).
struct Stencil {
    int ii[4], jj[4], kk[4];
    float Bx[4], By[4], Bz[4];
    float dBx[4], dBy[4], dBz[4];
    float d2Bx[4], d2By[4], d2Bz[4];
    int fx, fy, fz;
    float px, py, pz;   // fractional coordinates
};

__device__ __forceinline__ void make_stencil(const DevGrid &g, float x, float y, float z,
                                             Stencil &s, bool second)
{
    const float qx = (x - g.ox) / g.hx, qy = (y - g.oy) / g.hy, qz = (z - g.oz) / g.hz;
    // the cell is taken from the coordinate clamped to +-1e6 cells, so that a non-finite point
    // still converts to a valid integer; its fraction (and hence its weights) stays non-finite
    const float fx = floorf(fminf(fmaxf(qx, -1.0e6f), 1.0e6f));
    const float fy = floorf(fminf(fmaxf(qy, -1.0e6f), 1.0e6f));
    const float fz = floorf(fminf(fmaxf(qz, -1.0e6f), 1.0e6f));
    s.fx = (int)fx;
    s.fy = (int)fy;
    s.fz = (int)fz;
    s.px = qx - fx;
    s.py = qy - fy;
    s.pz = qz - fz;
    bspline4(s.px, s.Bx);
    bspline4(s.py, s.By);
    bspline4(s.pz, s.Bz);
    bspline4_d(s.px, s.dBx);
    bspline4_d(s.py, s.dBy);
    bspline4_d(s.pz, s.dBz);
    const float ihx = 1.0f / g.hx, ihy = 1.0f / g.hy, ihz = 1.0f / g.hz;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        s.ii[l] = clampi(s.fx - 1 + l, g.nx);
        s.jj[l] = clampi(s.fy - 1 + l, g.ny);
        s.kk[l] = clampi(s.fz - 1 + l, g.nz);
        s.dBx[l] *= ihx;
        s.dBy[l] *= ihy;
        s.dBz[l] *= ihz;
    }
    if (second) {
        bspline4_dd(s.px, s.d2Bx);
        bspline4_dd(s.py, s.d2By);
        bspline4_dd(s.pz, s.d2Bz);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            s.d2Bx[l] *= ihx * ihx;
            s.d2By[l] *= ihy * ihy;
            s.d2Bz[l] *= ihz * ihz;
        }
    }
}

// element n of a 4-array without dynamic register indexing (selects, no scratch)
template <class T>
__device__ __forceinline__ T pick4(const T (&v)[4], int n)
{
    return n == 0 ? v[0] : (n == 1 ? v[1] : (n == 2 ? v[2] : v[3]));
}

// Where the control points of the lattice are read from. A source's row(r, k, j) points at
// control point (0, j, k) of rank r, so that row(r, k, j) + 3 i is point (i, j, k) (three floats).
// LatticeRows: the caller's coefficient array in device memory, coef[R][nz][ny][nx][3].
struct LatticeRows {
    const float *coef;
    int nx, ny, nz;
    __device__ const float *row(int r, int k, int j) const
    {
        return coef + ((((size_t)r * nz + k) * ny + j) * nx) * 3;
    }
};

// BrickRows: a box of control points [x0, x0 + bx) x [y0, y0 + by) x [z0, z0 + bz) of every rank
// staged in LDS as b[R][bz][by][bx][3] (see stage_brick); only points inside the box are valid.
struct BrickRows {
    const float *b;
    int x0, y0, z0, bx, by, bz;
    __device__ const float *row(int r, int k, int j) const
    {
        return b + ((((r * bz + (k - z0)) * by + (j - y0)) * bx) - x0) * 3;
    }
};

// u_r and grad u_r (row-major, J[3a+b] = du_a/dx_b) of one rank at the stencil's point.
// With NZ < 4, only the stencil's z index nz0 (its partial sum; the caller adds the four).
template <int NZ = 4, class Rows>
__device__ __forceinline__ void ffd_rank_rows(const Rows &rows, int r, const Stencil &s,
                                              float u[3], float J[9], int nz0 = 0)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) J[k] = 0.f;
#pragma unroll
    for (int nn = 0; nn < NZ; ++nn) {
        // z index n (selected without dynamic register indexing when it is a run-time value)
        const int n = NZ == 4 ? nn : nz0;
        const int kk = NZ == 4 ? s.kk[nn] : pick4(s.kk, n);
        const float Bz = NZ == 4 ? s.Bz[nn] : pick4(s.Bz, n);
        const float dBz = NZ == 4 ? s.dBz[nn] : pick4(s.dBz, n);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const float *row = rows.row(r, kk, s.jj[m]);
            float sx[3] = {0.f, 0.f, 0.f}, sdx[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const float *d = row + s.ii[l] * 3;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float v = d[a];
                    sx[a] = fmaf(s.Bx[l], v, sx[a]);
                    sdx[a] = fmaf(s.dBx[l], v, sdx[a]);
                }
            }
            const float wyz = s.By[m] * Bz, wdy = s.dBy[m] * Bz, wdz = s.By[m] * dBz;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[a] = fmaf(wyz, sx[a], u[a]);
                J[3 * a + 0] = fmaf(wyz, sdx[a], J[3 * a + 0]);
                J[3 * a + 1] = fmaf(wdy, sx[a], J[3 * a + 1]);
                J[3 * a + 2] = fmaf(wdz, sx[a], J[3 * a + 2]);
            }
        }
    }
}

template <int NZ = 4>
__device__ __forceinline__ void ffd_rank(const DevGrid &g, const float *__restrict__ coef, int r,
                                         const Stencil &s, float u[3], float J[9], int nz0 = 0)
{
    ffd_rank_rows<NZ>(LatticeRows{coef, g.nx, g.ny, g.nz}, r, s, u, J, nz0);
}

// sum_{a,b} Q[3a+b] * d^2 u_a / dx_b dx_c for one rank (the term of dL/dmu through K(mu)),
// accumulated into h[c] (over the stencil's z indices n0..n1-1). The z and y loops stay rolled
// (registers); their per-index values are selected.
template <class Rows>
__device__ __forceinline__ void ffd_rank_hessian_contract(const Rows &rows, int r,
                                                          const Stencil &s, const float Q[9],
                                                          float h[3], int n0 = 0, int n1 = 4)
{
#pragma unroll 1
    for (int n = n0; n < n1; ++n) {
        const int kk = pick4(s.kk, n);
        const float Bz = pick4(s.Bz, n), dBz = pick4(s.dBz, n), d2Bz = pick4(s.d2Bz, n);
#pragma unroll 1
        for (int m = 0; m < 4; ++m) {
            const int jj = pick4(s.jj, m);
            const float By = pick4(s.By, m), dBy = pick4(s.dBy, m), d2By = pick4(s.d2By, m);
            const float *row = rows.row(r, kk, jj);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const float *d = row + s.ii[l] * 3;
                // y_b = sum_a Q[a][b] d_a
                float y[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) y[b] = Q[b] * d[0] + Q[3 + b] * d[1] + Q[6 + b] * d[2];
                const float wxx = s.d2Bx[l] * By * Bz;
                const float wyy = s.Bx[l] * d2By * Bz;
                const float wzz = s.Bx[l] * By * d2Bz;
                const float wxy = s.dBx[l] * dBy * Bz;
                const float wxz = s.dBx[l] * By * dBz;
                const float wyz = s.Bx[l] * dBy * dBz;
                h[0] += wxx * y[0] + wxy * y[1] + wxz * y[2];
                h[1] += wxy * y[0] + wyy * y[1] + wyz * y[2];
                h[2] += wxz * y[0] + wyz * y[1] + wzz * y[2];
            }
        }
    }
}

// The control points that a workgroup's Gaussians reach, staged in LDS (`lds`, at most `cap`
// floats): every thread passes its Gaussian's stencil (valid false for a thread without one),
// and the box of the stencils' clamped lattice indices is loaded for every rank, row by row
// (rows of the box are contiguous runs of the lattice). red: 24 ints of LDS for the reduction.
// Returns false, for the whole workgroup, when the box needs more than `cap` floats or no thread
// has a Gaussian (the caller then reads the lattice in device memory). Every thread of the
// workgroup must call it (it synchronises the workgroup); blockDim.x is a multiple of 64, at most
// 256.
__device__ __forceinline__ bool stage_brick(const DevGrid &g, const float *__restrict__ coef,
                                            const Stencil &s, bool valid, float *lds, int cap,
                                            int *red, BrickRows &b)
{
    int v[6] = {valid ? s.ii[0] : INT_MAX, valid ? s.jj[0] : INT_MAX, valid ? s.kk[0] : INT_MAX,
                valid ? -s.ii[3] : INT_MAX, valid ? -s.jj[3] : INT_MAX,
                valid ? -s.kk[3] : INT_MAX};   // minima of the low ends and of minus the high ends
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] = min(v[k], __shfl_xor(v[k], off, 64));
    const int wave = threadIdx.x / 64, nwaves = blockDim.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k) red[wave * 6 + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[k] = red[k];
        for (int w = 1; w < nwaves; ++w) v[k] = min(v[k], red[w * 6 + k]);
    }
    __syncthreads();   // red may be reused after the call
    if (v[0] == INT_MAX) return false;   // no Gaussian in the workgroup
    b.b = lds;
    b.x0 = v[0];
    b.y0 = v[1];
    b.z0 = v[2];
    b.bx = -v[3] - v[0] + 1;
    b.by = -v[4] - v[1] + 1;
    b.bz = -v[5] - v[2] + 1;
    const int rowlen = b.bx * 3, nrows = g.R * b.bz * b.by;
    if ((long long)rowlen * nrows > cap) return false;
    for (int e = threadIdx.x; e < rowlen * nrows; e += blockDim.x) {
        const int row = e / rowlen, off = e - row * rowlen;
        const int r = row / (b.bz * b.by), zy = row - r * (b.bz * b.by);
        const int z = zy / b.by, y = zy - z * b.by;
        lds[e] = coef[((((size_t)r * g.nz + b.z0 + z) * g.ny + b.y0 + y) * g.nx + b.x0) * 3 + off];
    }
    __syncthreads();
    return true;
}
