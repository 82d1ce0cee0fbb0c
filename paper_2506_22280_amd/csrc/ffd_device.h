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

// u_r and grad u_r (row-major, J[3a+b] = du_a/dx_b) of one rank at the stencil's point.
// With NZ < 4, only the stencil's z index nz0 (its partial sum; the caller adds the four).
template <int NZ = 4>
__device__ __forceinline__ void ffd_rank(const DevGrid &g, const float *__restrict__ coef, int r,
                                         const Stencil &s, float u[3], float J[9], int nz0 = 0)
{
    const float *base = coef + (size_t)r * g.nz * g.ny * g.nx * 3;
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
            const float *row = base + ((size_t)(kk * g.ny + s.jj[m]) * g.nx) * 3;
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

// sum_{a,b} Q[3a+b] * d^2 u_a / dx_b dx_c for one rank (the term of dL/dmu through K(mu)),
// accumulated into h[c] (over the stencil's z indices n0..n1-1). The z and y loops stay rolled (registers); their per-index values are
// selected.
__device__ __forceinline__ void ffd_rank_hessian_contract(const DevGrid &g,
                                                          const float *__restrict__ coef, int r,
                                                          const Stencil &s, const float Q[9],
                                                          float h[3], int n0 = 0, int n1 = 4)
{
    const float *base = coef + (size_t)r * g.nz * g.ny * g.nx * 3;
#pragma unroll 1
    for (int n = n0; n < n1; ++n) {
        const int kk = pick4(s.kk, n);
        const float Bz = pick4(s.Bz, n), dBz = pick4(s.dBz, n), d2Bz = pick4(s.d2Bz, n);
#pragma unroll 1
        for (int m = 0; m < 4; ++m) {
            const int jj = pick4(s.jj, m);
            const float By = pick4(s.By, m), dBy = pick4(s.dBy, m), d2By = pick4(s.d2By, m);
            const float *row = base + ((size_t)(kk * g.ny + jj) * g.nx) * 3;
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
