// common.h -- device helpers shared by the libdigs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/digs.h"

#define DIGS_WAVE 64
#define DIGS_TILE 16                 // default detector tile edge (pixels)
#define DIGS_TILE_PX 256             // pixels of the largest tile (four 8x8 blocks)
#define DIGS_BIN_ITEMS 1024          // items (Gaussians) per binning workgroup: 4 waves x 256
#define DIGS_BIN_ITEMS_SMALL 256     // the same when a launch would have few workgroups
#define DIGS_REC_FLOATS 16           // per-(t,n) projected record, 64 bytes
#define DIGS_PART_FLOATS 12          // per-instance backward partial sums, 48 bytes

// Record layout (per projection t and Gaussian n), all float32:
//  0 us, 1 vs          footprint centre in pixel-index coordinates (column, row)
//  2 Huu', 3 Huv', 4 Hvv'   c2*H~uu, 2*c2*H~uv, c2*H~vv with c2 = -log2(e)/2 (exp2 argument)
//  5 gu2, 6 gv2        2*g~u, 2*g~v
//  7 Guu, 8 Guv2, 9 Gvv    G~uu, 2*G~uv, G~vv
//  10 amp              rho*sqrt(2 pi / Q*)
//  11 a00, 12 a01, 13 a11, 14 cx, 15 cy    the cut-off footprint as the ellipse
//                      (p - c)^T A (p - c) <= 1 in pixel-index coordinates (A = 0: not an ellipse)
// The per-pixel value is |e_ij| * amp * q^-1/2 * 2^(E' / q) with
// q = 1 + gu2 du + gv2 dv + Guu du^2 + Guv2 du dv + Gvv dv^2 and E' = Huu' du^2 + Huv' du dv
// + Hvv' dv^2, du = i - us, dv = j - vs.

struct DevGeom {
    float sid, sdd;
    int nu, nv;
    float pitch_u, pitch_v, off_u, off_v;
    int tiles_x, tiles_y, ntiles;
    // tile shape: tile_w x tile_h pixels (8, 16 or 32 each), a grid of tile_bx x (tile_nb /
    // tile_bx) blocks of 8x8 pixels with tile_nb in {1, 2, 4}; tile_lw, tile_lh = log2 of the edges
    int tile_w, tile_h, tile_lw, tile_lh, tile_bx, tile_nb;
    int ewa;                 // projection model: 0 exact line integral, 1 EWA 2D approximation
};

struct DevGrid {
    int R, nx, ny, nz;
    float ox, oy, oz;
    float hx, hy, hz;
};

struct DiagBlock {           // device copy of digs_diag plus internal totals
    unsigned long long instances;
    unsigned long long capacity;
    unsigned long long stat[3];   // digs_count_pairs
    unsigned int overflow;
    unsigned int nonfinite;
    unsigned int folded;
    unsigned int behind_source;
    unsigned int wide;
    unsigned int reserved[1];
    unsigned long long max_instances;   // largest `instances` of any call since the last reset
    unsigned long long stamp;           // DIAG_STAMP once the block has been cleared
};

// A workspace's diagnostics block counts as cleared only while it holds this stamp; the first call
// on a new workspace (whatever its memory held) clears it.
#define DIAG_STAMP 0x6469677364696167ull

__device__ __forceinline__ void diag_clear(DiagBlock *d)
{
    d->instances = 0;
    d->capacity = 0;
    d->stat[0] = d->stat[1] = d->stat[2] = 0;
    d->overflow = 0;
    d->nonfinite = 0;
    d->folded = 0;
    d->behind_source = 0;
    d->wide = 0;
    d->reserved[0] = 0;
    d->max_instances = 0;
    d->stamp = DIAG_STAMP;
}

__device__ __forceinline__ int lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// the set bits of a wave mask below this lane (its rank among the mask's lanes)
__device__ __forceinline__ int lane_rank(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <typename T>
__device__ __forceinline__ T uniform(T v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ float uniformf(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Uniform cubic B-spline pieces (Eq. 10), first and second derivatives in the fraction u.
__device__ __forceinline__ void bspline4(float u, float B[4])
{
    float v = 1.0f - u, u2 = u * u, u3 = u2 * u;
    const float s = 1.0f / 6.0f;
    B[0] = v * v * v * s;
    B[1] = (3.0f * u3 - 6.0f * u2 + 4.0f) * s;
    B[2] = (-3.0f * u3 + 3.0f * u2 + 3.0f * u + 1.0f) * s;
    B[3] = u3 * s;
}

__device__ __forceinline__ void bspline4_d(float u, float dB[4])
{
    float v = 1.0f - u;
    dB[0] = -0.5f * v * v;
    dB[1] = 0.5f * (3.0f * u * u - 4.0f * u);
    dB[2] = 0.5f * (-3.0f * u * u + 2.0f * u + 1.0f);
    dB[3] = 0.5f * u * u;
}

__device__ __forceinline__ void bspline4_dd(float u, float d2B[4])
{
    d2B[0] = 1.0f - u;
    d2B[1] = 3.0f * u - 2.0f;
    d2B[2] = 1.0f - 3.0f * u;
    d2B[3] = u;
}

__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// rotation of the normalised quaternion (w,x,y,z)
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float R[9])
{
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// dL/dq (normalised) from dL/dR for R(q) above
__device__ __forceinline__ void quat_rot_adjoint(float w, float x, float y, float z,
                                                 const float g[9], float gq[4])
{
    gq[0] = 2.0f * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    gq[1] = 2.0f * (y * g[1] + z * g[2] + y * g[3] - 2.0f * x * g[4] - w * g[5] + z * g[6] +
                    w * g[7] - 2.0f * x * g[8]);
    gq[2] = 2.0f * (-2.0f * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] +
                    z * g[7] - 2.0f * y * g[8]);
    gq[3] = 2.0f * (-2.0f * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0f * z * g[4] +
                    y * g[5] + x * g[6] + y * g[7]);
}

// row-major 3x3 inverse by cofactors; returns the determinant
__device__ __forceinline__ float inv3(const float A[9], float Ai[9])
{
    float c0 = A[4] * A[8] - A[5] * A[7];
    float c1 = A[5] * A[6] - A[3] * A[8];
    float c2 = A[3] * A[7] - A[4] * A[6];
    float det = A[0] * c0 + A[1] * c1 + A[2] * c2;
    float id = 1.0f / det;
    Ai[0] = c0 * id;
    Ai[3] = c1 * id;
    Ai[6] = c2 * id;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return det;
}

// wave-wide sum in a fixed order (deterministic)
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// host-side helpers ---------------------------------------------------------------------------
int digs_set_hip_error(hipError_t e);
