// render.hip -- forward and backward of the deformation-informed Gaussian X-ray renderer.
//
// Forward (per call of T projections):
//   k_ffd_canonical  u_r, grad u_r at every canonical mean (Eq. 10-11), once per call
//   k_setup          per (t, n): the warp of Eq. 7-9 (mu', Sigma' = M M^T, M = K R diag(s)) and
//                    the projected record of the Gaussian's exact line integral (see below),
//                    its cut-off bounding box and the detector tiles it touches
//   k_bin_count/fill per projection, lists of Gaussians per 16x16 tile (bin.h)
//   k_splat_fwd      one workgroup per (projection, tile), one wave per 8x8 pixel block; lane =
//                    (Gaussian slot, column), eight Gaussians at a time, rows by forward
//                    differences; every pixel is written once (no atomics)
// Backward:
//   k_splat_bwd      one lane per (list entry, 8x8 block) pair, looping over the block's 64 pixels
//                    and accumulating 12 moment sums; one partial per instance (no atomics)
//   k_tn_bwd         per Gaussian and chunk of views: sums the instance partials, runs the set-up
//                    and warp adjoints per view and folds them into per-Gaussian sums; per-wave
//                    partial sums of dL/dw
//   k_gauss_reduce   per Gaussian, over the chunks in order: reduces to the canonical parameters
//                    (with the second-derivative term) and emits the sources of dL/dcoef
//   k_cell_*         stable radix sort of the Gaussians by lattice cell
//   k_coef_grad      each control point gathers from the Gaussians of its 4x4x4 cells
//
// The exact line integral of one Gaussian (Eq. 2 along the ray of Eq. 1, the quantity that
// Eq. 4 approximates) is evaluated in a whitened, cancellation-free form: with W = M^-1,
// m = source - mu', m_w = W m, the centre ray through mu' meeting the detector at pixel
// coordinates (us, vs), D_u = W e_u pitch_u, D_v = W e_v pitch_v, and delta = (i - us, j - vs),
//   I_ij = |e_ij| amp q^-1/2 exp(-E / (2 q)),
//   q = 1 + 2 g.delta + delta^T G delta,  E = delta^T H delta,
//   H = beta^2 D_perp^T D_perp,  g = -beta (m_w.D)/c,  G = beta^2 D^T D / c,
//   amp = rho sqrt(2 pi) beta / sqrt(c),  beta = (n.m)/SDD, c = |m_w|^2,
// where D_perp removes the m_w component. This equals rho |e| sqrt(2 pi / a) exp(-(c - b^2/a)/2)
// of the plain closed form without subtracting two large numbers.
#include "bin.h"
#include "ffd_device.h"
#include "kernels.h"
#include "prof.h"

#define SETUP_TCHUNK 8
#define WS(a, off, type) reinterpret_cast<type>((a).ws + (a).L.off)
#define SQRT_2PI 2.5066282746310002f
#define C2_EXP2 (-0.72134752044448170f)   // -log2(e)/2
#define LN2 0.69314718055994531f

// ------------------------------------------------------------------------------------------
// Diagnostics and small fills
__global__ void k_diag_begin(DiagBlock *d, unsigned long long cap, uint32_t *cnt_last)
{
    if (d->stamp != DIAG_STAMP) diag_clear(d);
    d->instances = 0;
    d->capacity = cap;
    *cnt_last = 0;
}

__global__ void k_diag_check(DiagBlock *d)
{
    if (d->instances > d->capacity) d->overflow = 1u;
    if (d->instances > d->max_instances) d->max_instances = d->instances;
}

__global__ void k_fill_f32(float *p, size_t count, float v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

hipError_t render_zero(float *p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    unsigned blocks = (unsigned)(((count + 255) / 256) < 65536 ? ((count + 255) / 256) : 65536);
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, s, p, count, 0.0f);
    return hipGetLastError();
}

static hipError_t fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    unsigned blocks = (unsigned)(((count + 255) / 256) < 65536 ? ((count + 255) / 256) : 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// a1: FFD at the canonical means, uv = [U (R x 3) ; V (R x 9)] x N, and the Gaussians' parameters
// gs = [mu (3); scale (3); quat (4); rho] x N, both in cell order (entry i belongs to Gaussian
// order[i]). With a per-Gaussian basis (the second ablation of Sec. 4.3: the spatial basis
// stored per Gaussian instead of interpolated from the lattice), U and V are gathered from it.
#define FFD_BRICK_FLOATS 8192   // LDS for a workgroup's control points, all ranks (32 KB)
// Staging pays only when other workgroups hide its extra round trip to memory: calls with fewer
// Gaussians (a few workgroups per CU) read the lattice through the caches (STAGE false).
#define FFD_STAGE_MIN_GAUSSIANS 65536
template <bool STAGE>
__global__ __launch_bounds__(256) void k_ffd_canonical(DevGrid g, const float *__restrict__ coef,
                                                       const float *__restrict__ basis,
                                                       int n, const float *__restrict__ mu,
                                                       const float *__restrict__ scale,
                                                       const float *__restrict__ quat,
                                                       const float *__restrict__ rho,
                                                       const uint32_t *__restrict__ order,
                                                       float *__restrict__ uv,
                                                       float *__restrict__ gs)
{
    // four lanes per Gaussian: lane `part` takes the stencil's z index part, and the four partial
    // sums are added in a fixed order. The control points the workgroup's 64 Gaussians reach
    // (neighbours in cell order) are staged in LDS first.
    __shared__ float brick[STAGE ? FFD_BRICK_FLOATS : 1];
    __shared__ int red[24];
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gt >> 2, part = gt & 3;
    const bool valid = i < n;
    const size_t src = order[valid ? i : 0];
    float *U = uv, *V = uv + (size_t)3 * g.R * n;
    if (valid && part == 0) {
        // the Gaussian's parameters, gathered once into cell order: mu (3), scale (3), quat (4),
        // rho
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gs[(size_t)a * n + i] = mu[(size_t)a * n + src];
            gs[(size_t)(3 + a) * n + i] = scale[(size_t)a * n + src];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) gs[(size_t)(6 + a) * n + i] = quat[(size_t)a * n + src];
        gs[(size_t)10 * n + i] = rho[src];
    }
    if (basis) {
        if (!valid || part != 0) return;
        for (int r = 0; r < g.R; ++r) {
            const float *b = basis + (size_t)r * 12 * n + src;
#pragma unroll
            for (int a = 0; a < 3; ++a) U[((size_t)r * 3 + a) * n + i] = b[(size_t)a * n];
#pragma unroll
            for (int k = 0; k < 9; ++k) V[((size_t)r * 9 + k) * n + i] = b[(size_t)(3 + k) * n];
        }
        return;
    }
    Stencil st;
    make_stencil(g, mu[src], mu[n + src], mu[2 * n + src], st, false);
    BrickRows br;
    const bool staged =
        STAGE && stage_brick(g, coef, st, valid, brick, FFD_BRICK_FLOATS, red, br);
    if (!valid) return;
    for (int r = 0; r < g.R; ++r) {
        float u[3], J[9];
        if (staged) ffd_rank_rows<1>(br, r, st, u, J, part);
        else ffd_rank<1>(g, coef, r, st, u, J, part);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] += __shfl_xor(u[a], 1, DIGS_WAVE);
            u[a] += __shfl_xor(u[a], 2, DIGS_WAVE);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            J[k] += __shfl_xor(J[k], 1, DIGS_WAVE);
            J[k] += __shfl_xor(J[k], 2, DIGS_WAVE);
        }
        if (part == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) U[((size_t)r * 3 + a) * n + i] = u[a];
#pragma unroll
            for (int k = 0; k < 9; ++k) V[((size_t)r * 9 + k) * n + i] = J[k];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Per-(t,n) geometry shared by the set-up and its adjoint.
struct ViewTrig {
    float ct, st;
};

// record part 2 of an idle Gaussian slot: with parts 0 and 1 zero, q = 1, E = 0 and
// log2|amp| = -inf, so the slot adds exactly zero
__device__ __forceinline__ float4 idle_rec2() { return make_float4(0.0f, 0.0f, -INFINITY, 0.0f); }

struct SetupFwd {
    // deformation
    float K[9], Kinv[9], detK, mup[3], W[9];
    // projection set-up
    float alpha, xu, xv, m[3], mw[3], Du[3], Dv[3], c, ic, pa, pb, Dup[3], Dvp[3], beta, kap;
    float Huu, Huv, Hvv, gu, gv, Guu, Guv, Gvv, amp, us, vs;
    float ee;   // EWA: |e*|, the length of the ray through the mean to the detector; exact: 1
    bool ok;
};

__device__ __forceinline__ float dot3(const float *a, const float *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// R = R(q_hat) row-major, RS = R diag(s); U [R][3], V [R][9], w [R]
template <int NR>
__device__ __forceinline__ void setup_forward(const DevGeom &G, const float *mu0,
                                              const float *inv_s, const float *Rm,
                                              const float (*U)[3], const float (*V)[9],
                                              const float *wt, float rho, ViewTrig vt,
                                              SetupFwd &f)
{
    // Eq. 9 and 11: mu' = mu + sum_r w_r u_r(mu), K = I + sum_r w_r grad u_r(mu)
#pragma unroll
    for (int k = 0; k < 9; ++k) f.K[k] = (k % 4 == 0) ? 1.0f : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) f.mup[a] = mu0[a];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int a = 0; a < 3; ++a) f.mup[a] = fmaf(wt[r], U[r][a], f.mup[a]);
#pragma unroll
        for (int k = 0; k < 9; ++k) f.K[k] = fmaf(wt[r], V[r][k], f.K[k]);
    }
    f.detK = inv3(f.K, f.Kinv);
    // W = M^-1 = diag(1/s) R^T K^-1 (Eq. 8 with Sigma = R S S^T R^T)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            f.W[3 * a + b] = inv_s[a] * (Rm[a] * f.Kinv[b] + Rm[3 + a] * f.Kinv[3 + b] +
                                         Rm[6 + a] * f.Kinv[6 + b]);
    const float ct = vt.ct, st = vt.st;
    f.alpha = G.sid - (ct * f.mup[0] + st * f.mup[1]);
    f.xu = st * f.mup[0] - ct * f.mup[1];
    f.xv = -f.mup[2];
    f.ok = isfinite(f.detK) && f.detK != 0.0f && f.alpha > 1e-3f * G.sid;
    const float ia = 1.0f / f.alpha;
    f.us = (-G.sdd * f.xu * ia - G.off_u) / G.pitch_u + 0.5f * (float)(G.nu - 1);
    f.vs = (-G.sdd * f.xv * ia - G.off_v) / G.pitch_v + 0.5f * (float)(G.nv - 1);
    f.m[0] = G.sid * ct - f.mup[0];
    f.m[1] = G.sid * st - f.mup[1];
    f.m[2] = -f.mup[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *Wa = f.W + 3 * a;
        f.mw[a] = Wa[0] * f.m[0] + Wa[1] * f.m[1] + Wa[2] * f.m[2];
        f.Du[a] = G.pitch_u * (-st * Wa[0] + ct * Wa[1]);
        f.Dv[a] = G.pitch_v * Wa[2];
    }
    f.c = dot3(f.mw, f.mw);
    f.ic = 1.0f / f.c;
    f.pa = dot3(f.mw, f.Du) * f.ic;
    f.pb = dot3(f.mw, f.Dv) * f.ic;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.Dup[a] = f.Du[a] - f.pa * f.mw[a];
        f.Dvp[a] = f.Dv[a] - f.pb * f.mw[a];
    }
    f.beta = f.alpha / G.sdd;
    f.kap = f.beta * f.beta;
    f.Huu = f.kap * dot3(f.Dup, f.Dup);
    f.Huv = f.kap * dot3(f.Dup, f.Dvp);
    f.Hvv = f.kap * dot3(f.Dvp, f.Dvp);
    f.gu = -f.beta * f.pa;
    f.gv = -f.beta * f.pb;
    f.Guu = f.kap * dot3(f.Du, f.Du) * f.ic;
    f.Guv = f.kap * dot3(f.Du, f.Dv) * f.ic;
    f.Gvv = f.kap * dot3(f.Dv, f.Dv) * f.ic;
    f.amp = rho * SQRT_2PI * f.beta * sqrtf(f.ic);
    // EWA (Eq. 4): the affine approximation at the mean drops the perspective terms (q = 1), and
    // the 2D Gaussian's peak is the line integral along the ray through the mean, |e*| amp
    f.ee = 1.0f;
    if (G.ewa) {
        f.ee = G.sdd * sqrtf(1.0f + (f.xu * f.xu + f.xv * f.xv) * (ia * ia));
        f.gu = f.gv = f.Guu = f.Guv = f.Gvv = 0.0f;
    }
    f.ok = f.ok && isfinite(f.us) && isfinite(f.vs) && isfinite(f.Huu) && isfinite(f.Huv) &&
           isfinite(f.Hvv) && isfinite(f.Guu) && isfinite(f.Guv) && isfinite(f.Gvv) &&
           isfinite(f.amp) && isfinite(f.gu) && isfinite(f.gv);
}

// The cut-off footprint {delta : E/q <= r^2} = {delta^T (H - r^2 G) delta - 2 r^2 g.delta - r^2 <= 0}
// in centred, normalised form (p - c)^T A (p - c) <= 1 (p in pixel-index coordinates), and its
// bounding box (inclusive pixel ranges, clamped to the detector). Returns false when the conic is
// not an ellipse: then the box is the whole detector and A = 0 (every block is kept).
struct Footprint {
    float cx, cy, a00, a01, a11;
};

__device__ __forceinline__ bool footprint_box(const DevGeom &G, const SetupFwd &f, float r,
                                              int &x0, int &x1, int &y0, int &y1, Footprint &fp)
{
    const float r2 = r * r;
    const float b00 = f.Huu - r2 * f.Guu, b01 = f.Huv - r2 * f.Guv, b11 = f.Hvv - r2 * f.Gvv;
    const float det = b00 * b11 - b01 * b01;
    if (!(b00 > 0.0f && det > 0.0f)) {
        x0 = 0; x1 = G.nu - 1; y0 = 0; y1 = G.nv - 1;
        fp.cx = f.us; fp.cy = f.vs; fp.a00 = fp.a01 = fp.a11 = 0.0f;
        return false;
    }
    const float id = 1.0f / det;
    const float i00 = b11 * id, i01 = -b01 * id, i11 = b00 * id;
    const float cu = r2 * (i00 * f.gu + i01 * f.gv), cv = r2 * (i01 * f.gu + i11 * f.gv);
    const float k2 = r2 + (f.gu * cu + f.gv * cv) * r2;
    const float hu = sqrtf(fmaxf(k2 * i00, 0.0f)), hv = sqrtf(fmaxf(k2 * i11, 0.0f));
    const float ik = 1.0f / k2;
    fp.cx = f.us + cu;
    fp.cy = f.vs + cv;
    fp.a00 = b00 * ik;
    fp.a01 = b01 * ik;
    fp.a11 = b11 * ik;
    if (!(k2 > 0.0f) || !isfinite(ik)) fp.a00 = fp.a01 = fp.a11 = 0.0f;
    const float lo_u = fp.cx - hu - 1e-3f, hi_u = fp.cx + hu + 1e-3f;
    const float lo_v = fp.cy - hv - 1e-3f, hi_v = fp.cy + hv + 1e-3f;
    // clamp in float before converting (boxes far off the detector stay empty)
    x0 = (int)ceilf(fminf(fmaxf(lo_u, -1.0f), (float)G.nu));
    x1 = (int)floorf(fminf(fmaxf(hi_u, -1.0f), (float)G.nu));
    y0 = (int)ceilf(fminf(fmaxf(lo_v, -1.0f), (float)G.nv));
    y1 = (int)floorf(fminf(fmaxf(hi_v, -1.0f), (float)G.nv));
    x0 = max(x0, 0); y0 = max(y0, 0);
    x1 = min(x1, G.nu - 1); y1 = min(y1, G.nv - 1);
    return true;
}

// The cut-off ellipse by horizontal chords: at y = cy + dy the chord is
// x in cx - s dy -+ sqrt((1 - D dy^2) ia), |dy| <= ry; its leftmost point is at dy = ryl and its
// rightmost at dy = -ryl (1 carries a slack of 1e-5). ell is false for a footprint that is not an
// ellipse (it meets everything).
struct FootEll {
    float cx, cy, s, ia, D, ry, ryl;
    bool ell;
    __device__ void init(float a00, float a01, float a11, float ccx, float ccy)
    {
        cx = ccx;
        cy = ccy;
        s = ia = D = ry = ryl = 0.0f;
        const float d = a11 - a01 * (a01 / a00);
        ell = a00 > 0.0f && d > 0.0f && isfinite(d);
        if (ell) {
            s = a01 / a00;
            ia = 1.0f / a00;
            D = d;
            ry = sqrtf(1.00001f / d);
            ryl = a01 / sqrtf(a00 * a11) * ry;
        }
    }
    // x-extent [L, R] of the ellipse within the strip y in [ya, yb]; false if it misses
    __device__ bool strip(float ya, float yb, float &L, float &R) const
    {
        const float lo = fmaxf(ya - cy, -ry), hi = fminf(yb - cy, ry);
        if (!(lo <= hi)) return false;
        // (ryl clamped to [lo, hi]: the median of the three, one instruction)
        const float dl = __builtin_amdgcn_fmed3f(ryl, lo, hi);
        const float dr = __builtin_amdgcn_fmed3f(-ryl, lo, hi);
        L = cx - s * dl - __builtin_amdgcn_sqrtf(fmaxf(0.0f, fmaf(-D * dl, dl, 1.00001f)) * ia);
        R = cx - s * dr + __builtin_amdgcn_sqrtf(fmaxf(0.0f, fmaf(-D * dr, dr, 1.00001f)) * ia);
        return true;
    }
};

// The instances of a (view, Gaussian): the tiles of its footprint's bounding rectangle that the
// footprint ellipse meets. rect = (tx0 | tx1 << 16, ty0 | ty1 << 16, m, 0): for a rectangle of at
// most 32 tiles bit k of m marks tile k (row-major) as an instance; a larger rectangle has all its
// tiles as instances. Instance j of the (view, Gaussian) sits at slot goff + j, in row-major order.
struct TileRect {
    int tx0, ty0, w, h, R;
    uint32_t m;
    __device__ static TileRect from(int4 r)
    {
        TileRect q;
        q.tx0 = r.x & 0xffff;
        q.ty0 = r.y & 0xffff;
        const int tx1 = r.x >> 16, ty1 = r.y >> 16;
        q.w = tx1 - q.tx0 + 1;
        q.h = ty1 - q.ty0 + 1;
        q.R = (tx1 >= q.tx0 && ty1 >= q.ty0) ? q.w * q.h : 0;
        q.m = (uint32_t)r.z;   // the set-up stores it restricted to the rectangle's R tiles
        return q;
    }
    __device__ int count() const { return R > 32 ? R : __popc(m); }
    // rectangle tile (row-major index) of instance j < count()
    __device__ int tile_of(int j) const
    {
        if (R > 32) return j;
        uint32_t v = m;
        int p = 0;
#pragma unroll
        for (int b = 16; b >= 1; b >>= 1) {
            const int c = __popc(v & ((1u << b) - 1u));
            if (j >= c) {
                j -= c;
                v >>= b;
                p += b;
            }
        }
        return p;
    }
    // instance index of rectangle tile k (an instance)
    __device__ int inst_of(int k) const { return R > 32 ? k : __popc(m & ((1u << k) - 1u)); }
};

// Instance mask of a footprint rectangle of R <= 32 tiles (see TileRect): in each row of tiles,
// the tiles whose tw columns meet the ellipse's x-extent over the row's th pixel rows. (This
// keeps every tile in which a list entry could mark an 8x8 block; a kept tile with no such block
// only costs an empty entry.)
__device__ uint32_t footprint_tiles(const Footprint &fp, int tx0, int ty0, int w, int h, int tw,
                                    int th)
{
    FootEll fe;
    fe.init(fp.a00, fp.a01, fp.a11, fp.cx, fp.cy);
    if (!fe.ell) return ~0u;
    uint32_t m = 0u;
    const float inv = 1.0f / (float)tw;   // exact: tw is a power of two
    for (int r = 0; r < h; ++r) {
        const float y0 = (float)((ty0 + r) * th);
        float L, R;
        if (!fe.strip(y0, y0 + (float)(th - 1), L, R)) continue;
        // columns c with (tx0 + c) tw <= R and (tx0 + c) tw + tw - 1 >= L
        const int c0 = max(0, (int)ceilf(fmaxf((L - (float)(tw - 1)) * inv, -1.0f)) - tx0);
        const int c1 = min(w - 1, (int)floorf(fminf(R * inv, 65536.0f)) - tx0);
        if (c0 <= c1) m |= (((1u << (c1 - c0)) << 1) - 1u) << (r * w + c0);
    }
    return m;
}

template <int NR>
__global__ __launch_bounds__(256) void k_setup(DevGeom G, int n, int T,
                                               const float *__restrict__ gs,
                                               const float *__restrict__ angles,
                                               const float *__restrict__ w,
                                               const float *__restrict__ uv, float cull,
                                               float4 *__restrict__ rec,
                                               int4 *__restrict__ rect,
                                               uint32_t *__restrict__ gcount,
                                               DiagBlock *__restrict__ diag)
{
    __shared__ unsigned long long wsum[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // position in cell order
    const bool valid = i < n;
    const int ii = valid ? i : 0;
    float mu0[3], s[3], q[4], Rm[9], inv_s[3];
    float U[NR][3], V[NR][9];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mu0[a] = gs[(size_t)a * n + ii];
        s[a] = gs[(size_t)(3 + a) * n + ii];
        inv_s[a] = 1.0f / s[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) q[a] = gs[(size_t)(6 + a) * n + ii];
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    quat_to_rot(q[0] * qn, q[1] * qn, q[2] * qn, q[3] * qn, Rm);
    const float rh = gs[(size_t)10 * n + ii];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int a = 0; a < 3; ++a) U[r][a] = uv[((size_t)r * 3 + a) * n + ii];
#pragma unroll
        for (int k = 0; k < 9; ++k) V[r][k] = uv[((size_t)3 * NR + r * 9 + k) * n + ii];
    }
    bool inputs_ok = isfinite(mu0[0]) && isfinite(mu0[1]) && isfinite(mu0[2]) && s[0] > 0.0f &&
                     s[1] > 0.0f && s[2] > 0.0f && isfinite(inv_s[0] * inv_s[1] * inv_s[2]) &&
                     isfinite(qn) && isfinite(rh);
    unsigned long long mycount = 0;
    const int t0 = blockIdx.y * SETUP_TCHUNK, t1 = min(T, t0 + SETUP_TCHUNK);
    for (int t = t0; t < t1; ++t) {
        float wt[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) wt[r] = w[(size_t)t * NR + r];
        ViewTrig vt;
        sincosf(angles[t], &vt.st, &vt.ct);
        SetupFwd f;
        setup_forward<NR>(G, mu0, inv_s, Rm, U, V, wt, rh, vt, f);
        int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
        Footprint fp = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        bool ok = inputs_ok && f.ok;
        if (valid) {
            if (!inputs_ok || !(isfinite(f.detK) && f.detK != 0.0f))
                atomicAdd(&diag->nonfinite, 1u);
            else if (!(f.alpha > 1e-3f * G.sid))
                atomicAdd(&diag->behind_source, 1u);
            else if (!f.ok)
                atomicAdd(&diag->nonfinite, 1u);
            if (ok && f.detK <= 0.0f) atomicAdd(&diag->folded, 1u);
        }
        if (ok) {
            if (!footprint_box(G, f, cull, x0, x1, y0, y1, fp) && valid)
                atomicAdd(&diag->wide, 1u);
        }
        uint32_t count = 0;
        int4 rr = make_int4(1, 0, 0, 0);
        if (valid && ok && x0 <= x1 && y0 <= y1) {
            const int tx0 = x0 >> G.tile_lw, tx1 = x1 >> G.tile_lw;
            const int ty0 = y0 >> G.tile_lh, ty1 = y1 >> G.tile_lh;
            const int w = tx1 - tx0 + 1, h = ty1 - ty0 + 1;
            count = (uint32_t)(w * h);
            uint32_t m = ~0u;
            if (w * h <= 32) {
                m = footprint_tiles(fp, tx0, ty0, w, h, G.tile_w, G.tile_h);
                if (w * h < 32) m &= (1u << (w * h)) - 1u;
                count = (uint32_t)__popc(m);
            }
            rr = make_int4(tx0 | (tx1 << 16), ty0 | (ty1 << 16), (int)m, 0);
        } else {
            x0 = 1; x1 = 0; y0 = 1; y1 = 0;
        }
        mycount += count;
        if (valid) {
            const size_t o = (size_t)t * n + i;
            if (ok) {
                rec[o * 4 + 0] = make_float4(f.us, f.vs, C2_EXP2 * f.Huu, 2.0f * C2_EXP2 * f.Huv);
                rec[o * 4 + 1] = make_float4(C2_EXP2 * f.Hvv, 2.0f * f.gu, 2.0f * f.gv, f.Guu);
                // the splats take amp as log2|amp| (-inf for 0) with its sign on Gvv (>= +0)
                const float ampr = f.amp * f.ee;
                rec[o * 4 + 2] = make_float4(2.0f * f.Guv, copysignf(f.Gvv, ampr),
                                             log2f(fabsf(ampr)), fp.a00);
                rec[o * 4 + 3] = make_float4(fp.a01, fp.a11, fp.cx, fp.cy);
            } else {   // an idle record: adds zero wherever it is evaluated
                const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                rec[o * 4 + 0] = z;
                rec[o * 4 + 1] = z;
                rec[o * 4 + 2] = idle_rec2();
                rec[o * 4 + 3] = z;
            }
            rect[o] = rr;
            gcount[o] = count;
        }
    }
    // exact total of instances (64-bit) for the capacity check
    unsigned long long v = mycount;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane_id() == 0) wsum[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (tot) atomicAdd(&diag->instances, tot);
    }
}

// ------------------------------------------------------------------------------------------
// a4: binning sources. A tile list entry is the Gaussian's index in the low 24 bits; above it two
// bits per 8x8 pixel block b of the tile (at most four blocks, in row-major order: block column
// b % tile_bx, block row b / tile_bx): bit LIST_BLOCK_SHIFT + 2b is set when the cut-off footprint
// ellipse meets rows 0-3 of the block, the next bit when it meets rows 4-7. The splats evaluate
// only those rows.
#define LIST_INDEX_MASK 0x00FFFFFFu
#define LIST_BLOCK_SHIFT 24

// Per 8x8 block b of tile (tx, ty) of a TW x TH tile shape, which 4-row halves the cut-off ellipse
// meets (bits 2b and 2b + 1; blocks in row-major order).
template <int TW, int TH>
__device__ __forceinline__ uint32_t block_mask(const FootEll &fe, int tx, int ty)
{
    uint32_t m = 0u;
    const float x0 = (float)(tx * TW), y0 = (float)(ty * TH);
#pragma unroll
    for (int s4 = 0; s4 < TH / 4; ++s4) {   // 4-row strips; block row s4 >> 1, half s4 & 1
        float L, R;
        if (fe.strip(y0 + (float)(4 * s4), y0 + (float)(4 * s4 + 3), L, R)) {
            const int b = (s4 >> 1) * (TW / 8), h = s4 & 1;
#pragma unroll
            for (int c = 0; c < TW / 8; ++c) {   // block columns
                const float xb = x0 + (float)(8 * c);
                if (xb <= R && xb + 7.0f >= L) m |= 1u << (2 * (b + c) + h);
            }
        }
    }
    return m;
}

template <int TW, int TH>   // tile shape (pixels)
struct TileSrc {
    const int4 *rect;        // [T][N] footprint rectangles and instance masks (TileRect)
    const float4 *rec;       // [T][N][4] projected records (footprint conic in rec[2].w, rec[3])
    uint32_t *list;
    size_t cap;
    int items;               // N
    int tiles_x;
    float inv_tiles_x;       // 1 / tiles_x
    struct Item {
        TileRect tr;
        int cnt, tiles_x;
        float inv_w;
        FootEll fe;          // the cut-off ellipse (prepare)
        __device__ int nkeys() const { return cnt; }
        // tile of instance k (row-major in the rectangle; k / w in float: exact for k < 2^21)
        __device__ void tile(int k, int &tx, int &ty) const
        {
            const int p = tr.tile_of(k);
            const int q = (int)(((float)p + 0.5f) * inv_w);
            tx = tr.tx0 + (p - __mul24(q, tr.w));
            ty = tr.ty0 + q;
        }
        __device__ int key(int k) const
        {
            int tx, ty;
            tile(k, tx, ty);
            return __mul24(ty, tiles_x) + tx;
        }
        // one count per instance tile, by rows of the rectangle (no instance search)
        __device__ void count(uint32_t *h) const
        {
            if (cnt == 0) return;
            const uint32_t rowmask = tr.w >= 32 ? ~0u : ((1u << tr.w) - 1u);
            for (int r = 0; r < tr.h; ++r) {
                const int row = __mul24(tr.ty0 + r, tiles_x) + tr.tx0;
                if (tr.R > 32) {
                    for (int c = 0; c < tr.w; ++c) atomicAdd(&h[row + c], 1u);
                } else {
                    for (uint32_t v = (tr.m >> (r * tr.w)) & rowmask; v; v &= v - 1u)
                        atomicAdd(&h[row + __builtin_ctz(v)], 1u);
                }
            }
        }
    };
    __device__ Item load(int t, int item) const
    {
        Item it;
        it.tr = TileRect::from(rect[(size_t)t * items + item]);
        it.cnt = it.tr.count();
        it.inv_w = it.cnt > 0 ? 1.0f / (float)it.tr.w : 0.0f;
        it.tiles_x = tiles_x;
        it.fe.cx = it.fe.cy = it.fe.s = it.fe.ia = it.fe.D = it.fe.ry = it.fe.ryl = 0.0f;
        it.fe.ell = false;
        return it;
    }
    __device__ void prepare(int t, int item, Item &it) const
    {
        const float4 *r = rec + ((size_t)t * items + item) * 4;
        const float4 c = r[2], d = r[3];
        it.fe.init(c.w, d.x, d.y, d.z, d.w);
    }
    // the entry: the Gaussian's index and, per 8x8 block, which 4-row halves its ellipse meets
    // (a footprint that is not an ellipse meets them all)
    __device__ void emit(int, int item, const Item &it, int, unsigned key, uint32_t pos) const
    {
        if (pos >= cap) return;
        // the tile from its key (key / tiles_x in float: exact for keys below 2^21)
        const int ty = (int)(((float)key + 0.5f) * inv_tiles_x);
        const int tx = (int)key - __mul24(ty, tiles_x);
        // (bits of blocks the tile does not have are never read)
        const uint32_t m = it.fe.ell ? block_mask<TW, TH>(it.fe, tx, ty) : 0xFFu;
        list[pos] = (uint32_t)item | (m << LIST_BLOCK_SHIFT);
    }
};

// ------------------------------------------------------------------------------------------
// Workgroup -> (view, tile). The hardware hands consecutive workgroups of a launch to the 8 XCDs
// in turn (b mod 8). When T is a multiple of 8, XCD x is given the views t = x (mod 8) one after
// another, tile by tile in row-major order, so the records and lists one XCD reads at a time
// belong to a band of tile rows of one view and stay in that XCD's L2.
__device__ __forceinline__ void map_block(int b, int ntiles, int T, int &t, int &tile)
{
    if ((T & 7) == 0) {
        const int x = b & 7, k = b >> 3, q = k / ntiles;
        t = x + 8 * q;
        tile = k - q * ntiles;
    } else {
        t = b / ntiles;
        tile = b - t * ntiles;
    }
}

// Entries [begin, end) of one tile list cut into nsl slices of `round` -entry multiples (the
// last ones may be short or empty); slice sl keeps its part.
__device__ __forceinline__ void slice_range(uint32_t &begin, uint32_t &end, int sl, int nsl,
                                            uint32_t round)
{
    if (nsl <= 1) return;
    const uint64_t len = end - begin;
    uint64_t per = (len + (uint64_t)nsl - 1u) / (uint64_t)nsl;
    per = (per + round - 1u) / round * round;
    const uint64_t b = min(len, per * (uint64_t)sl), e = min(len, per * (uint64_t)(sl + 1));
    end = begin + (uint32_t)e;
    begin = begin + (uint32_t)b;
}

// ------------------------------------------------------------------------------------------
// a5: forward splat. One workgroup per (view, tile), one wave per 8x8 pixel block (with
// WAVES == 1 a single wave takes the tile's four blocks in turn). The wave walks the tile's list
// in chunks of 64 entries and appends the Gaussians whose footprint meets its block (bits of the
// list entry) to one of three queues in LDS: those that meet both 4-row halves of the block, only
// the upper, only the lower. It evaluates each queue 8 Gaussians at a time, over the rows its
// Gaussians meet, and carries the remainder (fewer than 8) over to the next chunk, so that only
// each queue's last group has idle lanes. lane = (Gaussian slot, column); each lane runs down the
// rows of its column with forward differences of the two quadratic forms (two adds each per row).
// The amplitude enters as log2|amp| added to the exponent (one multiply less per pixel); positive
// and negative amplitudes go to separate row sums, the negative ones in a second pass that only
// groups holding one take. The per-lane row sums are reduced over the 8 slots at the end in a
// fixed order, and every pixel is written once.
#define FWD_QUEUE (DIGS_WAVE + 8)

// Adds rows [R0, R0 + NR) of one Gaussian at the lane's column into acc: from the row quadratics
// q (and its first and second differences) and E, with la = log2|amp| (-inf: adds zero). EWA:
// q = 1, so a pixel costs one exp2 and the E recurrence.
template <bool EWA, int R0, int NR>
__device__ __forceinline__ void splat_fwd_rows(float q, float dq, float ddq, float e, float de,
                                               float dde, float la, float *acc)
{
    if constexpr (EWA) {
        e += la;   // amp 2^E = 2^(E + log2 amp)
#pragma unroll
        for (int row = 0; row < NR; ++row) {
            acc[R0 + row] += __builtin_amdgcn_exp2f(e);
            e += de;
            de += dde;
        }
    } else {
        // amp rs 2^x = rs 2^(x + log2 amp)
#pragma unroll
        for (int row = 0; row < NR; ++row) {
            const float rs = __builtin_amdgcn_rsqf(q);
            const float x = fmaf(e, rs * rs, la);
            acc[R0 + row] = fmaf(rs, __builtin_amdgcn_exp2f(x), acc[R0 + row]);
            q += dq;
            dq += ddq;
            e += de;
            de += dde;
        }
    }
}

// Evaluates the wave's queued Gaussians [0, ns) (a multiple of 8 unless TAIL: the queue's last
// group) over rows [R0, R0 + NR) of the block: positive amplitudes into the lane's row sums acc,
// negative ones (by magnitude, in a second pass taken only when the group has any) into accn.
// The queue holds the byte offsets of the Gaussians' records from rt.
template <bool EWA, int R0, int NR, bool TAIL>
__device__ __forceinline__ void splat_fwd_group(const float4 *__restrict__ rt,
                                                const uint32_t *__restrict__ qid, int ns,
                                                int gslot, float fi, float fby, float *acc,
                                                float *accn)
{
    for (int j = 0; j < ns; j += 8) {
        // (TAIL) a slot past the queue's end repeats its last Gaussian with amplitude 0
        const int sn = j + gslot;
        const bool live = !TAIL || sn < ns;
        const float4 *rg =
            (const float4 *)((const char *)rt + qid[TAIL ? min(sn, ns - 1) : sn]);
        const float4 r0 = rg[0], r1 = rg[1], r2 = rg[2];
        // r0 = (us, vs, Huu', Huv'), r1 = (Hvv', gu2, gv2, Guu),
        // r2 = (Guv2, Gvv carrying the sign of amp, log2|amp|, -)
        const float du = fi - r0.x, dv0 = (fby + (float)R0) - r0.y;
        const float Aq = fmaf(du, fmaf(r1.w, du, r1.y), 1.0f);
        const float Bq = fmaf(r2.x, du, r1.z), Cq = fabsf(r2.y);
        const float AE = r0.z * du * du, BE = r0.w * du, CE = r1.x;
        const float s1 = fmaf(2.0f, dv0, 1.0f);
        const float q = fmaf(dv0, fmaf(Cq, dv0, Bq), Aq);
        const float dq = fmaf(Cq, s1, Bq);
        const float e = fmaf(dv0, fmaf(CE, dv0, BE), AE);
        const float de = fmaf(CE, s1, BE);
        const bool neg = signbit(r2.y);
        splat_fwd_rows<EWA, R0, NR>(q, dq, 2.0f * Cq, e, de, 2.0f * CE,
                                    (live && !neg) ? r2.z : -INFINITY, acc);
        if (__ballot(live && neg) != 0ull)
            splat_fwd_rows<EWA, R0, NR>(q, dq, 2.0f * Cq, e, de, 2.0f * CE,
                                        (live && neg) ? r2.z : -INFINITY, accn);
    }
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// With nsl > 1 the workgroup renders slice sl of the tile's list into its own partial image
// spart[sl][t][tile][256] (without the |e| factor); k_slice_reduce adds the slices in order.
template <int WAVES, bool EWA>
__device__ __forceinline__ void splat_fwd_tile(const DevGeom &G, int n, int t, int tile,
                                               const float4 *__restrict__ rec,
                                               const uint32_t *__restrict__ list,
                                               const uint32_t *__restrict__ cnt, int nblk,
                                               unsigned cap, float *__restrict__ proj,
                                               uint32_t (*ids)[3][FWD_QUEUE], int sl, int nsl,
                                               int T, float *__restrict__ spart)
{
    const int tx = tile % G.tiles_x, ty = tile / G.tiles_x;
    const int wave = uniform((int)(threadIdx.x / DIGS_WAVE)), lane = lane_id();
    const int gslot = lane >> 3, col = lane & 7;
    const size_t cidx = ((size_t)t * G.ntiles + tile) * nblk;
    uint32_t begin = cnt[cidx], end = cnt[cidx + nblk];
    begin = min(begin, cap);
    end = min(max(end, begin), cap);
    slice_range(begin, end, sl, nsl, DIGS_WAVE);
    const float4 *rt = rec + (size_t)t * n * 4;
    // the wave's three queues: Gaussians that meet rows 0-7 of the block, only rows 0-3, only 4-7
    uint32_t(*qs)[FWD_QUEUE] = ids[wave];
    // WAVES > 1 is launched only with one wave per block of the tile; a single wave takes the
    // tile's blocks in turn
    const int lbx = G.tile_lw - 3;   // log2 of the blocks per tile row
    const int nblocks = WAVES > 1 ? 1 : G.tile_nb;
    for (int pass = 0; pass < nblocks; ++pass) {
        const int blkid = WAVES > 1 ? wave : pass;
        const int bx = tx * G.tile_w + (blkid & (G.tile_bx - 1)) * 8;
        const int by = ty * G.tile_h + (blkid >> lbx) * 8;
        const float fi = (float)(bx + col), fby = (float)by;
        float acc[8], accn[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = accn[r] = 0.0f;
        // queued Gaussians carried over from earlier chunks (fewer than 8 per queue)
        int pend0 = 0, pend1 = 0, pend2 = 0;
        for (uint32_t c0 = begin; c0 < end; c0 += DIGS_WAVE) {
            const uint32_t k = c0 + lane;
            uint32_t g = 0, h = 0;
            if (k < end) {
                const uint32_t e = list[k];
                g = e & LIST_INDEX_MASK;
                h = g < (uint32_t)n ? (e >> (LIST_BLOCK_SHIFT + 2 * blkid)) & 3u : 0u;
            }
            const unsigned long long m0 = __ballot(h == 3u), m1 = __ballot(h == 1u),
                                     m2 = __ballot(h == 2u);
            // a masked store per queue (the empty asm keeps the compiler from merging them into
            // one store whose queue, count and mask each lane selects)
            // (the queues hold the records' byte offsets, g * 64 < 2^30)
            const uint32_t go = g << 6;
            if (h == 3u) qs[0][pend0 + lane_rank(m0)] = go;
            asm volatile("" ::: "memory");
            if (h == 1u) qs[1][pend1 + lane_rank(m1)] = go;
            asm volatile("" ::: "memory");
            if (h == 2u) qs[2][pend2 + lane_rank(m2)] = go;
            const int ns0 = pend0 + __popcll(m0), ns1 = pend1 + __popcll(m1),
                      ns2 = pend2 + __popcll(m2);
            const int f0 = ns0 & ~7, f1 = ns1 & ~7, f2 = ns2 & ~7;
            wave_sync_lds();
            if (f0 > 0)
                splat_fwd_group<EWA, 0, 8, false>(rt, qs[0], f0, gslot, fi, fby, acc, accn);
            if (f1 > 0)
                splat_fwd_group<EWA, 0, 4, false>(rt, qs[1], f1, gslot, fi, fby, acc, accn);
            if (f2 > 0)
                splat_fwd_group<EWA, 4, 4, false>(rt, qs[2], f2, gslot, fi, fby, acc, accn);
            if ((f0 | f1 | f2) > 0) {
                // move each queue's remainder to its front: lane 8c + i moves entry i of queue c
                const int qc = lane >> 3, qi = lane & 7;
                const int fc = qc == 0 ? f0 : (qc == 1 ? f1 : f2);
                const int lc = (qc == 0 ? ns0 : (qc == 1 ? ns1 : ns2)) - fc;
                const bool mv = qc < 3 && qi < lc;
                const uint32_t keep = mv ? qs[qc][fc + qi] : 0u;
                wave_sync_lds();
                if (mv) qs[qc][qi] = keep;
                wave_sync_lds();
            }
            pend0 = ns0 - f0;
            pend1 = ns1 - f1;
            pend2 = ns2 - f2;
        }
        if (pend0 > 0)
            splat_fwd_group<EWA, 0, 8, true>(rt, qs[0], pend0, gslot, fi, fby, acc, accn);
        if (pend1 > 0)
            splat_fwd_group<EWA, 0, 4, true>(rt, qs[1], pend1, gslot, fi, fby, acc, accn);
        if (pend2 > 0)
            splat_fwd_group<EWA, 4, 4, true>(rt, qs[2], pend2, gslot, fi, fby, acc, accn);
        wave_sync_lds();
        // sum over the 8 Gaussian slots (lane bits 3..5) in a fixed order
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            acc[r] -= accn[r];
            acc[r] += __shfl_xor(acc[r], 8, 64);
            acc[r] += __shfl_xor(acc[r], 16, 64);
            acc[r] += __shfl_xor(acc[r], 32, 64);
        }
        float v = acc[0];
#pragma unroll
        for (int r = 1; r < 8; ++r) v = (gslot == r) ? acc[r] : v;
        const int px = bx + col, py = by + gslot;
        if (nsl > 1) {
            const int p = (py - ty * G.tile_h) * G.tile_w + (px - tx * G.tile_w);
            spart[(((size_t)sl * T + t) * G.ntiles + tile) * (G.tile_w * G.tile_h) + p] = v;
        } else if (px < G.nu && py < G.nv) {
            // exact: times the pixel's ray length |e| (EWA: |e*| is in each amplitude)
            if constexpr (!EWA) {
                const float xu = ((float)px - 0.5f * (float)(G.nu - 1)) * G.pitch_u + G.off_u;
                const float yv = ((float)py - 0.5f * (float)(G.nv - 1)) * G.pitch_v + G.off_v;
                v *= sqrtf(G.sdd * G.sdd + xu * xu + yv * yv);
            }
            proj[((size_t)t * G.nv + py) * G.nu + px] = v;
        }
    }
}

// Work items of a persistent launch: with T a multiple of 8 there is one queue per XCD (queue x
// holds the views t = x mod 8, tile by tile, like map_block); a workgroup takes items from the
// queue of its XCD (workgroups of a launch start on XCD b mod 8) and, once that is empty, from the
// others in turn. Returns -1 when every queue is empty, so every workgroup ends.
__device__ __forceinline__ int next_item(uint32_t *__restrict__ queue, int home, int ntiles,
                                         int T)
{
    const int nq = ((T & 7) == 0) ? 8 : 1;
    const uint32_t per = (uint32_t)(T / nq) * (uint32_t)ntiles;
    for (int k = 0; k < nq; ++k) {
        const int x = (home + k) % nq;
        const uint32_t j = atomicAdd(&queue[x], 1u);
        if (j < per) return (nq == 8) ? (int)(j * 8u + (uint32_t)x) : (int)j;
    }
    return -1;
}

// blockIdx.x: (view, tile); blockIdx.y: slice of the tile's list (gridDim.y slices)
template <int WAVES, bool EWA>
__global__ __launch_bounds__(64 * WAVES) void k_splat_fwd(DevGeom G, int n, int T,
                                                          const float4 *__restrict__ rec,
                                                          const uint32_t *__restrict__ list,
                                                          const uint32_t *__restrict__ cnt,
                                                          int nblk, unsigned cap,
                                                          float *__restrict__ proj,
                                                          float *__restrict__ spart)
{
    __shared__ uint32_t ids[WAVES][3][FWD_QUEUE];
    int t, tile;
    map_block(blockIdx.x, G.ntiles, T, t, tile);
    splat_fwd_tile<WAVES, EWA>(G, n, t, tile, rec, list, cnt, nblk, cap, proj, ids, blockIdx.y,
                               gridDim.y, T, spart);
}

// The slices' partial images added in slice order, times the pixel's ray length |e| (exact
// model; EWA: |e*| is in each amplitude): one thread per pixel.
template <bool EWA>
__global__ __launch_bounds__(256) void k_slice_reduce(DevGeom G, int T, int nsl,
                                                      const float *__restrict__ spart,
                                                      float *__restrict__ proj)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)G.nu * G.nv;
    if (i >= npx * T) return;
    const int t = (int)(i / npx);
    const int rem = (int)(i - (size_t)t * npx);
    const int py = rem / G.nu, px = rem - py * G.nu;
    const int tile = (py >> G.tile_lh) * G.tiles_x + (px >> G.tile_lw);
    const int p = (py & (G.tile_h - 1)) * G.tile_w + (px & (G.tile_w - 1));
    const int tpx = G.tile_w * G.tile_h;
    const size_t stride = (size_t)T * G.ntiles * tpx;
    const float *src = spart + ((size_t)t * G.ntiles + tile) * tpx + p;
    float v = src[0];
    for (int s = 1; s < nsl; ++s) v += src[(size_t)s * stride];
    if constexpr (!EWA) {
        const float xu = ((float)px - 0.5f * (float)(G.nu - 1)) * G.pitch_u + G.off_u;
        const float yv = ((float)py - 0.5f * (float)(G.nv - 1)) * G.pitch_v + G.off_v;
        v *= sqrtf(G.sdd * G.sdd + xu * xu + yv * yv);
    }
    proj[i] = v;
}

// Persistent variant: a grid sized to the machine loops over the work queues.
template <int WAVES, bool EWA>
__global__ __launch_bounds__(64 * WAVES) void k_splat_fwd_persist(
    DevGeom G, int n, int T, const float4 *__restrict__ rec, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ cnt, int nblk, unsigned cap, float *__restrict__ proj,
    uint32_t *__restrict__ queue)
{
    __shared__ uint32_t ids[WAVES][3][FWD_QUEUE];
    __shared__ int s_item;
    const int home = blockIdx.x & 7;
    for (;;) {
        if (threadIdx.x == 0) s_item = next_item(queue, home, G.ntiles, T);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item < 0) break;
        int t, tile;
        map_block(item, G.ntiles, T, t, tile);
        splat_fwd_tile<WAVES, EWA>(G, n, t, tile, rec, list, cnt, nblk, cap, proj, ids, 0, 1, T,
                                   nullptr);
    }
}

// Measurement only: the pairs inside each footprint and on the detector, and the pairs the forward
// and backward splats evaluate (per 8x8 block that a footprint ellipse meets, 64, or 32 when it
// meets only one 4-row half of the block; the same in both).
__global__ __launch_bounds__(256) void k_count_pairs(DevGeom G, int n, int T, float cull,
                                                     const float *__restrict__ rec,
                                                     const uint32_t *__restrict__ list,
                                                     const uint32_t *__restrict__ cnt, int nblk,
                                                     unsigned cap, DiagBlock *__restrict__ diag)
{
    __shared__ unsigned long long tot[3];
    if (threadIdx.x < 3) tot[threadIdx.x] = 0;
    __syncthreads();
    int t, tile;
    map_block(blockIdx.x, G.ntiles, T, t, tile);
    const int tx = tile % G.tiles_x, ty = tile / G.tiles_x;
    const int wave = threadIdx.x / DIGS_WAVE, lane = lane_id();
    const size_t cidx = ((size_t)t * G.ntiles + tile) * nblk;
    uint32_t begin = cnt[cidx], end = cnt[cidx + nblk];
    begin = min(begin, cap);
    end = min(max(end, begin), cap);
    const int bx = tx * G.tile_w + (wave & (G.tile_bx - 1)) * 8;
    const int by = ty * G.tile_h + (wave >> (G.tile_lw - 3)) * 8;
    const int px = bx + (lane & 7), py = by + (lane >> 3);
    const bool on_det = px < G.nu && py < G.nv;
    if (wave >= G.tile_nb) begin = end;   // the tile has fewer blocks than waves
    const float c2r2 = (-0.72134752044448170f) * cull * cull;   // exp2 argument at the cut-off
    unsigned long long in_fp = 0, eval_f = 0;
    for (uint32_t k = begin; k < end; ++k) {
        const uint32_t ent = uniform(list[k]);
        const uint32_t g = ent & LIST_INDEX_MASK;
        const uint32_t h = (ent >> (LIST_BLOCK_SHIFT + 2 * wave)) & 3u;
        if (g >= (uint32_t)n || h == 0u) continue;
        const float *r = rec + ((size_t)t * n + g) * DIGS_REC_FLOATS;
        eval_f += h == 3u ? 64 : 32;
        const float du = (float)px - r[0], dv = (float)py - r[1];
        const float q = fmaf(du, fmaf(r[7], du, fmaf(r[8], dv, r[5])),
                             fmaf(dv, fmaf(fabsf(r[9]), dv, r[6]), 1.0f));
        const float e = fmaf(du, fmaf(r[2], du, r[3] * dv), r[4] * dv * dv);
        const bool inside = on_det && q > 0.0f && e >= c2r2 * q;
        in_fp += __popcll(__ballot(inside));
    }
    if (lane == 0) {
        atomicAdd(&tot[0], in_fp);
        atomicAdd(&tot[1], eval_f);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&diag->stat[0], tot[0]);
        atomicAdd(&diag->stat[1], tot[1]);
        atomicAdd(&diag->stat[2], tot[1]);   // the backward splat walks the same blocks
    }
}

__global__ void k_stat_reset(DiagBlock *d) { d->stat[0] = d->stat[1] = d->stat[2] = 0; }

hipError_t render_count_pairs(const RenderArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_stat_reset, dim3(1), dim3(1), 0, s, WS(a, diag, DiagBlock *));
    hipLaunchKernelGGL(k_count_pairs, dim3(a.geom.ntiles * a.T), dim3(256), 0, s, a.geom, a.n,
                       a.T, a.cull, WS(a, rec, const float *), WS(a, list, const uint32_t *),
                       WS(a, cnt, const uint32_t *), a.L.nblk, (unsigned)a.L.cap,
                       WS(a, diag, DiagBlock *));
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// a6: backward splat. One workgroup per (projection, tile); the tile's dL/dI (times |e|) is staged
// in LDS (row stride 18 keeps the four 8x8 blocks in distinct banks). Each wave takes chunks of
// 64 list entries and appends the (entry, 8x8 block) pairs whose footprint ellipse meets the block
// (block-major) to one of two pair queues in LDS: pairs whose ellipse meets both 4-row halves of
// the block run over its 8 rows, the others over the one half they meet. Each queue is evaluated
// 64 pairs at a time, one pair per lane, and its remainder is carried over to the next chunk, so
// that lanes idle only when a chunk must be finished early (below) and in the tile's last groups
// (the four waves' remainders, pooled and evaluated by one wave). A
// lane runs over its pair's 64 (or 32) pixels with forward differences along each row and
// accumulates twelve moment sums, which are added into the entry's LDS slot in block order (fixed
// order, no atomics). Entry slots belong to
// two chunks in turn; once the pairs of a chunk are all evaluated (by the end of the next chunk's
// step, with a partial group if no full one forms), its entries are written as the instances'
// partials, at each instance's slot in Gaussian-major order (so that the per-Gaussian reduction
// reads each Gaussian's partials contiguously). Per pixel, with a = g r 2^x r^2 (EWA: g 2^x),
// dL/dE = -amp/2 a and dL/dq = -amp/2 a (1 + 2 ln2 x); the partial holds the sums without the
// factor -amp/2, which is the same for every pixel of a (view, Gaussian) and is applied once by
// the adjoint of the set-up, which also forms the dL/dq sums from those of a and a x:
//  0 sum g r 2^x  (dL/damp)
//  1, 2, 3    sum a du^2, a du dv, a dv^2
//  4, 5, 6    sum a x du^2, a x du dv, a x dv^2  (exact model only; EWA: 0)
//  7, 8       sum a x du, a x dv                  (exact only)
//  9          sum a (1 + 2 ln2 x)                 (exact only)
//  10, 11     sum a du, a dv
// dL/dI of the tile in LDS: rows of tile_w + 2 floats (18 for 16-pixel rows)
#define GPX_FLOATS 320              // the largest tile's rows: 32 x (8 + 2) or 16 x 18 or 8 x 34
#define BWD_QUEUE (5 * DIGS_WAVE)   // carried (< 64) + one chunk's pairs (<= 256)
struct BwdShared {
    float gpx[GPX_FLOATS];
    uint32_t pairs[4][2][BWD_QUEUE];       // (entry slot << 3) | (half << 2) | block
    uint32_t gid[4][2 * DIGS_WAVE];        // record byte offset (Gaussian x 64) of each entry slot
    float accS[4][2 * DIGS_WAVE][13];      // moment sums of each entry slot
    int pend[2][4];                        // each wave's pairs left at the end of the tile
};

// Evaluates queued pairs [j0, j0 + cnt) of the wave (cnt <= 64), one per lane, over NROWS rows of
// the pair's block (with NROWS == 4 the half that bit 2 of the pair names), and adds their moment
// sums into the entries' slots (NB blocks per tile). EWA: q = 1 (no dL/dq moments), one exp2 per
// pixel. TW: tile width in pixels (the LDS rows of dL/dI hold TW + 2 floats).
template <bool EWA, int NROWS, int TW, int NB>
__device__ __forceinline__ void splat_bwd_group(const float4 *__restrict__ rt,
                                                const uint32_t *__restrict__ pq,
                                                const uint32_t *__restrict__ gid,
                                                float (*accS)[13], const float *__restrict__ gpx,
                                                int j0, int cnt, int tx0, int ty0)
{
    // products are not contracted into sums here: each product feeds several sums, and a
    // contraction would compute it twice
#pragma clang fp contract(off)
    constexpr int GPX_STRIDE = TW + 2, BXL = TW == 8 ? 0 : (TW == 16 ? 1 : 2);
    const int lane = lane_id();
    // a lane past the group's end evaluates its last pair again and adds nothing
    const bool active = lane < cnt;
    const uint32_t pr = pq[j0 + min(lane, cnt - 1)];
    const int slot = (int)(pr >> 3), blk = (int)(pr & 3u);
    const float4 *rg = (const float4 *)((const char *)rt + gid[slot]);
    const float4 r0 = rg[0], r1 = rg[1], r2 = rg[2];
    // r0 = (us, vs, Huu', Huv'), r1 = (Hvv', gu2, gv2, Guu),
    // r2 = (Guv2, Gvv carrying the sign of amp, log2|amp|, -)
    const int lbx = (blk & ((1 << BXL) - 1)) * 8;
    const int lby = (blk >> BXL) * 8 + (NROWS == 4 ? (int)((pr >> 2) & 1u) * 4 : 0);
    const float du0 = (float)(tx0 + lbx) - r0.x, dv0 = (float)(ty0 + lby) - r0.y;
    const float Cq = r1.w, CE = r0.z, Gvv = fabsf(r2.y);
    const float s1 = fmaf(2.0f, du0, 1.0f), t1 = fmaf(2.0f, dv0, 1.0f);
    // Per pixel, with a = g r 2^x r^2 (dL/dE up to the factor -amp/2), the
    // lane accumulates a and a x weighted by 1, c and c^2 (c = 0..7, the column inside the block,
    // a compile-time constant) over all its rows. The row moments come from prefix sums: with P_r
    // the sum through row r, sum_r r c_r = (R-1) P_{R-1} - sum_{r<R-1} P_r and
    // sum_r r^2 c_r = (R-1)^2 P_{R-1} - sum_{r<R-1} (2r+1) P_r, so a row costs three adds per
    // accumulated quantity; dv = dv0 + r and the column offset du0 are applied at the end. dL/dq
    // (up to the same factor) is b = a (1 + 2 ln2 x): its moments are those of a plus 2 ln2 times
    // those of a x (formed by the adjoint of the set-up, except the constant one). Each row starts from q and E at its first pixel, carried down the rows by
    // their differences (q and E are quadratic in du and dv).
    const float ddq = 2.0f * Cq, dde = 2.0f * CE;
    float er = fmaf(du0, fmaf(CE, du0, r0.w * dv0), r1.x * (dv0 * dv0));
    float ve = fmaf(r1.x, t1, r0.w * du0);
    const float vve = 2.0f * r1.x;
    float der = fmaf(CE, s1, r0.w * dv0);
    const float Rm = (float)(NROWS - 1);
    // (the sums start at -0, which adding the first term leaves exactly that term)
    float S[12];
    if constexpr (EWA) {
        // per pixel a = g 2^x (dL/dE up to the factor -amp/2); dL/damp = sum a
        float e0 = -0.f, e1 = -0.f, e2 = -0.f, Q0 = -0.f, Q1 = -0.f, W0 = -0.f;
        const float *gp = gpx + lby * GPX_STRIDE + lbx;
#pragma unroll
        for (int row = 0; row < NROWS; ++row) {
            if (row > 0) {   // (row 0 adds P_{-1} = 0)
                Q0 += e0;
                Q1 += e1;
                W0 = fmaf((float)(2 * row - 1), e0, W0);
            }
            float ee = er, de = der;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float a = gp[row * GPX_STRIDE + c] * __builtin_amdgcn_exp2f(ee);
                e0 += a;
                if (c > 0) {
                    e1 = fmaf((float)c, a, e1);
                    e2 = fmaf((float)(c * c), a, e2);
                }
                ee += de;
                de += dde;
            }
            er += ve;
            ve += vve;
            der += r0.w;
        }
        const float R0 = fmaf(Rm, e0, -Q0), R1 = fmaf(Rm, e1, -Q1), RR0 = fmaf(Rm * Rm, e0, -W0);
        const float EV0 = fmaf(dv0, e0, R0), EV1 = fmaf(dv0, e1, R1);
        const float EW0 = fmaf(dv0, fmaf(dv0, e0, 2.0f * R0), RR0);
        S[0] = e0;
        S[1] = fmaf(du0, fmaf(du0, e0, 2.0f * e1), e2);
        S[2] = fmaf(du0, EV0, EV1);
        S[3] = EW0;
        S[4] = S[5] = S[6] = S[7] = S[8] = S[9] = 0.0f;   // (not accumulated below)
        S[10] = fmaf(du0, e0, e1);
        S[11] = EV0;
    } else {
        const float Bq0 = fmaf(r2.x, dv0, r1.y);
        float qr = fmaf(du0, fmaf(Cq, du0, Bq0), fmaf(dv0, fmaf(Gvv, dv0, r1.z), 1.0f));
        float vq = fmaf(Gvv, t1, fmaf(r2.x, du0, r1.z));
        const float vvq = 2.0f * Gvv;
        float dqr = fmaf(Cq, s1, Bq0);
        float S0 = -0.f, e0 = -0.f, e1 = -0.f, e2 = -0.f, x0 = -0.f, x1 = -0.f, x2 = -0.f;
        float Qe0 = -0.f, Qe1 = -0.f, We0 = -0.f, Qx0 = -0.f, Qx1 = -0.f, Wx0 = -0.f;
        const float *gp = gpx + lby * GPX_STRIDE + lbx;
#pragma unroll
        for (int row = 0; row < NROWS; ++row) {
            if (row > 0) {   // (row 0 adds P_{-1} = 0)
                Qe0 += e0;
                Qe1 += e1;
                We0 = fmaf((float)(2 * row - 1), e0, We0);
                Qx0 += x0;
                Qx1 += x1;
                Wx0 = fmaf((float)(2 * row - 1), x0, Wx0);
            }
            // along the row: q(du) and E(du) by forward differences from the row's first pixel
            float q = qr, dq = dqr, ee = er, de = der;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float gval = gp[row * GPX_STRIDE + c];
                const float rs = __builtin_amdgcn_rsqf(q);
                const float r2s = rs * rs;
                const float x = ee * r2s;
                const float gr = (gval * rs) * __builtin_amdgcn_exp2f(x);
                const float a = gr * r2s;
                const float ax = a * x;
                S0 += gr;
                e0 += a;
                x0 += ax;
                if (c > 0) {
                    e1 = fmaf((float)c, a, e1);
                    e2 = fmaf((float)(c * c), a, e2);
                    x1 = fmaf((float)c, ax, x1);
                    x2 = fmaf((float)(c * c), ax, x2);
                }
                q += dq;
                dq += ddq;
                ee += de;
                de += dde;
            }
            qr += vq;
            vq += vvq;
            dqr += r2.x;
            er += ve;
            ve += vve;
            der += r0.w;
        }
        // row-index moments, then dv = dv0 + r
        const float Re0 = fmaf(Rm, e0, -Qe0), Re1 = fmaf(Rm, e1, -Qe1);
        const float RRe0 = fmaf(Rm * Rm, e0, -We0);
        const float Rx0 = fmaf(Rm, x0, -Qx0), Rx1 = fmaf(Rm, x1, -Qx1);
        const float RRx0 = fmaf(Rm * Rm, x0, -Wx0);
        const float EV0 = fmaf(dv0, e0, Re0), EV1 = fmaf(dv0, e1, Re1);
        const float EW0 = fmaf(dv0, fmaf(dv0, e0, 2.0f * Re0), RRe0);
        const float XV0 = fmaf(dv0, x0, Rx0), XV1 = fmaf(dv0, x1, Rx1);
        const float XW0 = fmaf(dv0, fmaf(dv0, x0, 2.0f * Rx0), RRx0);
        // the twelve partial sums (du = du0 + c)
        S[0] = S0;
        S[1] = fmaf(du0, fmaf(du0, e0, 2.0f * e1), e2);   // sum a du^2
        S[2] = fmaf(du0, EV0, EV1);                        // sum a du dv
        S[3] = EW0;                                        // sum a dv^2
        S[4] = fmaf(du0, fmaf(du0, x0, 2.0f * x1), x2);   // sum a x du^2
        S[5] = fmaf(du0, XV0, XV1);                        // sum a x du dv
        S[6] = XW0;                                        // sum a x dv^2
        S[7] = fmaf(du0, x0, x1);                          // sum a x du
        S[8] = XV0;                                        // sum a x dv
        S[9] = fmaf(2.0f * LN2, x0, e0);                   // sum a (1 + 2 ln2 x)
        S[10] = fmaf(du0, e0, e1);                         // sum a du
        S[11] = EV0;                                       // sum a dv
    }
    // add into the entry's slot, one block at a time (an entry has at most one pair per block)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (active && blk == b) {
            float *dst = accS[slot];
#pragma unroll
            for (int c = 0; c < 12; ++c)
                if (!EWA || c < 4 || c > 9) dst[c] += S[c];
        }
        wave_sync_lds();
    }
}

// Writes the partial of the entry in slot `slot` (Gaussian g of view t, this tile).
__device__ __forceinline__ void splat_bwd_write(int n, int t, int tx, int ty, uint32_t g,
                                                const float *acc, unsigned cap,
                                                const int4 *__restrict__ rect,
                                                const uint32_t *__restrict__ goff,
                                                float4 *__restrict__ part)
{
    // instance slot of (t, g, this tile): the Gaussian's instances are contiguous, in row-major
    // order over its tile rectangle
    const size_t o = (size_t)t * n + g;
    const TileRect tr = TileRect::from(rect[o]);
    const size_t slot = (size_t)goff[o] + (size_t)tr.inst_of((ty - tr.ty0) * tr.w + (tx - tr.tx0));
    if (slot < cap) {
        part[slot * 3 + 0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        part[slot * 3 + 1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
        part[slot * 3 + 2] = make_float4(acc[8], acc[9], acc[10], acc[11]);
    }
}

// With nsl > 1 the workgroup takes slice sl of the tile's list (every entry's partial is still
// complete: an entry is in one slice, and its blocks are summed in order as before).
template <bool EWA, int TW, int TH>
__device__ __forceinline__ void splat_bwd_tile(const DevGeom &G, int n, int t, int tile,
                                               const float4 *__restrict__ rec,
                                               const uint32_t *__restrict__ list,
                                               const uint32_t *__restrict__ cnt, int nblk,
                                               unsigned cap, const int4 *__restrict__ rect,
                                               const uint32_t *__restrict__ goff,
                                               const float *__restrict__ grad_proj,
                                               float4 *__restrict__ part, BwdShared &sh,
                                               int sl = 0, int nsl = 1)
{
    constexpr int GPX_STRIDE = TW + 2, NB = (TW / 8) * (TH / 8);
    float *gpx = sh.gpx;
    const int tx = tile % G.tiles_x, ty = tile / G.tiles_x;
    const int wave = uniform((int)(threadIdx.x / DIGS_WAVE)), lane = lane_id();
    if ((int)threadIdx.x < TW * TH) {   // one thread per pixel of the tile
        const int p = threadIdx.x;
        const int px = tx * TW + (p % TW), py = ty * TH + p / TW;
        float gv = 0.0f;
        if (px < G.nu && py < G.nv) {
            gv = grad_proj[((size_t)t * G.nv + py) * G.nu + px];
            if constexpr (!EWA) {   // times the pixel's ray length |e|
                const float xu = ((float)px - 0.5f * (float)(G.nu - 1)) * G.pitch_u + G.off_u;
                const float yv = ((float)py - 0.5f * (float)(G.nv - 1)) * G.pitch_v + G.off_v;
                gv *= sqrtf(G.sdd * G.sdd + xu * xu + yv * yv);
            }
        }
        gpx[(p / TW) * GPX_STRIDE + (p % TW)] = gv;
    }
    __syncthreads();
    const size_t cidx = ((size_t)t * G.ntiles + tile) * nblk;
    uint32_t begin = cnt[cidx], end = cnt[cidx + nblk];
    begin = min(begin, cap);
    end = min(max(end, begin), cap);
    slice_range(begin, end, sl, nsl, 4 * DIGS_WAVE);
    const float4 *rt = rec + (size_t)t * n * 4;
    const int tx0 = tx * TW, ty0 = ty * TH;
    uint32_t *pq0 = sh.pairs[wave][0];   // pairs over all 8 rows of the block
    uint32_t *pq1 = sh.pairs[wave][1];   // pairs over 4 rows (one half of the block)
    uint32_t *gid = sh.gid[wave];
    float(*accS)[13] = sh.accS[wave];
    int pend0 = 0, pend1 = 0;  // queued pairs carried over (all of the previous chunk), < 64 each
    int it = 0;
    bool prev_valid = false;   // the previous chunk's entry of this lane
    uint32_t prev_g = 0;
    for (uint32_t c0 = begin + wave * DIGS_WAVE; c0 < end; c0 += 4 * DIGS_WAVE, ++it) {
        const int ring = (it & 1) * DIGS_WAVE;
        const uint32_t k = c0 + lane;
        bool valid = k < end;
        const uint32_t ent = valid ? list[k] : 0u;
        const uint32_t g = ent & LIST_INDEX_MASK;
        valid = valid && g < (uint32_t)n;
        gid[ring + lane] = g << 6;   // the record's byte offset (g * 64 < 2^30)
#pragma unroll
        for (int c = 0; c < 12; ++c) accS[ring + lane][c] = 0.0f;
        int np0 = pend0, np1 = pend1;
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            const uint32_t h = valid ? (ent >> (LIST_BLOCK_SHIFT + 2 * blk)) & 3u : 0u;
            const bool whole = h == 3u, half = h == 1u || h == 2u;
            const unsigned long long mw = __ballot(whole), mh = __ballot(half);
            const uint32_t pe = ((uint32_t)(ring + lane) << 3) | (uint32_t)blk;
            // a masked store per queue (the empty asm keeps them from being merged into one)
            if (whole) pq0[np0 + lane_rank(mw)] = pe;
            asm volatile("" ::: "memory");
            if (half) pq1[np1 + lane_rank(mh)] = pe | ((h >> 1) << 2);
            np0 += __popcll(mw);
            np1 += __popcll(mh);
        }
        wave_sync_lds();
        // full groups; if pairs of the previous chunk are queued and no full group forms, they
        // are evaluated now in a partial group (with everything queued) to finish that chunk
        int done0 = np0 & ~(DIGS_WAVE - 1), done1 = np1 & ~(DIGS_WAVE - 1);
        if (done0 == 0 && pend0 > 0) done0 = np0;
        if (done1 == 0 && pend1 > 0) done1 = np1;
        for (int j = 0; j < done0; j += DIGS_WAVE)
            splat_bwd_group<EWA, 8, TW, NB>(rt, pq0, gid, accS, gpx, j,
                                            min(DIGS_WAVE, done0 - j), tx0, ty0);
        for (int j = 0; j < done1; j += DIGS_WAVE)
            splat_bwd_group<EWA, 4, TW, NB>(rt, pq1, gid, accS, gpx, j,
                                            min(DIGS_WAVE, done1 - j), tx0, ty0);
        if (it > 0 && prev_valid)
            splat_bwd_write(n, t, tx, ty, prev_g, accS[(ring ^ DIGS_WAVE) + lane], cap, rect, goff,
                            part);
        const int left0 = np0 - done0, left1 = np1 - done1;
        if ((done0 > 0 && left0 > 0) || (done1 > 0 && left1 > 0)) {
            const uint32_t keep0 = (lane < left0) ? pq0[done0 + lane] : 0u;
            const uint32_t keep1 = (lane < left1) ? pq1[done1 + lane] : 0u;
            wave_sync_lds();
            if (lane < left0) pq0[lane] = keep0;
            if (lane < left1) pq1[lane] = keep1;
        }
        wave_sync_lds();
        pend0 = left0;
        pend1 = left1;
        prev_valid = valid;
        prev_g = g;
    }
    // The waves' last pairs (fewer than 64 per queue each, all of their last chunk) are pooled in
    // wave order and evaluated by wave 0 in fewer, fuller groups; the pooled pairs name their
    // entry slots across the four waves (slot + 128 wave), and a single wave evaluates them all,
    // so no two groups that add into one slot run at once.
    if (lane == 0) {
        sh.pend[0][wave] = pend0;
        sh.pend[1][wave] = pend1;
    }
    const uint32_t wslot = (uint32_t)(wave * 2 * DIGS_WAVE) << 3;
    const uint32_t keep0 = lane < pend0 ? pq0[lane] + wslot : 0u;
    const uint32_t keep1 = lane < pend1 ? pq1[lane] + wslot : 0u;
    __syncthreads();
    int o0 = 0, o1 = 0, n0 = 0, n1 = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int c0 = sh.pend[0][w], c1 = sh.pend[1][w];
        if (w < wave) {
            o0 += c0;
            o1 += c1;
        }
        n0 += c0;
        n1 += c1;
    }
    uint32_t *pool0 = sh.pairs[0][0], *pool1 = sh.pairs[0][1];   // 4 x 63 < BWD_QUEUE entries
    if (lane < pend0) pool0[o0 + lane] = keep0;
    if (lane < pend1) pool1[o1 + lane] = keep1;
    __syncthreads();
    if (wave == 0) {
#pragma unroll 1
        for (int j = 0; j < n0; j += DIGS_WAVE)
            splat_bwd_group<EWA, 8, TW, NB>(rt, pool0, sh.gid[0], sh.accS[0], gpx, j,
                                            min(DIGS_WAVE, n0 - j), tx0, ty0);
#pragma unroll 1
        for (int j = 0; j < n1; j += DIGS_WAVE)
            splat_bwd_group<EWA, 4, TW, NB>(rt, pool1, sh.gid[0], sh.accS[0], gpx, j,
                                            min(DIGS_WAVE, n1 - j), tx0, ty0);
    }
    __syncthreads();
    if (it > 0 && prev_valid)
        splat_bwd_write(n, t, tx, ty, prev_g, accS[((it - 1) & 1) * DIGS_WAVE + lane], cap, rect,
                        goff, part);
    wave_sync_lds();
}

template <bool EWA, int TW, int TH>
__global__ __launch_bounds__(256) void k_splat_bwd(DevGeom G, int n, int T,
                                                   const float4 *__restrict__ rec,
                                                   const uint32_t *__restrict__ list,
                                                   const uint32_t *__restrict__ cnt, int nblk,
                                                   unsigned cap, const int4 *__restrict__ rect,
                                                   const uint32_t *__restrict__ goff,
                                                   const float *__restrict__ grad_proj,
                                                   float4 *__restrict__ part)
{
    __shared__ BwdShared sh;
    int t, tile;
    map_block(blockIdx.x, G.ntiles, T, t, tile);
    splat_bwd_tile<EWA, TW, TH>(G, n, t, tile, rec, list, cnt, nblk, cap, rect, goff, grad_proj,
                                part, sh, blockIdx.y, gridDim.y);
}

template <bool EWA, int TW, int TH>
__global__ __launch_bounds__(256) void k_splat_bwd_persist(
    DevGeom G, int n, int T, const float4 *__restrict__ rec, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ cnt, int nblk, unsigned cap, const int4 *__restrict__ rect,
    const uint32_t *__restrict__ goff, const float *__restrict__ grad_proj,
    float4 *__restrict__ part, uint32_t *__restrict__ queue)
{
    __shared__ BwdShared sh;
    __shared__ int s_item;
    const int home = blockIdx.x & 7;
    for (;;) {
        if (threadIdx.x == 0) s_item = next_item(queue, home, G.ntiles, T);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item < 0) break;
        int t, tile;
        map_block(item, G.ntiles, T, t, tile);
        splat_bwd_tile<EWA, TW, TH>(G, n, t, tile, rec, list, cnt, nblk, cap, rect, goff,
                                    grad_proj, part, sh);
    }
}

__global__ void k_queue_reset(uint32_t *q)
{
    if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

// ------------------------------------------------------------------------------------------
// a7: adjoint of the set-up and of the warp. k_tn_bwd runs one thread per Gaussian and a chunk
// of the call's views: for each view it sums the instance partials of (t, n), recomputes the
// set-up, back-propagates the record gradients to dL/dmu', dL/dK, dL/d(R diag(s)) and dL/drho, and
// folds them into per-Gaussian sums over the chunk's views (in view order) together with the
// w-weighted sums that the B-spline term needs; it also forms the per-(t, n) terms of dL/dw[t][r]
// and reduces them per wave in a fixed order. k_gauss_reduce then adds the chunks (fixed order),
// adds the term through K(mu) (second derivatives of the B-spline), and finishes the chain to the
// canonical parameters.
#define TN_FIELDS 22   // per view: gmu' (3), gK (9), gRS (9), grho (1)
// per Gaussian and chunk: sum gmu' (3), sum gRS (9), sum grho (1), then per rank r
// P_r = sum_t w[t][r] gmu' (3) and Q_r = sum_t w[t][r] gK (9)
#define TACC_FIELDS(R) (13 + 12 * (R))

// Ranks 1-3 keep the w-weighted sums P_r, Q_r in LDS (one column per thread, 12R x 1 KB per
// workgroup) instead of registers: the kernel then fits 168 VGPRs, three waves per SIMD instead of
// two (its loads of the instance partials are latency-bound). Higher ranks keep them in registers
// (more LDS would cost more occupancy than it frees).
template <int NR>
__global__ __launch_bounds__(256, NR <= 3 ? 3 : 1) void k_tn_bwd(
    DevGeom G, int n, int T, int tpc, const float *__restrict__ gs,
    const float *__restrict__ angles, const float *__restrict__ w, const float *__restrict__ uv,
    const int4 *__restrict__ rect,
    const uint32_t *__restrict__ goff,
    const float4 *__restrict__ part, unsigned cap,
    float *__restrict__ tacc, float *__restrict__ gwpart, int nparts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y, nch = gridDim.y;
    const int t0 = chunk * tpc, t1 = min(T, t0 + tpc);
    const bool valid = i < n;
    const int ii = valid ? i : 0;
    const int lane = lane_id(), wave = threadIdx.x / DIGS_WAVE;
    // the Gaussian's canonical parameters and B-spline fields, once for all views
    float mu0[3], s[3], inv_s[3], q[4], Rm[9];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mu0[a] = gs[(size_t)a * n + ii];
        s[a] = gs[(size_t)(3 + a) * n + ii];
        inv_s[a] = 1.0f / s[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) q[a] = gs[(size_t)(6 + a) * n + ii];
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    quat_to_rot(q[0] * qn, q[1] * qn, q[2] * qn, q[3] * qn, Rm);
    const float rh = gs[(size_t)10 * n + ii];
    float U[NR][3], V[NR][9];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int a = 0; a < 3; ++a) U[r][a] = uv[((size_t)r * 3 + a) * n + ii];
#pragma unroll
        for (int k = 0; k < 9; ++k) V[r][k] = uv[((size_t)3 * NR + r * 9 + k) * n + ii];
    }
    constexpr bool kLdsPQ = NR <= 3;
    constexpr int kPQ = kLdsPQ ? 12 * NR : 1;
    __shared__ float pq_lds[kPQ][256];
    float pq_reg[kLdsPQ ? 1 : 12 * NR];
    // P_r[a] at index 3r + a, Q_r[k] at 3NR + 9r + k
    auto pq = [&](int idx) -> float & {
        if constexpr (kLdsPQ) return pq_lds[idx][threadIdx.x];
        else return pq_reg[idx];
    };
    float gsum[3] = {0.f, 0.f, 0.f}, gRS[9], grho = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) gRS[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 12 * NR; ++k) pq(k) = 0.0f;
    for (int t = t0; t < t1; ++t) {
        const size_t o = (size_t)t * n + ii;
        const int cntk = valid ? TileRect::from(rect[o]).count() : 0;
        float gwc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) gwc[r] = 0.0f;
        if (cntk > 0) {
            float S[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) S[c] = 0.0f;
            const size_t base = goff[o];
            // the instances of (t, n) are contiguous; four are loaded at once (more loads in
            // flight) and added in instance order
            const int kend = (int)min((size_t)cntk, cap > base ? cap - base : (size_t)0);
            int k = 0;
            for (; k + 4 <= kend; k += 4) {
                float4 v[12];
#pragma unroll
                for (int j = 0; j < 12; ++j) v[j] = part[(base + k) * 3 + j];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 a = v[3 * j], b = v[3 * j + 1], c = v[3 * j + 2];
                    S[0] += a.x; S[1] += a.y; S[2] += a.z; S[3] += a.w;
                    S[4] += b.x; S[5] += b.y; S[6] += b.z; S[7] += b.w;
                    S[8] += c.x; S[9] += c.y; S[10] += c.z; S[11] += c.w;
                }
            }
            for (; k < kend; ++k) {
                const size_t p = base + k;
                const float4 a = part[p * 3 + 0], b = part[p * 3 + 1], c = part[p * 3 + 2];
                S[0] += a.x; S[1] += a.y; S[2] += a.z; S[3] += a.w;
                S[4] += b.x; S[5] += b.y; S[6] += b.z; S[7] += b.w;
                S[8] += c.x; S[9] += c.y; S[10] += c.z; S[11] += c.w;
            }
            float wt[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) wt[r] = w[(size_t)t * NR + r];
            ViewTrig vt;
            sincosf(angles[t], &vt.st, &vt.ct);
            SetupFwd f;
            setup_forward<NR>(G, mu0, inv_s, Rm, U, V, wt, rh, vt, f);
            float out[TN_FIELDS];
            // the moment sums of dL/dE and dL/dq: the partials' sums of a, a x times -amp/2 (the
            // record's amplitude), dL/dq's from a (1 + 2 ln2 x)
            {
                const float cA = -0.5f * (f.amp * f.ee), k2 = 2.0f * LN2;
                const float quu = fmaf(k2, S[4], S[1]), quv = fmaf(k2, S[5], S[2]);
                const float qvv = fmaf(k2, S[6], S[3]), qu = fmaf(k2, S[7], S[10]);
                const float qv = fmaf(k2, S[8], S[11]);
                S[4] = cA * quu;
                S[5] = cA * quv;
                S[6] = cA * qvv;
                S[7] = cA * qu;
                S[8] = cA * qv;
                S[9] *= cA;
                S[1] *= cA;
                S[2] *= cA;
                S[3] *= cA;
                S[10] *= cA;
                S[11] *= cA;
                if (G.ewa) S[4] = S[5] = S[6] = S[7] = S[8] = S[9] = 0.0f;
            }
            // record gradients from the moment sums
            const float gHuu = S[1], gHuv = 2.0f * S[2], gHvv = S[3];
            // (EWA: g and G are the constant zero, and the record's amplitude is amp |e*|)
            const float gGuu = G.ewa ? 0.0f : S[4], gGuv = G.ewa ? 0.0f : 2.0f * S[5];
            const float gGvv = G.ewa ? 0.0f : S[6];
            const float ggu = G.ewa ? 0.0f : 2.0f * S[7], ggv = G.ewa ? 0.0f : 2.0f * S[8];
            const float gamp = S[0] * f.ee, gee = S[0] * f.amp;
            const float gus = -2.0f * (f.Huu * S[10] + f.Huv * S[11] + f.gu * S[9] + f.Guu * S[7] +
                                       f.Guv * S[8]);
            const float gvs = -2.0f * (f.Huv * S[10] + f.Hvv * S[11] + f.gv * S[9] + f.Guv * S[7] +
                                       f.Gvv * S[8]);
            // reverse of the record formulas
            const float sic = sqrtf(f.ic);
            const float grho_t = gamp * SQRT_2PI * f.beta * sic;
            float gbeta = gamp * rh * SQRT_2PI * sic;
            float gc = -0.5f * gamp * f.amp * f.ic;
            const float Duu = dot3(f.Du, f.Du), Duv = dot3(f.Du, f.Dv), Dvv = dot3(f.Dv, f.Dv);
            float gkap = (gGuu * Duu + gGuv * Duv + gGvv * Dvv) * f.ic;
            gc -= (gGuu * f.Guu + gGuv * f.Guv + gGvv * f.Gvv) * f.ic;
            float gDu[3], gDv[3], gmw[3], gDup[3], gDvp[3];
            const float kic = f.kap * f.ic;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gDu[a] = kic * (2.0f * gGuu * f.Du[a] + gGuv * f.Dv[a]);
                gDv[a] = kic * (2.0f * gGvv * f.Dv[a] + gGuv * f.Du[a]);
            }
            gbeta -= ggu * f.pa + ggv * f.pb;
            float gpa = -ggu * f.beta, gpb = -ggv * f.beta;
            gkap += gHuu * dot3(f.Dup, f.Dup) + gHuv * dot3(f.Dup, f.Dvp) +
                    gHvv * dot3(f.Dvp, f.Dvp);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gDup[a] = f.kap * (2.0f * gHuu * f.Dup[a] + gHuv * f.Dvp[a]);
                gDvp[a] = f.kap * (2.0f * gHvv * f.Dvp[a] + gHuv * f.Dup[a]);
            }
            gbeta += 2.0f * f.beta * gkap;
            gpa -= dot3(gDup, f.mw);
            gpb -= dot3(gDvp, f.mw);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gDu[a] += gDup[a];
                gDv[a] += gDvp[a];
                gmw[a] = -f.pa * gDup[a] - f.pb * gDvp[a];
            }
            const float gdu = gpa * f.ic, gdv = gpb * f.ic;
            gc -= (gpa * f.pa + gpb * f.pb) * f.ic;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gmw[a] += gdu * f.Du[a] + gdv * f.Dv[a] + 2.0f * gc * f.mw[a];
                gDu[a] += gdu * f.mw[a];
                gDv[a] += gdv * f.mw[a];
            }
            float galpha = gbeta / G.sdd;
            const float ia = 1.0f / f.alpha;
            const float kuf = G.sdd * ia / G.pitch_u, kvf = G.sdd * ia / G.pitch_v;
            float gxu = -gus * kuf, gxv = -gvs * kvf;
            galpha += gus * kuf * f.xu * ia + gvs * kvf * f.xv * ia;
            if (G.ewa) {   // |e*| = SDD sqrt(1 + (xu^2 + xv^2) / alpha^2)
                const float k = gee * G.sdd * G.sdd * ia * ia / f.ee;
                gxu += k * f.xu;
                gxv += k * f.xv;
                galpha -= k * (f.xu * f.xu + f.xv * f.xv) * ia;
            }
            // mw = W m, Du = pu W e_u, Dv = pv W e_v
            const float eu[3] = {-vt.st, vt.ct, 0.0f};
            float gW[9], gm[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    gW[3 * a + b] = gmw[a] * f.m[b] + G.pitch_u * gDu[a] * eu[b] +
                                    (b == 2 ? G.pitch_v * gDv[a] : 0.0f);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                gm[b] = f.W[b] * gmw[0] + f.W[3 + b] * gmw[1] + f.W[6 + b] * gmw[2];
            float gmup[3] = {-gm[0], -gm[1], -gm[2]};
            gmup[0] += -vt.ct * galpha + vt.st * gxu;
            gmup[1] += -vt.st * galpha - vt.ct * gxu;
            gmup[2] += -gxv;
            // W = M^-1: dL/dM = -W^T gW W^T
            float T1[9], gM[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    T1[3 * a + b] =
                        f.W[a] * gW[b] + f.W[3 + a] * gW[3 + b] + f.W[6 + a] * gW[6 + b];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    gM[3 * a + b] = -(T1[3 * a] * f.W[3 * b] + T1[3 * a + 1] * f.W[3 * b + 1] +
                                      T1[3 * a + 2] * f.W[3 * b + 2]);
            // M = K (R S): dL/dK = gM (RS)^T, dL/d(RS) = K^T gM
            float RS[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) RS[3 * a + b] = Rm[3 * a + b] * s[b];
#pragma unroll
            for (int a = 0; a < 3; ++a) out[a] = gmup[a];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    out[3 + 3 * a + b] = gM[3 * a] * RS[3 * b] + gM[3 * a + 1] * RS[3 * b + 1] +
                                         gM[3 * a + 2] * RS[3 * b + 2];
                    out[12 + 3 * a + b] = f.K[a] * gM[b] + f.K[3 + a] * gM[3 + b] +
                                          f.K[6 + a] * gM[6 + b];
                }
            out[21] = grho_t;
            // per-(t, n) term of dL/dw[t][r] = u_r . dL/dmu' + grad u_r : dL/dK
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                float c = 0.0f;
#pragma unroll
                for (int a = 0; a < 3; ++a) c = fmaf(U[r][a], out[a], c);
#pragma unroll
                for (int k = 0; k < 9; ++k) c = fmaf(V[r][k], out[3 + k], c);
                gwc[r] = c;
            }
            // per-Gaussian sums over the chunk's views, in view order
#pragma unroll
            for (int a = 0; a < 3; ++a) gsum[a] += out[a];
#pragma unroll
            for (int k = 0; k < 9; ++k) gRS[k] += out[12 + k];
            grho += out[21];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int a = 0; a < 3; ++a) pq(3 * r + a) = fmaf(wt[r], out[a], pq(3 * r + a));
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    pq(3 * NR + 9 * r + k) = fmaf(wt[r], out[3 + k], pq(3 * NR + 9 * r + k));
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const float sm = wave_sum(gwc[r]);
            if (lane == 0) gwpart[((size_t)t * NR + r) * nparts + blockIdx.x * 4 + wave] = sm;
        }
    }
    if (valid) {
        float *dst = tacc + (size_t)chunk * n + i;
        const size_t fs = (size_t)nch * n;
#pragma unroll
        for (int a = 0; a < 3; ++a) dst[a * fs] = gsum[a];
#pragma unroll
        for (int k = 0; k < 9; ++k) dst[(3 + k) * fs] = gRS[k];
        dst[12 * fs] = grho;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int a = 0; a < 3; ++a) dst[(13 + 12 * r + a) * fs] = pq(3 * r + a);
#pragma unroll
            for (int k = 0; k < 9; ++k) dst[(16 + 12 * r + k) * fs] = pq(3 * NR + 9 * r + k);
        }
    }
}

template <int NR>
__global__ __launch_bounds__(256) void k_gauss_reduce(
    DevGrid grid, int n, int nch, const float *__restrict__ coef, const float *__restrict__ gpar,
    const float *__restrict__ uv, const float *__restrict__ tacc,
    const uint32_t *__restrict__ order, float *__restrict__ g_mu, float *__restrict__ g_scale,
    float *__restrict__ g_quat, float *__restrict__ g_rho, float *__restrict__ gq, int gq_stride,
    float *__restrict__ g_basis)
{
    // four lanes per Gaussian: lane `part` takes the stencil's z index part in the second-
    // derivative term (partial sums added in a fixed order); lane 0 writes the results. (The
    // lattice is read through the caches here: staging the workgroup's control points in LDS, as
    // the canonical FFD does, made this kernel slower.)
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gt >> 2, part = gt & 3;
    if (i >= n) return;
    float gsum[3] = {0.f, 0.f, 0.f}, gRS[9], P[NR][3], Q[NR][9], grho = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) gRS[k] = 0.0f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int a = 0; a < 3; ++a) P[r][a] = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) Q[r][k] = 0.0f;
    }
    // the chunks of views, in order
    const size_t fs = (size_t)nch * n;
    for (int c = 0; c < nch; ++c) {
        const float *src = tacc + (size_t)c * n + i;
#pragma unroll
        for (int a = 0; a < 3; ++a) gsum[a] += src[a * fs];
#pragma unroll
        for (int k = 0; k < 9; ++k) gRS[k] += src[(3 + k) * fs];
        grho += src[12 * fs];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int a = 0; a < 3; ++a) P[r][a] += src[(13 + 12 * r + a) * fs];
#pragma unroll
            for (int k = 0; k < 9; ++k) Q[r][k] += src[(16 + 12 * r + k) * fs];
        }
    }
    // dL/dmu = sum_t dL/dmu' + sum_r V_r^T P_r + sum_r Q_r : d(grad u_r)/dmu (with a per-Gaussian
    // basis, u and V do not depend on mu: the first term only)
    float gmu[3] = {gsum[0], gsum[1], gsum[2]};
    const size_t src = order[i];   // i is the position in cell order
    Stencil st;
    if (!g_basis) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float *V = uv + ((size_t)3 * NR + r * 9) * n + i;
                gmu[c] += V[c * (size_t)n] * P[r][0] + V[(3 + c) * (size_t)n] * P[r][1] +
                          V[(6 + c) * (size_t)n] * P[r][2];
            }
        const float mu0[3] = {gpar[i], gpar[(size_t)n + i], gpar[(size_t)2 * n + i]};
        make_stencil(grid, mu0[0], mu0[1], mu0[2], st, true);
        const LatticeRows lr{coef, grid.nx, grid.ny, grid.nz};
        float hs[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < NR; ++r) ffd_rank_hessian_contract(lr, r, st, Q[r], hs, part, part + 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            hs[a] += __shfl_xor(hs[a], 1, DIGS_WAVE);
            hs[a] += __shfl_xor(hs[a], 2, DIGS_WAVE);
            gmu[a] += hs[a];
        }
    }
    // R diag(s) -> s, R(q)
    const float s[3] = {gpar[(size_t)3 * n + i], gpar[(size_t)4 * n + i], gpar[(size_t)5 * n + i]};
    float q[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) q[a] = gpar[(size_t)(6 + a) * n + i];
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    // a Gaussian whose inputs the set-up rejects (non-finite mean, quaternion or density, a scale
    // that is not positive) was skipped in every view: all its gradients are zero, and it adds
    // nothing to dL/dcoef (its B-spline weights may be NaN, and NaN * 0 is NaN)
    const float mu0[3] = {gpar[i], gpar[(size_t)n + i], gpar[(size_t)2 * n + i]};
    const bool inputs_ok = isfinite(mu0[0]) && isfinite(mu0[1]) && isfinite(mu0[2]) &&
                           s[0] > 0.0f && s[1] > 0.0f && s[2] > 0.0f &&
                           isfinite(1.0f / s[0] * (1.0f / s[1]) * (1.0f / s[2])) && isfinite(qn) &&
                           isfinite(gpar[(size_t)10 * n + i]);
    if (!inputs_ok) {
#pragma unroll
        for (int a = 0; a < 3; ++a) gmu[a] = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) gRS[k] = 0.0f;
        grho = 0.0f;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int a = 0; a < 3; ++a) P[r][a] = 0.0f;
#pragma unroll
            for (int k = 0; k < 9; ++k) Q[r][k] = 0.0f;
        }
    }
    const float qh[4] = {q[0] * qn, q[1] * qn, q[2] * qn, q[3] * qn};
    float Rm[9];
    quat_to_rot(qh[0], qh[1], qh[2], qh[3], Rm);
    float gR[9], gs[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        gs[b] = gRS[b] * Rm[b] + gRS[3 + b] * Rm[3 + b] + gRS[6 + b] * Rm[6 + b];
#pragma unroll
        for (int a = 0; a < 3; ++a) gR[3 * a + b] = gRS[3 * a + b] * s[b];
    }
    float gqh[4];
    quat_rot_adjoint(qh[0], qh[1], qh[2], qh[3], gR, gqh);
    const float dq = gqh[0] * qh[0] + gqh[1] * qh[1] + gqh[2] * qh[2] + gqh[3] * qh[3];
    if (part != 0) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g_mu[(size_t)a * n + src] = gmu[a];
        g_scale[(size_t)a * n + src] = gs[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
        g_quat[(size_t)a * n + src] = inputs_ok ? (gqh[a] - dq * qh[a]) * qn : 0.0f;
    if (!inputs_ok) {
#pragma unroll
        for (int a = 0; a < 3; ++a) g_scale[(size_t)a * n + src] = 0.0f;
    }
    g_rho[src] = grho;
    if (g_basis) {   // dL/du_r = P_r, dL/dV_r = Q_r, at the Gaussian's own index
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            float *b = g_basis + (size_t)r * 12 * n + src;
#pragma unroll
            for (int a = 0; a < 3; ++a) b[(size_t)a * n] = P[r][a];
#pragma unroll
            for (int k = 0; k < 9; ++k) b[(size_t)(3 + k) * n] = Q[r][k];
        }
        return;
    }
    // sources of dL/dcoef in cell order: clamped cell, fraction, P_r, Q_r
    float *o = gq + (size_t)i * gq_stride;
    o[0] = __int_as_float(max(-2, min(st.fx, grid.nx + 1)));
    o[1] = __int_as_float(max(-2, min(st.fy, grid.ny + 1)));
    o[2] = __int_as_float(max(-2, min(st.fz, grid.nz + 1)));
    o[3] = inputs_ok ? st.px : 0.0f;
    o[4] = inputs_ok ? st.py : 0.0f;
    o[5] = inputs_ok ? st.pz : 0.0f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int a = 0; a < 3; ++a) o[6 + 12 * r + a] = P[r][a];
#pragma unroll
        for (int k = 0; k < 9; ++k) o[6 + 12 * r + 3 + k] = Q[r][k];
    }
}

// One workgroup per (t, r): strided per-thread sums over the per-wave parts, then a fixed tree.
__global__ __launch_bounds__(256) void k_gw_final(const float *__restrict__ gwpart, int nparts,
                                                  float *__restrict__ g_w)
{
    __shared__ float red[256];
    const float *p = gwpart + (size_t)blockIdx.x * nparts;
    float v = 0.0f;
    for (int k = threadIdx.x; k < nparts; k += 256) v += p[k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) g_w[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------------------------
// a8: cell sort and the control-point gather of dL/dcoef
__global__ void k_cell_keys(DevGrid g, int n, const float *__restrict__ mu,
                            uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float q[3] = {(mu[i] - g.ox) / g.hx, (mu[n + i] - g.oy) / g.hy,
                        (mu[2 * n + i] - g.oz) / g.hz};
    const int dims[3] = {g.nx, g.ny, g.nz};
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = floorf(q[a]);
        f = fminf(fmaxf(f, -2.0f), (float)(dims[a] + 1));   // NaN-safe clamp
        c[a] = (f == f) ? (int)f + 2 : 0;
    }
    keys[i] = ((uint32_t)c[2] * (g.ny + 4) + c[1]) * (g.nx + 4) + c[0];
    vals[i] = (uint32_t)i;
}

// cell_start[k] = number of Gaussians whose cell key is below k (for every key 0..ncells), by a
// binary search of the sorted keys per cell; order[p] = the Gaussian at position p in cell order
__global__ void k_cell_start(int n, int ncells, const uint32_t *__restrict__ keys,
                             const uint32_t *__restrict__ vals, uint32_t *__restrict__ cell_start,
                             uint32_t *__restrict__ order)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p <= ncells) {
        int lo = 0, hi = n;   // first position whose key is >= p
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (keys[mid] < (uint32_t)p) lo = mid + 1;
            else hi = mid;
        }
        cell_start[p] = (uint32_t)lo;
    }
    if (p < n) order[p] = min(vals[p], (uint32_t)(n - 1));
}

// One wave per control point: for each (cz, cy) row of its candidate cells the Gaussians of
// the cells cx = lx..hx are contiguous in cell order; the lanes take the rows' Gaussians 64 at a
// time over all rows together, and the per-lane sums are reduced over the wave in a fixed order.
template <int NR>
__global__ __launch_bounds__(256) void k_coef_grad(DevGrid g, const float *__restrict__ gq,
                                                   int gq_stride,
                                                   const uint32_t *__restrict__ cell_start,
                                                   float *__restrict__ g_coef)
{
    const int idx = blockIdx.x * 4 + threadIdx.x / DIGS_WAVE;
    const int lane = lane_id();
    const int npts = g.nx * g.ny * g.nz;
    if (idx >= npts) return;
    const int i = idx % g.nx, j = (idx / g.nx) % g.ny, k = idx / (g.nx * g.ny);
    float acc[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0f;
    const int lx = (i == 0) ? -2 : i - 2, hx = (i == g.nx - 1) ? g.nx + 1 : i + 1;
    const int ly = (j == 0) ? -2 : j - 2, hy = (j == g.ny - 1) ? g.ny + 1 : j + 1;
    const int lz = (k == 0) ? -2 : k - 2, hz = (k == g.nz - 1) ? g.nz + 1 : k + 1;
    const float ihx = 1.0f / g.hx, ihy = 1.0f / g.hy, ihz = 1.0f / g.hz;
    // The support's cell rows (cz, cy), at most 5 x 5, each a contiguous range of Gaussians in
    // cell order: lane r < nrows holds row r's range, and the rows' Gaussians are taken 64 at a
    // time over all rows together (a row holds only a few Gaussians).
    const int nry = hy - ly + 1, nrows = (hz - lz + 1) * nry;
    uint32_t rb = 0, rlen = 0;
    if (lane < nrows) {
        const int cz = lz + lane / nry, cy = ly + lane % nry;
        const uint32_t row = ((uint32_t)(cz + 2) * (g.ny + 4) + (cy + 2)) * (g.nx + 4);
        rb = cell_start[row + (lx + 2)];
        rlen = cell_start[row + (hx + 2) + 1] - rb;
    }
    // inclusive prefix sum of the row lengths over lanes 0..31 (nrows <= 25)
    uint32_t incl = rlen;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, DIGS_WAVE);
        if (lane >= off) incl += y;
    }
    const uint32_t total = __shfl(incl, 31, DIGS_WAVE);
    for (uint32_t q0 = 0; q0 < total; q0 += DIGS_WAVE) {
        // the row of flattened index q: the first lane whose inclusive sum exceeds q (the
        // shuffles run with every lane active; lanes past the end then skip the work)
        const uint32_t q = q0 + (uint32_t)lane;
        int row = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1)
            if (__shfl(incl, row + step - 1, DIGS_WAVE) <= q) row += step;
        row = min(row, 31);
        const uint32_t p = __shfl(rb, row, DIGS_WAVE) + q -
                           (__shfl(incl, row, DIGS_WAVE) - __shfl(rlen, row, DIGS_WAVE));
        if (q >= total) continue;
        const float *o = gq + (size_t)p * gq_stride;
        // the Gaussian's (clamped) cell
        const int cx = __float_as_int(o[0]), cy = __float_as_int(o[1]), cz = __float_as_int(o[2]);
        float B[4], dB[4];
        float wx = 0.f, dwx = 0.f, wy = 0.f, dwy = 0.f, wz = 0.f, dwz = 0.f;
        bspline4(o[3], B);
        bspline4_d(o[3], dB);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (clampi(cx - 1 + l, g.nx) == i) { wx += B[l]; dwx += dB[l]; }
        bspline4(o[4], B);
        bspline4_d(o[4], dB);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (clampi(cy - 1 + l, g.ny) == j) { wy += B[l]; dwy += dB[l]; }
        bspline4(o[5], B);
        bspline4_d(o[5], dB);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (clampi(cz - 1 + l, g.nz) == k) { wz += B[l]; dwz += dB[l]; }
        const float w0 = wx * wy * wz, w1 = dwx * ihx * wy * wz, w2 = wx * dwy * ihy * wz,
                    w3 = wx * wy * dwz * ihz;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const float *Pr = o + 6 + 12 * r, *Qr = Pr + 3;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                acc[r][a] += w0 * Pr[a] + w1 * Qr[3 * a] + w2 * Qr[3 * a + 1] + w3 * Qr[3 * a + 2];
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = wave_sum(acc[r][a]);
            if (lane == 0) g_coef[((size_t)r * npts + idx) * 3 + a] = v;
        }
}

// ------------------------------------------------------------------------------------------
// host orchestration
template <int NR>
static hipError_t setup_dispatch(const RenderArgs &a, hipStream_t s)
{
    const int n = a.n, T = a.T;
    dim3 grid((n + 255) / 256, (T + SETUP_TCHUNK - 1) / SETUP_TCHUNK);
    hipLaunchKernelGGL(k_setup<NR>, grid, dim3(256), 0, s, a.geom, n, T,
                       WS(a, gsort, const float *), a.angles, a.w, WS(a, uv, const float *), a.cull,
                       WS(a, rec, float4 *), WS(a, rect, int4 *), WS(a, gcount, uint32_t *),
                       WS(a, diag, DiagBlock *));
    return hipGetLastError();
}

// Cell sort of the Gaussians by the lattice cell of their canonical mean (LSD radix, 8 bits per
// pass): every per-Gaussian array of a call is laid out in this order, so that the records and
// partials of Gaussians that are near each other in space (and hence on the detector) are near
// each other in memory.
static hipError_t cell_sort(const RenderArgs &a, hipStream_t s)
{
    ProfScope ps(PS_CELL_SORT, s);
    hipError_t e;
    const int n = a.n;
    uint32_t *ka = WS(a, keys_a, uint32_t *), *va = WS(a, vals_a, uint32_t *);
    uint32_t *kb = WS(a, keys_b, uint32_t *), *vb = WS(a, vals_b, uint32_t *);
    hipLaunchKernelGGL(k_cell_keys, dim3((n + 255) / 256), dim3(256), 0, s, a.grid, n, a.mu, ka,
                       va);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nblk_r = (n + DIGS_BIN_ITEMS - 1) / DIGS_BIN_ITEMS;
    const int kbits = bits_for(a.L.ncells);
    for (int shift = 0; shift < kbits; shift += 8) {
        RadixSrc src;
        src.keys_in = ka;
        src.vals_in = va;
        src.keys_out = kb;
        src.vals_out = vb;
        src.items = n;
        src.shift = shift;
        e = launch_binning(src, 1, 256, nblk_r, 8, WS(a, rhist, uint32_t *),
                           (size_t)256 * nblk_r, WS(a, scratch, uint32_t *), s, DIGS_BIN_ITEMS,
                           false);
        if (e != hipSuccess) return e;
        uint32_t *t0 = ka; ka = kb; kb = t0;
        t0 = va; va = vb; vb = t0;
    }
    const int cs_threads = std::max(n, a.L.ncells + 1);
    hipLaunchKernelGGL(k_cell_start, dim3((cs_threads + 255) / 256), dim3(256), 0, s, n,
                       a.L.ncells,
                       ka, va, WS(a, cell_start, uint32_t *), WS(a, order, uint32_t *));
    return hipGetLastError();
}

// The per-Gaussian stage (cell order, the Gaussians gathered into it, the FFD at the canonical
// means): a function of the Gaussians and the lattice alone, shared by every view of a call.
hipError_t render_forward_canonical(const RenderArgs &a, hipStream_t s)
{
    hipError_t e;
    if ((e = cell_sort(a, s)) != hipSuccess) return e;
    {
        ProfScope ps(PS_FFD, s);
        auto kernel = a.n >= FFD_STAGE_MIN_GAUSSIANS ? k_ffd_canonical<true>
                                                     : k_ffd_canonical<false>;
        hipLaunchKernelGGL(kernel, dim3((unsigned)(((size_t)4 * a.n + 255) / 256)),
                           dim3(256), 0, s, a.grid,
                           a.coef, a.basis, a.n, a.mu, a.scale, a.quat, a.rho,
                           WS(a, order, const uint32_t *), WS(a, uv, float *), WS(a, gsort, float *));
    }
    return hipGetLastError();
}

hipError_t render_forward_setup(const RenderArgs &a, hipStream_t s)
{
    hipError_t e = render_forward_canonical(a, s);
    if (e != hipSuccess) return e;
    return render_forward_views(a, s);
}

// The tile lists of the call's (view, Gaussian) instances, binned for a TW x TH tile shape.
template <int TW, int TH>
static hipError_t bin_tiles(const RenderArgs &a, uint32_t *cnt, size_t cnt_elems,
                            uint32_t *scratch, hipStream_t s)
{
    TileSrc<TW, TH> src;
    src.rect = WS(a, rect, const int4 *);
    src.rec = WS(a, rec, const float4 *);
    src.list = WS(a, list, uint32_t *);
    src.cap = a.L.cap;
    src.items = a.n;
    src.tiles_x = a.geom.tiles_x;
    src.inv_tiles_x = 1.0f / (float)a.geom.tiles_x;
    return launch_binning(src, a.T, a.geom.ntiles, a.L.nblk, bits_for(a.geom.ntiles), cnt,
                          cnt_elems + 1, scratch, s, a.L.bin_items);
}

// The per-view stages: the warp and projected records, instance offsets and the tile lists.
hipError_t render_forward_views(const RenderArgs &a, hipStream_t s)
{
    hipError_t e;
    const size_t cnt_elems = (size_t)a.T * a.geom.ntiles * a.L.nblk;
    uint32_t *cnt = WS(a, cnt, uint32_t *);
    hipLaunchKernelGGL(k_diag_begin, dim3(1), dim3(1), 0, s, WS(a, diag, DiagBlock *),
                       (unsigned long long)a.L.cap, cnt + cnt_elems);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        ProfScope ps(PS_SETUP, s);
        switch (a.grid.R) {
        case 1: e = setup_dispatch<1>(a, s); break;
        case 2: e = setup_dispatch<2>(a, s); break;
        case 3: e = setup_dispatch<3>(a, s); break;
        case 4: e = setup_dispatch<4>(a, s); break;
        case 5: e = setup_dispatch<5>(a, s); break;
        case 6: e = setup_dispatch<6>(a, s); break;
        case 7: e = setup_dispatch<7>(a, s); break;
        default: e = setup_dispatch<8>(a, s); break;
        }
    }
    if (e != hipSuccess) return e;
    uint32_t *scratch = WS(a, scratch, uint32_t *);
    // the tile lists (the per-(t,n) instance offsets, which only the backward needs, are its
    // first step)
    const int tw = a.geom.tile_w, th = a.geom.tile_h;
    if (tw == 16 && th == 16) e = bin_tiles<16, 16>(a, cnt, cnt_elems, scratch, s);
    else if (tw == 32) e = bin_tiles<32, 8>(a, cnt, cnt_elems, scratch, s);
    else if (tw == 16) e = bin_tiles<16, 8>(a, cnt, cnt_elems, scratch, s);
    else if (th == 32) e = bin_tiles<8, 32>(a, cnt, cnt_elems, scratch, s);
    else if (th == 16) e = bin_tiles<8, 16>(a, cnt, cnt_elems, scratch, s);
    else e = bin_tiles<8, 8>(a, cnt, cnt_elems, scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_check, dim3(1), dim3(1), 0, s, WS(a, diag, DiagBlock *));
    return hipGetLastError();
}

// Workgroups of a persistent launch: enough to fill every CU at the kernel's occupancy, never more
// than there are work items.
// The device queries run once per kernel (the first launch happens before any graph capture).
template <class K>
static unsigned persistent_grid(K kernel, int threads, size_t items)
{
    static int cus = 0;
    static const void *known[32];
    static int known_per_cu[32];
    static int nknown = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    int per_cu = 0;
    for (int i = 0; i < nknown; ++i)
        if (known[i] == (const void *)kernel) per_cu = known_per_cu[i];
    if (per_cu == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 1;
        if (nknown < 32) {
            known[nknown] = (const void *)kernel;
            known_per_cu[nknown++] = per_cu;
        }
    }
    const size_t g = (size_t)cus * (size_t)per_cu;
    return (unsigned)(g < items ? g : items);
}

template <bool EWA>
static void prepare_bwd_shapes()
{
    (void)persistent_grid(k_splat_bwd_persist<EWA, 16, 16>, 256, 1);
    (void)persistent_grid(k_splat_bwd_persist<EWA, 32, 8>, 256, 1);
    (void)persistent_grid(k_splat_bwd_persist<EWA, 8, 32>, 256, 1);
    (void)persistent_grid(k_splat_bwd_persist<EWA, 16, 8>, 256, 1);
    (void)persistent_grid(k_splat_bwd_persist<EWA, 8, 16>, 256, 1);
    (void)persistent_grid(k_splat_bwd_persist<EWA, 8, 8>, 256, 1);
}

// Run the device queries of the persistent launches now (before any graph capture).
void render_prepare_launch_shapes()
{
    (void)persistent_grid(k_splat_fwd_persist<1, false>, 64, 1);
    (void)persistent_grid(k_splat_fwd_persist<2, false>, 128, 1);
    (void)persistent_grid(k_splat_fwd_persist<4, false>, 256, 1);
    (void)persistent_grid(k_splat_fwd_persist<1, true>, 64, 1);
    (void)persistent_grid(k_splat_fwd_persist<2, true>, 128, 1);
    (void)persistent_grid(k_splat_fwd_persist<4, true>, 256, 1);
    prepare_bwd_shapes<false>();
    prepare_bwd_shapes<true>();
}

template <int WAVES, bool EWA>
static void launch_splat_fwd(const RenderArgs &a, float *proj, uint32_t *queue, size_t items,
                             hipStream_t s)
{
    const unsigned cap = (unsigned)a.L.cap;
    const int nsl = a.L.slices;
    if (nsl > 1) {   // list slices into partial images, then their fixed-order sum
        float *spart = WS(a, spart, float *);
        hipLaunchKernelGGL((k_splat_fwd<WAVES, EWA>), dim3((unsigned)items, (unsigned)nsl),
                           dim3(64 * WAVES), 0, s, a.geom, a.n, a.T, WS(a, rec, const float4 *),
                           WS(a, list, const uint32_t *), WS(a, cnt, const uint32_t *), a.L.nblk,
                           cap, proj, spart);
        const size_t npx = (size_t)a.T * a.geom.nu * a.geom.nv;
        hipLaunchKernelGGL((k_slice_reduce<EWA>), dim3((unsigned)((npx + 255) / 256)), dim3(256),
                           0, s, a.geom, a.T, nsl, (const float *)spart, proj);
        return;
    }
    if (a.persistent)
        hipLaunchKernelGGL((k_splat_fwd_persist<WAVES, EWA>),
                           dim3(persistent_grid(k_splat_fwd_persist<WAVES, EWA>, 64 * WAVES,
                                                items)),
                           dim3(64 * WAVES), 0, s, a.geom, a.n, a.T, WS(a, rec, const float4 *),
                           WS(a, list, const uint32_t *), WS(a, cnt, const uint32_t *), a.L.nblk,
                           cap, proj, queue);
    else
        hipLaunchKernelGGL((k_splat_fwd<WAVES, EWA>), dim3((unsigned)items), dim3(64 * WAVES), 0, s,
                           a.geom, a.n, a.T, WS(a, rec, const float4 *),
                           WS(a, list, const uint32_t *), WS(a, cnt, const uint32_t *), a.L.nblk,
                           cap, proj, (float *)nullptr);
}

hipError_t render_forward_splat(const RenderArgs &a, float *proj, hipStream_t s)
{
    const size_t items = (size_t)a.geom.ntiles * a.T;
    uint32_t *queue = WS(a, queue, uint32_t *);
    if (a.persistent && a.L.slices <= 1) {
        hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps(PS_SPLAT_FWD, s);
    // waves per workgroup: the tuning's, at most one per 8x8 block of the tile
    const int waves = std::min(a.splat_waves, a.geom.tile_nb);
    if (waves == 1) {
        if (a.geom.ewa) launch_splat_fwd<1, true>(a, proj, queue, items, s);
        else launch_splat_fwd<1, false>(a, proj, queue, items, s);
    } else if (waves == 2) {
        if (a.geom.ewa) launch_splat_fwd<2, true>(a, proj, queue, items, s);
        else launch_splat_fwd<2, false>(a, proj, queue, items, s);
    } else {
        if (a.geom.ewa) launch_splat_fwd<4, true>(a, proj, queue, items, s);
        else launch_splat_fwd<4, false>(a, proj, queue, items, s);
    }
    return hipGetLastError();
}

template <int NR>
static hipError_t backward_dispatch(const RenderArgs &a, float *g_mu, float *g_scale,
                                    float *g_quat, float *g_rho, float *g_coef, float *g_w,
                                    hipStream_t s)
{
    const int n = a.n, T = a.T;
    const int nb = (n + 255) / 256;
    const int nparts = nb * 4;
    hipError_t e;
    {
        ProfScope ps(PS_GAUSS_BWD, s);
        hipLaunchKernelGGL(k_tn_bwd<NR>, dim3(nb, a.L.tchunks), dim3(256), 0, s, a.geom, n, T,
                           a.L.tpc, WS(a, gsort, const float *), a.angles, a.w,
                           WS(a, uv, const float *), WS(a, rect, const int4 *),
                           WS(a, goff, const uint32_t *),
                           WS(a, part, const float4 *),
                           (unsigned)a.L.cap, WS(a, tacc, float *), WS(a, gwpart, float *),
                           nparts);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gauss_reduce<NR>, dim3((unsigned)(((size_t)4 * n + 255) / 256)),
                               dim3(256), 0, s, a.grid, n,
                               a.L.tchunks, a.coef, WS(a, gsort, const float *),
                               WS(a, uv, const float *), WS(a, tacc, const float *),
                               WS(a, order, const uint32_t *), g_mu, g_scale, g_quat, g_rho,
                               WS(a, gq, float *), a.L.gq_stride, a.basis ? g_coef : nullptr);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(PS_OTHER, s);
        if (T * NR > 0)
            hipLaunchKernelGGL(k_gw_final, dim3(T * NR), dim3(256), 0, s,
                               WS(a, gwpart, const float *), nparts, g_w);
        e = hipGetLastError();
    }
    if (e != hipSuccess || a.basis) return e;   // (a per-Gaussian basis has no lattice gather)
    {
        ProfScope ps(PS_COEF_GRAD, s);
        const int npts = a.grid.nx * a.grid.ny * a.grid.nz;
        hipLaunchKernelGGL(k_coef_grad<NR>, dim3((npts + 3) / 4), dim3(256), 0, s, a.grid,
                           WS(a, gq, const float *), a.L.gq_stride,
                           WS(a, cell_start, const uint32_t *), g_coef);
        e = hipGetLastError();
    }
    return e;
}

template <bool EWA, int TW, int TH>
static void launch_splat_bwd(const RenderArgs &a, const float *grad_proj, uint32_t *queue,
                             size_t items, hipStream_t s)
{
    if (a.persistent && a.L.slices <= 1)
        hipLaunchKernelGGL((k_splat_bwd_persist<EWA, TW, TH>),
                           dim3(persistent_grid(k_splat_bwd_persist<EWA, TW, TH>, 256, items)),
                           dim3(256),
                           0, s, a.geom, a.n, a.T, WS(a, rec, const float4 *),
                           WS(a, list, const uint32_t *), WS(a, cnt, const uint32_t *), a.L.nblk,
                           (unsigned)a.L.cap, WS(a, rect, const int4 *),
                           WS(a, goff, const uint32_t *), grad_proj, WS(a, part, float4 *),
                           queue);
    else
        hipLaunchKernelGGL((k_splat_bwd<EWA, TW, TH>),
                           dim3((unsigned)items, (unsigned)a.L.slices), dim3(256),
                           0, s, a.geom, a.n,
                           a.T, WS(a, rec, const float4 *), WS(a, list, const uint32_t *),
                           WS(a, cnt, const uint32_t *), a.L.nblk, (unsigned)a.L.cap,
                           WS(a, rect, const int4 *), WS(a, goff, const uint32_t *), grad_proj,
                           WS(a, part, float4 *));
}

// the backward splat specialised for the call's tile shape
template <bool EWA>
static void launch_splat_bwd_shape(const RenderArgs &a, const float *grad_proj, uint32_t *queue,
                                   size_t items, hipStream_t s)
{
    const int tw = a.geom.tile_w, th = a.geom.tile_h;
    if (tw == 16 && th == 16) launch_splat_bwd<EWA, 16, 16>(a, grad_proj, queue, items, s);
    else if (tw == 32) launch_splat_bwd<EWA, 32, 8>(a, grad_proj, queue, items, s);
    else if (tw == 16) launch_splat_bwd<EWA, 16, 8>(a, grad_proj, queue, items, s);
    else if (th == 32) launch_splat_bwd<EWA, 8, 32>(a, grad_proj, queue, items, s);
    else if (th == 16) launch_splat_bwd<EWA, 8, 16>(a, grad_proj, queue, items, s);
    else launch_splat_bwd<EWA, 8, 8>(a, grad_proj, queue, items, s);
}

hipError_t render_backward(const RenderArgs &a, const float *grad_proj, float *g_mu,
                           float *g_scale, float *g_quat, float *g_rho, float *g_coef,
                           float *g_w, hipStream_t s)
{
    hipError_t e;
    // per-(t,n) instance offsets (Gaussian-major) from the forward's instance counts, into their
    // own array (the counts stay, so a second backward of the same forward finds them)
    {
        ProfScope ps(PS_SCAN, s);
        e = launch_exclusive_scan(WS(a, goff, uint32_t *), (size_t)a.T * a.n,
                                  WS(a, scratch, uint32_t *), s, WS(a, gcount, const uint32_t *));
    }
    if (e != hipSuccess) return e;
    // a6: per-instance moment sums
    {
        const size_t items = (size_t)a.geom.ntiles * a.T;
        uint32_t *queue = WS(a, queue, uint32_t *);
        if (a.persistent && a.L.slices <= 1) {
            hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        ProfScope ps(PS_SPLAT_BWD, s);
        if (a.geom.ewa) launch_splat_bwd_shape<true>(a, grad_proj, queue, items, s);
        else launch_splat_bwd_shape<false>(a, grad_proj, queue, items, s);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    switch (a.grid.R) {
    case 1: return backward_dispatch<1>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 2: return backward_dispatch<2>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 3: return backward_dispatch<3>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 4: return backward_dispatch<4>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 5: return backward_dispatch<5>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 6: return backward_dispatch<6>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    case 7: return backward_dispatch<7>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    default: return backward_dispatch<8>(a, g_mu, g_scale, g_quat, g_rho, g_coef, g_w, s);
    }
}
