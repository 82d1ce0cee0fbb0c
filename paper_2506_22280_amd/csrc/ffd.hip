// ffd.hip -- the low-rank cubic B-spline FFD (Sec. 3.3, Eq. 9-11) and the deformation-informed
// warp of the Gaussians (Sec. 3.2, Eq. 7-8) as standalone entry points.
//
// Layout: one thread per query point; control lattice coef[R][nz][ny][nx][3] read through the
// cache (the lattice of a realistic problem is well under a megabyte per rank and stays L2
// resident). Each 4x4x4 stencil is evaluated separably: a row of four control points along x is
// reduced with B(phi_x) and B'(phi_x) first, then weighted by the y/z pieces.
#include "ffd_device.h"
#include "kernels.h"

__global__ __launch_bounds__(256) void k_ffd_eval(DevGrid g, const float *__restrict__ coef,
                                                  int n, const float *__restrict__ x, int T,
                                                  const float *__restrict__ w,
                                                  float *__restrict__ disp,
                                                  float *__restrict__ jac)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Stencil st;
    make_stencil(g, x[i], x[n + i], x[2 * n + i], st, false);
    float U[DIGS_MAX_RANK][3], J[DIGS_MAX_RANK][9];
    for (int r = 0; r < g.R; ++r) ffd_rank(g, coef, r, st, U[r], J[r]);
    if (!w) {
        for (int r = 0; r < g.R; ++r) {
            for (int a = 0; a < 3; ++a) disp[((size_t)r * 3 + a) * n + i] = U[r][a];
            if (jac)
                for (int k = 0; k < 9; ++k) jac[((size_t)r * 9 + k) * n + i] = J[r][k];
        }
        return;
    }
    for (int t = 0; t < T; ++t) {
        float u[3] = {0.f, 0.f, 0.f}, jj[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < g.R; ++r) {
            const float wr = w[(size_t)t * g.R + r];
            for (int a = 0; a < 3; ++a) u[a] = fmaf(wr, U[r][a], u[a]);
            for (int k = 0; k < 9; ++k) jj[k] = fmaf(wr, J[r][k], jj[k]);
        }
        for (int a = 0; a < 3; ++a) disp[((size_t)t * 3 + a) * n + i] = u[a];
        if (jac)
            for (int k = 0; k < 9; ++k) jac[((size_t)t * 9 + k) * n + i] = jj[k];
    }
}

__global__ __launch_bounds__(256) void k_deform(DevGrid g, const float *__restrict__ coef, int n,
                                                const float *__restrict__ mu,
                                                const float *__restrict__ scale,
                                                const float *__restrict__ quat, int T,
                                                const float *__restrict__ w,
                                                float *__restrict__ mu_t,
                                                float *__restrict__ cov_t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float m0[3] = {mu[i], mu[n + i], mu[2 * n + i]};
    Stencil st;
    make_stencil(g, m0[0], m0[1], m0[2], st, false);
    float U[DIGS_MAX_RANK][3], J[DIGS_MAX_RANK][9];
    for (int r = 0; r < g.R; ++r) ffd_rank(g, coef, r, st, U[r], J[r]);
    float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
    const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    float Rm[9];
    quat_to_rot(qw * qn, qx * qn, qy * qn, qz * qn, Rm);
    const float s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
    float RS[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) RS[3 * a + b] = Rm[3 * a + b] * s[b];
    for (int t = 0; t < T; ++t) {
        float K[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        float mt[3] = {m0[0], m0[1], m0[2]};
        for (int r = 0; r < g.R; ++r) {
            const float wr = w[(size_t)t * g.R + r];
            for (int a = 0; a < 3; ++a) mt[a] = fmaf(wr, U[r][a], mt[a]);
            for (int k = 0; k < 9; ++k) K[k] = fmaf(wr, J[r][k], K[k]);
        }
        float M[9];  // M = K R diag(s), Sigma' = M M^T
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                M[3 * a + b] = K[3 * a] * RS[b] + K[3 * a + 1] * RS[3 + b] + K[3 * a + 2] * RS[6 + b];
        float C[6];
        const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
        for (int c = 0; c < 6; ++c) {
            const float *ra = M + 3 * pa[c], *rb = M + 3 * pb[c];
            C[c] = ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2];
        }
        for (int a = 0; a < 3; ++a) mu_t[((size_t)t * 3 + a) * n + i] = mt[a];
        for (int c = 0; c < 6; ++c) cov_t[((size_t)t * 6 + c) * n + i] = C[c];
    }
}

hipError_t launch_ffd_eval(const DevGrid &g, const float *coef, int n, const float *x, int T,
                           const float *w, float *disp, float *jac, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ffd_eval, dim3((n + 255) / 256), dim3(256), 0, s, g, coef, n, x, T, w,
                       disp, jac);
    return hipGetLastError();
}

hipError_t launch_deform(const DevGrid &g, const float *coef, int n, const float *mu,
                         const float *scale, const float *quat, int T, const float *w,
                         float *mu_t, float *cov_t, hipStream_t s)
{
    if (n <= 0 || T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_deform, dim3((n + 255) / 256), dim3(256), 0, s, g, coef, n, mu, scale,
                       quat, T, w, mu_t, cov_t);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Temporal weights of the low-rank motion model: a 1-D cubic B-spline in time over control
// values placed every dt from t0 (Sec. 3.3 after Eq. 11; Sec. 4.2 puts one every 4 time points),
// with the lattice's 0-based knot and clamping convention. One thread per (t, r).
__global__ __launch_bounds__(256) void k_temporal_fwd(int Ct, int R, const float *__restrict__ ctrl,
                                                      float t0, float idt, int T,
                                                      const float *__restrict__ times,
                                                      float *__restrict__ w)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= T * R) return;
    const int t = idx / R, r = idx % R;
    const float p = (times[t] - t0) * idt, f = floorf(p);
    float B[4];
    bspline4(p - f, B);
    const int fi = (int)fminf(fmaxf(f, -4.0f), (float)Ct + 4.0f);
    float acc = 0.0f;
#pragma unroll
    for (int l = 0; l < 4; ++l) acc = fmaf(B[l], ctrl[(size_t)clampi(fi - 1 + l, Ct) * R + r], acc);
    w[idx] = acc;
}

// Adjoint: each control value gathers, in time order, the pieces of the time points whose
// stencil (after clamping) lands on it. One thread per (control point, r); no atomics.
__global__ __launch_bounds__(256) void k_temporal_bwd(int Ct, int R, float t0, float idt, int T,
                                                      const float *__restrict__ times,
                                                      const float *__restrict__ g_w,
                                                      float *__restrict__ g_ctrl)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ct * R) return;
    const int j = idx / R, r = idx % R;
    float acc = 0.0f;
    for (int t = 0; t < T; ++t) {
        const float p = (times[t] - t0) * idt, f = floorf(p);
        const int fi = (int)fminf(fmaxf(f, -4.0f), (float)Ct + 4.0f);
        if (clampi(fi - 1, Ct) > j || clampi(fi + 2, Ct) < j) continue;
        float B[4];
        bspline4(p - f, B);
        float s = 0.0f;
#pragma unroll
        for (int l = 0; l < 4; ++l) s += (clampi(fi - 1 + l, Ct) == j) ? B[l] : 0.0f;
        acc = fmaf(s, g_w[(size_t)t * R + r], acc);
    }
    g_ctrl[idx] = acc;
}

hipError_t launch_temporal_fwd(int Ct, int R, const float *ctrl, float t0, float dt, int T,
                               const float *times, float *w, hipStream_t s)
{
    const int m = T * R;
    hipLaunchKernelGGL(k_temporal_fwd, dim3((m + 255) / 256), dim3(256), 0, s, Ct, R, ctrl, t0,
                       1.0f / dt, T, times, w);
    return hipGetLastError();
}

hipError_t launch_temporal_bwd(int Ct, int R, float t0, float dt, int T, const float *times,
                               const float *g_w, float *g_ctrl, hipStream_t s)
{
    const int m = Ct * R;
    hipLaunchKernelGGL(k_temporal_bwd, dim3((m + 255) / 256), dim3(256), 0, s, Ct, R, t0,
                       1.0f / dt, T, times, g_w, g_ctrl);
    return hipGetLastError();
}
