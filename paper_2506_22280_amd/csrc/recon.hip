// recon.hip -- kernels of the reconstruction loop around the renderer (Sec. 4.2): the L2
// projection loss with its gradient, and the Adam step on a parameter group kept in an
// unconstrained parameterisation (the renderer takes linear scales and densities; the loop
// optimises log-scales and softplus-densities, so the map and its derivative are applied here).
#include "kernels.h"

#define RES_THREADS 1024

static int rc(hipError_t e) { return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e); }

// grad = proj - meas, and per workgroup 1/2 the sum of grad^2 over its grid-stride share
// (per-thread sums, then a fixed tree) into part[blockIdx.x]; k_l2_total adds the parts in order,
// so the value is the same on every run.
__global__ __launch_bounds__(RES_THREADS) void k_l2_residual(size_t n,
                                                             const float *__restrict__ proj,
                                                             const float *__restrict__ meas,
                                                             float *__restrict__ grad,
                                                             float *__restrict__ part)
{
    __shared__ float red[RES_THREADS];
    float s = 0.0f;
    const size_t stride = (size_t)gridDim.x * RES_THREADS;
    for (size_t i = (size_t)blockIdx.x * RES_THREADS + threadIdx.x; i < n; i += stride) {
        const float d = proj[i] - meas[i];
        grad[i] = d;
        s = fmaf(d, d, s);
    }
    if (!part) return;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = RES_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = 0.5f * red[0];
}

__global__ void k_l2_total(int nparts, float *__restrict__ loss)
{
    float s = 0.0f;
    for (int b = 0; b < nparts; ++b) s += loss[1 + b];
    loss[0] = s;
}

// softplus(x) = log(1 + e^x), written so that it neither overflows nor loses small values
__device__ __forceinline__ float softplus(float x)
{
    return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

// One bias-corrected Adam step on the unconstrained raw[i] given dL/dvalue[i], value = map(raw):
// map 0 identity, 1 exp, 2 softplus. value is rewritten from the updated raw (with map 0 it is
// raw itself, hence no restrict on the two).
__global__ __launch_bounds__(256) void k_adam_mapped(int n, float *raw, float *value,
                                                     const float *__restrict__ g_value,
                                                     float *__restrict__ m, float *__restrict__ v,
                                                     float lr, float b1, float b2, float eps,
                                                     float c1, float c2, int map)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = raw[i];
    float g = g_value[i];
    if (map == 1) g *= value[i];                               // d e^x / dx = e^x
    else if (map == 2) g *= 1.0f / (1.0f + expf(-x));          // d softplus / dx = sigmoid
    const float mi = fmaf(b1, m[i], (1.0f - b1) * g);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * g * g);
    m[i] = mi;
    v[i] = vi;
    const float xn = x - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    raw[i] = xn;
    value[i] = (map == 1) ? expf(xn) : (map == 2) ? softplus(xn) : xn;
}

extern "C" int digs_l2_residual(int64_t n, const float *proj, const float *meas, float *grad,
                                float *loss, void *stream)
{
    if (n < 0 || (n > 0 && (!proj || !meas || !grad))) return DIGS_EINVAL;
    if (n == 0) {   // L = 0: the total of no parts
        if (!loss) return DIGS_OK;
        hipLaunchKernelGGL(k_l2_total, dim3(1), dim3(1), 0, (hipStream_t)stream, 0, loss);
        return rc(hipGetLastError());
    }
    const int64_t want = (n + RES_THREADS * 8 - 1) / (RES_THREADS * 8);
    const int blocks = (int)(want < DIGS_L2_PARTS ? want : DIGS_L2_PARTS);
    hipLaunchKernelGGL(k_l2_residual, dim3(blocks), dim3(RES_THREADS), 0, (hipStream_t)stream,
                       (size_t)n, proj, meas, grad, loss ? loss + 1 : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return rc(e);
    hipLaunchKernelGGL(k_l2_total, dim3(1), dim3(1), 0, (hipStream_t)stream, blocks, loss);
    return rc(hipGetLastError());
}

extern "C" int digs_adam_mapped(int n, float *raw, float *value, const float *g_value, float *m,
                                float *v, float lr, float b1, float b2, float eps, int step,
                                int map, void *stream)
{
    if (n < 0 || step < 1 || !(lr >= 0.0f) || map < 0 || map > 2 ||
        (n > 0 && (!raw || !value || !g_value || !m || !v)) || (map == 0 && value != raw))
        return DIGS_EINVAL;
    if (n == 0) return DIGS_OK;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam_mapped, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       n, raw, value, g_value, m, v, lr, b1, b2, eps, c1, c2, map);
    return rc(hipGetLastError());
}
