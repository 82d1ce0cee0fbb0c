// warmstart.hip -- kernels of the per-projection temporal-weight fit and of its learned warm start.
//
// The plain fit finds, for each view t, the rank-R weights w_t of the low-rank motion model
// (Sec. 3.3, Eq. 9) that minimise the projection residual 1/2 ||I(w_t) - P_t||^2 by
// Levenberg-Marquardt; k_lm_normal_eq forms its normal equations from rendered images. The learned
// warm start is a small MLP (downsampled projection and gantry angle in, w_t out) whose matrix
// products run on the gfx950 matrix cores: BF16 operands, FP32 accumulation (k_gemm_bf16), with
// FP32 master weights updated by Adam.
#include "kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ __bf16 to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

// ------------------------------------------------------------------------------------------
// C[M][N] = epilogue(A . B) with op(A) [M][K] and op(B) [K][N] read from FP32 memory, rounded to
// BF16 in LDS and multiplied on v_mfma_f32_32x32x16_bf16 with FP32 accumulation. A is stored
// [M][K] (lda) or, with TA, [K][M]; B is stored [K][N] (ldb) or, with TB, [N][K]. Epilogue, in
// order: + C (accumulate), + bias[col], max(., 0) (relu), zero where gate[row][col] <= 0 (gate has
// the leading dimension ldc). One workgroup (4 waves) per 64x64 tile of C, each wave a 32x32 block;
// K is staged through LDS 32 at a time.
#define GT_M 64
#define GT_N 64
#define GT_K 32
#define GT_LDS 40   // bf16 per LDS row: 80 bytes, so every 8-element fragment is 16-byte aligned

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const float *__restrict__ A,
                                                   int lda, const float *__restrict__ B, int ldb,
                                                   float *__restrict__ C, int ldc,
                                                   const float *__restrict__ bias,
                                                   const float *__restrict__ gate, int relu,
                                                   int accumulate)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[GT_M * GT_LDS];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[GT_N * GT_LDS];
    const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
    const int tid = threadIdx.x, wave = tid / DIGS_WAVE, lane = lane_id();
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += GT_K) {
        for (int e = tid; e < GT_M * GT_K; e += 256) {
            const int r = TA ? e % GT_M : e / GT_K, c = TA ? e / GT_M : e % GT_K;
            const int m = m0 + r, k = k0 + c;
            float v = 0.0f;
            if (m < M && k < K) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            As[r * GT_LDS + c] = to_bf16(v);
        }
        for (int e = tid; e < GT_N * GT_K; e += 256) {
            const int r = TB ? e / GT_K : e % GT_N, c = TB ? e % GT_K : e / GT_N;
            const int nn = n0 + r, k = k0 + c;
            float v = 0.0f;
            if (nn < N && k < K) v = TB ? B[(size_t)nn * ldb + k] : B[(size_t)k * ldb + nn];
            Bs[r * GT_LDS + c] = to_bf16(v);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < GT_K; s += 16) {
            const int kk = s + 8 * (lane >> 5);
            const bf16x8 a = *(const bf16x8 *)&As[(wm + (lane & 31)) * GT_LDS + kk];
            const bf16x8 b = *(const bf16x8 *)&Bs[(wn + (lane & 31)) * GT_LDS + kk];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // result lane layout: element r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = n0 + wn + (lane & 31);
        if (row < M && col < N) {
            const size_t o = (size_t)row * ldc + col;
            float v = acc[r];
            if (accumulate) v += C[o];
            if (bias) v += bias[col];
            if (relu) v = fmaxf(v, 0.0f);
            if (gate && !(gate[o] > 0.0f)) v = 0.0f;
            C[o] = v;
        }
    }
}

// out[j] = sum_i X[i][j], rows summed in order (bias gradients)
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float *__restrict__ X, int ldx,
                                                float *__restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += X[(size_t)i * ldx + j];
    out[j] = s;
}

// Mean squared error against standardised targets, (pred - (target - mean)/std)^2 averaged over
// the B x R entries: dpred = its gradient; loss[0] = its value. One workgroup, fixed order.
__global__ __launch_bounds__(256) void k_mse(int B, int R, const float *__restrict__ pred,
                                             const float *__restrict__ target,
                                             const float *__restrict__ mean,
                                             const float *__restrict__ stdv,
                                             float *__restrict__ dpred, float *__restrict__ loss)
{
    __shared__ float part[256];
    const int m = B * R;
    const float inv = 1.0f / (float)m;
    float s = 0.0f;
    for (int i = threadIdx.x; i < m; i += 256) {
        const int r = i % R;
        const float d = pred[i] - (target[i] - mean[r]) / stdv[r];
        dpred[i] = 2.0f * d * inv;
        s = fmaf(d, d, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = part[0] * inv;
}

// Adam on FP32 master weights (bias-corrected moments; c1 = 1 - b1^t, c2 = 1 - b2^t)
__global__ __launch_bounds__(256) void k_adam(int n, float *__restrict__ w,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Network input of view t: the projection averaged over fy x fx pixel blocks (row-major,
// (nv/fy) x (nu/fx) values) times `scale`, standardised per feature if fmean/fistd are given
// ((x - fmean[i]) * fistd[i]), then sin and cos of the gantry angle.
__global__ __launch_bounds__(256) void k_downsample(int T, int nv, int nu, int fy, int fx,
                                                    const float *__restrict__ proj,
                                                    const float *__restrict__ angles,
                                                    float scale, const float *__restrict__ fmean,
                                                    const float *__restrict__ fistd,
                                                    float *__restrict__ out, int ld_out)
{
    const int oy = nv / fy, ox = nu / fx;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (t >= T) return;
    float *o = out + (size_t)t * ld_out;
    if (i < oy * ox) {
        const int Y = i / ox, X = i % ox;
        const float *src = proj + ((size_t)t * nv + (size_t)Y * fy) * nu + (size_t)X * fx;
        float s = 0.0f;
        for (int a = 0; a < fy; ++a)
            for (int b = 0; b < fx; ++b) s += src[(size_t)a * nu + b];
        float v = s * scale / (float)(fy * fx);
        if (fmean) v = (v - fmean[i]) * fistd[i];
        o[i] = v;
    } else if (i == oy * ox && angles) {
        float sn, cs;
        sincosf(angles[t], &sn, &cs);
        o[i] = sn;
        o[i + 1] = cs;
    }
}

// X[i][j] = (X[i][j] - mean[j]) * istd[j] for the first N columns of M rows (in place)
__global__ __launch_bounds__(256) void k_standardize(int M, int N, float *__restrict__ X, int ldx,
                                                     const float *__restrict__ mean,
                                                     const float *__restrict__ istd)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)M * N) return;
    const int i = (int)(idx / N), j = (int)(idx % N);
    float *x = X + (size_t)i * ldx + j;
    *x = (*x - mean[j]) * istd[j];
}

// ------------------------------------------------------------------------------------------
// Normal equations of one Levenberg-Marquardt step per view. imgs holds, per view t, R + 1
// rendered images (base weights, then the base with w_r raised by h[r]), each npix long; meas the
// measured image. With J_r = (I_r - I_0)/h_r and res = I_0 - P:
//   out[t] = (JtJ upper triangle, row-major (R(R+1)/2), Jt res (R), res.res (1)).
// One workgroup per view; each thread sums a fixed strided subset of pixels, then a fixed-order
// tree reduction.
template <int R>
__global__ __launch_bounds__(256) void k_lm_normal_eq(int T, int npix, const float *__restrict__ imgs,
                                                      const float *__restrict__ meas,
                                                      const float *__restrict__ h,
                                                      float *__restrict__ out)
{
    constexpr int NOUT = R * (R + 1) / 2 + R + 1;
    __shared__ float red[256];
    const int t = blockIdx.x;
    const float *base = imgs + (size_t)t * (R + 1) * npix;
    const float *P = meas + (size_t)t * npix;
    float acc[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) acc[k] = 0.0f;
    float ih[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ih[r] = 1.0f / h[r];
    for (int p = threadIdx.x; p < npix; p += 256) {
        const float i0 = base[p];
        const float res = i0 - P[p];
        float J[R];
#pragma unroll
        for (int r = 0; r < R; ++r) J[r] = (base[(size_t)(r + 1) * npix + p] - i0) * ih[r];
        int k = 0;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = a; b < R; ++b) acc[k++] += J[a] * J[b];
#pragma unroll
        for (int a = 0; a < R; ++a) acc[k++] += J[a] * res;
        acc[k] += res * res;
    }
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[(size_t)t * NOUT + k] = red[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
static int wrc(hipError_t e) { return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e); }

extern "C" int digs_gemm_bf16(int M, int N, int K, const float *A, int lda, int transA,
                              const float *B, int ldb, int transB, float *C, int ldc,
                              const float *bias, const float *gate, int relu, int accumulate,
                              void *stream)
{
    if (M < 0 || N < 0 || K < 0 || M > (1 << 24) || N > (1 << 24) || K > (1 << 24))
        return DIGS_EINVAL;
    if (M == 0 || N == 0) return DIGS_OK;
    if (!A || !B || !C || lda <= 0 || ldb <= 0 || ldc < N) return DIGS_EINVAL;
    if ((transA ? lda < M : lda < K) || (transB ? ldb < K : ldb < N)) return DIGS_EINVAL;
    const dim3 grid((N + GT_N - 1) / GT_N, (M + GT_M - 1) / GT_M);
    hipStream_t s = (hipStream_t)stream;
    if (!transA && !transB)
        hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda,
                           B, ldb, C, ldc, bias, gate, relu, accumulate);
    else if (transA && !transB)
        hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B,
                           ldb, C, ldc, bias, gate, relu, accumulate);
    else if (!transA && transB)
        hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B,
                           ldb, C, ldc, bias, gate, relu, accumulate);
    else
        hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B,
                           ldb, C, ldc, bias, gate, relu, accumulate);
    return wrc(hipGetLastError());
}

extern "C" int digs_colsum(int M, int N, const float *X, int ldx, float *out, void *stream)
{
    if (M < 0 || N < 0 || (N > 0 && (!X || !out || ldx < N))) return DIGS_EINVAL;
    if (N == 0) return DIGS_OK;
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, M, N,
                       X, ldx, out);
    return wrc(hipGetLastError());
}

extern "C" int digs_mse(int B, int R, const float *pred, const float *target, const float *mean,
                        const float *stdv, float *dpred, float *loss, void *stream)
{
    if (B <= 0 || R <= 0 || !pred || !target || !mean || !stdv || !dpred) return DIGS_EINVAL;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, (hipStream_t)stream, B, R, pred, target,
                       mean, stdv, dpred, loss);
    return wrc(hipGetLastError());
}

extern "C" int digs_adam(int n, float *w, const float *g, float *m, float *v, float lr, float b1,
                         float b2, float eps, int step, void *stream)
{
    if (n < 0 || step < 1 || !(lr >= 0.0f) || (n > 0 && (!w || !g || !m || !v)))
        return DIGS_EINVAL;
    if (n == 0) return DIGS_OK;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, w, g,
                       m, v, lr, b1, b2, eps, c1, c2);
    return wrc(hipGetLastError());
}

extern "C" int digs_downsample(int T, int nv, int nu, int fy, int fx, const float *proj,
                               const float *angles, float scale, const float *fmean,
                               const float *fistd, float *out, int ld_out, void *stream)
{
    if (T < 0 || nv <= 0 || nu <= 0 || fy <= 0 || fx <= 0 || nv % fy || nu % fx) return DIGS_EINVAL;
    const int nfeat = (nv / fy) * (nu / fx);
    if (T == 0) return DIGS_OK;
    if (!proj || !out || ld_out < nfeat + (angles ? 2 : 0) || (!fmean != !fistd))
        return DIGS_EINVAL;
    hipLaunchKernelGGL(k_downsample, dim3((nfeat + 2 + 255) / 256, T), dim3(256), 0,
                       (hipStream_t)stream, T, nv, nu, fy, fx, proj, angles, scale, fmean, fistd,
                       out, ld_out);
    return wrc(hipGetLastError());
}

extern "C" int digs_standardize(int M, int N, float *X, int ldx, const float *mean,
                                const float *istd, void *stream)
{
    if (M < 0 || N < 0 || (M > 0 && N > 0 && (!X || !mean || !istd || ldx < N)))
        return DIGS_EINVAL;
    const size_t m = (size_t)M * N;
    if (m == 0) return DIGS_OK;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, M, N, X, ldx, mean, istd);
    return wrc(hipGetLastError());
}

extern "C" int digs_lm_normal_eq(int T, int R, int npix, const float *imgs, const float *meas,
                                 const float *h, float *out, void *stream)
{
    if (T < 0 || R < 1 || R > DIGS_MAX_RANK || npix < 0) return DIGS_EINVAL;
    if (T == 0) return DIGS_OK;
    if (!imgs || !meas || !h || !out) return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    switch (R) {
#define LM_CASE(r)                                                                               \
    case r:                                                                                      \
        hipLaunchKernelGGL(k_lm_normal_eq<r>, dim3(T), dim3(256), 0, s, T, npix, imgs, meas, h,   \
                           out);                                                                 \
        break;
        LM_CASE(1) LM_CASE(2) LM_CASE(3) LM_CASE(4) LM_CASE(5) LM_CASE(6) LM_CASE(7) LM_CASE(8)
#undef LM_CASE
    }
    return wrc(hipGetLastError());
}
