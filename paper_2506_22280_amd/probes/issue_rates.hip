// issue_rates.hip -- measured issue rate of the VALU instructions the splat kernels are made of
// (v_fma_f32, v_exp_f32, v_rsq_f32), alone and mixed, on the whole chip: 8192 workgroups of 256
// lanes, 8 independent dependency chains per lane, 4096 iterations. The rates set how many VALU
// issue slots a transcendental takes in the splat kernels' ALU roofline.
//
// Build: built next to this file by paper_2506_22280_amd.build (executable `issue_rates`).
#include <hip/hip_runtime.h>
#include <stdio.h>
template <int OP>
__global__ __launch_bounds__(256) void k(float *out, int iters, float c)
{
    float x[8], y[8];
    for (int j = 0; j < 8; ++j) { x[j] = 0.5f + 1e-3f * (threadIdx.x + j); y[j] = x[j]; }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (OP == 0) x[j] = fmaf(x[j], c, 0.25f);
            else if (OP == 1) x[j] = __builtin_amdgcn_exp2f(-x[j]);
            else if (OP == 2) x[j] = __builtin_amdgcn_rsqf(x[j]);
            else if (OP == 3) {   // 1 exp + 4 fma on independent chains
                x[j] = __builtin_amdgcn_exp2f(-x[j]);
                y[j] = fmaf(y[j], c, 0.25f); y[j] = fmaf(y[j], c, 0.25f);
                y[j] = fmaf(y[j], c, 0.25f); y[j] = fmaf(y[j], c, 0.25f);
            }
        }
    }
    float s = 0; for (int j = 0; j < 8; ++j) s += x[j] + y[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
int main()
{
    const int blocks = 256 * 32, threads = 256, iters = 4096;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * blocks * threads) != hipSuccess) return 1;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    const char *names[4] = {"fma", "exp2", "rsq", "exp2+4fma"};
    for (int op = 0; op < 4; ++op) {
        for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(a);
            if (op == 0) hipLaunchKernelGGL(k<0>, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f);
            if (op == 1) hipLaunchKernelGGL(k<1>, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.f);
            if (op == 2) hipLaunchKernelGGL(k<2>, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.f);
            if (op == 3) hipLaunchKernelGGL(k<3>, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f);
            (void)hipEventRecord(b);
            (void)hipEventSynchronize(b);
            float ms; (void)hipEventElapsedTime(&ms, a, b);
            double inst = (double)blocks * threads * iters * 8 * (op == 3 ? 5 : 1);
            if (rep) printf("%s: %.3f ms, %.2f T lane-instr/s\n", names[op], ms, inst / ms / 1e9);
        }
    }
    (void)hipFree(out);
    return 0;
}
