// scan.hip -- device-wide exclusive prefix sum of uint32 (fixed order, deterministic).
//
// Used for the (projection, tile, Gaussian-block) instance counts of the tile binning, the
// per-Gaussian instance offsets, and the digit histograms of the cell sort. Each workgroup
// scans 2048 elements (256 threads x 8 consecutive elements), from src into data (src may be
// data itself). With at most 2048 blocks, a
// second launch adds to each block the sum of the block totals before it (each workgroup sums
// them itself); with more, the block totals are scanned recursively and added back.
#include "kernels.h"

#define SCAN_THREADS 256
#define SCAN_PER_THREAD 8
#define SCAN_BLOCK (SCAN_THREADS * SCAN_PER_THREAD)

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_block(uint32_t *data, const uint32_t *src,
                                                             size_t n,
                                                             uint32_t *__restrict__ bsum)
{
    __shared__ uint32_t wave_tot[SCAN_THREADS / DIGS_WAVE];
    const size_t base = (size_t)blockIdx.x * SCAN_BLOCK + (size_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        size_t i = base + k;
        uint32_t x = (i < n) ? src[i] : 0u;
        v[k] = run;
        run += x;
    }
    // inclusive scan of thread totals within the wave
    const int lane = lane_id();
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < DIGS_WAVE; off <<= 1) {
        uint32_t y = __shfl_up(incl, off, DIGS_WAVE);
        if (lane >= off) incl += y;
    }
    const int wave = threadIdx.x / DIGS_WAVE;
    if (lane == DIGS_WAVE - 1) wave_tot[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / DIGS_WAVE; ++w) {
        uint32_t t = wave_tot[w];
        if (w < wave) woff += t;
        btot += t;
    }
    const uint32_t toff = woff + incl - run;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        size_t i = base + k;
        if (i < n) data[i] = v[k] + toff;
    }
    if (threadIdx.x == 0 && bsum) bsum[blockIdx.x] = btot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(uint32_t *__restrict__ data, size_t n,
                                                           const uint32_t *__restrict__ bsum)
{
    const uint32_t add = bsum[blockIdx.x];
    const size_t base = (size_t)blockIdx.x * SCAN_BLOCK;
    for (int k = threadIdx.x; k < SCAN_BLOCK; k += SCAN_THREADS) {
        size_t i = base + k;
        if (i < n) data[i] += add;
    }
}

// Adds to block b of data the sum of bsum[0..b) (b < SCAN_BLOCK: one pass over at most 2048
// totals per workgroup, summed in a fixed order).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add_prefix(uint32_t *__restrict__ data,
                                                                  size_t n,
                                                                  const uint32_t *__restrict__ bsum)
{
    __shared__ uint32_t wave_tot[SCAN_THREADS / DIGS_WAVE];
    const int b = blockIdx.x;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        const int i = (int)threadIdx.x * SCAN_PER_THREAD + k;
        if (i < b) v += bsum[i];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, DIGS_WAVE);
    if (lane_id() == 0) wave_tot[threadIdx.x / DIGS_WAVE] = v;
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / DIGS_WAVE; ++w) add += wave_tot[w];
    const size_t base = (size_t)b * SCAN_BLOCK;
    for (int k = threadIdx.x; k < SCAN_BLOCK; k += SCAN_THREADS) {
        const size_t i = base + k;
        if (i < n) data[i] += add;
    }
}

size_t scan_scratch_elems(size_t n)
{
    size_t total = 0;
    while (n > 1) {
        n = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
        total += n;
    }
    return total + 1;
}

hipError_t launch_exclusive_scan(uint32_t *data, size_t n, uint32_t *scratch, hipStream_t s,
                                 const uint32_t *src)
{
    if (n == 0) return hipSuccess;
    const size_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data,
                       src ? src : (const uint32_t *)data, n, nb > 1 ? scratch : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    if (nb <= SCAN_BLOCK) {
        hipLaunchKernelGGL(k_scan_add_prefix, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data,
                           n, (const uint32_t *)scratch);
        return hipGetLastError();
    }
    e = launch_exclusive_scan(scratch, nb, scratch + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n,
                       scratch);
    return hipGetLastError();
}
