// bin.h -- deterministic, atomics-free-in-global-memory binning of items into keyed lists.
//
// Each item (a Gaussian of one projection, or one key of a radix pass) contributes nkeys()
// keys: key(k) is its k-th, and count(h) adds one to h[key] for each of them (in any order);
// before its keys are placed, prepare() may load what emit() needs beyond the keys. k_bin_count builds per-wave key histograms in LDS (integer LDS atomics: exact counts)
// and writes one count per (slice, key, item block), and beside it the offsets of the block's
// waves 1-3 within it (10 bits each, packed). After an exclusive scan of the counts in (slice,
// key, block) order, k_bin_fill forms per-wave running offsets from both and places every
// (item, key) pair: the rank among equal keys in
// one wave step comes from ballots over the key bits (a wave-level match), so the order
// inside every list is a fixed function of the input and the whole binning is bitwise
// reproducible.
#pragma once

#include "common.h"
#include "kernels.h"
#include "prof.h"

#define BIN_THREADS 256
#define BIN_WAVES (BIN_THREADS / DIGS_WAVE)
// ITEMS: items per workgroup (DIGS_BIN_ITEMS, or DIGS_BIN_ITEMS_SMALL for launches with few
// workgroups); each wave takes ITEMS / BIN_WAVES of them, 64 per step

// lanes whose key equals this lane's key (among active lanes), from the ballots of its bits. A bit
// that all active lanes share (the usual case for the high bits of nearby keys) selects nothing
// and is skipped (a uniform branch on its ballot).
__device__ __forceinline__ unsigned long long wave_match(unsigned key, bool active, int nbits)
{
    const unsigned long long act = __ballot(active);
    unsigned mlo = (unsigned)act, mhi = (unsigned)(act >> 32);
    for (int b = 0; b < nbits; ++b) {
        const unsigned bit = (key >> b) & 1u;
        const unsigned long long ones = __ballot(bit != 0u) & act;
        if (ones != 0ull && ones != act) {
            asm volatile("");   // keeps this a (uniform) branch rather than a select
            const unsigned nb = bit - 1u;   // lanes with the bit keep ones, the others ~ones
            mlo &= (unsigned)ones ^ nb;
            mhi &= (unsigned)(ones >> 32) ^ nb;
        }
    }
    return ((unsigned long long)mhi << 32) | mlo;
}

// (a wave takes ITEMS / BIN_WAVES items, each with at most one instance of a key, so the offsets
// of waves 1-3 within a block, at most 3 ITEMS / BIN_WAVES, fit 10 bits each)
template <class Src, int ITEMS>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_count(Src src, uint32_t *__restrict__ cnt,
                                                           uint32_t *__restrict__ pre, int nbins,
                                                           int nblk)
{
    static_assert(3 * (ITEMS / BIN_WAVES) < 1024 && BIN_WAVES == 4, "wave offsets: 3 x 10 bits");
    extern __shared__ uint32_t hist[];   // [BIN_WAVES][nbins]
    const int slice = blockIdx.y, blk = blockIdx.x;
    const int wave = threadIdx.x / DIGS_WAVE, lane = lane_id();
    for (int k = threadIdx.x; k < BIN_WAVES * nbins; k += BIN_THREADS) hist[k] = 0;
    __syncthreads();
    uint32_t *h = hist + wave * nbins;
    constexpr int PER_WAVE = ITEMS / BIN_WAVES;
    const int base = blk * ITEMS + wave * PER_WAVE;
    for (int step = 0; step < PER_WAVE / DIGS_WAVE; ++step) {
        const int item = base + step * DIGS_WAVE + lane;
        if (item < src.items) src.load(slice, item).count(h);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += BIN_THREADS) {
        const uint32_t c0 = hist[b], c1 = hist[nbins + b], c2 = hist[2 * nbins + b];
        const uint32_t c3 = hist[3 * nbins + b];
        cnt[((size_t)slice * nbins + b) * nblk + blk] = c0 + c1 + c2 + c3;
        // (the offsets in workgroup-major order: each workgroup writes, and reads, one run)
        pre[((size_t)slice * nblk + blk) * nbins + b] =
            c0 | ((c0 + c1) << 10) | ((c0 + c1 + c2) << 20);
    }
}

template <class Src, int ITEMS>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_fill(Src src,
                                                          const uint32_t *__restrict__ cnt_scan,
                                                          const uint32_t *__restrict__ pre,
                                                          int nbins, int nblk, int nbits)
{
    extern __shared__ uint32_t hist[];   // per-wave running offsets
    const int slice = blockIdx.y, blk = blockIdx.x;
    const int wave = threadIdx.x / DIGS_WAVE, lane = lane_id();
    uint32_t *h = hist + wave * nbins;
    constexpr int PER_WAVE = ITEMS / BIN_WAVES;
    const int base = blk * ITEMS + wave * PER_WAVE;
    // each wave's first position per key: the block's (scanned) plus the wave's offset within it
    for (int b = threadIdx.x; b < nbins; b += BIN_THREADS) {
        const uint32_t run = cnt_scan[((size_t)slice * nbins + b) * nblk + blk];
        const uint32_t p = pre[((size_t)slice * nblk + blk) * nbins + b];
        hist[b] = run;
        hist[nbins + b] = run + (p & 1023u);
        hist[2 * nbins + b] = run + ((p >> 10) & 1023u);
        hist[3 * nbins + b] = run + (p >> 20);
    }
    __syncthreads();
    // Emit: the step's (item, key) pairs are flattened in (lane, key) order and placed 64 at a time,
    // so items with many keys do not leave the rest of the wave idle.
    __shared__ int starts[BIN_WAVES][DIGS_WAVE];
    __shared__ typename Src::Item items[BIN_WAVES][DIGS_WAVE];
    for (int step = 0; step < PER_WAVE / DIGS_WAVE; ++step) {
        const int item0 = base + step * DIGS_WAVE;
        const int item = item0 + lane;
        const bool valid = item < src.items;
        typename Src::Item it = src.load(slice, valid ? item : 0);
        if (valid) src.prepare(slice, item, it);
        const int nk = valid ? it.nkeys() : 0;
        int incl = nk;
#pragma unroll
        for (int off = 1; off < DIGS_WAVE; off <<= 1) {
            const int y = __shfl_up(incl, off, DIGS_WAVE);
            if (lane >= off) incl += y;
        }
        const int total = __shfl(incl, DIGS_WAVE - 1, DIGS_WAVE);
        starts[wave][lane] = incl - nk;
        items[wave][lane] = it;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int c0 = 0; c0 < total; c0 += DIGS_WAVE) {
            const int idx = c0 + lane;
            const bool active = idx < total;
            // owner: the last lane whose start is <= idx (it has at least one key)
            int j = 0;
#pragma unroll
            for (int b = DIGS_WAVE / 2; b >= 1; b >>= 1)
                if (starts[wave][j + b] <= idx) j += b;
            const int k = idx - starts[wave][j];
            const typename Src::Item o = items[wave][j];
            const unsigned key = active ? (unsigned)o.key(k) : 0u;
            const unsigned long long peers = wave_match(key, active, nbits);
            uint32_t pos = 0;
            const int rank = lane_rank(peers);
            if (active) pos = h[key] + (uint32_t)rank;
            if (active && rank == 0) h[key] = pos + (uint32_t)__popcll(peers);
            if (active) src.emit(slice, item0 + j, o, k, key, pos);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Stable LSD radix pass source: 8 bits of 32-bit keys from `shift`, values carried along.
struct RadixSrc {
    const uint32_t *keys_in, *vals_in;
    uint32_t *keys_out, *vals_out;
    int items;
    int shift;
    struct Item {
        uint32_t k;
        __device__ int nkeys() const { return 1; }
        __device__ int key(int) const { return (int)k; }
        __device__ void count(uint32_t *h) const { atomicAdd(&h[k], 1u); }
    };
    __device__ Item load(int, int item) const
    {
        Item it;
        it.k = (keys_in[item] >> shift) & 255u;
        return it;
    }
    __device__ void prepare(int, int, Item &) const {}
    __device__ void emit(int, int item, const Item &, int, unsigned, uint32_t pos) const
    {
        if (pos < (uint32_t)items) {
            keys_out[pos] = keys_in[item];
            vals_out[pos] = vals_in[item];
        }
    }
};

// Count, scan and place (see above); the scan runs over (slice, key, block) counts, which cnt
// holds followed by the waves' offsets (2 cnt_elems words).
// items: items per workgroup, DIGS_BIN_ITEMS or DIGS_BIN_ITEMS_SMALL (nblk = ceil(items of a
// slice / items)). stages: time the three launches as their own stages (false when the caller
// times the whole binning as one stage)
template <class Src>
static inline hipError_t launch_binning(const Src &src, int slices, int nbins, int nblk, int nbits,
                                        uint32_t *cnt, size_t cnt_elems, uint32_t *scratch,
                                        hipStream_t s, int items = DIGS_BIN_ITEMS,
                                        bool stages = true)
{
    // cnt holds 2 cnt_elems words: the counts (scanned in place), then the waves' offsets
    uint32_t *pre = cnt + cnt_elems;
    const size_t lds = (size_t)BIN_WAVES * nbins * sizeof(uint32_t);
    const bool small = items == DIGS_BIN_ITEMS_SMALL;
    {
        ProfScope ps(stages ? PS_BIN_COUNT : -1, s);
        if (small)
            hipLaunchKernelGGL((k_bin_count<Src, DIGS_BIN_ITEMS_SMALL>), dim3(nblk, slices),
                               dim3(BIN_THREADS), lds, s, src, cnt, pre, nbins, nblk);
        else
            hipLaunchKernelGGL((k_bin_count<Src, DIGS_BIN_ITEMS>), dim3(nblk, slices),
                               dim3(BIN_THREADS), lds, s, src, cnt, pre, nbins, nblk);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps(stages ? PS_SCAN : -1, s);
        e = launch_exclusive_scan(cnt, cnt_elems, scratch, s);
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(stages ? PS_BIN_FILL : -1, s);
        if (small)
            hipLaunchKernelGGL((k_bin_fill<Src, DIGS_BIN_ITEMS_SMALL>), dim3(nblk, slices),
                               dim3(BIN_THREADS), lds, s, src, cnt, pre, nbins, nblk, nbits);
        else
            hipLaunchKernelGGL((k_bin_fill<Src, DIGS_BIN_ITEMS>), dim3(nblk, slices),
                               dim3(BIN_THREADS), lds, s, src, cnt, pre, nbins, nblk, nbits);
    }
    return hipGetLastError();
}

static inline int bits_for(int nbins)
{
    int b = 0;
    while ((1 << b) < nbins) ++b;
    return b < 1 ? 1 : b;
}


// Stable sort of (key, value) pairs by the low `kbits` bits of the key, 8 bits per pass. The
// pairs start in (ka, va); the sorted pairs end in (ka, va) if *swapped is false, else in
// (kb, vb). rhist needs 2 * 256 * ceil(n / DIGS_BIN_ITEMS) words, scratch the scan's scratch.
static inline hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb,
                                          int n, int kbits, uint32_t *rhist, uint32_t *scratch,
                                          bool *swapped, hipStream_t s)
{
    *swapped = false;
    const int nblk = (n + DIGS_BIN_ITEMS - 1) / DIGS_BIN_ITEMS;
    for (int shift = 0; shift < kbits; shift += 8) {
        RadixSrc src;
        src.keys_in = *swapped ? kb : ka;
        src.vals_in = *swapped ? vb : va;
        src.keys_out = *swapped ? ka : kb;
        src.vals_out = *swapped ? va : vb;
        src.items = n;
        src.shift = shift;
        hipError_t e = launch_binning(src, 1, 256, nblk, 8, rhist, (size_t)256 * nblk, scratch, s);
        if (e != hipSuccess) return e;
        *swapped = !*swapped;
    }
    return hipSuccess;
}
