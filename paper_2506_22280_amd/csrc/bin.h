// bin.h -- deterministic, atomics-free-in-global-memory binning of items into keyed lists.
//
// Each item (a Gaussian of one projection, or one key of a radix pass) contributes nkeys()
// keys; before its keys are placed, prepare() may load what emit() needs beyond the keys. k_bin_count builds per-wave key histograms in LDS (integer LDS atomics: exact counts)
// and writes one count per (slice, key, item block). After an exclusive scan of those counts
// in (slice, key, block) order, k_bin_fill recomputes the per-wave histograms, turns them into
// per-wave running offsets, and places every (item, key) pair: the rank among equal keys in
// one wave step comes from ballots over the key bits (a wave-level match), so the order
// inside every list is a fixed function of the input and the whole binning is bitwise
// reproducible.
#pragma once

#include "common.h"

#define BIN_THREADS 256
#define BIN_WAVES (BIN_THREADS / DIGS_WAVE)
#define BIN_PER_WAVE (DIGS_BIN_ITEMS / BIN_WAVES)   // 256 items per wave, 4 steps of 64

// lanes whose key equals this lane's key (among active lanes)
__device__ __forceinline__ unsigned long long wave_match(unsigned key, bool active, int nbits)
{
    unsigned long long m = __ballot(active);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1u;
        const unsigned long long ones = __ballot(active && bit);
        m &= bit ? ones : ~ones;
    }
    return m;
}

template <class Src>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_count(Src src, uint32_t *__restrict__ cnt,
                                                           int nbins, int nblk)
{
    extern __shared__ uint32_t hist[];   // [BIN_WAVES][nbins]
    const int slice = blockIdx.y, blk = blockIdx.x;
    const int wave = threadIdx.x / DIGS_WAVE, lane = lane_id();
    for (int k = threadIdx.x; k < BIN_WAVES * nbins; k += BIN_THREADS) hist[k] = 0;
    __syncthreads();
    uint32_t *h = hist + wave * nbins;
    const int base = blk * DIGS_BIN_ITEMS + wave * BIN_PER_WAVE;
    for (int step = 0; step < BIN_PER_WAVE / DIGS_WAVE; ++step) {
        const int item = base + step * DIGS_WAVE + lane;
        if (item < src.items) {
            typename Src::Item it = src.load(slice, item);
            const int nk = it.nkeys();
            for (int k = 0; k < nk; ++k) atomicAdd(&h[it.key(k)], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += BIN_THREADS) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < BIN_WAVES; ++w) c += hist[w * nbins + b];
        cnt[((size_t)slice * nbins + b) * nblk + blk] = c;
    }
}

template <class Src>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_fill(Src src,
                                                          const uint32_t *__restrict__ cnt_scan,
                                                          int nbins, int nblk, int nbits)
{
    extern __shared__ uint32_t hist[];   // per-wave counts, then per-wave running offsets
    const int slice = blockIdx.y, blk = blockIdx.x;
    const int wave = threadIdx.x / DIGS_WAVE, lane = lane_id();
    for (int k = threadIdx.x; k < BIN_WAVES * nbins; k += BIN_THREADS) hist[k] = 0;
    __syncthreads();
    uint32_t *h = hist + wave * nbins;
    const int base = blk * DIGS_BIN_ITEMS + wave * BIN_PER_WAVE;
    for (int step = 0; step < BIN_PER_WAVE / DIGS_WAVE; ++step) {
        const int item = base + step * DIGS_WAVE + lane;
        if (item < src.items) {
            typename Src::Item it = src.load(slice, item);
            const int nk = it.nkeys();
            for (int k = 0; k < nk; ++k) atomicAdd(&h[it.key(k)], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += BIN_THREADS) {
        uint32_t run = cnt_scan[((size_t)slice * nbins + b) * nblk + blk];
#pragma unroll
        for (int w = 0; w < BIN_WAVES; ++w) {
            const uint32_t c = hist[w * nbins + b];
            hist[w * nbins + b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int step = 0; step < BIN_PER_WAVE / DIGS_WAVE; ++step) {
        const int item = base + step * DIGS_WAVE + lane;
        const bool valid = item < src.items;
        typename Src::Item it = src.load(slice, valid ? item : 0);
        if (valid) src.prepare(slice, item, it);
        const int nk = valid ? it.nkeys() : 0;
        for (int k = 0;; ++k) {
            const bool active = k < nk;
            if (!__any(active)) break;
            const unsigned key = active ? (unsigned)it.key(k) : 0u;
            const unsigned long long peers = wave_match(key, active, nbits);
            uint32_t pos = 0;
            const int rank = __popcll(peers & lanemask_lt());
            if (active) pos = h[key] + (uint32_t)rank;
            if (active && rank == 0) h[key] = pos + (uint32_t)__popcll(peers);
            if (active) src.emit(slice, item, it, k, pos);
        }
    }
}
