// Stable block-level ranking by one 8-bit digit, shared by the radix sort's
// scatter and by the fused binning passes.
//
// A block of kSortThreads threads holds ITEMS items per thread in registers
// (kSortItems unless stated), assigned wave-striped -- wave w owns chunk
// positions [w*P, (w+1)*P), P = 64 ITEMS, and in step i lane l holds position
// w*P + i*64 + l --
// so lane order, then step order, then wave order is the input order.  Each
// wave ranks its items with eight ballots per step (the lanes sharing the
// digit) and a running per-digit count in LDS; per-digit wave prefixes and a
// block scan then order the waves.  The ranked chunk is staged in LDS in
// (digit, input) order and handed to the caller's writer by consecutive
// threads, so each digit's run leaves the block as contiguous stores.
#pragma once
#include "gsr_internal.hpp"

namespace gsr {

constexpr int kRankWaves = kSortThreads / kWave;

struct RankSmem {
    uint32_t wcnt[kRankWaves][256];  // per-wave running digit counts, then wave prefixes
    uint32_t gbase[256];             // global output start of each digit for this block
    uint32_t dstart[256];            // block-local start of each digit
    uint32_t wt[kRankWaves];
};

// Zero the per-wave counts; the caller then fills gbase and issues a barrier.
__device__ __forceinline__ void rank_init(RankSmem &sm) {
    for (int i = threadIdx.x; i < kRankWaves * 256; i += kSortThreads) (&sm.wcnt[0][0])[i] = 0;
}

// Chunk position of item i of this thread, for blocks that hold ITEMS items
// per thread (ITEMS * kSortThreads per block).
template <int ITEMS = kSortItems>
__device__ __forceinline__ int rank_pos(int i) {
    return (threadIdx.x / kWave) * (ITEMS * kWave) + i * kWave + (threadIdx.x & (kWave - 1));
}

// Ranks the block's items by digit (key >> shift) & 255 and, for each valid
// item, computes payload = fetch(key, val) and calls store(dst, key, payload),
// where dst = gbase[digit] + the item's stable rank within its digit.  Every
// thread runs all its fetches (loads may be in flight together) before its
// stores.  Items at positions >= cnt are invalid.  skey / sval: ITEMS*256-entry
// LDS staging arrays, which may alias memory the caller no longer reads (item
// generation must be complete).  Contains barriers; the caller must have run
// rank_init, set gbase and issued a barrier.
// sval may be null when the values are not needed (fetch then gets 0).
// Output positions are below 2^32 (capacities are 32-bit).
template <int ITEMS, class Fetch, class Store>
__device__ __forceinline__ void rank_stage_write(const uint32_t (&key)[ITEMS],
                                                 const uint32_t (&val)[ITEMS], int cnt,
                                                 int shift, RankSmem &sm, uint32_t *skey,
                                                 uint32_t *sval, Fetch fetch, Store store) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t rank[ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = rank_pos<ITEMS>(i) < cnt;
        const uint32_t d = (key[i] >> shift) & 255u;
        // lanes whose digit differs from this lane's in some bit: per bit the
        // ballot XOR this lane's bit spread over 32 bits, OR-accumulated in the
        // two 32-lane halves (cheaper than selecting ballot or ~ballot per lane)
        uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t spread = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);  // 0 or ~0
            const uint64_t m = __ballot((int32_t)spread < 0);
            dlo |= (uint32_t)m ^ spread;
            dhi |= (uint32_t)(m >> 32) ^ spread;
        }
        const uint64_t peers = __ballot(valid) & ~(((uint64_t)dhi << 32) | dlo);
        const uint32_t before = sm.wcnt[wid][d];
        rank[i] = before + (uint32_t)__popcll(peers & lt);
        // the highest lane of each digit group advances the running count
        if (valid && (peers >> lane) == 1ull) sm.wcnt[wid][d] = before + (uint32_t)__popcll(peers);
        if (!valid) rank[i] = 0xffffffffu;
    }
    __syncthreads();
    uint32_t tot_d = 0;
    {   // exclusive prefix over waves per digit; thread t owns digit t
        const int d = threadIdx.x;
#pragma unroll
        for (int w = 0; w < kRankWaves; ++w) {
            const uint32_t c = sm.wcnt[w][d];
            sm.wcnt[w][d] = tot_d;
            tot_d += c;
        }
    }
    uint32_t all;
    sm.dstart[threadIdx.x] = block_exclusive_scan<kSortThreads, uint32_t>(tot_d, sm.wt, &all);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (rank[i] == 0xffffffffu) continue;
        const uint32_t d = (key[i] >> shift) & 255u;
        const uint32_t p = sm.dstart[d] + sm.wcnt[wid][d] + rank[i];
        skey[p] = key[i];
        if (sval) sval[p] = val[i];
    }
    __syncthreads();
    // position p = threadIdx.x + i * kSortThreads: consecutive threads take
    // consecutive staged items, so each digit's run is stored contiguously
    uint32_t k[ITEMS], pay[ITEMS], dst[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int p = threadIdx.x + i * kSortThreads;
        if (p < cnt) {
            k[i] = skey[p];
            const uint32_t d = (k[i] >> shift) & 255u;
            dst[i] = sm.gbase[d] + ((uint32_t)p - sm.dstart[d]);
            pay[i] = fetch(k[i], sval ? sval[p] : 0u);
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (threadIdx.x + i * kSortThreads < cnt) store((int64_t)dst[i], k[i], pay[i]);
}

}  // namespace gsr
