// rsi_rank.h -- stable ranking of a workgroup's tile by an 8-bit digit
// (wave64 ballots, LDS counts per round and wave, one 256-entry scan), shared
// by the radix sort and the adjoint's per-triangle grouping.  Workgroups of
// kThreads = 256 threads; item r of thread x is tile element r * 256 + x, so
// the stable order of a tile is (round, wave, lane).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsi {
namespace rank {

constexpr int kThreads = 256;
constexpr int kRadix = 256;
constexpr int kWaves = kThreads / 64;

__device__ inline uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Exclusive scan of 256 per-digit values held one per thread, done by the
// first wave (four digits per lane).
__device__ inline void scan256(const uint32_t *in, uint32_t *out)
{
    const int tid = threadIdx.x;
    if (tid < 64) {
        uint32_t c0 = in[4 * tid], c1 = in[4 * tid + 1], c2 = in[4 * tid + 2], c3 = in[4 * tid + 3];
        uint32_t s4 = c0 + c1 + c2 + c3;
        uint32_t incl = s4;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t v = __shfl_up(incl, off, 64);
            if ((int)__lane_id() >= off) incl += v;
        }
        uint32_t ex = incl - s4;
        out[4 * tid] = ex;
        out[4 * tid + 1] = ex + c0;
        out[4 * tid + 2] = ex + c0 + c1;
        out[4 * tid + 3] = ex + c0 + c1 + c2;
    }
}

// Stable rank of one tile held in registers (item r of thread x is tile
// element r * kThreads + x; `valid` marks live elements): on return pos[r]
// is the item's position in the tile ordered by digit (ties in tile order),
// run[d] the tile's count of digit d and start[d] its exclusive scan.
// `wcnt` is LDS scratch of IPT * kWaves * kRadix words.
template <int IPT>
__device__ inline void rank_tile(const uint32_t (&dig)[IPT], const bool (&valid)[IPT], uint32_t (&pos)[IPT],
                                 uint32_t *wcnt, uint32_t *run, uint32_t *start)
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
#pragma unroll
    for (int r = 0; r < IPT; ++r)
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[(r * kWaves + w) * kRadix + tid] = 0;
    __syncthreads();
    // per round: the lanes of this wave holding the same digit (8 ballots);
    // the lowest of them records the group size
    uint32_t below[IPT];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t d = dig[r];
        uint64_t peers = __ballot(valid[r]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        below[r] = (uint32_t)__popcll(peers & lt);
        if (valid[r] && below[r] == 0) wcnt[(r * kWaves + wave) * kRadix + d] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // digit tid: exclusive prefix over (round, wave) in tile order
    {
        uint32_t acc = 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[(r * kWaves + w) * kRadix + tid];
                wcnt[(r * kWaves + w) * kRadix + tid] = acc;
                acc += c;
            }
        run[tid] = acc;
    }
    __syncthreads();
    scan256(run, start);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) pos[r] = start[dig[r]] + wcnt[(r * kWaves + wave) * kRadix + dig[r]] + below[r];
}

}  // namespace rank
}  // namespace rsi
