// sort.hip -- stable LSD radix sort of (uint64 key, uint32 value) pairs,
// 8-bit digits, LDS-staged (the Morton-code sorting step timed in the paper's
// Table 2, which there ran on the host).
//
// One pass per digit:
//   k_hist     per-tile digit histogram in LDS -> hist[digit][tile]
//   k_scan     one workgroup turns hist into exclusive global offsets
//              (digit-major, so the offset of (digit, tile) is the count of
//              all smaller digits plus this digit in earlier tiles)
//   k_scatter  per tile: stable rank of every element among equal digits
//              via wave64 ballots, reorder the tile in LDS by digit, then
//              write each digit run to its global offset (contiguous runs)
// With at most 64 tiles (inputs up to 128k elements, where the passes are
// latency bound) every scatter workgroup derives its own offsets from the
// raw histograms (no k_scan) and also counts the next pass's digits of the
// elements it writes, per destination tile, so only the first pass needs
// k_hist: one launch per pass.  Three histogram buffers rotate: pass p reads
// H[p % 3], adds into H[(p + 1) % 3] and clears H[(p + 2) % 3] for pass p + 1.
// Tiles are 256 threads x 8 items in striped order (item r of thread x is
// element r*256 + x), which fixes the stable order (r, wave, lane).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsi_host.h"
#include "rsi_rank.h"

namespace rsi {
namespace {

using rank::kThreads;
using rank::kRadix;
using rank::kWaves;
using rank::lanemask_lt;
using rank::scan256;
using rank::rank_tile;
constexpr int kItems = 8;                // elements per thread in large sorts
constexpr int kTile = kThreads * kItems;
constexpr int kFusedTiles = 64;  // up to this many tiles each workgroup scans the histograms itself

// Digit of an element for one pass: 8 bits of the key, or (for batches)
// 8 bits of the mesh that the element's value (a triangle index) belongs to.
struct Digit {
    const int64_t *off;  // null: key digits
    int32_t M;
    int shift;
    __device__ inline uint32_t operator()(uint64_t key, uint32_t val) const
    {
        if (off) return ((uint32_t)mesh_of(off, M, (int64_t)val) >> shift) & (kRadix - 1);
        return (uint32_t)(key >> shift) & (kRadix - 1);
    }
};

template <int IPT>
__global__ __launch_bounds__(kThreads) void k_hist(const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ vals, int64_t n, Digit dg,
                                                   uint32_t *__restrict__ hist, int ntiles,
                                                   uint32_t *__restrict__ clear)
{
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    // `clear` (may be null): a histogram buffer the next scatter adds into
    if (clear) clear[(int64_t)tid * ntiles + blockIdx.x] = 0;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kThreads * IPT);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        int64_t i = base + r * kThreads + tid;
        if (i < n) atomicAdd(&h[dg(keys[i], dg.off ? vals[i] : 0u)], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Exclusive scan of n counts in place by one workgroup of 1024 threads:
// each thread sums a contiguous chunk, the chunk sums are scanned in LDS,
// then each thread rewrites its chunk.
__global__ __launch_bounds__(1024) void k_scan(uint32_t *__restrict__ a, int64_t n)
{
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = tid * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    uint32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += a[i];
    part[tid] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = tid ? part[tid - 1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

// Large tables (many tiles): a three-launch scan.  k_part_sums reduces
// blocks of kScanChunk counts, k_scan scans those sums (one workgroup), and
// k_part_apply rescans each block from its offset.
constexpr int kScanChunk = 4096;

__global__ __launch_bounds__(256) void k_part_sums(const uint32_t *__restrict__ a, int64_t n,
                                                   uint32_t *__restrict__ part)
{
    __shared__ uint32_t ws[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t s = 0;
    for (int k = threadIdx.x; k < kScanChunk; k += 256) {
        const int64_t i = base + k;
        if (i < n) s += a[i];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (__lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void k_part_apply(uint32_t *__restrict__ a, int64_t n,
                                                    const uint32_t *__restrict__ part)
{
    // each thread owns 16 consecutive counts of the block's 4096
    __shared__ uint32_t ts[256];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * 16;
    uint32_t v[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = base + k < n ? a[base + k] : 0u;
        s += v[k];
    }
    ts[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t x = (int)threadIdx.x >= off ? ts[threadIdx.x - off] : 0u;
        __syncthreads();
        ts[threadIdx.x] += x;
        __syncthreads();
    }
    uint32_t run = part[blockIdx.x] + ts[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
}

// FUSED: `offs` holds the raw per-tile histograms and each workgroup forms
// its own global digit offsets (few tiles: this saves the separate scan
// launch); it then also adds the next pass's digit counts of the elements it
// writes into `hnext` (per destination tile) and clears `hclear`.  Otherwise
// `offs` is the scanned table.
template <bool FUSED, int IPT>
__global__ __launch_bounds__(kThreads) void k_scatter(const uint64_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                      int64_t n, Digit dg, const uint32_t *__restrict__ offs,
                                                      int ntiles, Digit dnext, uint32_t *__restrict__ hnext,
                                                      uint32_t *__restrict__ hclear)
{
    // wcnt[r][w][d]: elements with digit d held by wave w in round r; after
    // the scan, the number of elements with digit d before (r, w) in the tile
    __shared__ uint32_t wcnt[IPT][kWaves][kRadix];
    __shared__ uint32_t run[kRadix];    // the tile's count of each digit
    __shared__ uint32_t start[kRadix];  // exclusive scan of run[]
    __shared__ uint32_t gbase[kRadix];  // global offset of (digit, this tile)
    __shared__ uint64_t skey[(kThreads * IPT)];
    __shared__ uint32_t sval[(kThreads * IPT)];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * (kThreads * IPT);

    // all loads first: one memory latency for the whole tile
    uint64_t key[IPT];
    uint32_t val[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t i = base + r * kThreads + tid;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0u;
    }
    if (FUSED && hclear) hclear[(int64_t)tid * ntiles + blockIdx.x] = 0;
#pragma unroll
    for (int r = 0; r < IPT; ++r)
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[r][w][tid] = 0;
    if (FUSED) {
        // digit tid: elements in earlier tiles and in all tiles
        uint32_t before = 0, total = 0;
        for (int b = 0; b < ntiles; ++b) {
            const uint32_t c = offs[(int64_t)tid * ntiles + b];
            before += b < (int)blockIdx.x ? c : 0u;
            total += c;
        }
        start[tid] = total;
        __syncthreads();
        scan256(start, gbase);
        __syncthreads();
        gbase[tid] += before;
    } else {
        gbase[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
        __syncthreads();
    }

    // per round: the lanes of this wave holding the same digit (8 ballots);
    // the lowest of them records the group size
    uint32_t dig[IPT];
    uint32_t below[IPT];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = base + r * kThreads + tid < n;
        const uint32_t d = valid ? dg(key[r], val[r]) : 0u;
        dig[r] = d;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        below[r] = (uint32_t)__popcll(peers & lt);
        if (valid && below[r] == 0) wcnt[r][wave][d] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // digit tid: exclusive prefix over (round, wave) in the tile's stable order
    {
        uint32_t acc = 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[r][w][tid];
                wcnt[r][w][tid] = acc;
                acc += c;
            }
        run[tid] = acc;
    }
    __syncthreads();
    scan256(run, start);
    __syncthreads();

#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (base + r * kThreads + tid < n) {
            const uint32_t p = start[dig[r]] + wcnt[r][wave][dig[r]] + below[r];
            skey[p] = key[r];
            sval[p] = val[r];
        }
    }
    __syncthreads();

    const int64_t rem = n - base;
    const int cnt = rem < (kThreads * IPT) ? (int)rem : (kThreads * IPT);
    for (int p = tid; p < cnt; p += kThreads) {
        const uint64_t k = skey[p];
        const uint32_t v = sval[p];
        const uint32_t d = dg(k, v);
        const int64_t dst = (int64_t)gbase[d] + (p - start[d]);
        kout[dst] = k;
        vout[dst] = v;
        if (FUSED && hnext) atomicAdd(&hnext[(int64_t)dnext(k, v) * ntiles + dst / (kThreads * IPT)], 1u);
    }
}

// A bucket of at most IPT * kThreads elements: all low passes in LDS.
template <int IPT>
__device__ inline void sort_bucket_lds(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                       uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t b0,
                                       uint32_t bn, int nlow, uint32_t *wcnt, uint32_t *run, uint32_t *start,
                                       uint64_t *skey, uint32_t *sval)
{
    const int tid = threadIdx.x;
    uint64_t key[IPT];
    uint32_t val[IPT], dig[IPT], pos[IPT];
    bool valid[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t i = (uint32_t)(r * kThreads + tid);
        valid[r] = i < bn;
        key[r] = valid[r] ? kin[b0 + i] : 0ull;
        val[r] = valid[r] ? vin[b0 + i] : 0u;
    }
    for (int p = 0; p < nlow; ++p) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) dig[r] = valid[r] ? (uint32_t)(key[r] >> (8 * p)) & (kRadix - 1) : 0u;
        rank_tile<IPT>(dig, valid, pos, wcnt, run, start);
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (valid[r]) {
                skey[pos[r]] = key[r];
                sval[pos[r]] = val[r];
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (valid[r]) {
                key[r] = skey[r * kThreads + tid];
                val[r] = sval[r * kThreads + tid];
            }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (valid[r]) {
            kout[b0 + r * kThreads + tid] = key[r];
            vout[b0 + r * kThreads + tid] = val[r];
        }
}

// A small bucket (at most 2 * kThreads keys, all with the same top digit):
// every key's place is the number of keys below it, equal keys counted by
// their index, i.e. the place of a stable sort by the whole key, which is
// what the low passes compute; the keys are read from LDS by all threads at
// the same index (broadcast).  About bn compares per thread instead of
// nlow stable ranking rounds.
__device__ inline void sort_bucket_count(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                         uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t b0,
                                         uint32_t bn, uint64_t *skey)
{
    const int tid = threadIdx.x;
    uint64_t key[2];
    uint32_t val[2], below[2] = {0u, 0u};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t i = (uint32_t)(r * kThreads + tid);
        key[r] = i < bn ? kin[b0 + i] : ~0ull;
        val[r] = i < bn ? vin[b0 + i] : 0u;
        if (i < bn) skey[i] = key[r];
    }
    __syncthreads();
    for (uint32_t j = 0; j < bn; ++j) {
        const uint64_t kj = skey[j];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t i = (uint32_t)(r * kThreads + tid);
            below[r] += (kj < key[r] || (kj == key[r] && j < i)) ? 1u : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t i = (uint32_t)(r * kThreads + tid);
        if (i < bn) {
            kout[b0 + below[r]] = key[r];
            vout[b0 + below[r]] = val[r];
        }
    }
}

// A larger bucket: the same stable low passes over its range in device
// memory, one histogram sweep and one tile-by-tile scatter sweep per pass,
// alternating between the range in kin and in kout (the result ends in kout).
__device__ inline void sort_bucket_global(uint64_t *__restrict__ kin, uint32_t *__restrict__ vin,
                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t b0,
                                          uint32_t bn, int nlow, uint32_t *wcnt, uint32_t *run, uint32_t *start,
                                          uint32_t *gcount, uint32_t *gbase)
{
    const int tid = threadIdx.x;
    uint64_t *ks = kin, *kd = kout;
    uint32_t *vs = vin, *vd = vout;
    for (int p = 0; p < nlow; ++p) {
        const int shift = 8 * p;
        gcount[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < bn; i += kThreads)
            atomicAdd(&gcount[(uint32_t)(ks[b0 + i] >> shift) & (kRadix - 1)], 1u);
        __syncthreads();
        // a digit that every element of the bucket shares changes no order
        if (gcount[(uint32_t)(ks[b0] >> shift) & (kRadix - 1)] == bn) {
            __syncthreads();
            continue;
        }
        scan256(gcount, gbase);
        __syncthreads();
        for (uint32_t c0 = 0; c0 < bn; c0 += kTile) {
            uint64_t key[kItems];
            uint32_t val[kItems], dig[kItems], pos[kItems];
            bool valid[kItems];
#pragma unroll
            for (int r = 0; r < kItems; ++r) {
                const uint32_t i = c0 + (uint32_t)(r * kThreads + tid);
                valid[r] = i < bn;
                key[r] = valid[r] ? ks[b0 + i] : 0ull;
                val[r] = valid[r] ? vs[b0 + i] : 0u;
                dig[r] = valid[r] ? (uint32_t)(key[r] >> shift) & (kRadix - 1) : 0u;
            }
            rank_tile<kItems>(dig, valid, pos, wcnt, run, start);
#pragma unroll
            for (int r = 0; r < kItems; ++r)
                if (valid[r]) {
                    const uint32_t dst = b0 + gbase[dig[r]] + (pos[r] - start[dig[r]]);
                    kd[dst] = key[r];
                    vd[dst] = val[r];
                }
            __syncthreads();
            gbase[tid] += run[tid];
            __syncthreads();
        }
        uint64_t *tk = ks; ks = kd; kd = tk;
        uint32_t *tv = vs; vs = vd; vd = tv;
    }
    if (ks != kout) {  // an even number of passes left the result in kin's range
        for (uint32_t i = tid; i < bn; i += kThreads) {
            kout[b0 + i] = ks[b0 + i];
            vout[b0 + i] = vs[b0 + i];
        }
    }
}

// One workgroup per top-digit bucket.  kin/vin hold the elements grouped
// by their top digit (stable); `hist` holds that digit's per-tile counts
// (digit-major), raw or (`scanned`) as the exclusive scan of the whole
// table, whose entry (d, tile 0) is bucket d's offset.  Each bucket is
// sorted by its `nlow` lower digits and written to the same offsets in
// kout/vout: in LDS up to kBucketLds elements, else over device memory.
constexpr int kBucketLds = 16 * kThreads;

__global__ __launch_bounds__(kThreads) void k_bucket_sort(uint64_t *__restrict__ kin, uint32_t *__restrict__ vin,
                                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                          const uint32_t *__restrict__ hist, int ntiles, int64_t n,
                                                          int scanned, int nlow)
{
    __shared__ uint32_t wcnt[16 * kWaves * kRadix];
    __shared__ uint32_t run[kRadix], start[kRadix], gcount[kRadix], gbase[kRadix];
    __shared__ uint64_t skey[kBucketLds];
    __shared__ uint32_t sval[kBucketLds];
    const int tid = threadIdx.x;
    uint32_t b0, bn;
    if (scanned) {
        const int d = blockIdx.x;
        b0 = hist[(int64_t)d * ntiles];
        const uint32_t end = d + 1 < kRadix ? hist[(int64_t)(d + 1) * ntiles] : (uint32_t)n;
        bn = end - b0;
    } else {
        // bucket sizes and offsets: digit tid's total over the tiles, scanned
        uint32_t tot = 0;
        for (int b = 0; b < ntiles; ++b) tot += hist[(int64_t)tid * ntiles + b];
        gcount[tid] = tot;
        __syncthreads();
        scan256(gcount, gbase);
        __syncthreads();
        b0 = gbase[blockIdx.x];
        bn = gcount[blockIdx.x];
        __syncthreads();
    }
    if (bn == 0) return;
    if (bn <= 2u * kThreads)
        sort_bucket_count(kin, vin, kout, vout, b0, bn, skey);
    else if (bn <= (uint32_t)kTile)
        sort_bucket_lds<kItems>(kin, vin, kout, vout, b0, bn, nlow, wcnt, run, start, skey, sval);
    else if (bn <= (uint32_t)kBucketLds)
        sort_bucket_lds<16>(kin, vin, kout, vout, b0, bn, nlow, wcnt, run, start, skey, sval);
    else
        sort_bucket_global(kin, vin, kout, vout, b0, bn, nlow, wcnt, run, start, gcount, gbase);
}

__global__ void k_copy_pairs(const uint64_t *__restrict__ ks, const uint32_t *__restrict__ vs,
                             uint64_t *__restrict__ kd, uint32_t *__restrict__ vd, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

}  // namespace

hipError_t ensure_sort_scratch(SortScratch &sc, int64_t n)
{
    hipError_t e = hipSuccess;
    if (n > sc.cap) {
        if (sc.keys_alt) (void)hipFree(sc.keys_alt);
        if (sc.vals_alt) (void)hipFree(sc.vals_alt);
        sc.keys_alt = nullptr;
        sc.vals_alt = nullptr;
        sc.cap = 0;
        if ((e = hipMalloc(&sc.keys_alt, sizeof(uint64_t) * n)) != hipSuccess) return e;
        if ((e = hipMalloc(&sc.vals_alt, sizeof(uint32_t) * n)) != hipSuccess) return e;
        sc.cap = n;
    }
    const int64_t ntiles = (n + kTile - 1) / kTile;
    // fused path: three rotating histograms; else one table plus the
    // partial sums of the three-launch scan
    const int64_t hn = (ntiles <= kFusedTiles ? 3 * kFusedTiles * kRadix
                                                  : ntiles * kRadix + (ntiles * kRadix + kScanChunk - 1) / kScanChunk);
    if (hn > sc.hist_cap) {
        if (sc.hist) (void)hipFree(sc.hist);
        sc.hist = nullptr;
        sc.hist_cap = 0;
        if ((e = hipMalloc(&sc.hist, sizeof(uint32_t) * hn)) != hipSuccess) return e;
        sc.hist_cap = hn;
    }
    return e;
}

void free_sort_scratch(SortScratch &sc)
{
    if (sc.keys_alt) (void)hipFree(sc.keys_alt);
    if (sc.vals_alt) (void)hipFree(sc.vals_alt);
    if (sc.hist) (void)hipFree(sc.hist);
    sc = SortScratch();
}

// The passes of a small sort (at most kFusedTiles tiles of kThreads * IPT):
// H[0] from k_hist (which also clears H[1]), then one scatter per pass.
template <int IPT>
void fused_passes(uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n, const Digit *passes, int np,
                  SortScratch &sc, hipStream_t s)
{
    const int ntiles = (int)((n + kThreads * IPT - 1) / (kThreads * IPT));
    const int64_t hsz = (int64_t)ntiles * kRadix;
    uint32_t *H[3] = {sc.hist, sc.hist + hsz, sc.hist + 2 * hsz};
    hipLaunchKernelGGL(k_hist<IPT>, dim3(ntiles), dim3(kThreads), 0, s, ka, va, n, passes[0], H[0], ntiles,
                       np > 1 ? H[1] : nullptr);
    for (int p = 0; p < np; ++p) {
        const Digit dn = p + 1 < np ? passes[p + 1] : passes[p];
        hipLaunchKernelGGL((k_scatter<true, IPT>), dim3(ntiles), dim3(kThreads), 0, s, ka, va, kb, vb, n, passes[p],
                           H[p % 3], ntiles, dn, p + 1 < np ? H[(p + 1) % 3] : nullptr,
                           p + 2 < np ? H[(p + 2) % 3] : nullptr);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
}

// Exclusive scan of a digit-major histogram table in place: one workgroup
// for small tables, else block sums, their scan and a rescan of each block.
static void scan_table(uint32_t *hist, int64_t hsz, hipStream_t s)
{
    if (hsz <= 4 * kScanChunk) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, hist, hsz);
    } else {
        const int64_t nparts = (hsz + kScanChunk - 1) / kScanChunk;
        uint32_t *part = hist + hsz;
        hipLaunchKernelGGL(k_part_sums, dim3((unsigned)nparts), dim3(256), 0, s, hist, hsz, part);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, part, nparts);
        hipLaunchKernelGGL(k_part_apply, dim3((unsigned)nparts), dim3(256), 0, s, hist, hsz, part);
    }
}

// Inputs up to kRadix * kBucketLarge keys take the bucket sort (an average
// bucket of at most kBucketLarge keys per workgroup).
constexpr uint32_t kBucketLarge = 16384;

hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, SortScratch &sc,
                            hipStream_t s, const int64_t *mesh_off, int32_t M, int first_bit, uint64_t **kres,
                            uint32_t **vres)
{
    if (kres) *kres = keys;
    if (vres) *vres = vals;
    if (n <= 1 || key_bits <= first_bit) return hipSuccess;
    hipError_t e = ensure_sort_scratch(sc, n);
    if (e != hipSuccess) return e;
    const int ntiles = (int)((n + kTile - 1) / kTile);
    // key digits first, then (batches) the mesh id as the most significant
    // digits, so each mesh's elements end up contiguous in key order
    Digit passes[16];
    int np = 0;
    for (int b = first_bit; b < key_bits; b += 8) passes[np++] = Digit{nullptr, 0, b};
    if (mesh_off && M > 1) {
        passes[np++] = Digit{mesh_off, M, 0};
        if (M > 256) passes[np++] = Digit{mesh_off, M, 8};
    }
    uint64_t *ka = keys, *kb = sc.keys_alt;
    uint32_t *va = vals, *vb = sc.vals_alt;
    const int64_t hsz = (int64_t)ntiles * kRadix;
    // Key digits by buckets: one stable pass on the top 8 bits groups the
    // elements into 256 buckets, then one workgroup per bucket sorts it by
    // the lower digits (k_bucket_sort), so three or four launches replace
    // one or more per digit.  Inputs up to kRadix * kBucketLarge keys take
    // this path without looking at the data (nothing is read back, so the
    // call stays stream-ordered and can be captured): buckets up to
    // kBucketLds keys sort in LDS, a larger one streams through device
    // memory inside its workgroup, which is slower but only meets meshes
    // whose triangles crowd into a few of the top-level Morton cells.
    int p0 = 0;  // first pass still to run
    if (key_bits > 8 && first_bit == 0) {
        const int top = key_bits - 8;
        const Digit dtop{nullptr, 0, top};
        const int nlow = (top + 7) / 8;
        if (ntiles <= kFusedTiles) {
            hipLaunchKernelGGL(k_hist<kItems>, dim3(ntiles), dim3(kThreads), 0, s, ka, va, n, dtop, sc.hist, ntiles,
                               nullptr);
            hipLaunchKernelGGL((k_scatter<true, kItems>), dim3(ntiles), dim3(kThreads), 0, s, ka, va, kb, vb, n,
                               dtop, sc.hist, ntiles, dtop, nullptr, nullptr);
            hipLaunchKernelGGL(k_bucket_sort, dim3(kRadix), dim3(kThreads), 0, s, kb, vb, ka, va, sc.hist, ntiles, n,
                               0, nlow);
            p0 = (key_bits + 7) / 8;
        } else if (n <= (int64_t)kRadix * kBucketLarge) {  // else even the average bucket is too large
            hipLaunchKernelGGL(k_hist<kItems>, dim3(ntiles), dim3(kThreads), 0, s, ka, va, n, dtop, sc.hist, ntiles,
                               nullptr);
            scan_table(sc.hist, hsz, s);
            hipLaunchKernelGGL((k_scatter<false, kItems>), dim3(ntiles), dim3(kThreads), 0, s, ka, va, kb, vb, n,
                               dtop, sc.hist, ntiles, dtop, nullptr, nullptr);
            hipLaunchKernelGGL(k_bucket_sort, dim3(kRadix), dim3(kThreads), 0, s, kb, vb, ka, va, sc.hist, ntiles, n,
                               1, nlow);
            p0 = (key_bits + 7) / 8;
        }
    }
    if (p0 == np) return hipGetLastError();
    if (ntiles <= kFusedTiles) {
        // (smaller tiles, hence more workgroups, measured slower: each
        // workgroup then scans more histograms and the next-pass counters
        // see more atomic traffic)
        fused_passes<kItems>(ka, va, kb, vb, n, passes + p0, np - p0, sc, s);
        if ((np - p0) & 1) {
            uint64_t *tk = ka; ka = kb; kb = tk;
            uint32_t *tv = va; va = vb; vb = tv;
        }
    } else {
        for (int p = p0; p < np; ++p) {
            const Digit dg = passes[p];
            hipLaunchKernelGGL(k_hist<kItems>, dim3(ntiles), dim3(kThreads), 0, s, ka, va, n, dg, sc.hist, ntiles,
                               nullptr);
            scan_table(sc.hist, hsz, s);
            hipLaunchKernelGGL((k_scatter<false, kItems>), dim3(ntiles), dim3(kThreads), 0, s, ka, va, kb, vb, n, dg,
                               sc.hist, ntiles, dg, nullptr, nullptr);
            uint64_t *tk = ka; ka = kb; kb = tk;
            uint32_t *tv = va; va = vb; vb = tv;
        }
    }
    if (kres && vres) {  // the caller takes the result where it is
        *kres = ka;
        *vres = va;
        return hipGetLastError();
    }
    if (ka != keys) {
        const int blk = 256;
        hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, s, ka, va, keys,
                           vals, n);
    }
    return hipGetLastError();
}

}  // namespace rsi
