// order.hip -- Morton order of segments (the paper's v2.2 step, Section 4.1:
// rays sorted so that neighbouring threads follow similar paths through the
// tree).  The key of a segment is the octant of its direction (3 bits, most
// significant) above the 30-bit Morton code of its midpoint quantised to
// 2^10 levels per axis inside the midpoints' bounding box; the radix sort of
// the build orders (key, index) pairs stably.  A caller computes the order
// once and reuses it for every mesh the segments are tested against, and
// gathers the segments into that order (rsi_gather_segments).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsi_host.h"

namespace rsi {
namespace {

__global__ void k_seg_bounds_init(int32_t *b)
{
    if (threadIdx.x < 3) b[threadIdx.x] = 0x7FFFFFFF;      // ordered min
    else if (threadIdx.x < 6) b[threadIdx.x] = (int32_t)0x80000000;  // ordered max
}

// Bounding box of the midpoints (block min/max in LDS, one ordered-int
// atomic per block and bound).
__global__ __launch_bounds__(256) void k_seg_bounds(const float *__restrict__ S, const float *__restrict__ E,
                                                    int64_t n, int32_t *__restrict__ b)
{
    __shared__ int32_t lb[6][256];
    int32_t mn[3] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
    int32_t mx[3] = {(int32_t)0x80000000, (int32_t)0x80000000, (int32_t)0x80000000};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int k = 0; k < 3; ++k) {
            const int32_t m = float_to_ordered(0.5f * (S[3 * i + k] + E[3 * i + k]));
            mn[k] = m < mn[k] ? m : mn[k];
            mx[k] = m > mx[k] ? m : mx[k];
        }
    }
    for (int k = 0; k < 3; ++k) {
        lb[k][threadIdx.x] = mn[k];
        lb[3 + k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int k = 0; k < 3; ++k) {
                const int32_t a = lb[k][threadIdx.x + h], c = lb[3 + k][threadIdx.x + h];
                if (a < lb[k][threadIdx.x]) lb[k][threadIdx.x] = a;
                if (c > lb[3 + k][threadIdx.x]) lb[3 + k][threadIdx.x] = c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) atomicMin(&b[threadIdx.x], lb[threadIdx.x][0]);
    else if (threadIdx.x < 6) atomicMax(&b[threadIdx.x], lb[threadIdx.x][0]);
}

__device__ inline uint32_t spread10(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x30000FFu;
    v = (v | (v << 8)) & 0x300F00Fu;
    v = (v | (v << 4)) & 0x30C30C3u;
    v = (v | (v << 2)) & 0x9249249u;
    return v;
}

__global__ __launch_bounds__(256) void k_seg_keys(const float *__restrict__ S, const float *__restrict__ E,
                                                  int64_t n, const int32_t *__restrict__ b,
                                                  uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    uint32_t oct = 0;
    for (int k = 0; k < 3; ++k) {
        const float lo = ordered_to_float(b[k]), hi = ordered_to_float(b[3 + k]);
        const float m = 0.5f * (S[3 * i + k] + E[3 * i + k]);
        const float ext = hi - lo;
        float x = ext > 0.0f ? (m - lo) / ext * 1024.0f : 0.0f;
        x = fminf(fmaxf(x, 0.0f), 1023.0f);
        q[k] = (uint32_t)x;
        oct |= (E[3 * i + k] < S[3 * i + k] ? 1u : 0u) << k;
    }
    const uint32_t code = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
    keys[i] = ((uint64_t)oct << 30) | code;
    vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_gather_segments(const float *__restrict__ S, const float *__restrict__ E,
                                                         const int32_t *__restrict__ order, int64_t n,
                                                         float *__restrict__ So, float *__restrict__ Eo)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t i = order[k];
    if (i < 0 || i >= n) i = 0;  // every read stays inside S and E
    for (int c = 0; c < 3; ++c) {
        So[3 * k + c] = S[3 * i + c];
        Eo[3 * k + c] = E[3 * i + c];
    }
}

}  // namespace

hipError_t launch_segment_order(rsi_bvh *h, const float *S, const float *E, int64_t n, int32_t *order,
                                hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (h->seg_key_cap < n) {
        if (h->seg_keys) (void)hipFree(h->seg_keys);
        h->seg_keys = nullptr;
        h->seg_key_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&h->seg_keys), sizeof(uint64_t) * (size_t)n)) != hipSuccess)
            return e;
        h->seg_key_cap = n;
    }
    int32_t *b = h->scalars + kSegBounds;
    hipLaunchKernelGGL(k_seg_bounds_init, dim3(1), dim3(64), 0, s, b);
    int dev = 0, n_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4 * (int64_t)n_cu) blocks = 4 * (int64_t)n_cu;
    hipLaunchKernelGGL(k_seg_bounds, dim3((unsigned)blocks), dim3(256), 0, s, S, E, n, b);
    hipLaunchKernelGGL(k_seg_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, E, n, b, h->seg_keys,
                       reinterpret_cast<uint32_t *>(order));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return radix_sort_pairs(h->seg_keys, reinterpret_cast<uint32_t *>(order), n, 33, h->seg_sort, s);
}

hipError_t launch_gather_segments(rsi_bvh *h, const float *S, const float *E, const int32_t *order, int64_t n,
                                  float *So, float *Eo, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    (void)h;
    hipLaunchKernelGGL(k_gather_segments, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, E, order, n, So,
                       Eo);
    return hipGetLastError();
}

}  // namespace rsi
