// Device-wide exclusive prefix sums (reduce / scan-of-block-sums / down-sweep).
// Used for stream compaction in the octree build and the tree walk, where the
// scan keeps the compacted order identical to the input order (deterministic).
#include "common.h"

namespace tfmm {
namespace {

constexpr int SB = 256;            // threads per block
constexpr int SI = 8;              // items per thread
constexpr int STILE = SB * SI;     // items per block

__device__ __forceinline__ U3 operator+(U3 x, U3 y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }
__device__ __forceinline__ U3 vsub(U3 x, U3 y) { return {x.a - y.a, x.b - y.b, x.c - y.c}; }
__device__ __forceinline__ uint32_t vsub(uint32_t x, uint32_t y) { return x - y; }

template <typename V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ uint32_t vzero<uint32_t>() { return 0u; }
template <> __device__ __forceinline__ U3 vzero<U3>() { return {0u, 0u, 0u}; }

__device__ __forceinline__ uint32_t shfl_up(uint32_t v, int d) { return __shfl_up(v, d, kWave); }
__device__ __forceinline__ U3 shfl_up(U3 v, int d) {
    return {(uint32_t)__shfl_up(v.a, d, kWave), (uint32_t)__shfl_up(v.b, d, kWave),
            (uint32_t)__shfl_up(v.c, d, kWave)};
}

// Inclusive scan over the block of one value per thread; returns the inclusive
// prefix and writes the block total.
template <typename V>
__device__ V block_inclusive(V v, V& total, V* wsum) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        V u = shfl_up(v, d);
        if (lane >= d) v = v + u;
    }
    if (lane == kWave - 1) wsum[w] = v;
    __syncthreads();
    V off = vzero<V>();
    V tot = vzero<V>();
#pragma unroll
    for (int i = 0; i < SB / kWave; ++i) {
        V x = wsum[i];
        if (i < w) off = off + x;
        tot = tot + x;
    }
    __syncthreads();
    total = tot;
    return off + v;
}

template <typename V>
__global__ __launch_bounds__(SB) void scan_reduce_kernel(const V* __restrict__ in, int64_t n,
                                                         V* __restrict__ bsum) {
    __shared__ V wsum[SB / kWave];
    const int64_t base = (int64_t)blockIdx.x * STILE + (int64_t)threadIdx.x * SI;
    V s = vzero<V>();
#pragma unroll
    for (int i = 0; i < SI; ++i)
        if (base + i < n) s = s + in[base + i];
    V tot;
    block_inclusive(s, tot, wsum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block scans the block sums (exclusive, in place) and writes the total.
template <typename V>
__global__ __launch_bounds__(SB) void scan_top_kernel(V* __restrict__ bsum, int64_t nb,
                                                      V* __restrict__ total) {
    __shared__ V wsum[SB / kWave];
    V carry = vzero<V>();
    for (int64_t c0 = 0; c0 < nb; c0 += STILE) {
        const int64_t base = c0 + (int64_t)threadIdx.x * SI;
        V loc[SI];
        V s = vzero<V>();
#pragma unroll
        for (int i = 0; i < SI; ++i) {
            loc[i] = (base + i < nb) ? bsum[base + i] : vzero<V>();
            s = s + loc[i];
        }
        V tot;
        const V incl = block_inclusive(s, tot, wsum);
        V start = carry + vsub(incl, s);
#pragma unroll
        for (int i = 0; i < SI; ++i) {
            if (base + i < nb) bsum[base + i] = start;
            start = start + loc[i];
        }
        carry = carry + tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

template <typename V>
__global__ __launch_bounds__(SB) void scan_down_kernel(const V* __restrict__ in, V* __restrict__ out,
                                                       int64_t n, const V* __restrict__ bsum) {
    __shared__ V wsum[SB / kWave];
    const int64_t base = (int64_t)blockIdx.x * STILE + (int64_t)threadIdx.x * SI;
    V loc[SI];
    V s = vzero<V>();
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        loc[i] = (base + i < n) ? in[base + i] : vzero<V>();
        s = s + loc[i];
    }
    V tot;
    const V incl = block_inclusive(s, tot, wsum);
    V start = bsum[blockIdx.x] + vsub(incl, s);
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        if (base + i < n) out[base + i] = start;
        start = start + loc[i];
    }
}

template <typename V>
void scan_impl(const V* in, V* out, int64_t n, void* scratch, V* total, hipStream_t s) {
    const int64_t nb = cdiv(n > 0 ? n : 1, STILE);
    V* bsum = static_cast<V*>(scratch);
    hipLaunchKernelGGL(scan_reduce_kernel<V>, dim3((unsigned)nb), dim3(SB), 0, s, in, n, bsum);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(scan_top_kernel<V>, dim3(1), dim3(SB), 0, s, bsum, nb, total);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(scan_down_kernel<V>, dim3((unsigned)nb), dim3(SB), 0, s, in, out, n,
                       (const V*)bsum);
    TFMM_LAUNCHED();
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    return (size_t)round_up(cdiv(n > 0 ? n : 1, STILE) * (int64_t)sizeof(U3), 256);
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                        uint32_t* total_dev, hipStream_t s) {
    scan_impl<uint32_t>(in, out, n, scratch, total_dev, s);
}

void exclusive_scan_u3(const U3* in, U3* out, int64_t n, void* scratch, U3* total_dev,
                       hipStream_t s) {
    scan_impl<U3>(in, out, n, scratch, total_dev, s);
}

}  // namespace tfmm
