// Device-wide exclusive prefix sums of uint32 values, one pass.
//
// Used for stream compaction in the octree build and the tree walk, where the
// scan keeps the compacted order identical to the input order (deterministic).
// Tiles of 4096 values take their index from an atomic ticket, scan locally
// (coalesced loads transposed through LDS, 16 consecutive values per thread),
// publish their total, and add the totals of earlier tiles found by looking
// back over the published words (decoupled look-back, one wavefront reading 64
// earlier words at a time; a tile publishes before it waits and only waits
// for tiles already running).  Each wait is bounded:
// past kSpinLimit polls the device error word is set and the kernel ends.
// In-place use (in == out) is allowed.  The input may also be gathered:
// value i = val[idx[i]].
#include "common.h"

namespace tfmm {
namespace {

constexpr int SB = 256;            // threads per block
constexpr int SI = 16;             // values per thread
constexpr int STILE = SB * SI;     // values per tile
constexpr uint32_t kSpinLimit = 1u << 20;

constexpr unsigned long long kFlagOwn = 1ull << 62;
constexpr unsigned long long kFlagTotal = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;

__device__ __forceinline__ int pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(SB) void scan_zero_kernel(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * SB + threadIdx.x; i < n; i += (int64_t)gridDim.x * SB) p[i] = 0ull;
}

struct ArrayIn {
    const uint32_t* p;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct GatherIn {
    const int32_t* idx;
    const int32_t* val;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const { return (uint32_t)val[idx[i]]; }
};

template <typename In>
__global__ __launch_bounds__(SB) void scan_lookback_kernel(In in, uint32_t* out, int64_t n,
                                                           unsigned long long* __restrict__ status,
                                                           uint32_t* __restrict__ ticket,
                                                           uint32_t* __restrict__ total, uint32_t* __restrict__ err) {
    __shared__ uint32_t sv[STILE + STILE / 32];
    __shared__ uint32_t wsum[SB / kWave];
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t t0 = tile * STILE;
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = t0 + r * SB + tid;
        sv[pad(r * SB + tid)] = i < n ? in(i) : 0u;
    }
    __syncthreads();
    uint32_t x[SI];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        x[k] = sv[pad(tid * SI + k)];
        sum += x[k];
    }
    // block scan of the per-thread sums
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += u;
    }
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    uint32_t woff = 0, tile_total = 0;
#pragma unroll
    for (int q = 0; q < SB / kWave; ++q) {
        if (q < wv) woff += wsum[q];
        tile_total += wsum[q];
    }
    const uint32_t texcl = woff + incl - sum;

    // look-back by the first wavefront: lane k reads the word of tile - 1 - k
    if (wv == 0) {
        unsigned long long* st = status + tile;
        if (lane == 0)
            __hip_atomic_store(st, (tile == 0 ? kFlagTotal : kFlagOwn) | (unsigned long long)tile_total,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long excl = 0;
        int64_t j0 = tile - 1;
        uint32_t spins = 0;
        while (j0 >= 0) {
            const int64_t j = j0 - lane;
            // words before the first tile count as a zero running total
            const unsigned long long y =
                j >= 0 ? __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kFlagTotal;
            const unsigned long long flag = y & ~kValMask;
            const unsigned long long totm = __ballot(flag == kFlagTotal);
            const unsigned long long zerom = __ballot(flag == 0ull);
            const int first_total = totm ? __ffsll((long long)totm) - 1 : kWave;
            const unsigned long long need = first_total >= kWave - 1 ? ~0ull : ((2ull << first_total) - 1ull);
            if (zerom & need) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(err, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            unsigned long long v = ((need >> lane) & 1ull) ? (y & kValMask) : 0ull;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
            excl += v;
            if (first_total < kWave) break;
            j0 -= kWave;
        }
        if (lane == 0) {
            if (tile > 0)
                __hip_atomic_store(st, kFlagTotal | (excl + tile_total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = excl;
            if (t0 + STILE >= n) *total = (uint32_t)(excl + tile_total);
        }
    }
    __syncthreads();
    uint32_t run = (uint32_t)s_prefix + texcl;
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        sv[pad(tid * SI + k)] = run;
        run += x[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = t0 + r * SB + tid;
        if (i < n) out[i] = sv[pad(r * SB + tid)];
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) { return (size_t)(cdiv(n > 0 ? n : 1, STILE) + 64) * 8 + 256; }

template <typename In>
void scan_run(In in, uint32_t* out, int64_t n, void* scratch, uint32_t* total_dev, uint32_t* err, hipStream_t s) {
    const int64_t nb = cdiv(n > 0 ? n : 1, STILE);
    auto* words = static_cast<unsigned long long*>(scratch);
    uint32_t* ticket = reinterpret_cast<uint32_t*>(words);  // first 64 words: ticket
    unsigned long long* status = words + 64;
    const int64_t nz = 64 + nb;
    hipLaunchKernelGGL(scan_zero_kernel, dim3((unsigned)std::min<int64_t>(1024, cdiv(nz, SB))), dim3(SB), 0, s, words,
                       nz);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL((scan_lookback_kernel<In>), dim3((unsigned)nb), dim3(SB), 0, s, in, out, n, status, ticket,
                       total_dev, err);
    TFMM_LAUNCHED();
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch, uint32_t* total_dev,
                        uint32_t* err, hipStream_t s) {
    scan_run(ArrayIn{in}, out, n, scratch, total_dev, err, s);
}

void exclusive_scan_gather_u32(const int32_t* idx, const int32_t* val, uint32_t* out, int64_t n, void* scratch,
                               uint32_t* total_dev, uint32_t* err, hipStream_t s) {
    scan_run(GatherIn{idx, val}, out, n, scratch, total_dev, err, s);
}

}  // namespace tfmm
