// Device-wide exclusive prefix sums of uint32 values (modulo 2^32).
//
// Used for stream compaction in the octree build and the list building, where
// the scan keeps the compacted order identical to the input order
// (deterministic).  Two launches of 256-thread workgroups: the first writes
// every tile's total; the second has every tile add up the totals before it
// (at most kDirectTiles of them; larger inputs scan the totals themselves
// first, the same way) and scan its values from there.  No workgroup waits on
// another, no scratch word needs clearing between scans, and every workgroup
// is small, so a scan beside a long kernel on another stream still finds room
// on the device.  (A one-pass scan with decoupled look-back needed a clearing
// launch per scan and spent most of its time in the chain of look-backs; one
// large workgroup for the tile totals waited for whole compute units to
// drain.)  In-place use (in == out) is allowed: a tile is read whole before it
// is written.  The input may also be gathered: value i = val[idx[i]].
#include <algorithm>

#include "common.h"

namespace tfmm {
namespace {

constexpr int SB = 256;             // threads of a tile workgroup
constexpr int SI = 16;              // values per thread
constexpr int STILE = SB * SI;      // values per tile
constexpr int64_t kDirectTiles = 1024;

__device__ __forceinline__ int pad(int i) { return i + (i >> 5); }

struct ArrayIn {
    const uint32_t* p;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct GatherIn {
    const int32_t* idx;
    const int32_t* val;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const { return (uint32_t)val[idx[i]]; }
};

// Exclusive scan of the per-thread sums over a workgroup of B threads; the
// workgroup total lands in tot.  wsum: B / kWave words of LDS.
template <int B>
__device__ __forceinline__ uint32_t block_excl(uint32_t sum, uint32_t* wsum, uint32_t& tot) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += u;
    }
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    uint32_t woff = 0, t = 0;
#pragma unroll
    for (int q = 0; q < B / kWave; ++q) {
        if (q < wv) woff += wsum[q];
        t += wsum[q];
    }
    __syncthreads();
    tot = t;
    return woff + incl - sum;
}

// Scans the tile of B * SI values starting at t0 from base: coalesced loads
// transposed through LDS so that every thread owns SI consecutive values.
// Returns the tile total.
template <int B, typename In>
__device__ __forceinline__ uint32_t tile_scan(In in, uint32_t* out, int64_t n, int64_t t0, uint32_t base,
                                              uint32_t* sv, uint32_t* wsum) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = t0 + r * B + tid;
        sv[pad(r * B + tid)] = i < n ? in(i) : 0u;
    }
    __syncthreads();
    uint32_t x[SI];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        x[k] = sv[pad(tid * SI + k)];
        sum += x[k];
    }
    uint32_t tot;
    uint32_t run = base + block_excl<B>(sum, wsum, tot);
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        sv[pad(tid * SI + k)] = run;
        run += x[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = t0 + r * B + tid;
        if (i < n) out[i] = sv[pad(r * B + tid)];
    }
    __syncthreads();
    return tot;
}

// Sum over the workgroup (every thread gets it).
__device__ __forceinline__ uint32_t block_total(uint32_t x, uint32_t* wsum) {
    uint32_t tot;
    (void)block_excl<SB>(x, wsum, tot);
    return tot;
}

// Up to two scans of n values each in one launch (blockIdx.y picks the job).
template <typename In>
struct Job {
    In in;
    uint32_t* out;
    uint32_t* sums;          // tile totals (or, with prefix, their exclusive scan)
    uint32_t* total;
};

template <typename In>
__global__ __launch_bounds__(SB) void scan_reduce_kernel(Job<In> j0, Job<In> j1, int64_t n) {
    __shared__ uint32_t wsum[SB / kWave];
    const Job<In> j = blockIdx.y == 0 ? j0 : j1;
    const int64_t t0 = (int64_t)blockIdx.x * STILE;
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = t0 + r * SB + threadIdx.x;
        if (i < n) sum += j.in(i);
    }
    const uint32_t tot = block_total(sum, wsum);
    if (threadIdx.x == 0) j.sums[blockIdx.x] = tot;
}

// prefixed: sums already holds exclusive prefixes of the tile totals.
template <typename In>
__global__ __launch_bounds__(SB) void scan_down_kernel(Job<In> j0, Job<In> j1, int64_t n, bool prefixed) {
    __shared__ uint32_t sv[STILE + STILE / 32];
    __shared__ uint32_t wsum[SB / kWave];
    const Job<In> j = blockIdx.y == 0 ? j0 : j1;
    const int64_t b = blockIdx.x;
    uint32_t base;
    if (prefixed) {
        base = j.sums[b];
    } else {
        uint32_t x = 0;
        for (int64_t k = threadIdx.x; k < b; k += SB) x += j.sums[k];
        base = block_total(x, wsum);
    }
    const uint32_t tot = tile_scan<SB>(j.in, j.out, n, b * STILE, base, sv, wsum);
    if (b == (int64_t)gridDim.x - 1 && threadIdx.x == 0) *j.total = base + tot;
}

// Scratch: the tile totals of this level, then the next level's scratch.
template <typename In>
void scan_jobs(Job<In> j0, Job<In> j1, int jobs, int64_t n, void* scratch, hipStream_t s);

inline uint32_t* level_scratch(void* scratch, int64_t nb, int job) {
    return static_cast<uint32_t*>(scratch) + job * round_up(nb, 64);
}

template <typename In>
void scan_jobs(Job<In> j0, Job<In> j1, int jobs, int64_t n, void* scratch, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, cdiv(n, STILE));
    j0.sums = level_scratch(scratch, nb, 0);
    j1.sums = level_scratch(scratch, nb, jobs - 1);
    const dim3 g((unsigned)nb, (unsigned)jobs);
    hipLaunchKernelGGL((scan_reduce_kernel<In>), g, dim3(SB), 0, s, j0, j1, n);
    TFMM_LAUNCHED();
    const bool prefixed = nb > kDirectTiles;
    if (prefixed) {
        // the tile totals scanned in place (their own totals are not needed)
        void* next = level_scratch(scratch, nb, jobs);
        uint32_t* junk = static_cast<uint32_t*>(next);
        void* next2 = junk + 64;
        const Job<ArrayIn> k0{ArrayIn{j0.sums}, j0.sums, nullptr, junk};
        const Job<ArrayIn> k1{ArrayIn{j1.sums}, j1.sums, nullptr, junk + 1};
        scan_jobs(k0, k1, jobs, nb, next2, s);
    }
    hipLaunchKernelGGL((scan_down_kernel<In>), g, dim3(SB), 0, s, j0, j1, n, prefixed);
    TFMM_LAUNCHED();
}

template <typename In>
void scan_run(In in, uint32_t* out, int64_t n, void* scratch, uint32_t* total_dev, hipStream_t s) {
    const Job<In> j{in, out, nullptr, total_dev};
    scan_jobs(j, j, 1, n, scratch, s);
}

}  // namespace

// Two jobs' tile totals per level, 64 words between levels, three levels at most.
size_t scan_scratch_bytes(int64_t n) {
    size_t words = 0;
    int64_t nb = std::max<int64_t>(1, cdiv(n, STILE));
    for (int lv = 0; lv < 3; ++lv) {
        words += 2 * round_up(nb, 64) + 64;
        if (nb <= kDirectTiles) break;
        nb = cdiv(nb, STILE);
    }
    return words * 4 + 256;
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch, uint32_t* total_dev,
                        hipStream_t s) {
    scan_run(ArrayIn{in}, out, n, scratch, total_dev, s);
}

void exclusive_scan2_u32(const uint32_t* in0, uint32_t* out0, uint32_t* total0, const uint32_t* in1,
                         uint32_t* out1, uint32_t* total1, int64_t n, void* scratch, hipStream_t s) {
    const Job<ArrayIn> j0{ArrayIn{in0}, out0, nullptr, total0}, j1{ArrayIn{in1}, out1, nullptr, total1};
    scan_jobs(j0, j1, 2, n, scratch, s);
}

void exclusive_scan_gather_u32(const int32_t* idx, const int32_t* val, uint32_t* out, int64_t n, void* scratch,
                               uint32_t* total_dev, hipStream_t s) {
    scan_run(GatherIn{idx, val}, out, n, scratch, total_dev, s);
}

}  // namespace tfmm
