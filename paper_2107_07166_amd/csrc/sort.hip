// Stable LSD radix sort of (key, int32 value) pairs, 8-bit digits.
//
// Per pass: a histogram kernel counts digits per 4096-key tile, a device scan
// turns the digit-major counts into global offsets, and a scatter kernel ranks
// every key inside its tile (wave ballots find the lanes sharing a digit, a
// per-wave LDS counter carries ranks across rounds), stages the tile in LDS in
// digit order and writes it out in contiguous runs.  Tile order = input order,
// so equal keys keep their input order (stable); with the identity as initial
// payload, ties are broken by the original index.
#include "common.h"

namespace tfmm {
namespace {

constexpr int RB = 256;          // threads per block
constexpr int RW = RB / kWave;   // waves per block
constexpr int RI = 16;           // keys per lane
constexpr int RTILE = RB * RI;   // keys per block
constexpr int RADIX = 256;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
}

// Lanes holding the same 8-bit digit (all 64 lanes must be active).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d) {
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

template <typename K>
__global__ __launch_bounds__(RB) void radix_hist_kernel(const K* __restrict__ kin, int64_t n, int shift,
                                                        uint32_t* __restrict__ hist, int nb) {
    __shared__ uint32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int64_t wbase = (int64_t)blockIdx.x * RTILE + (int64_t)w * (kWave * RI);
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)((kin[i] >> shift) & (RADIX - 1)) : (uint32_t)RADIX - 1;
        const uint64_t peers = digit_peers(d) & __ballot(valid);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(RB) void radix_scatter_kernel(const K* __restrict__ kin,
                                                           const int32_t* __restrict__ vin,
                                                           K* __restrict__ kout, int32_t* __restrict__ vout,
                                                           int64_t n, int shift,
                                                           const uint32_t* __restrict__ off, int nb) {
    __shared__ uint32_t wcnt[RW][RADIX];
    __shared__ uint32_t dstart[RADIX];
    __shared__ uint32_t gbase[RADIX];
    __shared__ uint32_t wsum[RW];
    __shared__ K skeys[RTILE];
    __shared__ int32_t svals[RTILE];

    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int ww = 0; ww < RW; ++ww) wcnt[ww][threadIdx.x] = 0;
    __syncthreads();

    const int64_t tile0 = (int64_t)blockIdx.x * RTILE;
    const int64_t wbase = tile0 + (int64_t)w * (kWave * RI);
    K k[RI];
    int32_t v[RI];
    uint32_t rank[RI];
    uint32_t dig[RI];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        k[r] = valid ? kin[i] : (K)0;
        v[r] = valid ? vin[i] : 0;
        const uint32_t d = valid ? (uint32_t)((k[r] >> shift) & (RADIX - 1)) : (uint32_t)RADIX - 1;
        dig[r] = d;
        const uint64_t peers = digit_peers(d);
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t base = wcnt[w][d];
        rank[r] = base + below;
        if (below == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // per digit: exclusive offsets across waves, then the digit totals' scan
    const int d = threadIdx.x;
    uint32_t tot = 0;
    for (int ww = 0; ww < RW; ++ww) {
        const uint32_t c = wcnt[ww][d];
        wcnt[ww][d] = tot;
        tot += c;
    }
    uint32_t incl = tot;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const uint32_t u = __shfl_up(incl, s, kWave);
        if (lane >= s) incl += u;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    gbase[d] = off[(int64_t)d * nb + blockIdx.x];
    __syncthreads();
    uint32_t woff = 0;
    for (int ww = 0; ww < w; ++ww) woff += wsum[ww];
    dstart[d] = woff + incl - tot;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const uint32_t pos = dstart[dig[r]] + wcnt[w][dig[r]] + rank[r];
        skeys[pos] = k[r];
        svals[pos] = v[r];
    }
    __syncthreads();

    const int64_t rem = n - tile0;
    const int valid_count = (int)(rem < RTILE ? rem : RTILE);
    for (int i = threadIdx.x; i < valid_count; i += RB) {
        const K kk = skeys[i];
        const uint32_t dd = (uint32_t)((kk >> shift) & (RADIX - 1));
        const int64_t dst = (int64_t)gbase[dd] + (i - (int64_t)dstart[dd]);
        kout[dst] = kk;
        vout[dst] = svals[i];
    }
}

template <typename K>
void radix_sort_impl(K* keys, int32_t* vals, K* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                     void* scratch, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int nb = (int)cdiv(n, RTILE);
    const int64_t nh = (int64_t)RADIX * nb;
    uint32_t* hist = static_cast<uint32_t*>(scratch);
    uint32_t* total = hist + round_up(nh, 64);
    void* scan_scr = total + 64;
    const int passes = (bits + 7) / 8;
    K* kin = keys;
    int32_t* vin = vals;
    K* kout = keys_alt;
    int32_t* vout = vals_alt;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(radix_hist_kernel<K>, dim3(nb), dim3(RB), 0, s, kin, n, shift, hist, nb);
        TFMM_LAUNCHED();
        exclusive_scan_u32(hist, hist, nh, scan_scr, total, s);
        hipLaunchKernelGGL(radix_scatter_kernel<K>, dim3(nb), dim3(RB), 0, s, kin, vin, kout, vout, n,
                           shift, (const uint32_t*)hist, nb);
        TFMM_LAUNCHED();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (kin != keys) {
        TFMM_HIP(hipMemcpyAsync(keys, kin, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
        TFMM_HIP(hipMemcpyAsync(vals, vin, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace

size_t sort_scratch_bytes(int64_t n) {
    const int64_t nb = cdiv(n > 0 ? n : 1, RTILE);
    const int64_t nh = (int64_t)RADIX * nb;
    return (size_t)(round_up(nh, 64) + 64) * sizeof(uint32_t) + scan_scratch_bytes(nh) + 256;
}

void radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n,
                    int bits, void* scratch, hipStream_t s) {
    radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s);
}

void radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
                    int bits, void* scratch, hipStream_t s) {
    radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s);
}

}  // namespace tfmm
