// Stable LSD radix sort of (key, int32 value) pairs, 8-bit digits.
//
// One histogram kernel counts the digits of every pass at once (the global
// digit totals do not depend on the order of the keys).  Each pass is then a
// single kernel over 4096-key tiles: a tile scans the pass's digit totals
// itself (the output start of every digit), ranks its keys (wave ballots find
// the lanes sharing a digit, a per-wave LDS counter carries ranks across
// rounds), publishes its per-digit counts, and finds the number of keys with
// the same digit in all earlier tiles by looking back over their published
// counts (decoupled look-back: a tile publishes its own count before it
// waits, and earlier tiles publish running totals, so the look-back usually
// stops after a tile or two).  Tiles take their index from an atomic ticket,
// so a tile only ever waits for tiles that are already running.  A status word
// carries its own value, so relaxed device-scope atomics suffice.  The tile is
// staged in LDS in digit order and written out in contiguous runs.  Tile
// order = input order, so equal keys keep their input order (stable).
//
// Every wait is bounded: a look-back that spins past kSpinLimit polls sets a
// device error word, which the host checks at its next read-back; the kernel
// always runs to its end.
//
// The histogram and the first pass read their input through a source: plain
// key and value arrays, or an array of node pairs read as directed entries
// (entry 2i = (x_i <- y_i), entry 2i + 1 = (y_i <- x_i)), which spares the
// lists an expansion pass before the sort.
#include <algorithm>

#include "common.h"

namespace tfmm {
namespace {

constexpr int kLookBack = 8;      // earlier tiles read per look-back step
constexpr int RB = 256;           // threads per block (one digit per thread)
constexpr int RW = RB / kWave;    // waves per block
// keys per lane (16 for every key type: measured against 8 and 32)
template <typename K, bool HV> constexpr int keys_per_lane() { return 16; }
template <typename K, bool HV> constexpr int tile_keys() { return RB * keys_per_lane<K, HV>(); }
constexpr int RADIX = 256;
constexpr int MAXP = 8;          // passes of a 64-bit key
constexpr int kHistBlocks = 1024;
// Sorts of at least this many tiles run reduce-then-scan passes (count, scan,
// scatter), so that no tile waits on another (decoupled look-back over
// thousands of tiles costs more than the extra launches).
constexpr int kRtsMinTiles = 1024;
constexpr int kHistKeysPerThread = 16;  // fewer blocks, fewer global atomics
constexpr uint32_t kSpinLimit = 1u << 20;

// Tile status word: bits 62..63 flag (0 none, 1 own count, 2 running total
// including this tile), low 62 bits the value.
constexpr unsigned long long kFlagOwn = 1ull << 62;
constexpr unsigned long long kFlagTotal = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;

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

// Input sources.  load(i) gives entry i's key and value.
template <typename K>
struct ArraySrc {
    const K* k;
    const int32_t* v;
    __device__ __forceinline__ void load(int64_t i, K& key, int32_t& val) const {
        key = k[i];
        val = v[i];
    }
};

// Directed entries of node pairs.  With self_dummy set, the second entry of a
// pair (x, x) gets the key self_key (above every node id), so it sorts after
// all real entries.
struct PairSrc {
    const int2* p;
    uint32_t self_key;
    int self_dummy;
    __device__ __forceinline__ void load(int64_t i, uint32_t& key, int32_t& val) const {
        const int2 q = p[i >> 1];
        if (i & 1) {
            key = (self_dummy && q.x == q.y) ? self_key : (uint32_t)q.y;
            val = q.x;
        } else {
            key = (uint32_t)q.x;
            val = q.y;
        }
    }
};

// Keys alone.
template <typename K>
struct KeySrc {
    const K* k;
    __device__ __forceinline__ void load(int64_t i, K& key, int32_t& val) const {
        key = k[i];
        val = 0;
    }
};

// Directed entries of node pairs packed into one word, (target << 16) |
// source, for node ids below 2^16; no values.
struct PairPack16Src {
    const int2* p;
    __device__ __forceinline__ void load(int64_t i, uint32_t& key, int32_t& val) const {
        const int2 q = p[i >> 1];
        const uint32_t x = (uint32_t)q.x, y = (uint32_t)q.y;
        key = (i & 1) ? ((y << 16) | x) : ((x << 16) | y);
        val = 0;
    }
};

__global__ __launch_bounds__(RB) void zero_u64_kernel(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) p[i] = 0ull;
}

// Digit totals of every pass: LDS counters per block, then global atomics.
template <typename K, typename Src>
__global__ __launch_bounds__(RB) void radix_hist_all_kernel(Src src, int64_t n, int shift0, int passes,
                                                            uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[MAXP][RADIX];
    for (int p = 0; p < MAXP; ++p) h[p][threadIdx.x] = 0u;
    __syncthreads();
    constexpr int U = kHistKeysPerThread;  // loads in flight per thread
    const int64_t stride = (int64_t)gridDim.x * RB * U;
    for (int64_t base = (int64_t)blockIdx.x * RB * U; base < n; base += stride) {
        K k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * RB + threadIdx.x;
            int32_t unused;
            k[u] = (K)0;
            if (i < n) src.load(i, k[u], unused);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + (int64_t)u * RB + threadIdx.x < n) {
                for (int p = 0; p < passes; ++p)
                    atomicAdd(&h[p][(uint32_t)(k[u] >> (shift0 + 8 * p)) & (RADIX - 1)], 1u);
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * RADIX + threadIdx.x], c);
    }
}

template <typename K, bool HV, typename Src>
__global__ __launch_bounds__(RB) void radix_pass_kernel(Src src, K* __restrict__ kout, int32_t* __restrict__ vout,
                                                        int64_t n,
                                                        int shift, const uint32_t* __restrict__ dcount,
                                                        unsigned long long* __restrict__ status,
                                                        uint32_t* __restrict__ ticket, uint32_t* __restrict__ err) {
    __shared__ uint32_t wcnt[RW][RADIX];
    __shared__ uint32_t dstart[RADIX];
    __shared__ unsigned long long gbase[RADIX];
    constexpr int RI = keys_per_lane<K, HV>();
    constexpr int RTILE = tile_keys<K, HV>();
    __shared__ uint32_t wsum[RW];
    __shared__ uint32_t hsum[RW];
    __shared__ K skeys[RTILE];
    __shared__ int32_t svals[HV ? RTILE : 1];
    __shared__ uint32_t s_tile;

    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    const uint32_t hc = dcount[threadIdx.x];  // all keys with this thread's digit
    for (int ww = 0; ww < RW; ++ww) wcnt[ww][threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = s_tile;

    const int64_t tile0 = tile * RTILE;
    const int64_t wbase = tile0 + (int64_t)w * (kWave * RI);
    K k[RI];
    int32_t v[RI];
    uint32_t rank[RI];
    uint32_t dig[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        k[r] = (K)0;
        v[r] = 0;
        if (i < n) src.load(i, k[r], v[r]);
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)((k[r] >> shift) & (RADIX - 1)) : (uint32_t)RADIX - 1;
        dig[r] = d;
        const uint64_t peers = digit_peers(d);
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t base = wcnt[w][d];
        rank[r] = base + below;
        if (below == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // per digit: exclusive offsets across waves and the tile's count
    const int d = threadIdx.x;
    uint32_t tot = 0;
    for (int ww = 0; ww < RW; ++ww) {
        const uint32_t c = wcnt[ww][d];
        wcnt[ww][d] = tot;
        tot += c;
    }
    // padding keys of the last tile were counted under digit 255: drop them
    const int64_t rem = n - tile0;
    const int valid_count = (int)(rem < RTILE ? rem : RTILE);
    const uint32_t real = (d == RADIX - 1) ? tot - (uint32_t)(RTILE - valid_count) : tot;

    // publish, look back over earlier tiles, publish the running total
    unsigned long long* st = status + tile * RADIX;
    unsigned long long excl = 0;
    if (tile == 0) {
        __hip_atomic_store(&st[d], kFlagTotal | (unsigned long long)real, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(&st[d], kFlagOwn | (unsigned long long)real, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // earlier tiles' words for this digit, kLook at a time (independent loads)
        constexpr int kLook = kLookBack;
        uint32_t spins = 0;
        int64_t j = tile - 1;
        bool done = false;
        while (!done && j >= 0) {
            unsigned long long y[kLook];
#pragma unroll
            for (int b = 0; b < kLook; ++b)
                y[b] = (j - b >= 0) ? __hip_atomic_load(&status[(j - b) * RADIX + d], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : kFlagTotal;
            bool stalled = false;
#pragma unroll
            for (int b = 0; b < kLook; ++b) {
                if (done || stalled) continue;
                const unsigned long long flag = y[b] & ~kValMask;
                if (flag == 0ull) {
                    stalled = true;  // reload from tile j
                } else {
                    excl += y[b] & kValMask;
                    --j;
                    if (flag == kFlagTotal) done = true;
                }
            }
            if (stalled) {
                if (++spins > kSpinLimit) {
                    atomicOr(err, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(&st[d], kFlagTotal | (excl + real), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // digit starts inside the tile and in the output (scans over digits)
    uint32_t incl = tot, hincl = hc;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const uint32_t u = __shfl_up(incl, s, kWave);
        const uint32_t hu = __shfl_up(hincl, s, kWave);
        if (lane >= s) {
            incl += u;
            hincl += hu;
        }
    }
    if (lane == kWave - 1) {
        wsum[w] = incl;
        hsum[w] = hincl;
    }
    __syncthreads();
    uint32_t woff = 0, hoff = 0;
    for (int ww = 0; ww < w; ++ww) {
        woff += wsum[ww];
        hoff += hsum[ww];
    }
    dstart[d] = woff + incl - tot;
    gbase[d] = (unsigned long long)(hoff + hincl - hc) + excl;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const uint32_t pos = dstart[dig[r]] + wcnt[w][dig[r]] + rank[r];
        skeys[pos] = k[r];
        if constexpr (HV) svals[pos] = v[r];
    }
    __syncthreads();

    for (int i = threadIdx.x; i < valid_count; i += RB) {
        const K kk = skeys[i];
        const uint32_t dd = (uint32_t)((kk >> shift) & (RADIX - 1));
        const int64_t dst = (int64_t)gbase[dd] + (i - (int64_t)dstart[dd]);
        kout[dst] = kk;
        if constexpr (HV) vout[dst] = svals[i];
    }
}

// ---- reduce-then-scan passes (large inputs) --------------------------------
// With thousands of tiles in flight, the look-back's chain of device-scope
// reads sets the pace of a pass.  Large sorts therefore split a pass into
// three launches with no waits: every tile counts its digits
// (radix_up_kernel), one scan over the counts in digit-major order gives
// every (digit, tile) run its output start, and every tile ranks its keys
// again and scatters them (radix_down_kernel).  The tile layout and ranking
// are those of the single-kernel pass, so the order is the same (stable).

// ATOM: count with LDS adds (for digits that vary across neighbouring keys);
// otherwise one add per distinct digit of a row, found with ballots (for
// digits that repeat, where per-lane adds would serialise).
template <typename K, bool HV, bool ATOM, typename Src>
__global__ __launch_bounds__(RB) void radix_up_kernel(Src src, int64_t n, int shift, int64_t ntiles,
                                                      uint32_t* __restrict__ cnt) {
    constexpr int RI = keys_per_lane<K, HV>();
    constexpr int RTILE = tile_keys<K, HV>();
    __shared__ uint32_t wcnt[RW][RADIX];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int ww = 0; ww < RW; ++ww) wcnt[ww][threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = blockIdx.x;
    const int64_t wbase = tile * RTILE + (int64_t)w * (kWave * RI);
    K k[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        int32_t unused;
        k[r] = (K)0;
        if (i < n) src.load(i, k[r], unused);
    }
    if constexpr (ATOM) {
        // counts only: order does not matter (a row whose lanes all share one
        // digit adds once)
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const bool valid = wbase + (int64_t)r * kWave + lane < n;
            const uint32_t d = (uint32_t)((k[r] >> shift) & (RADIX - 1));
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            const uint64_t vm = __ballot(valid);
            if (__ballot(valid && d != d0) == 0ull) {
                if (lane == 0 && vm) wcnt[w][d0] += (uint32_t)__popcll(vm);
            } else if (valid) {
                atomicAdd(&wcnt[w][d], 1u);
            }
        }
    } else {
        const uint64_t lt = lanemask_lt();
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const bool valid = wbase + (int64_t)r * kWave + lane < n;
            const uint32_t d = (uint32_t)((k[r] >> shift) & (RADIX - 1));
            const uint64_t peers = digit_peers(d) & __ballot(valid);
            if (valid && (peers & lt) == 0ull) wcnt[w][d] += (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int ww = 0; ww < RW; ++ww) tot += wcnt[ww][threadIdx.x];
    cnt[(int64_t)threadIdx.x * ntiles + tile] = tot;
}

template <typename K, bool HV, typename Src>
__global__ __launch_bounds__(RB) void radix_down_kernel(Src src, K* __restrict__ kout, int32_t* __restrict__ vout,
                                                        int64_t n, int shift, int64_t ntiles,
                                                        const uint32_t* __restrict__ off) {
    constexpr int RI = keys_per_lane<K, HV>();
    constexpr int RTILE = tile_keys<K, HV>();
    __shared__ uint32_t wcnt[RW][RADIX];
    __shared__ uint32_t dstart[RADIX];
    __shared__ uint32_t gbase[RADIX];
    __shared__ uint32_t wsum[RW];
    __shared__ K skeys[RTILE];
    __shared__ int32_t svals[HV ? RTILE : 1];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int64_t tile = blockIdx.x;
    const uint32_t gb = off[(int64_t)threadIdx.x * ntiles + tile];  // output start of this tile's digit run
    for (int ww = 0; ww < RW; ++ww) wcnt[ww][threadIdx.x] = 0;
    __syncthreads();

    const int64_t tile0 = tile * RTILE;
    const int64_t wbase = tile0 + (int64_t)w * (kWave * RI);
    K k[RI];
    int32_t v[RI];
    uint32_t rank[RI];
    uint32_t dig[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        k[r] = (K)0;
        v[r] = 0;
        if (i < n) src.load(i, k[r], v[r]);
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int64_t i = wbase + (int64_t)r * kWave + lane;
        const uint32_t d = i < n ? (uint32_t)((k[r] >> shift) & (RADIX - 1)) : (uint32_t)RADIX - 1;
        dig[r] = d;
        const uint64_t peers = digit_peers(d);
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t base = wcnt[w][d];
        rank[r] = base + below;
        if (below == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    const int d = threadIdx.x;
    uint32_t tot = 0;
    for (int ww = 0; ww < RW; ++ww) {
        const uint32_t c = wcnt[ww][d];
        wcnt[ww][d] = tot;
        tot += c;
    }
    const int64_t rem = n - tile0;
    const int valid_count = (int)(rem < RTILE ? rem : RTILE);
    uint32_t incl = tot;
#pragma unroll
    for (int sh = 1; sh < kWave; sh <<= 1) {
        const uint32_t u = __shfl_up(incl, sh, kWave);
        if (lane >= sh) incl += u;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t woff = 0;
    for (int ww = 0; ww < w; ++ww) woff += wsum[ww];
    dstart[d] = woff + incl - tot;
    gbase[d] = gb;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const uint32_t pos = dstart[dig[r]] + wcnt[w][dig[r]] + rank[r];
        skeys[pos] = k[r];
        if constexpr (HV) svals[pos] = v[r];
    }
    __syncthreads();

    // padding keys of the last tile sit after every valid key (digit 255, last)
    for (int i = threadIdx.x; i < valid_count; i += RB) {
        const K kk = skeys[i];
        const uint32_t dd = (uint32_t)((kk >> shift) & (RADIX - 1));
        const int64_t dst = (int64_t)gbase[dd] + (i - (int64_t)dstart[dd]);
        kout[dst] = kk;
        if constexpr (HV) vout[dst] = svals[i];
    }
}

// Scratch layout: digit counts [MAXP][RADIX] u32, tickets [MAXP] u32 (padded),
// then the tile status words [passes][tiles][RADIX] u64.
struct SortScratch {
    uint32_t* dcount;
    uint32_t* ticket;
    unsigned long long* status;
    int64_t zero_words;  // u64 words to clear from the start of the scratch
};

SortScratch carve(void* scratch, int64_t n, int passes, int rtile) {
    const int64_t nb = cdiv(n > 0 ? n : 1, rtile);
    auto* base = static_cast<unsigned long long*>(scratch);
    SortScratch s;
    s.dcount = reinterpret_cast<uint32_t*>(base);                          // MAXP*RADIX u32 = 1024 u64
    s.ticket = reinterpret_cast<uint32_t*>(base + MAXP * RADIX / 2);      // 64 u64 of room
    s.status = base + MAXP * RADIX / 2 + 64;
    s.zero_words = MAXP * RADIX / 2 + 64 + (int64_t)passes * nb * RADIX;
    return s;
}

// Sorts n entries read from src by bits [shift0, shift0 + bits) of the key;
// pass ps writes (kout, vout) when the number of passes after it is even,
// else the alternate arrays, so the last pass always lands in (kout, vout).
// Without values (HV false) the value arrays are not touched.
template <typename K, bool HV, typename Src>
void radix_sort_run(Src src, K* kout, int32_t* vout, K* kalt, int32_t* valt, int64_t n, int shift0, int bits,
                    void* scratch, uint32_t* err, hipStream_t s) {
    constexpr int RTILE = tile_keys<K, HV>();
    const int passes = (bits + 7) / 8;
    const int nb = (int)cdiv(n, RTILE);
    if (nb >= kRtsMinTiles && (int64_t)nb * RADIX <= (int64_t)UINT32_MAX && n <= (int64_t)UINT32_MAX) {
        // reduce-then-scan: counts [RADIX][nb] (in place: output starts), then the scan's scratch
        auto* base = static_cast<uint32_t*>(scratch);
        uint32_t* total = base;  // the scan's total (unused)
        uint32_t* cnt = base + 64;
        void* sscr = cnt + round_up((int64_t)nb * RADIX, 64);
        const int64_t nc = (int64_t)nb * RADIX;
        for (int ps = 0; ps < passes; ++ps) {
            const bool to_out = ((passes - 1 - ps) & 1) == 0;
            K* ko = to_out ? kout : kalt;
            int32_t* vo = to_out ? vout : valt;
            const int shift = shift0 + 8 * ps;
            if (ps == 0) {
                hipLaunchKernelGGL((radix_up_kernel<K, HV, true, Src>), dim3(nb), dim3(RB), 0, s, src, n, shift,
                                   (int64_t)nb, cnt);
                TFMM_LAUNCHED();
                exclusive_scan_u32(cnt, cnt, nc, sscr, total, s);
                hipLaunchKernelGGL((radix_down_kernel<K, HV, Src>), dim3(nb), dim3(RB), 0, s, src, ko, vo, n, shift,
                                   (int64_t)nb, (const uint32_t*)cnt);
                TFMM_LAUNCHED();
            } else if constexpr (HV) {
                const ArraySrc<K> prev{to_out ? kalt : kout, to_out ? valt : vout};
                hipLaunchKernelGGL((radix_up_kernel<K, HV, false, ArraySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, n, shift,
                                   (int64_t)nb, cnt);
                TFMM_LAUNCHED();
                exclusive_scan_u32(cnt, cnt, nc, sscr, total, s);
                hipLaunchKernelGGL((radix_down_kernel<K, HV, ArraySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, ko, vo, n,
                                   shift, (int64_t)nb, (const uint32_t*)cnt);
                TFMM_LAUNCHED();
            } else {
                const KeySrc<K> prev{to_out ? kalt : kout};
                hipLaunchKernelGGL((radix_up_kernel<K, HV, false, KeySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, n, shift,
                                   (int64_t)nb, cnt);
                TFMM_LAUNCHED();
                exclusive_scan_u32(cnt, cnt, nc, sscr, total, s);
                hipLaunchKernelGGL((radix_down_kernel<K, HV, KeySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, ko, vo, n,
                                   shift, (int64_t)nb, (const uint32_t*)cnt);
                TFMM_LAUNCHED();
            }
        }
        return;
    }
    const SortScratch sc = carve(scratch, n, passes, RTILE);
    const unsigned zb = (unsigned)std::min<int64_t>(2048, cdiv(sc.zero_words, RB));
    hipLaunchKernelGGL(zero_u64_kernel, dim3(zb), dim3(RB), 0, s, static_cast<unsigned long long*>(scratch),
                       sc.zero_words);
    TFMM_LAUNCHED();
    const unsigned hb = (unsigned)std::min<int64_t>(kHistBlocks, cdiv(n, RB * kHistKeysPerThread));
    hipLaunchKernelGGL((radix_hist_all_kernel<K, Src>), dim3(hb), dim3(RB), 0, s, src, n, shift0, passes,
                       sc.dcount);
    TFMM_LAUNCHED();
    for (int ps = 0; ps < passes; ++ps) {
        const bool to_out = ((passes - 1 - ps) & 1) == 0;
        K* ko = to_out ? kout : kalt;
        int32_t* vo = to_out ? vout : valt;
        const uint32_t* db = sc.dcount + ps * RADIX;
        unsigned long long* st = sc.status + (int64_t)ps * nb * RADIX;
        const int shift = shift0 + 8 * ps;
        if (ps == 0) {
            hipLaunchKernelGGL((radix_pass_kernel<K, HV, Src>), dim3(nb), dim3(RB), 0, s, src, ko, vo, n, shift,
                               db, st, sc.ticket, err);
        } else if constexpr (HV) {
            // the previous pass wrote the other pair of arrays
            const ArraySrc<K> prev{to_out ? kalt : kout, to_out ? valt : vout};
            hipLaunchKernelGGL((radix_pass_kernel<K, HV, ArraySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, ko, vo, n,
                               shift, db, st, sc.ticket + ps, err);
        } else {
            const KeySrc<K> prev{to_out ? kalt : kout};
            hipLaunchKernelGGL((radix_pass_kernel<K, HV, KeySrc<K>>), dim3(nb), dim3(RB), 0, s, prev, ko, vo, n,
                               shift, db, st, sc.ticket + ps, err);
        }
        TFMM_LAUNCHED();
    }
}

template <typename K>
void radix_sort_impl(K* keys, int32_t* vals, K* keys_alt, int32_t* vals_alt, int64_t n, int bits, void* scratch,
                     uint32_t* err, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int passes = (bits + 7) / 8;
    if (passes & 1) {
        // an odd number of passes ends in the alternate arrays: sort from a
        // copy there back into the caller's arrays
        TFMM_HIP(hipMemcpyAsync(keys_alt, keys, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
        TFMM_HIP(hipMemcpyAsync(vals_alt, vals, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        radix_sort_run<K, true>(ArraySrc<K>{keys_alt, vals_alt}, keys, vals, keys_alt, vals_alt, n, 0, bits, scratch,
                                err, s);
    } else {
        radix_sort_run<K, true>(ArraySrc<K>{keys, vals}, keys, vals, keys_alt, vals_alt, n, 0, bits, scratch, err,
                                s);
    }
}

}  // namespace

size_t sort_scratch_bytes(int64_t n, int bits) {
    const int passes = bits <= 0 ? 1 : (bits + 7) / 8;
    const int rtile = std::min({tile_keys<uint32_t, true>(), tile_keys<uint32_t, false>(), tile_keys<uint64_t, true>()});
    const size_t onesweep = (size_t)carve(nullptr, n, passes, rtile).zero_words * 8 + 256;
    const int64_t nc = cdiv(n > 0 ? n : 1, rtile) * RADIX;
    const size_t rts = (size_t)(64 + round_up(nc, 64)) * 4 + scan_scratch_bytes(nc) + 256;
    return std::max(onesweep, rts);
}

void radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                    void* scratch, uint32_t* err, hipStream_t s) {
    radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, err, s);
}

void radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                    void* scratch, uint32_t* err, hipStream_t s) {
    radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, err, s);
}

void radix_sort_pairs(const int2* pairs, int64_t np, bool self_dummy, uint32_t self_key, uint32_t* keys,
                      int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int bits, void* scratch, uint32_t* err,
                      hipStream_t s) {
    const int64_t n = 2 * np;
    if (n <= 0) return;
    radix_sort_run<uint32_t, true>(PairSrc{pairs, self_key, self_dummy ? 1 : 0}, keys, vals, keys_alt, vals_alt, n,
                                   0, bits > 0 ? bits : 1, scratch, err, s);
}

void radix_sort_pairs_packed16(const int2* pairs, int64_t np, uint32_t* keys, uint32_t* keys_alt, int bits,
                               void* scratch, uint32_t* err, hipStream_t s) {
    const int64_t n = 2 * np;
    if (n <= 0) return;
    radix_sort_run<uint32_t, false>(PairPack16Src{pairs}, keys, nullptr, keys_alt, nullptr, n, 16,
                                    bits > 0 ? std::min(bits, 16) : 1, scratch, err, s);
}

}  // namespace tfmm
