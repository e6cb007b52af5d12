// Mutual dual-tree walk and per-target interaction lists.
//
// The walk processes a frontier of unordered node pairs level-synchronously
// from (root, root) (one such pair per set of a forest; the children of a
// pair belong to its set, so nodes of different sets never meet, and each
// set may have its own theta).  For each pair:
//   A == B : a leaf gives a near (P2P) self pair; otherwise the children
//            pairs (c_i, c_j), i <= j, join the next frontier;
//   A != B : R = sqrt((dx*dx + dy*dy) + dz*dz), d = Z_A - Z_B.  The pair is a
//            far (M2L) pair iff R > 0 and r_A + r_B <= theta * R
//            (Eq. mac_criterion with theta = tan of the MAC angle); else two
//            leaves give a near pair; else one node is split (the non-leaf
//            if one is a leaf, else the larger r_max, then the lower level,
//            then the lower index) and its children are paired with the other.
// Counts are compacted with prefix sums, so the emitted lists are in a fixed
// order and the pair sets do not depend on scheduling.  FP64 without
// contraction so that every decision is reproducible.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>

#include "common.h"

namespace tfmm {
namespace {

constexpr int TB = 256;

// Per node, packed for the walk: geo = (centre of mass x, y, z, r_max),
// top = (child count, level, first child, set).  theta: per set (forests
// walked with several thetas), else nullptr and the passes' scalar applies.
struct WalkNodes {
    const double4* geo;
    const int4* top;
    const double* theta;
};

__global__ __launch_bounds__(TB) void walk_nodes_kernel(int64_t nn, const double4* __restrict__ Z,
                                                        const double* __restrict__ rmax,
                                                        const int32_t* __restrict__ nchild,
                                                        const int32_t* __restrict__ level,
                                                        const int32_t* __restrict__ child_first,
                                                        const int32_t* __restrict__ first,
                                                        const int64_t* __restrict__ set_off, int n_sets,
                                                        double4* __restrict__ geo, int4* __restrict__ top) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nn) return;
    const double4 z = Z[i];
    geo[i] = make_double4(z.x, z.y, z.z, rmax[i]);
    top[i] = make_int4(nchild[i], level[i], child_first[i], set_of(set_off, n_sets, first[i]));
}

struct Decision {
    int kind;      // 0 near, 1 far, 2 expand self, 3 split S against O
    int32_t S, O;  // for kind 3
    uint32_t nnew;
};

__device__ __forceinline__ Decision decide(const WalkNodes& w, int32_t A, int32_t B, double theta) {
    Decision d{0, -1, -1, 0u};
    const int4 ta = w.top[A];
    if (A == B) {
        const int32_t nc = ta.x;
        if (nc == 0) {
            d.kind = 0;
        } else {
            d.kind = 2;
            d.nnew = (uint32_t)(nc * (nc + 1) / 2);
        }
        return d;
    }
    const int4 tb = w.top[B];
    const double4 ga = w.geo[A], gb = w.geo[B];
    const double dx = ga.x - gb.x, dy = ga.y - gb.y, dz = ga.z - gb.z;
    const double R = sqrt((dx * dx + dy * dy) + dz * dz);
    const double ra = ga.w, rb = gb.w;
    const double th = w.theta ? w.theta[ta.w] : theta;
    if (R > 0.0 && ra + rb <= th * R) {
        d.kind = 1;
        return d;
    }
    const int32_t na = ta.x, nb = tb.x;
    if (na == 0 && nb == 0) {
        d.kind = 0;
        return d;
    }
    int32_t S;
    if (na == 0) S = B;
    else if (nb == 0) S = A;
    else if (ra > rb) S = A;
    else if (rb > ra) S = B;
    else if (ta.y < tb.y) S = A;
    else if (tb.y < ta.y) S = B;
    else S = A < B ? A : B;
    d.kind = 3;
    d.S = S;
    d.O = (S == A) ? B : A;
    d.nnew = (uint32_t)((S == A) ? na : nb);
    return d;
}


__device__ __forceinline__ U3 u3add(U3 x, U3 y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }

// Pass totals are carried in 64 bits so that a pass too large for 32-bit
// offsets is detected instead of wrapping.
struct U3L {
    unsigned long long a, b, c;
};
__device__ __forceinline__ U3L u3ladd(U3L x, U3 y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }
__device__ __forceinline__ U3L u3ladd(U3L x, U3L y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }

// Exclusive scan over the block (every thread calls it); the block total is
// returned in tot.  The shared array may be reused right after the call.
__device__ __forceinline__ U3 block_excl_scan(U3 c, U3* wsum, U3& tot) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    U3 v = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        U3 u{(uint32_t)__shfl_up(v.a, d, kWave), (uint32_t)__shfl_up(v.b, d, kWave),
             (uint32_t)__shfl_up(v.c, d, kWave)};
        if (lane >= d) v = u3add(v, u);
    }
    if (lane == kWave - 1) wsum[wv] = v;
    __syncthreads();
    U3 base{0u, 0u, 0u}, t{0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < TB / kWave; ++k) {
        if (k < wv) base = u3add(base, wsum[k]);
        t = u3add(t, wsum[k]);
    }
    __syncthreads();
    tot = t;
    return U3{base.a + v.a - c.a, base.b + v.b - c.b, base.c + v.c - c.c};
}

// Sum over the block (every thread calls it and gets the total).
__device__ __forceinline__ U3L block_sum(U3L x, U3L* wsum) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        x.a += __shfl_xor(x.a, d, kWave);
        x.b += __shfl_xor(x.b, d, kWave);
        x.c += __shfl_xor(x.c, d, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = x;
    __syncthreads();
    U3L t{0ull, 0ull, 0ull};
#pragma unroll
    for (int k = 0; k < TB / kWave; ++k) t = u3ladd(t, wsum[k]);
    __syncthreads();
    return t;
}

// ---- frontier passes ----------------------------------------------------------
// A pass has two kernels (the unsynchronised walk fuses them for small
// frontiers, below).  The counting kernel decides every frontier pair,
// stores the decision and scans the output counts (next-frontier pairs, far
// pairs, near pairs) inside its block; the emitting kernel adds the totals of
// the blocks before it and writes the outputs.  Block b of a pass takes a
// contiguous range of frontier tiles, so the outputs follow the frontier
// order whatever the grid: children of a pair in a fixed order (a self pair
// gives (c_a, c_b) for a <= b, row major; a split gives (c_a, O)).
//
// The frontier size and the running list lengths live on the device, double
// buffered by pass parity (a pass reads slot p and writes slot 1 - p), so
// passes can be queued without reading anything back.  A pass whose outputs
// would not fit sets a sticky flag and writes nothing; later passes then see
// an empty frontier.
constexpr int kMaxPasses = 64;  // a walk needs at most 2 * 21 + 1 passes
struct WalkState {
    uint32_t nf[2];
    uint32_t overflow;
    uint32_t passes;  // passes that found a non-empty frontier
    uint32_t max_nf;  // largest frontier seen
    uint32_t pad;
    unsigned long long n_far[2], n_near[2];
    uint32_t nf_pass[kMaxPasses];  // frontier size of every pass (sizes the next walk's grids)
    uint32_t ticket[kMaxPasses];   // tile tickets of the fused passes
};
constexpr int kWalkGrid = 1024;

__device__ __forceinline__ void block_tiles(uint32_t nf, int64_t& t0, int64_t& t1) {
    const int64_t tiles = ((int64_t)nf + TB - 1) / TB;
    const int64_t per = (tiles + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * per;
    t1 = t0 + per < tiles ? t0 + per : tiles;
}

// The first frontier: (k, k) for the root k of every set.
__global__ void walk_init_kernel(WalkState* __restrict__ st, int2* __restrict__ fr, int n_roots) {
    if (threadIdx.x == 0) {
        st->nf[0] = (uint32_t)n_roots;
        st->nf[1] = 0u;
        st->overflow = 0u;
        st->passes = 0u;
        st->max_nf = (uint32_t)n_roots;
        st->pad = 0u;
        st->n_far[0] = st->n_far[1] = 0ull;
        st->n_near[0] = st->n_near[1] = 0ull;
    }
    for (int k = threadIdx.x; k < n_roots; k += blockDim.x) fr[k] = make_int2(k, k);
    for (int k = threadIdx.x; k < kMaxPasses; k += blockDim.x) {
        st->nf_pass[k] = 0u;
        st->ticket[k] = 0u;
    }
}

__global__ __launch_bounds__(TB) void zero_words_kernel(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) p[i] = 0ull;
}

// Decision code: bits 0-1 kind (0 near, 1 far, 2 expand self, 3 split);
// bit 2 set when the split node is the pair's second node.
__global__ __launch_bounds__(TB) void walk_count_pass_kernel(WalkNodes w, const int2* __restrict__ fr,
                                                             const WalkState* __restrict__ st, int parity,
                                                             double theta, uint8_t* __restrict__ dec,
                                                             U3L* __restrict__ bsum) {
    __shared__ U3L wsum[TB / kWave];
    const uint32_t nf = st->overflow ? 0u : st->nf[parity];
    int64_t t0, t1;
    block_tiles(nf, t0, t1);
    U3L c{0ull, 0ull, 0ull};
    const int64_t iend = t1 * TB < (int64_t)nf ? t1 * TB : (int64_t)nf;
    for (int64_t i = t0 * TB + threadIdx.x; i < iend; i += TB) {
        const int2 pr = fr[i];
        const Decision d = decide(w, pr.x, pr.y, theta);
        if (d.kind == 0) c.c += 1u;
        else if (d.kind == 1) c.b += 1u;
        else c.a += d.nnew;
        dec[i] = (uint8_t)(d.kind | ((d.kind == 3 && d.S == pr.y) ? 4 : 0));
    }
    const U3L tot = block_sum(c, wsum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Sum of the block totals of a pass (one block), for the host-sized passes.
__global__ __launch_bounds__(TB) void walk_total_kernel(const U3L* __restrict__ bsum, int nb,
                                                        U3L* __restrict__ total) {
    __shared__ U3L wsum[TB / kWave];
    U3L x{0ull, 0ull, 0ull};
    for (int j = threadIdx.x; j < nb; j += TB) x = u3ladd(x, bsum[j]);
    const U3L t = block_sum(x, wsum);
    if (threadIdx.x == 0) *total = t;
}

// Every block sums the block totals itself (the pass total and its own
// offset), so no scan launch sits between counting and emitting; offsets
// inside the block come from a scan of the counts, recomputed from the
// stored decisions.
__global__ __launch_bounds__(TB) void walk_emit_pass_kernel(WalkNodes w, const int2* __restrict__ fr,
                                                            WalkState* __restrict__ st, int pass,
                                                            const uint8_t* __restrict__ dec,
                                                            const U3L* __restrict__ bsum,
                                                            int2* __restrict__ next, int2* __restrict__ far,
                                                            int2* __restrict__ near, uint32_t cap_next,
                                                            unsigned long long cap_far,
                                                            unsigned long long cap_near) {
    __shared__ U3L wsum[TB / kWave];
    __shared__ U3 wsum3[TB / kWave];
    U3L before{0ull, 0ull, 0ull}, all{0ull, 0ull, 0ull};
    for (int j = threadIdx.x; j < (int)gridDim.x; j += TB) {
        const U3L x = bsum[j];
        all = u3ladd(all, x);
        if (j < (int)blockIdx.x) before = u3ladd(before, x);
    }
    const U3L T = block_sum(all, wsum);
    const U3L B = block_sum(before, wsum);
    const int parity = pass & 1;
    const uint32_t nf = st->overflow ? 0u : st->nf[parity];
    const unsigned long long far0 = st->n_far[parity], near0 = st->n_near[parity];
    const unsigned long long lim = 0xffffffffull;
    const bool ovf = T.a > cap_next || T.b > lim || T.c > lim || far0 + T.b > cap_far || near0 + T.c > cap_near;
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    if (ovf) {
        if (leader) {
            st->overflow = 1u;
            st->nf[parity ^ 1] = 0u;
        }
        return;
    }
    if (leader) {
        st->nf[parity ^ 1] = (uint32_t)T.a;
        st->n_far[parity ^ 1] = far0 + T.b;
        st->n_near[parity ^ 1] = near0 + T.c;
        if (nf > 0u) st->passes += 1u;
        if ((uint32_t)T.a > st->max_nf) st->max_nf = (uint32_t)T.a;
        if (pass < kMaxPasses) st->nf_pass[pass] = nf;
    }
    int64_t t0, t1;
    block_tiles(nf, t0, t1);
    U3L carry = B;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t i = t * TB + threadIdx.x;
        int2 pr = make_int2(0, 0);
        int kind = -1;
        int32_t S = 0, O = 0, c0 = 0, nc = 0;
        U3 c{0u, 0u, 0u};
        if (i < (int64_t)nf) {
            pr = fr[i];
            const int code = dec[i];
            kind = code & 3;
            if (kind == 0) {
                c.c = 1u;
            } else if (kind == 1) {
                c.b = 1u;
            } else {
                S = (kind == 3 && (code & 4)) ? pr.y : pr.x;
                O = (S == pr.x) ? pr.y : pr.x;
                const int4 tp = w.top[S];
                c0 = tp.z;
                nc = tp.x;
                c.a = kind == 2 ? (uint32_t)(nc * (nc + 1) / 2) : (uint32_t)nc;
            }
        }
        U3 tot;
        const U3 e = block_excl_scan(c, wsum3, tot);
        if (kind >= 0) {
            const U3L o = u3ladd(carry, e);
            const int32_t lo = pr.x < pr.y ? pr.x : pr.y, hi = pr.x < pr.y ? pr.y : pr.x;
            if (kind == 0) {
                near[near0 + o.c] = make_int2(lo, hi);
            } else if (kind == 1) {
                far[far0 + o.b] = make_int2(lo, hi);
            } else if (kind == 2) {
                int2* q = next + o.a;
                for (int32_t x = 0; x < nc; ++x)
                    for (int32_t y = x; y < nc; ++y) *q++ = make_int2(c0 + x, c0 + y);
            } else {
                int2* q = next + o.a;
                for (int32_t x = 0; x < nc; ++x) q[x] = make_int2(c0 + x, O);
            }
        }
        carry = u3ladd(carry, tot);
    }
}

// ---- fused frontier pass ---------------------------------------------------
// One kernel per pass for the unsynchronised walk: a block takes tiles of
// kPassTile frontier pairs in ticket order, decides them, scans the three
// output counts inside the block, and finds the counts of all earlier tiles
// by decoupled look-back over per-tile status words (one word per count).
// Outputs land in frontier order, exactly as with the two-kernel pass.
// A status word holds (epoch << 44) | (flag << 42) | value; a word written by
// another pass carries another epoch and reads as unpublished, so the words
// need no clearing between passes.  The tile that comes last writes the pass
// totals into the state; with an empty frontier block 0 does.
constexpr int kPassPPT = 2;                    // consecutive pairs per thread
constexpr int kPassTile = TB * kPassPPT;       // pairs per tile
constexpr int kEpochBits = 20;
constexpr unsigned long long kPstOwn = 1ull << 42;
constexpr unsigned long long kPstTotal = 2ull << 42;
constexpr unsigned long long kPstVal = (1ull << 42) - 1;
constexpr uint32_t kPassSpinLimit = 1u << 20;
constexpr int kPassGrid = 2048;                // blocks of a fused pass (at most)
// Passes expected to hold at most this many pairs run fused.  Look-back over
// many tiles costs more than the second launch saves, so larger passes keep
// the two-kernel form.
constexpr int64_t kFuseMaxPairs = 4096;

__device__ __forceinline__ unsigned long long pst_word(uint32_t epoch, unsigned long long flag,
                                                       unsigned long long v) {
    return ((unsigned long long)epoch << 44) | flag | v;
}

__device__ __forceinline__ void pass_state_write(WalkState* st, int pass, uint32_t nf, U3L T,
                                                 unsigned long long far0, unsigned long long near0,
                                                 uint32_t cap_next, unsigned long long cap_far,
                                                 unsigned long long cap_near) {
    const int parity = pass & 1;
    const unsigned long long lim = 0xffffffffull;
    const bool ovf = T.a > cap_next || T.b > lim || T.c > lim || far0 + T.b > cap_far || near0 + T.c > cap_near;
    if (ovf) {
        st->overflow = 1u;
        st->nf[parity ^ 1] = 0u;
        return;
    }
    st->nf[parity ^ 1] = (uint32_t)T.a;
    st->n_far[parity ^ 1] = far0 + T.b;
    st->n_near[parity ^ 1] = near0 + T.c;
    if (nf > 0u) st->passes += 1u;
    if ((uint32_t)T.a > st->max_nf) st->max_nf = (uint32_t)T.a;
    if (pass < kMaxPasses) st->nf_pass[pass] = nf;
}

__global__ __launch_bounds__(TB) void walk_pass_kernel(WalkNodes w, const int2* __restrict__ fr,
                                                       WalkState* __restrict__ st, int pass, double theta,
                                                       int2* __restrict__ next, int2* __restrict__ far,
                                                       int2* __restrict__ near, uint32_t cap_next,
                                                       unsigned long long cap_far, unsigned long long cap_near,
                                                       unsigned long long* __restrict__ pst, uint32_t cap_tiles,
                                                       uint32_t epoch, uint32_t* __restrict__ err) {
    __shared__ U3 wsum[TB / kWave];
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_pre[3];
    const int parity = pass & 1;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nf = st->nf[parity];
    const unsigned long long far0 = st->n_far[parity], near0 = st->n_near[parity];
    const uint32_t ntiles = (uint32_t)(((uint64_t)nf + kPassTile - 1) / kPassTile);
    if (ntiles == 0u || ntiles > cap_tiles) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (ntiles == 0u) {
                pass_state_write(st, pass, 0u, U3L{0ull, 0ull, 0ull}, far0, near0, cap_next, cap_far, cap_near);
            } else {
                st->overflow = 1u;
                st->nf[parity ^ 1] = 0u;
            }
        }
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&st->ticket[pass], 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;

        // decide this thread's pairs (consecutive in the frontier)
        const int64_t i0 = (int64_t)tile * kPassTile + (int64_t)threadIdx.x * kPassPPT;
        int2 pr[kPassPPT];
        Decision dc[kPassPPT];
        U3 c{0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < kPassPPT; ++q) {
            dc[q] = Decision{-1, -1, -1, 0u};
            if (i0 + q < (int64_t)nf) {
                pr[q] = fr[i0 + q];
                dc[q] = decide(w, pr[q].x, pr[q].y, theta);
                if (dc[q].kind == 0) c.c += 1u;
                else if (dc[q].kind == 1) c.b += 1u;
                else c.a += dc[q].nnew;
            }
        }
        U3 tot;
        const U3 e = block_excl_scan(c, wsum, tot);

        // publish the tile's counts, then look back (first wavefront)
        if (threadIdx.x < kWave) {
            unsigned long long* my = pst + (size_t)tile * 3;
            const unsigned long long f0 = tile == 0u ? kPstTotal : kPstOwn;
            if (lane == 0) {
                __hip_atomic_store(&my[0], pst_word(epoch, f0, tot.a), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&my[1], pst_word(epoch, f0, tot.b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&my[2], pst_word(epoch, f0, tot.c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            unsigned long long acc[3] = {0ull, 0ull, 0ull};
            bool done[3] = {tile == 0u, tile == 0u, tile == 0u};
            int64_t j0 = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (j0 >= 0 && !(done[0] && done[1] && done[2])) {
                const int64_t j = j0 - lane;
                unsigned long long y[3];
                uint64_t need[3];
                int ft[3];
                bool stall = false;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    y[k] = 0ull;
                    need[k] = 0ull;
                    ft[k] = kWave;
                    if (done[k]) continue;
                    // words before the first tile count as a zero running total
                    y[k] = j >= 0 ? __hip_atomic_load(&pst[j * 3 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : pst_word(epoch, kPstTotal, 0ull);
                    const bool cur = (uint32_t)(y[k] >> 44) == epoch;
                    const unsigned long long flag = cur ? (y[k] & (3ull << 42)) : 0ull;
                    const uint64_t totm = __ballot(flag == kPstTotal);
                    const uint64_t zerom = __ballot(flag == 0ull);
                    ft[k] = totm ? __ffsll((long long)totm) - 1 : kWave;
                    need[k] = ft[k] >= kWave - 1 ? ~0ull : ((2ull << ft[k]) - 1ull);
                    if (zerom & need[k]) stall = true;
                }
                if (stall) {
                    if (++spins > kPassSpinLimit) {
                        if (lane == 0) atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (done[k]) continue;
                    unsigned long long v = ((need[k] >> lane) & 1ull) ? (y[k] & kPstVal) : 0ull;
#pragma unroll
                    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
                    acc[k] += v;
                    if (ft[k] < kWave) done[k] = true;
                }
                j0 -= kWave;
            }
            if (lane == 0) {
                if (tile > 0u) {
                    __hip_atomic_store(&my[0], pst_word(epoch, kPstTotal, acc[0] + tot.a), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&my[1], pst_word(epoch, kPstTotal, acc[1] + tot.b), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&my[2], pst_word(epoch, kPstTotal, acc[2] + tot.c), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
                s_pre[0] = acc[0];
                s_pre[1] = acc[1];
                s_pre[2] = acc[2];
            }
        }
        __syncthreads();
        const U3L P{s_pre[0], s_pre[1], s_pre[2]};
        const bool fits = P.a + tot.a <= cap_next && far0 + P.b + tot.b <= cap_far &&
                          near0 + P.c + tot.c <= cap_near;
        if (!fits) {
            if (threadIdx.x == 0) atomicOr(&st->overflow, 1u);
        } else {
            unsigned long long on = P.a + e.a, ofar = far0 + P.b + e.b, onear = near0 + P.c + e.c;
#pragma unroll
            for (int q = 0; q < kPassPPT; ++q) {
                const Decision d = dc[q];
                if (d.kind < 0) continue;
                const int32_t lo = pr[q].x < pr[q].y ? pr[q].x : pr[q].y;
                const int32_t hi = pr[q].x < pr[q].y ? pr[q].y : pr[q].x;
                if (d.kind == 0) {
                    near[onear++] = make_int2(lo, hi);
                } else if (d.kind == 1) {
                    far[ofar++] = make_int2(lo, hi);
                } else if (d.kind == 2) {
                    const int4 tp = w.top[pr[q].x];
                    const int32_t c0 = tp.z, nc = tp.x;
                    int2* o = next + on;
                    for (int32_t x = 0; x < nc; ++x)
                        for (int32_t yy = x; yy < nc; ++yy) *o++ = make_int2(c0 + x, c0 + yy);
                    on += d.nnew;
                } else {
                    const int4 tp = w.top[d.S];
                    const int32_t c0 = tp.z, nc = tp.x;
                    int2* o = next + on;
                    for (int32_t x = 0; x < nc; ++x) o[x] = make_int2(c0 + x, d.O);
                    on += d.nnew;
                }
            }
        }
        if (tile == ntiles - 1u && threadIdx.x == 0)
            pass_state_write(st, pass, nf, U3L{P.a + tot.a, P.b + tot.b, P.c + tot.c}, far0, near0, cap_next,
                             cap_far, cap_near);
        __syncthreads();
    }
}

// CSR offsets from targets sorted ascending (target = keys[i] >> shift):
// off[t] = first entry with target >= t, for t = 0..nn.  Entry boundary i
// (0..ne) writes off[t] for targets t in (target[i-1], target[i]], so each t
// is written by exactly one boundary, which also copies off[nn] (the number
// of entries below nn) to *below_nn if given.  Targets may equal nn (entries
// sorted after every real one).  A thread takes four boundaries and reads
// their keys with one 16-byte load.
__global__ __launch_bounds__(TB) void csr_offsets_kernel(const uint32_t* __restrict__ keys, int64_t ne,
                                                         int64_t nn, int shift, uint32_t* __restrict__ off,
                                                         uint32_t* __restrict__ below_nn) {
    const int64_t i0 = ((int64_t)blockIdx.x * TB + threadIdx.x) * 4;
    if (i0 > ne) return;
    int64_t kv[5];  // targets of entries i0 - 1 .. i0 + 3 (-1 before the first, nn after the last)
    kv[0] = i0 == 0 ? -1 : (int64_t)(keys[i0 - 1] >> shift);
    if (i0 + 4 <= ne) {
        const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
        kv[1] = q.x >> shift;
        kv[2] = q.y >> shift;
        kv[3] = q.z >> shift;
        kv[4] = q.w >> shift;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) kv[j + 1] = i0 + j < ne ? (int64_t)(keys[i0 + j] >> shift) : nn;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = i0 + j;
        if (i > ne) break;
        const int64_t lo = kv[j] + 1;
        const int64_t hi = kv[j + 1] < nn ? kv[j + 1] : nn;
        for (int64_t t = lo; t <= hi; ++t) off[t] = (uint32_t)i;
        if (below_nn && lo <= nn && nn <= hi) *below_nn = (uint32_t)i;
    }
}

__global__ __launch_bounds__(TB) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) p[i] = v;
}

// Directed near particle interactions: sum over directed leaf pairs of
// n_t * n_s (self pairs n (n - 1)).
__global__ __launch_bounds__(TB) void near_work_kernel(const uint32_t* __restrict__ tgt,
                                                       const int32_t* __restrict__ src, int64_t ne,
                                                       const int32_t* __restrict__ count,
                                                       unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sh[TB];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < ne; i += (int64_t)gridDim.x * TB) {
        const int32_t a = (int32_t)tgt[i], b = src[i];
        const unsigned long long na = (unsigned long long)count[a];
        s += (a == b) ? na * (na - 1) : na * (unsigned long long)count[b];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = TB / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, sh[0]);
}


// ---- near-field work items -------------------------------------------------
// A target leaf's near list is cut before entry q when the number of source
// particles preceding q in that list crosses a multiple of kItemSources, so no
// wavefront receives more than about kItemSources sources per target.  (The
// prefix is taken modulo 2^32; only differences inside one list are used.)
constexpr uint32_t kItemSources = 4096;

// Items of a node's near list: entry q (list start q0) belongs to item
// k = floor((P[q] - P[q0]) / kItemSources) of its leaf.  A source leaf holds
// at most 4096 particles, so k grows by at most one per entry and a list
// with last entry q1 - 1 has k_last + 1 items.  Only a leaf split into
// several items needs partial-sum rows (one per item and target particle).
__global__ __launch_bounds__(TB) void node_items_kernel(const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ P, int64_t nn,
                                                        const int32_t* __restrict__ count,
                                                        uint32_t* __restrict__ nitems, uint32_t* __restrict__ prows) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nn) return;
    const uint32_t q0 = off[i], q1 = off[i + 1];
    const uint32_t n = (q1 > q0) ? (P[q1 - 1] - P[q0]) / kItemSources + 1u : 0u;
    nitems[i] = n;
    prows[i] = n > 1u ? n * (uint32_t)count[i] : 0u;
}

// One thread per item (grid-stride over the item count on the device): its
// leaf is the last node whose first item is at or before it (nodes without
// items share their first-item index with the next node); item k of a list
// starts at its first entry q with P[q] - P[q0] >= k kItemSources (P grows
// along a list, by at most kItemSources per entry, so every item has a first
// entry), found by binary search, and ends where item k + 1 starts.
__device__ __forceinline__ uint32_t item_start(const uint32_t* __restrict__ P, uint32_t q0, uint32_t q1,
                                               uint32_t k) {
    if (k == 0u) return q0;
    const uint32_t p0 = P[q0], want = k * kItemSources;
    uint32_t lo = q0 + 1u, hi = q1 - 1u;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (P[mid] - p0 >= want) hi = mid;
        else lo = mid + 1u;
    }
    return lo;
}

__global__ __launch_bounds__(TB) void item_write_kernel(const uint32_t* __restrict__ P,
                                                        const uint32_t* __restrict__ off, int64_t nn,
                                                        const uint32_t* __restrict__ nitems,
                                                        const uint32_t* __restrict__ item0,
                                                        const uint32_t* __restrict__ n_items,
                                                        const uint32_t* __restrict__ pbase,
                                                        const int32_t* __restrict__ count,
                                                        int32_t* __restrict__ it_leaf, uint32_t* __restrict__ it_q0,
                                                        uint32_t* __restrict__ it_q1, uint32_t* __restrict__ it_pbase,
                                                        int32_t* __restrict__ leaf_item0,
                                                        int32_t* __restrict__ leaf_nitems,
                                                        int32_t* __restrict__ multi_leaf,
                                                        uint32_t* __restrict__ multi_count) {
    const uint32_t total = *n_items;
    for (uint32_t i = (uint32_t)(blockIdx.x * TB + threadIdx.x); i < total; i += gridDim.x * TB) {
        int64_t lo = 0, hi = nn - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (item0[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const int64_t L = lo;
        const uint32_t n = nitems[L], k = i - item0[L];
        const uint32_t q0 = off[L], q1 = off[L + 1];
        it_leaf[i] = (int32_t)L;
        it_q0[i] = item_start(P, q0, q1, k);
        it_q1[i] = k + 1u < n ? item_start(P, q0, q1, k + 1u) : q1;
        it_pbase[i] = n > 1u ? pbase[L] + k * (uint32_t)count[L] : 0u;
        if (k == 0u) {
            leaf_item0[L] = (int32_t)item0[L];
            leaf_nitems[L] = (int32_t)n;
            if (n > 1u) multi_leaf[atomicAdd(multi_count, 1u)] = (int32_t)L;
        }
    }
}

unsigned grid(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, TB); }

int bits_for(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

// Stable sort by target of the directed entries of np node pairs (read
// straight from the pair array), then CSR offsets from the sorted targets.
// With self_dummy, the second entry of a self pair gets key nn and sorts
// last, so the first off[nn] entries are the real ones; off[nn] is also
// written to *real_out if given.  The sources of every target stay in the
// walk's emission order.
void build_csr_pairs(Tree& t, const DevBuf& pairs, int64_t np, bool self_dummy, DevBuf& tgtbuf, DevBuf& srcbuf,
                     DevBuf& off, DevBuf& srcout, DevBuf& scr, DevBuf& scr2, uint32_t* real_out, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    const int64_t ne = 2 * np;
    const int64_t room = std::max<int64_t>(ne, 1);
    tgtbuf.ensure(ctx, (size_t)room * 4);
    srcbuf.ensure(ctx, (size_t)room * 4);
    scr2.ensure(ctx, (size_t)room * 8 + 256);
    uint32_t* kalt = scr2.as<uint32_t>();
    int32_t* valt = reinterpret_cast<int32_t*>(kalt + room);
    const int bits = bits_for(self_dummy ? nn + 1 : nn);
    scr.ensure(ctx, sort_scratch_bytes(ne, bits) + 1024);
    radix_sort_pairs(pairs.as<int2>(), np, self_dummy, (uint32_t)nn, tgtbuf.as<uint32_t>(), srcbuf.as<int32_t>(),
                     kalt, valt, bits, scr.p, ctx->dev_err, s);
    off.ensure(ctx, (size_t)(nn + 1) * 4);
    hipLaunchKernelGGL(csr_offsets_kernel, dim3(grid(cdiv(ne + 1, 4))), dim3(TB), 0, s,
                       (const uint32_t*)tgtbuf.as<uint32_t>(), ne, nn, 0, off.as<uint32_t>(), real_out);
    TFMM_LAUNCHED();
    std::swap(srcbuf.p, srcout.p);
    std::swap(srcbuf.cap, srcout.cap);
    std::swap(srcbuf.ctx, srcout.ctx);
}

// The far lists with node ids below 2^16: entries packed as (target << 16) |
// source and sorted as single words (half the bytes of separate arrays); the
// sorted words become the source list, read through the mask 0xffff.
void build_far_csr_packed(Tree& t, int64_t np, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    const int64_t ne = 2 * np;
    const int64_t room = std::max<int64_t>(ne, 1);
    t.w_tg.ensure(ctx, (size_t)room * 4);
    t.scratch2.ensure(ctx, (size_t)room * 4 + 256);
    const int bits = bits_for(nn);
    t.scratch.ensure(ctx, sort_scratch_bytes(ne, bits) + 1024);
    radix_sort_pairs_packed16(t.m2l_pairs.as<int2>(), np, t.w_tg.as<uint32_t>(), t.scratch2.as<uint32_t>(), bits,
                              t.scratch.p, ctx->dev_err, s);
    t.m2l_off.ensure(ctx, (size_t)(nn + 1) * 4);
    hipLaunchKernelGGL(csr_offsets_kernel, dim3(grid(cdiv(ne + 1, 4))), dim3(TB), 0, s,
                       (const uint32_t*)t.w_tg.as<uint32_t>(), ne, nn, 16, t.m2l_off.as<uint32_t>(), nullptr);
    TFMM_LAUNCHED();
    std::swap(t.w_tg.p, t.m2l_src.p);
    std::swap(t.w_tg.cap, t.m2l_src.cap);
    std::swap(t.w_tg.ctx, t.m2l_src.ctx);
    t.m2l_src_mask = 0xffffu;
}

// Frontier passes sized on the host: the totals of every pass are read back
// and the buffers grown before its outputs are written.  Used for the first
// walk of a tree and whenever the unsynchronised passes ran out of room.
void walk_bfs_sized(Tree& t, const WalkNodes& w, double theta, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    int64_t cap_far = (int64_t)(t.m2l_pairs.cap / 8), cap_near = (int64_t)(t.p2p_pairs.cap / 8);
    if (cap_far < 4096) {
        cap_far = std::max<int64_t>(4096, 64 * nn);
        t.m2l_pairs.ensure(ctx, (size_t)cap_far * 8);
    }
    if (cap_near < 4096) {
        cap_near = std::max<int64_t>(4096, 16 * nn);
        t.p2p_pairs.ensure(ctx, (size_t)cap_near * 8);
    }
    t.w_fr.ensure(ctx, (size_t)std::max(4096, t.n_sets) * 8);
    t.w_off.ensure(ctx, (size_t)kWalkGrid * sizeof(U3L));
    t.w_state.ensure(ctx, sizeof(WalkState));
    t.scratch2.ensure(ctx, 256);
    WalkState* st = t.w_state.as<WalkState>();
    U3L* tot = t.scratch2.as<U3L>();
    hipLaunchKernelGGL(walk_init_kernel, dim3(1), dim3(TB), 0, s, st, t.w_fr.as<int2>(), t.n_sets);
    TFMM_LAUNCHED();
    DevBuf* cur = &t.w_fr;
    DevBuf* nxt = &t.w_fr2;
    int64_t nf = t.n_sets, max_nf = t.n_sets, n_far = 0, n_near = 0;
    t.walk_hint_nf.clear();
    for (int k = 0; nf > 0; ++k) {
        const int parity = k & 1;
        t.walk_hint_nf.push_back(nf);
        const unsigned g = (unsigned)std::min<int64_t>(kWalkGrid, cdiv(nf, TB));
        // buffers resized here are idle: a resize waits for the device
        t.w_dec.ensure(ctx, (size_t)nf);
        hipLaunchKernelGGL(walk_count_pass_kernel, dim3(g), dim3(TB), 0, s, w, (const int2*)cur->as<int2>(),
                           (const WalkState*)st, parity, theta, t.w_dec.as<uint8_t>(), t.w_off.as<U3L>());
        TFMM_LAUNCHED();
        hipLaunchKernelGGL(walk_total_kernel, dim3(1), dim3(TB), 0, s, (const U3L*)t.w_off.as<U3L>(), (int)g, tot);
        TFMM_LAUNCHED();
        const U3L T = read_back(ctx, (const U3L*)tot, s);
        if (T.a > UINT32_MAX || T.b > UINT32_MAX || T.c > UINT32_MAX)
            fail(TFMM_ENOMEM, "walk: one frontier pass would emit more than 2^32 pairs");
        if (n_far + (int64_t)T.b > cap_far) {
            cap_far = std::max<int64_t>(2 * cap_far, n_far + (int64_t)T.b);
            t.m2l_pairs.ensure_keep(ctx, (size_t)cap_far * 8, s);
        }
        if (n_near + (int64_t)T.c > cap_near) {
            cap_near = std::max<int64_t>(2 * cap_near, n_near + (int64_t)T.c);
            t.p2p_pairs.ensure_keep(ctx, (size_t)cap_near * 8, s);
        }
        nxt->ensure(ctx, (size_t)std::max<unsigned long long>(T.a, 1) * 8);
        const size_t cap_next = std::min<size_t>(nxt->cap / 8, UINT32_MAX);
        hipLaunchKernelGGL(walk_emit_pass_kernel, dim3(g), dim3(TB), 0, s, w, (const int2*)cur->as<int2>(), st, k,
                           (const uint8_t*)t.w_dec.as<uint8_t>(), (const U3L*)t.w_off.as<U3L>(), nxt->as<int2>(), t.m2l_pairs.as<int2>(),
                           t.p2p_pairs.as<int2>(), (uint32_t)cap_next, (unsigned long long)(t.m2l_pairs.cap / 8),
                           (unsigned long long)(t.p2p_pairs.cap / 8));
        TFMM_LAUNCHED();
        n_far += (int64_t)T.b;
        n_near += (int64_t)T.c;
        nf = (int64_t)T.a;
        max_nf = std::max(max_nf, nf);
        std::swap(cur, nxt);
    }
    const WalkState h = read_back(ctx, (const WalkState*)st, s);
    if (h.overflow)
        fail(TFMM_EDEVICE, "walk: a host-sized frontier pass reported an overflow");
    t.n_m2l = n_far;
    t.n_p2p = n_near;
    t.walk_hint_fr = max_nf;
}

// Frontier passes with no host synchronisation (small ones fused into one
// kernel), sized from the previous walk of this tree plus a quarter.  A pair's level sum grows by at least one per
// expansion, a non-leaf sits above the deepest level and a pair of leaves is
// never expanded, so every frontier after pass 2 max_level is empty; the host
// checks that, and the overflow flag, once at the end.  Returns false (lists
// invalid) when the host-sized passes must be used instead.
bool walk_bfs_async(Tree& t, const WalkNodes& w, double theta, hipStream_t s) {
    Ctx* ctx = t.ctx;
    if (t.walk_hint_fr <= 0) return false;
    const int64_t want_fr = t.walk_hint_fr + t.walk_hint_fr / 4 + 4096;
    const int64_t want_far = t.walk_hint_far + t.walk_hint_far / 4 + 4096;
    const int64_t want_near = t.walk_hint_near + t.walk_hint_near / 4 + 4096;
    if (want_fr > (int64_t)UINT32_MAX) return false;
    t.w_fr.ensure(ctx, (size_t)want_fr * 8);
    t.w_fr2.ensure(ctx, (size_t)want_fr * 8);
    t.w_dec.ensure(ctx, (size_t)want_fr);
    t.w_off.ensure(ctx, (size_t)kWalkGrid * sizeof(U3L));
    t.m2l_pairs.ensure(ctx, (size_t)want_far * 8);
    t.p2p_pairs.ensure(ctx, (size_t)want_near * 8);
    t.w_state.ensure(ctx, sizeof(WalkState));
    const size_t cap_next = std::min({t.w_fr.cap / 8, t.w_fr2.cap / 8, t.w_dec.cap, (size_t)UINT32_MAX});
    const unsigned long long cap_far = t.m2l_pairs.cap / 8, cap_near = t.p2p_pairs.cap / 8;
    const int passes = 2 * t.max_level + 1;
    if (passes > kMaxPasses) return false;
    // tile status words (three per tile); cleared when new and when the pass
    // epoch would wrap, so a stale word never carries the current epoch
    const uint32_t cap_tiles = (uint32_t)cdiv((int64_t)cap_next, kPassTile);
    void* old_pst = t.w_pst.p;
    t.w_pst.ensure(ctx, (size_t)cap_tiles * 3 * 8);
    if (t.w_pst.p != old_pst || t.w_epoch + (uint32_t)passes >= (1u << kEpochBits)) {
        const int64_t nw = (int64_t)(t.w_pst.cap / 8);
        hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)std::min<int64_t>(1024, cdiv(nw, TB))), dim3(TB), 0, s,
                           t.w_pst.as<unsigned long long>(), nw);
        TFMM_LAUNCHED();
        t.w_epoch = 0;
    }
    WalkState* st = t.w_state.as<WalkState>();
    hipLaunchKernelGGL(walk_init_kernel, dim3(1), dim3(TB), 0, s, st, t.w_fr.as<int2>(), t.n_sets);
    TFMM_LAUNCHED();
    int64_t bound = t.n_sets;  // a pass's frontier is at most 36 times the previous one
    for (int k = 0; k < passes; ++k) {
        const int parity = k & 1;
        // grid from this pass's frontier in the previous walk (any grid covers
        // any frontier; a small one keeps small passes cheap)
        int64_t expect = bound;
        if (k < (int)t.walk_hint_nf.size()) expect = std::min(bound, t.walk_hint_nf[k] + t.walk_hint_nf[k] / 4 + 1024);
        int2* cur = parity ? t.w_fr2.as<int2>() : t.w_fr.as<int2>();
        int2* nxt = parity ? t.w_fr.as<int2>() : t.w_fr2.as<int2>();
        if (expect <= kFuseMaxPairs) {
            const unsigned g =
                (unsigned)std::min<int64_t>(kPassGrid, cdiv(std::max<int64_t>(expect, 1), kPassTile));
            const uint32_t epoch = ++t.w_epoch;
            hipLaunchKernelGGL(walk_pass_kernel, dim3(g), dim3(TB), 0, s, w, (const int2*)cur, st, k, theta, nxt,
                               t.m2l_pairs.as<int2>(), t.p2p_pairs.as<int2>(), (uint32_t)cap_next, cap_far,
                               cap_near, t.w_pst.as<unsigned long long>(), cap_tiles, epoch, ctx->dev_err);
            TFMM_LAUNCHED();
        } else {
            const unsigned g = (unsigned)std::min<int64_t>(kWalkGrid, cdiv(expect, TB));
            hipLaunchKernelGGL(walk_count_pass_kernel, dim3(g), dim3(TB), 0, s, w, (const int2*)cur,
                               (const WalkState*)st, parity, theta, t.w_dec.as<uint8_t>(), t.w_off.as<U3L>());
            TFMM_LAUNCHED();
            hipLaunchKernelGGL(walk_emit_pass_kernel, dim3(g), dim3(TB), 0, s, w, (const int2*)cur, st, k,
                               (const uint8_t*)t.w_dec.as<uint8_t>(), (const U3L*)t.w_off.as<U3L>(), nxt, t.m2l_pairs.as<int2>(), t.p2p_pairs.as<int2>(),
                               (uint32_t)cap_next, cap_far, cap_near);
            TFMM_LAUNCHED();
        }
        bound = std::min<int64_t>((int64_t)cap_next, 36 * bound);
    }
    const WalkState h = read_back(ctx, (const WalkState*)st, s);
    const int pf = passes & 1;
    if (h.overflow || h.nf[pf] != 0u) return false;
    t.n_m2l = (int64_t)h.n_far[pf];
    t.n_p2p = (int64_t)h.n_near[pf];
    t.walk_hint_fr = h.max_nf;
    t.walk_hint_nf.assign(h.nf_pass, h.nf_pass + passes);
    return true;
}

// Device slots of the list-building totals, read back together at the end.
struct WalkTotals {
    uint32_t multi;        // leaves split into several near-field items
    uint32_t near_entries; // directed near entries (check of 2 n_near - n_leaves)
    uint32_t items;        // near-field work items
    uint32_t partial;      // partial-sum rows of multi-item leaves
    uint32_t scratch[12];  // totals nobody reads
    unsigned long long near_int;
};

}  // namespace

// Fork the tree's second stream from s / join it back into s.
void aux_fork(Tree& t, hipStream_t s) {
    if (!t.aux) {
        TFMM_HIP(hipStreamCreateWithFlags(&t.aux, hipStreamNonBlocking));
        TFMM_HIP(hipEventCreateWithFlags(&t.fork_ev, hipEventDisableTiming));
        TFMM_HIP(hipEventCreateWithFlags(&t.join_ev, hipEventDisableTiming));
    }
    TFMM_HIP(hipEventRecord(t.fork_ev, s));
    TFMM_HIP(hipStreamWaitEvent(t.aux, t.fork_ev, 0));
}

void aux_join(Tree& t, hipStream_t s) {
    TFMM_HIP(hipEventRecord(t.join_ev, t.aux));
    TFMM_HIP(hipStreamWaitEvent(s, t.join_ev, 0));
}

// The frontier passes on s, then the far-list chain on the tree's second
// stream (after the passes) and the near-list chain on s.  walk_lists_end
// reads the totals back once the near chain is done.
void walk_lists_begin(Tree& t, const std::vector<double>& theta_in, hipStream_t s, hipEvent_t passes_done) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    if (theta_in.size() != 1 && theta_in.size() != (size_t)t.n_sets) fail(TFMM_EINVAL, "theta: one value or one per set");
    const std::vector<double> theta_keep = theta_in;  // the caller's vector may be the tree's own
    const double theta = theta_keep[0];
    const double* theta_dev = nullptr;
    if (theta_keep.size() > 1) {
        upload(t, t.set_theta, theta_keep.data(), theta_keep.size() * sizeof(double), 1, s);
        theta_dev = t.set_theta.as<double>();
    }
    t.w_geo.ensure(ctx, (size_t)std::max<int64_t>(nn, 1) * sizeof(double4));
    t.w_top.ensure(ctx, (size_t)std::max<int64_t>(nn, 1) * sizeof(int4));
    hipLaunchKernelGGL(walk_nodes_kernel, dim3(grid(nn)), dim3(TB), 0, s, nn, (const double4*)t.nd_Z.as<double4>(),
                       (const double*)t.nd_rmax.as<double>(), (const int32_t*)t.nd_nchild.as<int32_t>(),
                       (const int32_t*)t.nd_level.as<int32_t>(), (const int32_t*)t.nd_child_first.as<int32_t>(),
                       (const int32_t*)t.nd_first.as<int32_t>(),
                       t.n_sets > 1 ? (const int64_t*)t.set_off.as<int64_t>() : nullptr, t.n_sets,
                       t.w_geo.as<double4>(), t.w_top.as<int4>());
    TFMM_LAUNCHED();
    WalkNodes w{t.w_geo.as<double4>(), t.w_top.as<int4>(), theta_dev};
    t.walk_valid = false;
    if (!walk_bfs_async(t, w, theta, s)) walk_bfs_sized(t, w, theta, s);
    t.walk_hint_far = t.n_m2l;
    t.walk_hint_near = t.n_p2p;
    const int64_t n_far = t.n_m2l, n_near = t.n_p2p;
    if (passes_done) TFMM_HIP(hipEventRecord(passes_done, s));

    t.w_res.ensure(ctx, sizeof(WalkTotals));
    WalkTotals* res = t.w_res.as<WalkTotals>();
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(TB), 0, s, reinterpret_cast<int32_t*>(res),
                       (int64_t)(sizeof(WalkTotals) / 4), 0);
    TFMM_LAUNCHED();
    uint32_t* junk = res->scratch;

    // The far-list chain runs on the tree's second stream, the near-list chain
    // on s; they share no buffer.
    aux_fork(t, s);
    // far lists: directed, by target
    if (nn <= 65536) {
        build_far_csr_packed(t, n_far, t.aux);
    } else {
        build_csr_pairs(t, t.m2l_pairs, n_far, false, t.w_tg, t.w_sr, t.m2l_off, t.m2l_src, t.scratch, t.scratch2,
                        nullptr, t.aux);
        t.m2l_src_mask = 0xffffffffu;
    }
    DevBuf& tg = t.w_tg_b;
    DevBuf& sr = t.w_sr_b;
    // near lists: directed (self pairs once), by target.  Every leaf has
    // exactly one self pair, so the entry count is 2 n_near - n_leaves (the
    // count the sort leaves below its dummies is checked at the end).
    const int64_t ne = 2 * n_near - t.n_leaves;
    {
        build_csr_pairs(t, t.p2p_pairs, n_near, true, tg, sr, t.p2p_off, t.p2p_src, t.scratch_b, t.scratch2_b,
                        &res->near_entries, s);
        // work items over the sorted near entries (tg holds the sorted targets)
        t.w_c.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 4);
        uint32_t* P = t.w_c.as<uint32_t>();
        // the same scratch serves the scan over the entries and the two over the nodes
        t.scratch_b.ensure(ctx, scan_scratch_bytes(std::max<int64_t>(ne, nn)) + 256);
        // P[q] = source particles before entry q (gathered from the source leaf counts)
        exclusive_scan_gather_u32(t.p2p_src.as<int32_t>(), t.nd_count.as<int32_t>(), P, ne, t.scratch_b.p, junk, s);
        // per node: items and partial rows, then their offsets
        t.w_fl.ensure(ctx, (size_t)(nn + 1) * 16);
        uint32_t* nit = t.w_fl.as<uint32_t>();
        uint32_t* it0 = nit + (nn + 1);
        uint32_t* prw = it0 + (nn + 1);
        uint32_t* pbs = prw + (nn + 1);
        hipLaunchKernelGGL(node_items_kernel, dim3(grid(nn)), dim3(TB), 0, s, (const uint32_t*)t.p2p_off.as<uint32_t>(),
                           (const uint32_t*)P, nn, t.nd_count.as<int32_t>(), nit, prw);
        TFMM_LAUNCHED();
        exclusive_scan2_u32(nit, it0, &res->items, prw, pbs, &res->partial, nn, t.scratch_b.p, s);
        // there are at most ne items, so every item array is sized by ne
        const size_t ni = (size_t)std::max<int64_t>(ne, 1);
        t.it_leaf.ensure(ctx, ni * 4);
        t.it_q0.ensure(ctx, ni * 4);
        t.it_q1.ensure(ctx, ni * 4);
        t.it_pbase.ensure(ctx, ni * 4);
        t.leaf_item0.ensure(ctx, (size_t)(nn + 1) * 4);
        t.leaf_nitems.ensure(ctx, (size_t)(nn + 1) * 4);
        t.multi_leaf.ensure(ctx, (size_t)(nn + 1) * 4);
        t.multi_count = &res->multi;
        hipLaunchKernelGGL(item_write_kernel, dim3((unsigned)std::min<int64_t>(2048, grid(ne))), dim3(TB), 0, s,
                           (const uint32_t*)P, (const uint32_t*)t.p2p_off.as<uint32_t>(), nn, (const uint32_t*)nit,
                           (const uint32_t*)it0, (const uint32_t*)&res->items, (const uint32_t*)pbs,
                           t.nd_count.as<int32_t>(),
                           t.it_leaf.as<int32_t>(), t.it_q0.as<uint32_t>(), t.it_q1.as<uint32_t>(),
                           t.it_pbase.as<uint32_t>(), t.leaf_item0.as<int32_t>(), t.leaf_nitems.as<int32_t>(),
                           t.multi_leaf.as<int32_t>(), &res->multi);
        TFMM_LAUNCHED();
    }
    t.walk_theta = theta_keep;
}

void walk_lists_end(Tree& t, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t ne = 2 * t.n_p2p - t.n_leaves;
    const WalkTotals h = read_back_checked(ctx, t.w_res.as<WalkTotals>(), s);
    if ((int64_t)h.near_entries != ne)
        fail(TFMM_EDEVICE, "walk: near entry count " + std::to_string(h.near_entries) + " differs from " +
                               std::to_string(ne));
    t.n_near_int = -1;  // counted on request (near_interactions)
    t.n_items = h.items;
    t.n_partial = h.partial;
    t.walk_valid = true;
}

void walk_tree(Tree& t, const std::vector<double>& theta, hipStream_t s) {
    walk_lists_begin(t, theta, s);
    aux_join(t, s);
    walk_lists_end(t, s);
}

// Directed near particle interactions of the last walk (throughput
// accounting): one pass over the sorted near entries, on the null stream
// after the device is idle, counted once per walk.
int64_t near_interactions(Tree& t) {
    if (!t.walk_valid) return -1;
    if (t.n_near_int >= 0) return t.n_near_int;
    Ctx* ctx = t.ctx;
    TFMM_HIP(hipDeviceSynchronize());
    const int64_t ne = 2 * t.n_p2p - t.n_leaves;
    unsigned long long* acc = &t.w_res.as<WalkTotals>()->near_int;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(TB), 0, nullptr, reinterpret_cast<int32_t*>(acc), 2, 0);
    TFMM_LAUNCHED();
    const unsigned nb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(ne, TB)));
    hipLaunchKernelGGL(near_work_kernel, dim3(nb), dim3(TB), 0, nullptr, (const uint32_t*)t.w_tg_b.as<uint32_t>(),
                       (const int32_t*)t.p2p_src.as<int32_t>(), ne, t.nd_count.as<int32_t>(), acc);
    TFMM_LAUNCHED();
    t.n_near_int = (int64_t)read_back(ctx, (const unsigned long long*)acc, nullptr);
    return t.n_near_int;
}

}  // namespace tfmm
