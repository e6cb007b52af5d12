// Octree construction on the GPU.
//
// Every quantity that feeds the multipole acceptance criterion (keys, centres
// of mass, r_max) is computed in FP64 in one fixed operation order, without
// contraction, so the node table and the interaction lists are reproducible
// bit for bit:
//   keys   q_d = min(2^21 - 1, floor((X_d - lo_d) * scale)), 21 bits per axis
//          interleaved x, y, z from the most significant bit;
//   order  stable sort by key;
//   nodes  (level l, prefix = key >> 3(21 - l)), split while count > n_leaf
//          and l < 21, numbered level by level in Morton order;
//   M, S   leaf: left-to-right sums over its sorted particles of m and m X;
//          inner node: sums over its children in digit order; Z = S / M;
//   r_max  sqrt of the largest ((dx*dx + dy*dy) + dz*dz) over the node's
//          particles, d = X - Z (the r_max of Eq. mac_criterion).
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>

#include "common.h"

namespace tfmm {
namespace {

constexpr int TB = 256;
constexpr uint32_t QMAX = (1u << kLevels) - 1u;

__global__ __launch_bounds__(TB) void bbox_partial_kernel(const double* __restrict__ pos, int64_t n,
                                                          double* __restrict__ part) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t a = (int64_t)blockIdx.x * TB + threadIdx.x; a < n; a += (int64_t)gridDim.x * TB) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = pos[3 * a + d];
            bad |= !isfinite(v);
            lo[d] = v < lo[d] ? v : lo[d];
            hi[d] = v > hi[d] ? v : hi[d];
        }
    }
    __shared__ double sh[6][TB];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if (bad) s_bad = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int s = TB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double a = sh[d][threadIdx.x + s], b = sh[3 + d][threadIdx.x + s];
                if (a < sh[d][threadIdx.x]) sh[d][threadIdx.x] = a;
                if (b > sh[3 + d][threadIdx.x]) sh[3 + d][threadIdx.x] = b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[7 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 6) part[7 * blockIdx.x + 6] = s_bad ? 1.0 : 0.0;
}

// The cube of the keys: out[0..2] lo, [3..5] hi, [6] ext = the largest
// extent (1 if all extents are 0), [7] scale = 2^21 / ext, [8] 1 if any
// coordinate is not finite.  Exact FP64 operations, no contraction.
__device__ void write_cube(const double* lo, const double* hi, bool bad, double* __restrict__ out) {
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        out[d] = lo[d];
        out[3 + d] = hi[d];
        const double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    if (ext == 0.0) ext = 1.0;
    const double scale = 2097152.0 / ext;
    out[6] = ext;
    out[7] = scale;
    out[8] = (bad || !isfinite(ext) || !isfinite(scale)) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(TB) void bbox_final_kernel(const double* __restrict__ part, int nb,
                                                        double* __restrict__ out) {
    __shared__ double sh[6][TB];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += TB) {
        if (part[7 * b + 6] != 0.0) s_bad = 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double lo = part[7 * b + d], hi = part[7 * b + 3 + d];
            v[d] = lo < v[d] ? lo : v[d];
            v[3 + d] = hi > v[3 + d] ? hi : v[3 + d];
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) sh[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int s = TB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double a = sh[d][threadIdx.x + s], b = sh[3 + d][threadIdx.x + s];
                if (a < sh[d][threadIdx.x]) sh[d][threadIdx.x] = a;
                if (b > sh[3 + d][threadIdx.x]) sh[3 + d][threadIdx.x] = b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double lo[3] = {sh[0][0], sh[1][0], sh[2][0]}, hi[3] = {sh[3][0], sh[4][0], sh[5][0]};
        write_cube(lo, hi, s_bad != 0, out);
    }
}

// The cubes of the sets of a forest, one block per set (cube k at out + 16 k).
__global__ __launch_bounds__(TB) void bbox_sets_kernel(const double* __restrict__ pos,
                                                       const int64_t* __restrict__ off,
                                                       double* __restrict__ out) {
    const int64_t a0 = off[blockIdx.x], a1 = off[blockIdx.x + 1];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t a = a0 + threadIdx.x; a < a1; a += TB) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = pos[3 * a + d];
            bad |= !isfinite(v);
            lo[d] = v < lo[d] ? v : lo[d];
            hi[d] = v > hi[d] ? v : hi[d];
        }
    }
    __shared__ double sh[6][TB];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if (bad) s_bad = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int st = TB / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double x = sh[d][threadIdx.x + st], y = sh[3 + d][threadIdx.x + st];
                if (x < sh[d][threadIdx.x]) sh[d][threadIdx.x] = x;
                if (y > sh[3 + d][threadIdx.x]) sh[3 + d][threadIdx.x] = y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double l[3] = {sh[0][0], sh[1][0], sh[2][0]}, h[3] = {sh[3][0], sh[4][0], sh[5][0]};
        write_cube(l, h, s_bad != 0, out + 16 * (int64_t)blockIdx.x);
    }
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(TB) void morton_kernel(const double* __restrict__ pos, int64_t n,
                                                    const double* __restrict__ cubes,
                                                    const int64_t* __restrict__ set_off, int n_sets,
                                                    uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
    const int64_t a = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (a >= n) return;
    const double* cube = cubes + 16 * (int64_t)set_of(set_off, n_sets, a);
    const double lo[3] = {cube[0], cube[1], cube[2]};
    const double scale = cube[7];
    uint32_t q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = floor((pos[3 * a + d] - lo[d]) * scale);
        q[d] = (f >= (double)QMAX) ? QMAX : (uint32_t)f;
    }
    keys[a] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[a] = (int32_t)a;
}

// Forest: after the sort by key, a stable sort by set puts every set's
// particles in its own range in key order.  skey = set of each sorted
// particle, spos = its position; then the keys and the order follow spos.
__global__ __launch_bounds__(TB) void set_keys_kernel(const int32_t* __restrict__ perm, int64_t n,
                                                      const int64_t* __restrict__ set_off, int n_sets,
                                                      uint32_t* __restrict__ skey, int32_t* __restrict__ spos) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= n) return;
    skey[j] = (uint32_t)set_of(set_off, n_sets, perm[j]);
    spos[j] = (int32_t)j;
}

__global__ __launch_bounds__(TB) void set_apply_kernel(const int32_t* __restrict__ spos, int64_t n,
                                                       const uint64_t* __restrict__ keys,
                                                       const int32_t* __restrict__ perm,
                                                       uint64_t* __restrict__ keys_out, int32_t* __restrict__ perm_out) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= n) return;
    const int32_t q = spos[j];
    keys_out[j] = keys[q];
    perm_out[j] = perm[q];
}

// Sorted FP64 particles and the level at which a key boundary appears in front
// of each sorted position (22 = equal keys, never a boundary; 0 = the first
// particle of a set, where its root starts).
__global__ __launch_bounds__(TB) void gather_kernel(const double* __restrict__ pos,
                                                    const double* __restrict__ mass,
                                                    const uint64_t* __restrict__ keys,
                                                    const int32_t* __restrict__ perm, int64_t n,
                                                    const int64_t* __restrict__ set_off, int n_sets,
                                                    double4* __restrict__ Xm, uint8_t* __restrict__ lvlb) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= n) return;
    const int64_t a = perm[j];
    Xm[j] = make_double4(pos[3 * a], pos[3 * a + 1], pos[3 * a + 2], mass[a]);
    uint8_t lb = 0;
    if (j > 0 && (n_sets <= 1 || set_off[set_of(set_off, n_sets, j)] != j)) {
        const uint64_t x = keys[j - 1] ^ keys[j];
        lb = (x == 0) ? (uint8_t)(kLevels + 1) : (uint8_t)(kLevels - (63 - __clzll((long long)x)) / 3);
    }
    lvlb[j] = lb;
}

struct NodeArrays {
    int32_t* level;
    uint64_t* prefix;
    int32_t* first;
    int32_t* count;
    int32_t* child_first;
    int32_t* nchild;
    int32_t* parent;
};

// ---- octree from the sorted keys, all levels at once -------------------------
// With the split rule "count > n_leaf and level < 21", a particle's leaf level
// lambda(j) is one more than the deepest level at which its cell holds more
// than n_leaf particles (capped at 21; 0 when its whole set fits one leaf),
// and that happens exactly when some window of n_leaf + 1 consecutive sorted
// keys of its set around j shares the prefix of that level.  Position j then
// starts a node at every level l with lvlb[j] <= l <= lambda(j); the roots
// (level 0) start at the first particle of every set, so root k is node k.
// Node ids are level major and in position order inside a level, so an id is
// the level's first id plus the number of node starts at that level before j:
// per-level counts per block, scanned over blocks, plus wave ballots inside
// the block.
constexpr int NSLOT = kLevels + 2;  // levels 0..21 and a slot for the leaf count
constexpr int kMaxLeafWindow = 4096;

// cl[i] = deepest level shared by keys[i] and keys[i + n_leaf] (21 if equal,
// -1 if the two belong to different sets).
__global__ __launch_bounds__(TB) void window_level_kernel(const uint64_t* __restrict__ keys, int64_t nw, int n_leaf,
                                                          const int64_t* __restrict__ set_off, int n_sets,
                                                          int8_t* __restrict__ cl) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nw) return;
    if (n_sets > 1 && set_off[set_of(set_off, n_sets, i) + 1] <= i + n_leaf) {
        cl[i] = (int8_t)-1;
        return;
    }
    const uint64_t x = keys[i] ^ keys[i + n_leaf];
    cl[i] = (x == 0) ? (int8_t)kLevels : (int8_t)(kLevels - (63 - __clzll((long long)x)) / 3 - 1);
}

// lambda(j) from the largest cl over the n_leaf + 1 windows that contain j
// (a sparse-table maximum in LDS), and per-level counts of node starts and of
// leaf starts for the block.
__global__ __launch_bounds__(TB) void leaf_level_kernel(const int8_t* __restrict__ cl, int64_t n, int n_leaf,
                                                        const uint8_t* __restrict__ lvlb, uint8_t* __restrict__ lam,
                                                        uint32_t* __restrict__ cnt, int64_t nblk) {
    constexpr int VMAX = (TB + kMaxLeafWindow + TB - 1) / TB;
    __shared__ int8_t m[TB + kMaxLeafWindow];
    __shared__ uint32_t wc[TB / kWave][NSLOT];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t j0 = (int64_t)blockIdx.x * TB;
    const int64_t nw = n - n_leaf;
    const int TL = TB + n_leaf;
    for (int t = tid; t < TL; t += TB) {
        const int64_t i = j0 - n_leaf + t;
        m[t] = (i >= 0 && i < nw) ? cl[i] : (int8_t)-1;
    }
    __syncthreads();
    const int w = n_leaf + 1;
    int span = 1;
    while (2 * span <= w) {
        int8_t v[VMAX];
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int t = tid + q * TB;
            if (t < TL) {
                const int8_t x = m[t], y = (t + span < TL) ? m[t + span] : (int8_t)-1;
                v[q] = x > y ? x : y;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int t = tid + q * TB;
            if (t < TL) m[t] = v[q];
        }
        __syncthreads();
        span *= 2;
    }
    const int64_t j = j0 + tid;
    const bool valid = j < n;
    int a = 99, b = 0;
    if (valid) {
        // windows [tid, tid + w) of the tile; m[t] covers [t, t + span)
        const int8_t x = m[tid], y = m[tid + w - span];
        const int bd = x > y ? x : y;
        b = bd < 0 ? 0 : (bd + 1 < kLevels ? bd + 1 : kLevels);
        lam[j] = (uint8_t)b;
        a = lvlb[j];
    }
    for (int l = 0; l <= kLevels; ++l) {
        const unsigned long long bl = __ballot(a <= l && l <= b);
        if (lane == 0) wc[wv][l] = (uint32_t)__popcll(bl);
    }
    const unsigned long long leaf = __ballot(a <= b);
    if (lane == 0) wc[wv][NSLOT - 1] = (uint32_t)__popcll(leaf);
    __syncthreads();
    if (tid < NSLOT) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < TB / kWave; ++q) c += wc[q][tid];
        cnt[(int64_t)tid * nblk + blockIdx.x] = c;
    }
}

// Exclusive scan over the blocks of one slot's counts (one block per slot):
// every thread takes a contiguous run of the counts, the run totals are
// scanned across the block (wave scans, then the waves' totals), and each
// thread writes its run's exclusive prefixes.
__global__ __launch_bounds__(TB) void slot_scan_kernel(uint32_t* __restrict__ cnt, int64_t nblk,
                                                       uint32_t* __restrict__ tot) {
    __shared__ uint32_t wsum[TB / kWave];
    uint32_t* c = cnt + (int64_t)blockIdx.x * nblk;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t per = (nblk + TB - 1) / TB;
    const int64_t i0 = (int64_t)tid * per;
    const int64_t i1 = i0 + per < nblk ? i0 + per : nblk;
    uint32_t run = 0;
    for (int64_t i = i0; i < i1; ++i) run += c[i];
    uint32_t v = run;  // inclusive scan of the run totals over the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, d, kWave);
        if (lane >= d) v += u;
    }
    if (lane == kWave - 1) wsum[wv] = v;
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int q = 0; q < TB / kWave; ++q) {
        if (q < wv) base += wsum[q];
        all += wsum[q];
    }
    uint32_t acc = base + v - run;
    for (int64_t i = i0; i < i1; ++i) {
        const uint32_t x = c[i];
        c[i] = acc;
        acc += x;
    }
    if (tid == 0) tot[blockIdx.x] = all;
}

// Level boundaries and sizes of the octree (read back by the host once).
struct TreeHeader {
    int64_t LB[kLevels + 2];  // first node id of levels 0..21, then the node count
    int64_t max_level, n_nodes, n_leaves;
    int64_t nonfinite;        // a coordinate was not finite
};

__global__ void tree_header_kernel(const uint32_t* __restrict__ tot, const double* __restrict__ cubes, int n_sets,
                                   TreeHeader* __restrict__ h) {
    if (threadIdx.x != 0) return;
    int64_t bad = 0;
    for (int k = 0; k < n_sets; ++k) bad |= cubes[16 * k + 8] != 0.0 ? 1 : 0;
    h->nonfinite = bad;
    h->LB[0] = 0;
    int64_t ml = 0;
    for (int l = 0; l <= kLevels; ++l) {
        h->LB[l + 1] = h->LB[l] + tot[l];
        if (tot[l] > 0) ml = l;
    }
    h->max_level = ml;
    h->n_nodes = h->LB[kLevels + 1];
    h->n_leaves = (int64_t)tot[NSLOT - 1];
}

__global__ __launch_bounds__(TB) void node_create_kernel(NodeArrays nd, int64_t n, const uint64_t* __restrict__ keys,
                                                         const uint8_t* __restrict__ lvlb,
                                                         const uint8_t* __restrict__ lam,
                                                         const uint32_t* __restrict__ boff, int64_t nblk,
                                                         const TreeHeader* __restrict__ h,
                                                         int32_t* __restrict__ leaf_of,
                                                         int32_t* __restrict__ leaves) {
    __shared__ unsigned long long bal[TB / kWave][NSLOT];
    __shared__ uint32_t woff[TB / kWave][NSLOT];
    __shared__ int64_t sLB[kLevels + 2];
    __shared__ uint32_t sboff[NSLOT];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t j = (int64_t)blockIdx.x * TB + tid;
    const bool valid = j < n;
    const int a = valid ? (int)lvlb[j] : 99;
    const int b = valid ? (int)lam[j] : 0;
    for (int l = 0; l <= kLevels; ++l) {
        const unsigned long long bl = __ballot(a <= l && l <= b);
        if (lane == 0) bal[wv][l] = bl;
    }
    {
        const unsigned long long bl = __ballot(a <= b);  // a leaf starts here (at level b)
        if (lane == 0) bal[wv][NSLOT - 1] = bl;
    }
    if (tid < kLevels + 2) sLB[tid] = h->LB[tid];
    if (tid < NSLOT) sboff[tid] = boff[(int64_t)tid * nblk + blockIdx.x];
    __syncthreads();
    if (tid < NSLOT) {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < TB / kWave; ++q) {
            woff[q][tid] = run;
            run += (uint32_t)__popcll(bal[q][tid]);
        }
    }
    __syncthreads();
    if (!valid) return;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    auto rank = [&](int l) -> int64_t {
        return (int64_t)sboff[l] + woff[wv][l] + (uint32_t)__popcll(bal[wv][l] & lt);
    };
    auto incl = [&](int l) -> int64_t { return rank(l) + ((a <= l && l <= b) ? 1 : 0); };
    leaf_of[j] = (int32_t)(sLB[b] + incl(b) - 1);
    // the list of leaves, in particle order (every user takes each leaf on its own)
    if (a <= b) leaves[rank(NSLOT - 1)] = (int32_t)(sLB[b] + rank(b));
    for (int l = a; l <= b; ++l) {
        const int64_t id = sLB[l] + rank(l);
        nd.level[id] = l;
        nd.prefix[id] = keys[j] >> (3 * (kLevels - l));
        nd.first[id] = (int32_t)j;
        nd.count[id] = 0;
        nd.nchild[id] = 0;
        nd.parent[id] = (l == 0) ? -1 : (int32_t)(sLB[l - 1] + incl(l - 1) - 1);
        nd.child_first[id] = (l + 1 <= b) ? (int32_t)(sLB[l + 1] + rank(l + 1)) : -1;
    }
}

// Particle counts (a node ends where the next node of its level starts if
// that node has the same parent, else where its parent ends; the roots,
// parent -1, end where the next root starts) and child counts (written by the
// last child).
__global__ __launch_bounds__(TB) void node_finish_kernel(NodeArrays nd, int64_t nn, int64_t n,
                                                         const TreeHeader* __restrict__ h) {
    const int64_t c = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (c >= nn) return;
    const int l = nd.level[c];
    const int32_t P = nd.parent[c];
    int64_t x = c, end = n;
    for (int lx = l; lx >= 0; --lx) {
        const int64_t nx = x + 1;
        if (nx < h->LB[lx + 1] && nd.parent[nx] == nd.parent[x]) {
            end = nd.first[nx];
            break;
        }
        x = nd.parent[x];
    }
    nd.count[c] = (int32_t)(end - nd.first[c]);
    if (P >= 0 && (c + 1 >= h->LB[l + 1] || nd.parent[c + 1] != P))
        nd.nchild[P] = (int32_t)(c - nd.child_first[P] + 1);
}

// Mass and centre of mass of the leaves (all levels in one launch).
__global__ __launch_bounds__(TB) void geometry_leaf_kernel(const int32_t* __restrict__ leaves, int64_t n_leaves,
                                                           const int32_t* __restrict__ first,
                                                           const int32_t* __restrict__ count,
                                                           const double4* __restrict__ Xm, double4* __restrict__ S,
                                                           double4* __restrict__ Z) {
    const int64_t l = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (l >= n_leaves) return;
    const int32_t i = leaves[l];
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    // loads issued eight at a time, sums kept strictly left to right
    const int32_t s0 = first[i], s1 = s0 + count[i];
    for (int32_t q = s0; q < s1; q += 8) {
        double4 p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q + u < s1) p[u] = Xm[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (q + u < s1) {
                M = M + p[u].w;
                sx = sx + p[u].w * p[u].x;
                sy = sy + p[u].w * p[u].y;
                sz = sz + p[u].w * p[u].z;
            }
        }
    }
    S[i] = make_double4(sx, sy, sz, M);
    Z[i] = make_double4(sx / M, sy / M, sz / M, M);
}

// Inner node: sums over its children in digit order.
__device__ __forceinline__ void geometry_inner(int32_t i, const int32_t* __restrict__ child_first,
                                               const int32_t* __restrict__ nchild, double4* __restrict__ S,
                                               double4* __restrict__ Z) {
    const int32_t nc = nchild[i];
    if (nc == 0) return;  // a leaf: done by geometry_leaf_kernel
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    const int32_t c0 = child_first[i];
    for (int32_t c = c0; c < c0 + nc; ++c) {
        const double4 q = S[c];
        M = M + q.w;
        sx = sx + q.x;
        sy = sy + q.y;
        sz = sz + q.z;
    }
    S[i] = make_double4(sx, sy, sz, M);
    Z[i] = make_double4(sx / M, sy / M, sz / M, M);
}

// Inner nodes of one level (the level below is done).
__global__ __launch_bounds__(TB) void geometry_level_kernel(const int32_t* __restrict__ child_first,
                                                            const int32_t* __restrict__ nchild, int32_t lb,
                                                            int32_t le, double4* __restrict__ S,
                                                            double4* __restrict__ Z) {
    const int32_t i = lb + blockIdx.x * TB + threadIdx.x;
    if (i < le) geometry_inner(i, child_first, nchild, S, Z);
}

// Inner nodes of the top levels 0..top in one block, deepest first.
struct LevelBounds {
    int32_t b[kLevels + 2];
};
__global__ __launch_bounds__(TB) void geometry_top_kernel(const int32_t* __restrict__ child_first,
                                                          const int32_t* __restrict__ nchild, LevelBounds lv, int top,
                                                          double4* __restrict__ S, double4* __restrict__ Z) {
    for (int L = top; L >= 0; --L) {
        for (int32_t i = lv.b[L] + (int32_t)threadIdx.x; i < lv.b[L + 1]; i += TB) geometry_inner(i, child_first, nchild, S, Z);
        __syncthreads();
    }
}

__global__ __launch_bounds__(TB) void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exact r_max: the maximum squared distance of a node's particles from its
// centre of mass.  Work items are (node, chunk of at most RCH particles) so the
// root does not serialise on one wavefront; each item reduces its chunk across
// the wave and issues one atomicMax on the bits of the (non-negative) double.
// A maximum does not depend on the order of the atomics: deterministic.
constexpr int RCH = 4096;

__global__ __launch_bounds__(TB) void rmax_chunks_kernel(const int32_t* __restrict__ count, int64_t nn,
                                                         uint32_t* __restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < nn) c[i] = (uint32_t)((count[i] + RCH - 1) / RCH);
}

__global__ __launch_bounds__(TB) void rmax_items_kernel(int64_t nn, const uint32_t* __restrict__ c,
                                                        const uint32_t* __restrict__ base,
                                                        int2* __restrict__ items) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nn) return;
    for (uint32_t k = 0; k < c[i]; ++k) items[base[i] + k] = make_int2((int32_t)i, (int32_t)k);
}

__global__ __launch_bounds__(kWave) void rmax_kernel(const uint32_t* __restrict__ n_items,
                                                     const int2* __restrict__ items,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ count,
                                                     const double4* __restrict__ Xm, const double4* __restrict__ Z,
                                                     unsigned long long* __restrict__ r2bits) {
    if (blockIdx.x >= *n_items) return;
    const int2 it = items[blockIdx.x];
    const int32_t s0 = first[it.x] + it.y * RCH;
    const int32_t e = first[it.x] + count[it.x];
    const int32_t s1 = (s0 + RCH < e) ? s0 + RCH : e;
    const double4 z = Z[it.x];
    double m = 0.0;
    for (int32_t s = s0 + (int32_t)threadIdx.x; s < s1; s += kWave) {
        const double4 x = Xm[s];
        const double dx = x.x - z.x, dy = x.y - z.y, dz = x.z - z.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        m = d2 > m ? d2 : m;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double u = __shfl_xor(m, o, kWave);
        m = u > m ? u : m;
    }
    if (threadIdx.x == 0) atomicMax(&r2bits[it.x], (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(TB) void rmax_final_kernel(const unsigned long long* __restrict__ r2bits,
                                                        int64_t nn, double* __restrict__ rmax) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < nn) rmax[i] = sqrt(__longlong_as_double((long long)r2bits[i]));
}

template <typename T>
__global__ __launch_bounds__(TB) void sources_kernel(const double4* __restrict__ Xm,
                                                     const int32_t* __restrict__ leaf_of,
                                                     const double4* __restrict__ Z, int64_t n,
                                                     typename Vec4<T>::type* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= n) return;
    const double4 x = Xm[j];
    const double4 z = Z[leaf_of[j]];
    typename Vec4<T>::type r;
    r.x = (T)(x.x - z.x);
    r.y = (T)(x.y - z.y);
    r.z = (T)(x.z - z.z);
    r.w = (T)x.w;
    out[j] = r;
}

unsigned grid(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, TB); }

NodeArrays node_arrays(Tree& t) {
    return NodeArrays{t.nd_level.as<int32_t>(), t.nd_prefix.as<uint64_t>(), t.nd_first.as<int32_t>(),
                      t.nd_count.as<int32_t>(), t.nd_child_first.as<int32_t>(), t.nd_nchild.as<int32_t>(),
                      t.nd_parent.as<int32_t>()};
}

void ensure_nodes(Tree& t, int64_t cap, int64_t keep, hipStream_t s) {
    (void)keep;
    const size_t c = (size_t)cap;
    t.nd_level.ensure_keep(t.ctx, c * 4, s);
    t.nd_prefix.ensure_keep(t.ctx, c * 8, s);
    t.nd_first.ensure_keep(t.ctx, c * 4, s);
    t.nd_count.ensure_keep(t.ctx, c * 4, s);
    t.nd_child_first.ensure_keep(t.ctx, c * 4, s);
    t.nd_nchild.ensure_keep(t.ctx, c * 4, s);
    t.nd_parent.ensure_keep(t.ctx, c * 4, s);
}

}  // namespace

void upload(Tree& t, DevBuf& dst, const void* src, size_t bytes, int slot, hipStream_t s) {
    if (bytes > kStageSlot) fail(TFMM_EINVAL, "set table too large");
    if (!t.stage) {
        TFMM_HIP(hipHostMalloc(&t.stage, 2 * kStageSlot, hipHostMallocDefault));
        TFMM_HIP(hipEventCreateWithFlags(&t.stage_ev, hipEventDisableTiming));
    } else {
        // the previous copy out of the staging area has finished reading it
        TFMM_HIP(hipEventSynchronize(t.stage_ev));
    }
    char* h = static_cast<char*>(t.stage) + (size_t)slot * kStageSlot;
    std::memcpy(h, src, bytes);
    dst.ensure(t.ctx, bytes);
    TFMM_HIP(hipMemcpyAsync(dst.p, h, bytes, hipMemcpyHostToDevice, s));
    TFMM_HIP(hipEventRecord(t.stage_ev, s));
}

void build_tree(Tree& t, const double* pos, const double* mass, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t n = t.n;
    const size_t un = (size_t)n;

    // bounding cube and key scale of every set, on the device (no read-back)
    const int ns = t.n_sets;
    const int64_t* soff = ns > 1 ? t.set_off.as<int64_t>() : nullptr;
    const int nbb = (int)std::min<int64_t>(1024, cdiv(n, TB));
    t.scratch.ensure(ctx, std::max<size_t>({(size_t)nbb * 7 * 8 + 64, sort_scratch_bytes(n, 3 * kLevels) + 256,
                                            scan_scratch_bytes(n) + 256}));
    t.cube.ensure(ctx, (size_t)ns * 16 * sizeof(double));
    double* part = t.scratch.as<double>();
    double* cube = t.cube.as<double>();
    if (ns > 1) {
        hipLaunchKernelGGL(bbox_sets_kernel, dim3((unsigned)ns), dim3(TB), 0, s, pos, soff, cube);
        TFMM_LAUNCHED();
    } else {
        hipLaunchKernelGGL(bbox_partial_kernel, dim3(nbb), dim3(TB), 0, s, pos, n, part);
        TFMM_LAUNCHED();
        hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(TB), 0, s, (const double*)part, nbb, cube);
        TFMM_LAUNCHED();
    }

    // keys and stable order (by set, then by key)
    t.keys.ensure(ctx, un * 8);
    t.keys2.ensure(ctx, un * 8);
    t.perm.ensure(ctx, un * 4);
    t.perm2.ensure(ctx, un * 4);
    hipLaunchKernelGGL(morton_kernel, dim3(grid(n)), dim3(TB), 0, s, pos, n, (const double*)cube, soff, ns,
                       t.keys.as<uint64_t>(), t.perm.as<int32_t>());
    TFMM_LAUNCHED();
    radix_sort_u64(t.keys.as<uint64_t>(), t.perm.as<int32_t>(), t.keys2.as<uint64_t>(), t.perm2.as<int32_t>(),
                   n, 3 * kLevels, t.scratch.p, ctx->dev_err, s);
    if (ns > 1) {
        int bits = 1;
        while ((1 << bits) < ns) ++bits;
        t.set_sort.ensure(ctx, un * 16);
        uint32_t* skey = t.set_sort.as<uint32_t>();
        int32_t* spos = reinterpret_cast<int32_t*>(skey + n);
        uint32_t* skey2 = skey + 2 * n;
        int32_t* spos2 = reinterpret_cast<int32_t*>(skey + 3 * n);
        hipLaunchKernelGGL(set_keys_kernel, dim3(grid(n)), dim3(TB), 0, s, (const int32_t*)t.perm.as<int32_t>(), n,
                           soff, ns, skey, spos);
        TFMM_LAUNCHED();
        radix_sort_u32(skey, spos, skey2, spos2, n, bits, t.scratch.p, ctx->dev_err, s);
        hipLaunchKernelGGL(set_apply_kernel, dim3(grid(n)), dim3(TB), 0, s, (const int32_t*)spos, n,
                           (const uint64_t*)t.keys.as<uint64_t>(), (const int32_t*)t.perm.as<int32_t>(),
                           t.keys2.as<uint64_t>(), t.perm2.as<int32_t>());
        TFMM_LAUNCHED();
        std::swap(t.keys.p, t.keys2.p);
        std::swap(t.keys.cap, t.keys2.cap);
        std::swap(t.perm.p, t.perm2.p);
        std::swap(t.perm.cap, t.perm2.cap);
    }

    // sorted particles, boundary levels
    t.Xm.ensure(ctx, un * 32);
    t.lvlb.ensure(ctx, un);
    t.owner.ensure(ctx, un * 2);
    t.leaf_of.ensure(ctx, un * 4);
    hipLaunchKernelGGL(gather_kernel, dim3(grid(n)), dim3(TB), 0, s, pos, mass, t.keys.as<uint64_t>(),
                       t.perm.as<int32_t>(), n, soff, ns, t.Xm.as<double4>(), t.lvlb.as<uint8_t>());
    TFMM_LAUNCHED();

    // octree: leaf level of every particle, node starts per level, node table
    const int64_t nblk = cdiv(n, TB);
    const int64_t nw = n - t.n_leaf;  // windows of n_leaf + 1 consecutive keys
    // cl (int8, n) and lambda (uint8, n) share the owner buffer
    int8_t* cl = reinterpret_cast<int8_t*>(t.owner.as<int32_t>());
    uint8_t* lam = reinterpret_cast<uint8_t*>(cl + n);
    t.flags.ensure(ctx, std::max<size_t>(un * 8, (size_t)(NSLOT * nblk + NSLOT) * 4));
    uint32_t* cnt = t.flags.as<uint32_t>();
    uint32_t* tot = cnt + NSLOT * nblk;
    t.scratch2.ensure(ctx, sizeof(TreeHeader) + 256);
    TreeHeader* hdr = t.scratch2.as<TreeHeader>();
    if (nw > 0) {
        hipLaunchKernelGGL(window_level_kernel, dim3(grid(nw)), dim3(TB), 0, s, (const uint64_t*)t.keys.as<uint64_t>(),
                           nw, t.n_leaf, soff, ns, cl);
        TFMM_LAUNCHED();
    }
    hipLaunchKernelGGL(leaf_level_kernel, dim3((unsigned)nblk), dim3(TB), 0, s, (const int8_t*)cl, n, t.n_leaf,
                       (const uint8_t*)t.lvlb.as<uint8_t>(), lam, cnt, nblk);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(slot_scan_kernel, dim3(NSLOT), dim3(TB), 0, s, cnt, nblk, tot);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(tree_header_kernel, dim3(1), dim3(kWave), 0, s, (const uint32_t*)tot, (const double*)cube, ns,
                       hdr);
    TFMM_LAUNCHED();
    const TreeHeader H = read_back_checked(ctx, (const TreeHeader*)hdr, s);
    if (H.nonfinite) fail(TFMM_EINVAL, "positions contain non-finite values");
    t.n_nodes = H.n_nodes;
    t.max_level = (int)H.max_level;
    t.n_leaves = H.n_leaves;
    t.level_begin.assign((size_t)t.max_level + 2, 0);
    for (int l = 0; l <= t.max_level + 1; ++l) t.level_begin[(size_t)l] = H.LB[l];
    const int64_t nn = t.n_nodes;
    ensure_nodes(t, std::max<int64_t>(nn, 1), 0, s);
    NodeArrays nd = node_arrays(t);
    t.leaves.ensure(ctx, (size_t)std::max<int64_t>(t.n_leaves, 1) * 4);
    hipLaunchKernelGGL(node_create_kernel, dim3((unsigned)nblk), dim3(TB), 0, s, nd, n,
                       (const uint64_t*)t.keys.as<uint64_t>(), (const uint8_t*)t.lvlb.as<uint8_t>(),
                       (const uint8_t*)lam, (const uint32_t*)cnt, nblk, (const TreeHeader*)hdr,
                       t.leaf_of.as<int32_t>(), t.leaves.as<int32_t>());
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(node_finish_kernel, dim3(grid(nn)), dim3(TB), 0, s, nd, nn, n, (const TreeHeader*)hdr);
    TFMM_LAUNCHED();
    t.flags.ensure(ctx, (size_t)std::max<int64_t>(n, nn) * 4 * 2);
    t.scratch.ensure(ctx, scan_scratch_bytes(std::max<int64_t>(n, nn)) + 256);
    uint32_t* total = reinterpret_cast<uint32_t*>(t.scratch2.as<char>() + sizeof(TreeHeader));

    // geometry: leaves, then inner nodes level by level, deepest first; the
    // top levels (at most kTopNodes nodes together) in a single block
    t.nd_S.ensure(ctx, (size_t)nn * 32);
    t.nd_Z.ensure(ctx, (size_t)nn * 32);
    hipLaunchKernelGGL(geometry_leaf_kernel, dim3(grid(t.n_leaves)), dim3(TB), 0, s,
                       (const int32_t*)t.leaves.as<int32_t>(), t.n_leaves, nd.first, nd.count, t.Xm.as<double4>(),
                       t.nd_S.as<double4>(), t.nd_Z.as<double4>());
    TFMM_LAUNCHED();
    {
        constexpr int64_t kTopNodes = 1024;
        int top = -1;
        while (top + 1 <= t.max_level && t.level_begin[(size_t)top + 2] <= kTopNodes) ++top;
        for (int L = t.max_level - 1; L > top; --L) {
            const int32_t b = (int32_t)t.level_begin[L], e = (int32_t)t.level_begin[L + 1];
            if (e <= b) continue;
            hipLaunchKernelGGL(geometry_level_kernel, dim3(grid(e - b)), dim3(TB), 0, s, nd.child_first, nd.nchild,
                               b, e, t.nd_S.as<double4>(), t.nd_Z.as<double4>());
            TFMM_LAUNCHED();
        }
        if (top >= 0) {
            LevelBounds lv{};
            for (int L = 0; L <= top + 1; ++L) lv.b[L] = (int32_t)t.level_begin[L];
            hipLaunchKernelGGL(geometry_top_kernel, dim3(1), dim3(TB), 0, s, nd.child_first, nd.nchild, lv, top,
                               t.nd_S.as<double4>(), t.nd_Z.as<double4>());
            TFMM_LAUNCHED();
        }
    }
    t.nd_r2bits.ensure(ctx, (size_t)nn * 8);
    t.nd_rmax.ensure(ctx, (size_t)nn * 8);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid(nn)), dim3(TB), 0, s, t.nd_r2bits.as<uint64_t>(), nn,
                       (uint64_t)0);
    TFMM_LAUNCHED();
    {
        // items (node, chunk); the launch covers an upper bound and reads the count on the device
        const int64_t ub = nn + (int64_t)n * (t.max_level + 1) / RCH + 1;
        t.flags.ensure(ctx, (size_t)std::max<int64_t>(n, nn) * 4 * 2);
        uint32_t* c = t.flags.as<uint32_t>();
        uint32_t* base = c + std::max<int64_t>(n, nn);
        t.rmax_items.ensure(ctx, (size_t)ub * 8);
        hipLaunchKernelGGL(rmax_chunks_kernel, dim3(grid(nn)), dim3(TB), 0, s, nd.count, nn, c);
        TFMM_LAUNCHED();
        exclusive_scan_u32(c, base, nn, t.scratch.p, total, s);
        hipLaunchKernelGGL(rmax_items_kernel, dim3(grid(nn)), dim3(TB), 0, s, nn, (const uint32_t*)c,
                           (const uint32_t*)base, t.rmax_items.as<int2>());
        TFMM_LAUNCHED();
        hipLaunchKernelGGL(rmax_kernel, dim3((unsigned)ub), dim3(kWave), 0, s, (const uint32_t*)total,
                           (const int2*)t.rmax_items.as<int2>(), nd.first, nd.count, t.Xm.as<double4>(),
                           t.nd_Z.as<double4>(), t.nd_r2bits.as<unsigned long long>());
        TFMM_LAUNCHED();
    }
    hipLaunchKernelGGL(rmax_final_kernel, dim3(grid(nn)), dim3(TB), 0, s, t.nd_r2bits.as<unsigned long long>(),
                       nn, t.nd_rmax.as<double>());
    TFMM_LAUNCHED();

    t.walk_valid = false;
    t.mom_p = -1;
    t.src_prec = -1;
}

void prepare_sources(Tree& t, int precision, hipStream_t s) {
    if (t.src_prec == precision) return;
    const int64_t n = t.n;
    if (precision == TFMM_MIXED32) {
        t.src4.ensure(t.ctx, (size_t)n * 16);
        hipLaunchKernelGGL(sources_kernel<float>, dim3(grid(n)), dim3(TB), 0, s, t.Xm.as<double4>(),
                           t.leaf_of.as<int32_t>(), t.nd_Z.as<double4>(), n, t.src4.as<float4>());
    } else {
        t.src4.ensure(t.ctx, (size_t)n * 32);
        hipLaunchKernelGGL(sources_kernel<double>, dim3(grid(n)), dim3(TB), 0, s, t.Xm.as<double4>(),
                           t.leaf_of.as<int32_t>(), t.nd_Z.as<double4>(), n, t.src4.as<double4>());
    }
    TFMM_LAUNCHED();
    t.src_prec = precision;
}

}  // namespace tfmm
