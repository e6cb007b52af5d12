// Internal declarations shared by the libtfmm translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "tfmm.h"

namespace tfmm {

// Internal failures travel as exceptions and become status codes at the ABI.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

#define TFMM_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::tfmm::fail(TFMM_EDEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define TFMM_LAUNCHED() TFMM_HIP(hipGetLastError())

constexpr int kLevels = 21;       // key bits per axis = deepest octree level
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kMaxP = 8;

inline int c_le(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

struct Ctx;

// Grow-only device buffer, accounted against the owning context's budget.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Ctx* ctx = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void ensure(Ctx* c, size_t bytes);                 // contents not preserved
    void ensure_keep(Ctx* c, size_t bytes, hipStream_t s);  // contents preserved (async copy)
    void release();
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct Ctx {
    int device = 0;
    size_t budget = 0;  // 0 = unlimited
    size_t used = 0;    // device bytes held: live buffers plus the cache below
    // Released blocks kept for reuse (keyed by size): a block enters the cache
    // only once the device is idle, so a new owner never races an old kernel.
    std::multimap<size_t, void*> cache;
    size_t cached = 0;
    bool idle_release = false;  // set while an owner known to be idle releases its buffers
    void trim_cache();          // waits for the device, frees every cached block
    std::string err;
    bool broken = false;
    void* pinned = nullptr;  // small pinned host staging area
    size_t pinned_bytes = 0;
    uint32_t* mbox = nullptr;      // pinned, device-coherent read-back mailbox (host address)
    uint32_t* mbox_dev = nullptr;  // the same memory as the device sees it
    uint32_t mbox_seq = 0;         // sequence number of the last read-back
    uint32_t* dev_err = nullptr;  // device word set by a kernel whose bounded wait ran out
    int live_trees = 0;
    void* alloc(size_t bytes, size_t* got);  // *got: the block's size (>= bytes)
    void free(void* p, size_t bytes);
};

// 1/sqrt(x) in FP64: the v_rsq_f64 seed (about 2^-23 relative) refined by
// two Newton steps.
__device__ __forceinline__ double rsqrt_refined(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    return y;
}

// Per-precision scalar types for the interaction kernels.
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Largest number of particle sets in one tree (a forest of independent sets).
constexpr int kMaxSets = 4096;

// Block order for launches whose neighbouring blocks read the same data: the
// hardware hands workgroup b to XCD b % 8, each XCD with its own L2, so
// consecutive blocks would share nothing in L2.  This maps the first
// floor(G / (8 C)) * 8 C blocks so that each XCD runs chunks of C consecutive
// logical blocks (chunk j on XCD j % 8), keeping the load spread over the
// XCDs; the blocks past that stay in place.  A permutation of [0, G).  For
// M2L (neighbouring target nodes have overlapping far lists) and P2P
// (neighbouring target leaves share source leaves) on the 2^22-particle disk
// this took 1-2 % off the evaluation, with the same forces bit for bit.
template <int C>
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
    const uint32_t g0 = G / (8u * C) * (8u * C);
    if (b >= g0) return b;
    const uint32_t x = b & 7u, k = b >> 3;
    return ((k / C) * 8u + x) * C + (k % C);
}

// The set k of sorted position (or input index) j: off[k] <= j < off[k + 1]
// (off: n_sets + 1 ascending offsets; never read for a single set).
__device__ __forceinline__ int set_of(const int64_t* __restrict__ off, int n_sets, int64_t j) {
    if (n_sets <= 1) return 0;
    int lo = 0, hi = n_sets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Tree {
    Ctx* ctx = nullptr;
    int64_t n = 0;
    int n_leaf = 0;
    // Independent particle sets sharing this tree object (a forest): set k
    // is input particles [off[k], off[k + 1]), and after the sort the same
    // range of sorted positions.  Each set has its own key cube and root
    // (node k); the walk never pairs nodes of different sets.  One set for
    // an ordinary tree.
    int n_sets = 1;
    DevBuf set_off;            // int64, n_sets + 1 (device)
    DevBuf set_theta;          // FP64 theta of every set for the walk (device)
    DevBuf set_sort;           // forest sort scratch: set keys and positions
    void* stage = nullptr;     // pinned host staging of the set tables
    hipEvent_t stage_ev = nullptr;  // the last upload from it
    // tree sizes (host copies)
    int64_t n_nodes = 0, n_leaves = 0;
    int max_level = 0;
    std::vector<int64_t> level_begin;  // node index range of each level, size max_level + 2

    // particles (sorted order unless noted)
    DevBuf cube;               // FP64 key cube: lo x/y/z, hi x/y/z, ext, scale, non-finite flag
    DevBuf keys, keys2;        // uint64 Morton keys
    DevBuf perm, perm2;        // int32 sorted position -> original index
    DevBuf lvlb;               // uint8 level at which a key boundary appears before position j
    DevBuf owner, flags;       // octree-build scratch (window levels and leaf levels; counts and flags)
    DevBuf Xm;                 // double4 (x, y, z, m)
    DevBuf leaf_of;            // int32 leaf node of each sorted position
    DevBuf src4;               // float4/double4 (x, y, z relative to the leaf centre of mass, m)
    int src_prec = -1;

    // nodes (level-major, Morton order within a level)
    DevBuf nd_level, nd_prefix, nd_first, nd_count, nd_child_first, nd_nchild, nd_parent;
    DevBuf nd_S;               // double4 (sum m x, sum m y, sum m z, M)
    DevBuf nd_Z;               // double4 (centre of mass x, y, z, M)
    DevBuf nd_r2bits;          // uint64 bits of max squared distance (atomicMax target)
    DevBuf nd_rmax;            // double
    DevBuf leaves;             // int32 node ids of the leaves
    DevBuf rmax_items;         // int2 (node, chunk) work items of the r_max pass

    // walk and per-target interaction lists
    bool walk_valid = false;
    std::vector<double> walk_theta;  // theta of the last walk: one value, or one per set
    int64_t n_m2l = -1, n_p2p = -1, n_near_int = -1;
    DevBuf m2l_pairs, p2p_pairs;  // int2, lower node id first
    DevBuf m2l_off, m2l_src;      // per-target CSR, directed: source = m2l_src[q] & m2l_src_mask
    uint32_t m2l_src_mask = 0xffffffffu;  // 0xffff when entries are packed (target << 16) | source
    DevBuf p2p_off, p2p_src;
    DevBuf w_fr, w_fr2, w_cnt, w_off, w_tg, w_sr, w_fl, w_c;  // walk and list-building scratch
    DevBuf w_state, w_res, w_dec; // device-side walk counters, list totals, pair decisions
    DevBuf w_geo, w_top;          // per node, packed for the walk (COM + r_max; children, level)
    DevBuf w_pst;                 // tile status words of the fused frontier passes
    uint32_t w_epoch = 0;         // epoch of the last fused pass (tags its status words)
    // sizes seen by the previous walk of this tree (capacity hints for the
    // passes that run without host synchronisation; 0 = none yet)
    int64_t walk_hint_fr = 0, walk_hint_far = 0, walk_hint_near = 0;
    std::vector<int64_t> walk_hint_nf;  // frontier size of every pass
    // near-field work items: a target leaf's list cut into pieces of bounded
    // source count, each run by one wavefront into its own partial sums
    int64_t n_items = 0, n_partial = 0;
    DevBuf it_leaf, it_q0, it_q1, it_pbase;  // per item: leaf, entry range, partial offset
    DevBuf leaf_item0, leaf_nitems;           // per node: first item and item count of a leaf
    DevBuf multi_leaf;                        // leaves split into several items (any order)
    const uint32_t* multi_count = nullptr;    // device: number of entries in multi_leaf
    DevBuf partial;                           // FP64 partial near-field sums, 3 per (item, target)

    // expansions
    int mom_p = -1;
    DevBuf W32, W64;              // (-1)^|k| M_k / k!, NCP per node (FP32 / FP64 copies)
    DevBuf loc;                   // FP64 M2L locals per node (NLOC per node)
    DevBuf loc_leaf;              // FP64 gathered locals per leaf (per node when built level by level)
    DevBuf loc_has;               // uint8 per node: its gathered locals exist (level-by-level pass)
    DevBuf near3;                 // FP64 near-field acceleration (3 per sorted particle)
    DevBuf far3;                  // FP64 far-field acceleration (3 per sorted particle)
    DevBuf near_pot, partial_pot; // FP64 near-field potential (per sorted particle / per partial row)
    DevBuf loc_pot, loc_pot_leaf; // FP64 standard locals with L_0 (potential output only)

    // scratch
    DevBuf scratch;               // scans and sorts
    DevBuf scratch2;

    // a second stream for independent chains of kernels (the far- and
    // near-list builds of a walk), forked from and joined to the caller's
    // stream with events; default priority
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    DevBuf scratch_b, scratch2_b, w_tg_b, w_sr_b;  // the near-list chain's own scratch

    // timing: events of the latest timed evaluation, and the phase times of
    // the earlier ones added up (taken at the next timed evaluation, when its
    // events are complete, or when read).  ev[9], ev[10]: the latest timed
    // rebuild, folded at the next rebuild or when read; ev[11], ev[12]: the
    // walk of the latest evaluation (start, end of the frontier passes).
    bool timing = false;
    hipEvent_t ev[13] = {};
    bool ev_ready = false;
    bool ev_pending = false;
    bool ev_walked = false;        // the pending evaluation ran a walk
    bool build_pending = false;
    double t_sum[10] = {};
    int64_t t_count = 0, t_walks = 0, t_builds = 0;
};

// ---- scans (scan.hip) -----------------------------------------------------
struct U3 {
    uint32_t a, b, c;
};
size_t scan_scratch_bytes(int64_t n);
// Exclusive scan of n values (in == out allowed); writes the total to
// *total_dev (device).
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch, uint32_t* total_dev,
                        hipStream_t s);
// Two scans of n values each (one launch when n is small).
void exclusive_scan2_u32(const uint32_t* in0, uint32_t* out0, uint32_t* total0, const uint32_t* in1,
                         uint32_t* out1, uint32_t* total1, int64_t n, void* scratch, hipStream_t s);
// The same over gathered values: value i = val[idx[i]] (val non-negative).
void exclusive_scan_gather_u32(const int32_t* idx, const int32_t* val, uint32_t* out, int64_t n, void* scratch,
                               uint32_t* total_dev, hipStream_t s);

// ---- radix sort (sort.hip) ----------------------------------------------------
size_t sort_scratch_bytes(int64_t n, int bits);
// Stable LSD sort of (key, value) by the low `bits` bits of key; result ends in
// keys/vals (alt buffers are scratch of the same size).
void radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                    int64_t n, int bits, void* scratch, uint32_t* err, hipStream_t s);
void radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                    int64_t n, int bits, void* scratch, uint32_t* err, hipStream_t s);
// Stable sort by key of the 2 np directed entries of np node pairs: entry 2i
// is (key x_i, value y_i), entry 2i + 1 is (y_i, x_i); with self_dummy, the
// second entry of a pair (x, x) gets key self_key instead.  The sorted
// entries land in (keys, vals); the alternate arrays hold 2 np entries.
void radix_sort_pairs(const int2* pairs, int64_t np, bool self_dummy, uint32_t self_key, uint32_t* keys,
                      int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int bits, void* scratch,
                      uint32_t* err, hipStream_t s);
// The same entries packed as (x << 16) | y words (node ids below 2^16),
// stably sorted by their high half (its low `bits` bits); no values.
void radix_sort_pairs_packed16(const int2* pairs, int64_t np, uint32_t* keys, uint32_t* keys_alt, int bits,
                               void* scratch, uint32_t* err, hipStream_t s);

// Mailbox layout: word 0 the sequence number of the last read-back, word 1
// the device error word, the payload from word kBoxHeaderWords on.
constexpr int kBoxHeaderWords = 16;
constexpr size_t kBoxPayload = 32768;
constexpr size_t kBoxBytes = kBoxHeaderWords * 4 + kBoxPayload;
// Copies bytes (a multiple of 4, at most kBoxPayload) from device memory to
// out once the work queued on s before it is done; with check_err, fails if a
// kernel set the context's device error word.
void read_back_bytes(Ctx* ctx, const void* dev, size_t bytes, void* out, bool check_err, hipStream_t s);

template <typename V>
V read_back(Ctx* ctx, const V* dev, hipStream_t s) {
    V v;
    read_back_bytes(ctx, dev, sizeof(V), &v, false, s);
    return v;
}

// The same, failing if a kernel set the device error word.
template <typename V>
V read_back_checked(Ctx* ctx, const V* dev, hipStream_t s) {
    V v;
    read_back_bytes(ctx, dev, sizeof(V), &v, true, s);
    return v;
}

// ---- phases ---------------------------------------------------------------
void build_tree(Tree& t, const double* pos, const double* mass, hipStream_t s);
// Copies bytes from host memory to dst (device) on s through the tree's
// pinned staging area (slot 0 or 1, kStageSlot bytes each).
constexpr size_t kStageSlot = 48 << 10;
void upload(Tree& t, DevBuf& dst, const void* src, size_t bytes, int slot, hipStream_t s);
// theta: one value for every set, or one per set (n_sets values)
void walk_tree(Tree& t, const std::vector<double>& theta, hipStream_t s);
// passes_done: an event recorded on s once the frontier passes are queued
// (before the list chains), or nullptr
void walk_lists_begin(Tree& t, const std::vector<double>& theta, hipStream_t s, hipEvent_t passes_done = nullptr);
void walk_lists_end(Tree& t, hipStream_t s);
void aux_fork(Tree& t, hipStream_t s);
void aux_join(Tree& t, hipStream_t s);
int64_t near_interactions(Tree& t);
void compute_moments(Tree& t, int p, hipStream_t s);
void prepare_sources(Tree& t, int precision, hipStream_t s);
// kdeg: degree of the conserving projection scalar (p - 1 by default; above
// it the locals are of order kdeg + 1)
void run_m2l(Tree& t, int p, int variant, int precision, double eps2, hipStream_t s, int kdeg);
constexpr int kKnobMaxK = 6;  // largest scalar degree built for the GPU
void run_p2p(Tree& t, int precision, double eps2, bool with_pot, hipStream_t s);
void run_p2p_reduce(Tree& t, bool with_pot, hipStream_t s);
void run_m2l_pot(Tree& t, int p, int mom_p, int precision, double eps2, hipStream_t s);
void run_potential_down(Tree& t, int p, int precision, double eps2, double G, double* pot, hipStream_t s);
void run_l2l(Tree& t, int p, int variant, hipStream_t s);
// Far-field acceleration of every particle into t.far3 (after L2L, on the
// stream L2L ran on), then the forces G m (near + far) in caller order.
void run_l2p_far(Tree& t, int p, int variant, hipStream_t s);
void run_force_combine(Tree& t, double G, double* force, hipStream_t s);
void run_diagnostics(int64_t n, const double* pos, const double* vel, const double* mass,
                     const double* force, double* out_host, Ctx* ctx, hipStream_t s);
void diag_scratch_init(int device);  // with the device current
void run_diagnostics_noalloc(int64_t n, const double* pos, const double* vel, const double* mass,
                             const double* force, double* out_dev, int device, hipStream_t s);
// largest n of the allocation-free diagnostics (the library's particle limit)
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 30;
void run_kick(int64_t n, double* vel, const double* force, const double* mass, double h, hipStream_t s);
void run_drift(int64_t n, double* pos, const double* vel, double dt, hipStream_t s);

// number of FP64 local values per node for a variant
inline int n_local(int p, int variant) {
    return variant != TFMM_STANDARD ? 4 * c_le(p - 1) : c_le(p);
}

}  // namespace tfmm

struct tfmm_ctx : tfmm::Ctx {};
struct tfmm_tree : tfmm::Tree {};
