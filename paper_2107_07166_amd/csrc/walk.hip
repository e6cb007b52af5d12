// Mutual dual-tree walk and per-target interaction lists.
//
// The walk processes a frontier of unordered node pairs level-synchronously
// from (root, root).  For each pair:
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

struct WalkNodes {
    const int32_t* level;
    const int32_t* child_first;
    const int32_t* nchild;
    const double4* Z;
    const double* rmax;
};

struct Decision {
    int kind;      // 0 near, 1 far, 2 expand self, 3 split S against O
    int32_t S, O;  // for kind 3
    uint32_t nnew;
};

__device__ __forceinline__ Decision decide(const WalkNodes& w, int32_t A, int32_t B, double theta) {
    Decision d{0, -1, -1, 0u};
    if (A == B) {
        const int32_t nc = w.nchild[A];
        if (nc == 0) {
            d.kind = 0;
        } else {
            d.kind = 2;
            d.nnew = (uint32_t)(nc * (nc + 1) / 2);
        }
        return d;
    }
    const double4 za = w.Z[A], zb = w.Z[B];
    const double dx = za.x - zb.x, dy = za.y - zb.y, dz = za.z - zb.z;
    const double R = sqrt((dx * dx + dy * dy) + dz * dz);
    const double ra = w.rmax[A], rb = w.rmax[B];
    if (R > 0.0 && ra + rb <= theta * R) {
        d.kind = 1;
        return d;
    }
    const int32_t na = w.nchild[A], nb = w.nchild[B];
    if (na == 0 && nb == 0) {
        d.kind = 0;
        return d;
    }
    int32_t S;
    if (na == 0) S = B;
    else if (nb == 0) S = A;
    else if (ra > rb) S = A;
    else if (rb > ra) S = B;
    else if (w.level[A] < w.level[B]) S = A;
    else if (w.level[B] < w.level[A]) S = B;
    else S = A < B ? A : B;
    d.kind = 3;
    d.S = S;
    d.O = (S == A) ? B : A;
    d.nnew = (uint32_t)w.nchild[S];
    return d;
}

// Children of an expanded pair, in a fixed order: a self pair gives
// (c_a, c_b) for a <= b (row major), a split gives (c_a, O).
struct Kids {
    int kind;  // 2 self, 3 split
    int32_t c0, nc, O;
};

__device__ __forceinline__ Kids kids_of(const WalkNodes& w, int2 pr, const Decision& d) {
    if (d.kind == 2) return Kids{2, w.child_first[pr.x], w.nchild[pr.x], -1};
    return Kids{3, w.child_first[d.S], w.nchild[d.S], d.O};
}

// One walk step covers two tree levels: the pair's own decision and, when it
// is expanded, the decisions of its children; only grandchildren go to the
// next frontier.  Outputs are produced in a fixed order (children in order,
// each child's own output or its children), so counting and emitting agree.
template <bool EMIT>
__device__ __forceinline__ void walk_step(const WalkNodes& w, int2 pr, double theta, U3& c, int2* next, int2* far,
                                          int2* near) {
    auto put_final = [&](int kind, int32_t A, int32_t B) {
        const int32_t lo = A < B ? A : B, hi = A < B ? B : A;
        if (kind == 0) {
            if (EMIT) near[c.c] = make_int2(lo, hi);
            c.c++;
        } else {
            if (EMIT) far[c.b] = make_int2(lo, hi);
            c.b++;
        }
    };
    auto put_kids = [&](int2 q, const Decision& d) {
        const Kids k = kids_of(w, q, d);
        if (k.kind == 2) {
            for (int32_t a = 0; a < k.nc; ++a)
                for (int32_t b = a; b < k.nc; ++b) {
                    if (EMIT) next[c.a] = make_int2(k.c0 + a, k.c0 + b);
                    c.a++;
                }
        } else {
            for (int32_t a = 0; a < k.nc; ++a) {
                if (EMIT) next[c.a] = make_int2(k.c0 + a, k.O);
                c.a++;
            }
        }
    };
    const Decision d = decide(w, pr.x, pr.y, theta);
    if (d.kind <= 1) {
        put_final(d.kind, pr.x, pr.y);
        return;
    }
    const Kids k = kids_of(w, pr, d);
    for (int32_t a = 0; a < k.nc; ++a) {
        const int32_t bstart = (k.kind == 2) ? a : 0;
        const int32_t bend = (k.kind == 2) ? k.nc : 1;
        for (int32_t b = bstart; b < bend; ++b) {
            const int2 q = (k.kind == 2) ? make_int2(k.c0 + a, k.c0 + b) : make_int2(k.c0 + a, k.O);
            const Decision e = decide(w, q.x, q.y, theta);
            if (e.kind <= 1) put_final(e.kind, q.x, q.y);
            else put_kids(q, e);
        }
    }
}

__device__ __forceinline__ U3 u3add(U3 x, U3 y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }

// Per-pair output counts, scanned inside the block: off[i] = exclusive prefix
// within the block, bsum[block] = block total.
__global__ __launch_bounds__(TB) void walk_count_kernel(WalkNodes w, const int2* __restrict__ fr, int64_t nf,
                                                        double theta, U3* __restrict__ off, U3* __restrict__ bsum) {
    __shared__ U3 wsum[TB / kWave];
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    U3 c{0u, 0u, 0u};
    if (i < nf) walk_step<false>(w, fr[i], theta, c, nullptr, nullptr, nullptr);
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
    U3 base{0u, 0u, 0u}, tot{0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < TB / kWave; ++k) {
        if (k < wv) base = u3add(base, wsum[k]);
        tot = u3add(tot, wsum[k]);
    }
    if (i < nf) off[i] = U3{base.a + v.a - c.a, base.b + v.b - c.b, base.c + v.c - c.c};
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block totals in place (one block), total in *total.
__global__ __launch_bounds__(TB) void walk_top_kernel(U3* __restrict__ bsum, int64_t nb, U3* __restrict__ total) {
    __shared__ U3 sh[TB];
    U3 carry{0u, 0u, 0u};
    for (int64_t c0 = 0; c0 < nb; c0 += TB) {
        const int64_t i = c0 + threadIdx.x;
        const U3 x = (i < nb) ? bsum[i] : U3{0u, 0u, 0u};
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int d = 1; d < TB; d <<= 1) {
            const U3 y = (threadIdx.x >= (unsigned)d) ? sh[threadIdx.x - d] : U3{0u, 0u, 0u};
            __syncthreads();
            sh[threadIdx.x] = u3add(sh[threadIdx.x], y);
            __syncthreads();
        }
        const U3 incl = sh[threadIdx.x];
        if (i < nb) bsum[i] = U3{carry.a + incl.a - x.a, carry.b + incl.b - x.b, carry.c + incl.c - x.c};
        const U3 last = sh[TB - 1];
        __syncthreads();
        carry = u3add(carry, last);
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(TB) void walk_emit_kernel(WalkNodes w, const int2* __restrict__ fr, int64_t nf,
                                                       double theta, const U3* __restrict__ off,
                                                       const U3* __restrict__ bsum, int2* __restrict__ next,
                                                       int2* __restrict__ far, int64_t far_base,
                                                       int2* __restrict__ near, int64_t near_base) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nf) return;
    const U3 o = off[i], b = bsum[blockIdx.x];
    U3 c{0u, 0u, 0u};
    walk_step<true>(w, fr[i], theta, c, next + (o.a + b.a), far + (far_base + o.b + b.b),
                    near + (near_base + o.c + b.c));
}

// Directed entries of the far list: (A <- B) and (B <- A).
__global__ __launch_bounds__(TB) void far_entries_kernel(const int2* __restrict__ pairs, int64_t np,
                                                         uint32_t* __restrict__ tgt, int32_t* __restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= np) return;
    const int2 p = pairs[i];
    tgt[2 * i] = (uint32_t)p.x;
    src[2 * i] = p.y;
    tgt[2 * i + 1] = (uint32_t)p.y;
    src[2 * i + 1] = p.x;
}

__global__ __launch_bounds__(TB) void near_count_kernel(const int2* __restrict__ pairs, int64_t np,
                                                        uint32_t* __restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= np) return;
    const int2 p = pairs[i];
    c[i] = p.x == p.y ? 1u : 2u;
}

__global__ __launch_bounds__(TB) void near_entries_kernel(const int2* __restrict__ pairs, int64_t np,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t* __restrict__ tgt, int32_t* __restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= np) return;
    const int2 p = pairs[i];
    const uint32_t o = off[i];
    tgt[o] = (uint32_t)p.x;
    src[o] = p.y;
    if (p.x != p.y) {
        tgt[o + 1] = (uint32_t)p.y;
        src[o + 1] = p.x;
    }
}

// CSR offsets from targets sorted ascending: off[t] = first entry with target
// >= t, for t = 0..nn (each t written by exactly one thread).
__global__ __launch_bounds__(TB) void csr_offsets_kernel(const uint32_t* __restrict__ keys, int64_t ne,
                                                         int64_t nn, uint32_t* __restrict__ off) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i > ne) return;
    const int64_t lo = (i == 0) ? 0 : (int64_t)keys[i - 1] + 1;
    const int64_t hi = (i == ne) ? nn : (int64_t)keys[i];
    for (int64_t t = lo; t <= hi; ++t) off[t] = (uint32_t)i;
}

__global__ __launch_bounds__(TB) void nonempty_from_off_kernel(const uint32_t* __restrict__ off, int64_t n,
                                                               uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) flag[i] = off[i + 1] > off[i] ? 1u : 0u;
}

__global__ __launch_bounds__(TB) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(TB) void compact_kernel(const uint32_t* __restrict__ flag,
                                                     const uint32_t* __restrict__ excl, int64_t n,
                                                     int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n && flag[i]) out[excl[i]] = (int32_t)i;
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

__global__ __launch_bounds__(TB) void entry_sources_kernel(const int32_t* __restrict__ src, int64_t ne,
                                                           const int32_t* __restrict__ count,
                                                           uint32_t* __restrict__ c) {
    const int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q < ne) c[q] = (uint32_t)count[src[q]];
}

__global__ __launch_bounds__(TB) void item_flag_kernel(const uint32_t* __restrict__ tgt,
                                                       const uint32_t* __restrict__ P,
                                                       const uint32_t* __restrict__ off, int64_t ne,
                                                       uint32_t* __restrict__ flag) {
    const int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= ne) return;
    const uint32_t q0 = off[tgt[q]];
    uint32_t f = 1u;
    if ((uint32_t)q != q0) f = ((P[q] - P[q0]) / kItemSources != (P[q - 1] - P[q0]) / kItemSources) ? 1u : 0u;
    flag[q] = f;
}

__global__ __launch_bounds__(TB) void item_build_kernel(const uint32_t* __restrict__ flag,
                                                        const uint32_t* __restrict__ excl,
                                                        const uint32_t* __restrict__ tgt, int64_t ne,
                                                        int32_t* __restrict__ it_leaf, uint32_t* __restrict__ it_q0) {
    const int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= ne || !flag[q]) return;
    const uint32_t i = excl[q];
    it_q0[i] = (uint32_t)q;
    it_leaf[i] = (int32_t)tgt[q];
}

__global__ __launch_bounds__(TB) void item_finish_kernel(int64_t T, int64_t ne, const uint32_t* __restrict__ it_q0,
                                                         const int32_t* __restrict__ it_leaf,
                                                         const int32_t* __restrict__ count,
                                                         uint32_t* __restrict__ it_q1, uint32_t* __restrict__ pc,
                                                         int32_t* __restrict__ leaf_item0) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= T) return;
    it_q1[i] = (i + 1 < T) ? it_q0[i + 1] : (uint32_t)ne;
    const int32_t L = it_leaf[i];
    const bool first_of_leaf = (i == 0 || it_leaf[i - 1] != L);
    const bool last_of_leaf = (i + 1 == T || it_leaf[i + 1] != L);
    // a leaf with a single item writes its result directly: no partial space
    pc[i] = (first_of_leaf && last_of_leaf) ? 0u : (uint32_t)count[L];
    if (first_of_leaf) leaf_item0[L] = (int32_t)i;
}

__global__ __launch_bounds__(TB) void item_count_kernel(int64_t T, const int32_t* __restrict__ it_leaf,
                                                        const int32_t* __restrict__ leaf_item0,
                                                        int32_t* __restrict__ leaf_nitems) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= T) return;
    const int32_t L = it_leaf[i];
    if (i + 1 == T || it_leaf[i + 1] != L) leaf_nitems[L] = (int32_t)(i + 1 - leaf_item0[L]);
}

unsigned grid(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, TB); }

int bits_for(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

template <typename V>
V read_back(Ctx* ctx, const V* dev, hipStream_t s) {
    TFMM_HIP(hipMemcpyAsync(ctx->pinned, dev, sizeof(V), hipMemcpyDeviceToHost, s));
    TFMM_HIP(hipStreamSynchronize(s));
    V v;
    std::memcpy(&v, ctx->pinned, sizeof(V));
    return v;
}

// Stable sort of directed (target, source) entries by target, then CSR
// offsets from the sorted targets.  The sources of every target stay in the
// walk's emission order.
void build_csr(Tree& t, DevBuf& tgtbuf, DevBuf& srcbuf, int64_t ne, DevBuf& off, DevBuf& srcout,
               hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    t.scratch2.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 8 + 256);
    uint32_t* kalt = t.scratch2.as<uint32_t>();
    int32_t* valt = reinterpret_cast<int32_t*>(kalt + std::max<int64_t>(ne, 1));
    t.scratch.ensure(ctx, sort_scratch_bytes(ne) + 1024);
    radix_sort_u32(tgtbuf.as<uint32_t>(), srcbuf.as<int32_t>(), kalt, valt, ne, bits_for(nn), t.scratch.p, s);
    off.ensure(ctx, (size_t)(nn + 1) * 4);
    hipLaunchKernelGGL(csr_offsets_kernel, dim3(grid(ne + 1)), dim3(TB), 0, s, (const uint32_t*)tgtbuf.as<uint32_t>(),
                       ne, nn, off.as<uint32_t>());
    TFMM_LAUNCHED();
    std::swap(srcbuf.p, srcout.p);
    std::swap(srcbuf.cap, srcout.cap);
    std::swap(srcbuf.ctx, srcout.ctx);
}

}  // namespace

void walk_tree(Tree& t, double theta, hipStream_t s) {
    Ctx* ctx = t.ctx;
    const int64_t nn = t.n_nodes;
    WalkNodes w{t.nd_level.as<int32_t>(), t.nd_child_first.as<int32_t>(), t.nd_nchild.as<int32_t>(),
                t.nd_Z.as<double4>(), t.nd_rmax.as<double>()};

    // frontier (int2), per-pair counts and offsets (U3); all tree-owned, grow-only
    DevBuf& fr = t.w_fr;
    DevBuf& fr2 = t.w_fr2;
    DevBuf& cnt = t.w_cnt;
    DevBuf& off = t.w_off;
    fr.ensure(ctx, 4096 * 8);
    int64_t cap_far = (int64_t)(t.m2l_pairs.cap / 8), cap_near = (int64_t)(t.p2p_pairs.cap / 8);
    if (cap_far < 4096) {
        cap_far = std::max<int64_t>(4096, 64 * nn);
        t.m2l_pairs.ensure(ctx, (size_t)cap_far * 8);
    }
    if (cap_near < 4096) {
        cap_near = std::max<int64_t>(4096, 16 * nn);
        t.p2p_pairs.ensure(ctx, (size_t)cap_near * 8);
    }
    t.scratch2.ensure(ctx, 256);
    const int2 root = make_int2(0, 0);
    TFMM_HIP(hipMemcpyAsync(fr.p, &root, sizeof(int2), hipMemcpyHostToDevice, s));
    int64_t nf = 1, n_far = 0, n_near = 0;
    while (nf > 0) {
        // every buffer resized here is idle: the previous iteration ended with a sync
        const int64_t nb = cdiv(nf, TB);
        cnt.ensure(ctx, (size_t)nf * sizeof(U3));   // per-pair offsets inside the block
        off.ensure(ctx, (size_t)nb * sizeof(U3));   // block totals -> block offsets
        hipLaunchKernelGGL(walk_count_kernel, dim3((unsigned)nb), dim3(TB), 0, s, w, fr.as<int2>(), nf, theta,
                           cnt.as<U3>(), off.as<U3>());
        TFMM_LAUNCHED();
        U3* tot = t.scratch2.as<U3>();
        hipLaunchKernelGGL(walk_top_kernel, dim3(1), dim3(TB), 0, s, off.as<U3>(), nb, tot);
        TFMM_LAUNCHED();
        const U3 T = read_back(ctx, tot, s);
        if (n_far + (int64_t)T.b > cap_far) {
            cap_far = std::max<int64_t>(2 * cap_far, n_far + T.b);
            t.m2l_pairs.ensure_keep(ctx, (size_t)cap_far * 8, s);
        }
        if (n_near + (int64_t)T.c > cap_near) {
            cap_near = std::max<int64_t>(2 * cap_near, n_near + T.c);
            t.p2p_pairs.ensure_keep(ctx, (size_t)cap_near * 8, s);
        }
        fr2.ensure(ctx, (size_t)std::max<uint32_t>(T.a, 1) * 8);
        hipLaunchKernelGGL(walk_emit_kernel, dim3((unsigned)nb), dim3(TB), 0, s, w, fr.as<int2>(), nf, theta,
                           (const U3*)cnt.as<U3>(), (const U3*)off.as<U3>(), fr2.as<int2>(), t.m2l_pairs.as<int2>(),
                           n_far, t.p2p_pairs.as<int2>(), n_near);
        TFMM_LAUNCHED();
        n_far += T.b;
        n_near += T.c;
        nf = T.a;
        std::swap(fr.p, fr2.p);
        std::swap(fr.cap, fr2.cap);
        std::swap(fr.ctx, fr2.ctx);
    }
    t.n_m2l = n_far;
    t.n_p2p = n_near;

    DevBuf& tg = t.w_tg;
    DevBuf& sr = t.w_sr;
    // far lists: directed, by target
    {
        const int64_t ne = 2 * n_far;
        tg.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 4);
        sr.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 4);
        if (n_far > 0) {
            hipLaunchKernelGGL(far_entries_kernel, dim3(grid(n_far)), dim3(TB), 0, s, t.m2l_pairs.as<int2>(),
                               n_far, tg.as<uint32_t>(), sr.as<int32_t>());
            TFMM_LAUNCHED();
        }
        build_csr(t, tg, sr, ne, t.m2l_off, t.m2l_src, s);
        // targets with a non-empty far list
        t.w_fl.ensure(ctx, (size_t)(nn + 1) * 8);
        uint32_t* flag = t.w_fl.as<uint32_t>();
        uint32_t* ex = flag + nn + 1;
        hipLaunchKernelGGL(nonempty_from_off_kernel, dim3(grid(nn)), dim3(TB), 0, s,
                           (const uint32_t*)t.m2l_off.as<uint32_t>(), nn, flag);
        TFMM_LAUNCHED();
        t.scratch.ensure(ctx, scan_scratch_bytes(nn) + 256);
        uint32_t* tot = t.scratch2.as<uint32_t>();
        exclusive_scan_u32(flag, ex, nn, t.scratch.p, tot, s);
        t.n_m2l_targets = read_back(ctx, tot, s);
        t.m2l_targets.ensure(ctx, (size_t)std::max<int64_t>(t.n_m2l_targets, 1) * 4);
        hipLaunchKernelGGL(compact_kernel, dim3(grid(nn)), dim3(TB), 0, s, (const uint32_t*)flag,
                           (const uint32_t*)ex, nn, t.m2l_targets.as<int32_t>());
        TFMM_LAUNCHED();
    }
    // near lists: directed (self pairs once), by target
    {
        t.w_c.ensure(ctx, (size_t)std::max<int64_t>(n_near, 1) * 8);
        uint32_t* c = t.w_c.as<uint32_t>();
        uint32_t* o = c + std::max<int64_t>(n_near, 1);
        hipLaunchKernelGGL(near_count_kernel, dim3(grid(n_near)), dim3(TB), 0, s, t.p2p_pairs.as<int2>(), n_near, c);
        TFMM_LAUNCHED();
        t.scratch.ensure(ctx, scan_scratch_bytes(n_near) + 256);
        uint32_t* tot = t.scratch2.as<uint32_t>();
        exclusive_scan_u32(c, o, n_near, t.scratch.p, tot, s);
        const int64_t ne = read_back(ctx, tot, s);
        tg.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 4);
        sr.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 4);
        hipLaunchKernelGGL(near_entries_kernel, dim3(grid(n_near)), dim3(TB), 0, s, t.p2p_pairs.as<int2>(), n_near,
                           (const uint32_t*)o, tg.as<uint32_t>(), sr.as<int32_t>());
        TFMM_LAUNCHED();
        build_csr(t, tg, sr, ne, t.p2p_off, t.p2p_src, s);
        // directed near particle interactions (for throughput accounting)
        unsigned long long* acc = reinterpret_cast<unsigned long long*>(t.scratch2.as<char>() + 128);
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(TB), 0, s, reinterpret_cast<int32_t*>(acc), 2, 0);
        TFMM_LAUNCHED();
        const unsigned nb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(ne, TB)));
        hipLaunchKernelGGL(near_work_kernel, dim3(nb), dim3(TB), 0, s, (const uint32_t*)tg.as<uint32_t>(),
                           (const int32_t*)t.p2p_src.as<int32_t>(), ne, t.nd_count.as<int32_t>(), acc);
        TFMM_LAUNCHED();
        t.n_near_int = (int64_t)read_back(ctx, acc, s);

        // work items over the sorted near entries (tg holds the sorted targets)
        t.w_c.ensure(ctx, (size_t)std::max<int64_t>(ne, 1) * 16);
        uint32_t* ec = t.w_c.as<uint32_t>();
        uint32_t* P = ec + std::max<int64_t>(ne, 1);
        uint32_t* fl = P + std::max<int64_t>(ne, 1);
        uint32_t* ex = fl + std::max<int64_t>(ne, 1);
        t.scratch.ensure(ctx, scan_scratch_bytes(ne) + 256);
        hipLaunchKernelGGL(entry_sources_kernel, dim3(grid(ne)), dim3(TB), 0, s, (const int32_t*)t.p2p_src.as<int32_t>(),
                           ne, t.nd_count.as<int32_t>(), ec);
        TFMM_LAUNCHED();
        uint32_t* tot2 = t.scratch2.as<uint32_t>();
        exclusive_scan_u32(ec, P, ne, t.scratch.p, tot2, s);
        hipLaunchKernelGGL(item_flag_kernel, dim3(grid(ne)), dim3(TB), 0, s, (const uint32_t*)tg.as<uint32_t>(),
                           (const uint32_t*)P, (const uint32_t*)t.p2p_off.as<uint32_t>(), ne, fl);
        TFMM_LAUNCHED();
        exclusive_scan_u32(fl, ex, ne, t.scratch.p, tot2, s);
        const int64_t T = read_back(ctx, tot2, s);
        t.n_items = T;
        t.it_leaf.ensure(ctx, (size_t)std::max<int64_t>(T, 1) * 4);
        t.it_q0.ensure(ctx, (size_t)std::max<int64_t>(T, 1) * 4);
        t.it_q1.ensure(ctx, (size_t)std::max<int64_t>(T, 1) * 4);
        t.it_pbase.ensure(ctx, (size_t)std::max<int64_t>(T, 1) * 4);
        t.leaf_item0.ensure(ctx, (size_t)(nn + 1) * 4);
        hipLaunchKernelGGL(item_build_kernel, dim3(grid(ne)), dim3(TB), 0, s, (const uint32_t*)fl, (const uint32_t*)ex,
                           (const uint32_t*)tg.as<uint32_t>(), ne, t.it_leaf.as<int32_t>(), t.it_q0.as<uint32_t>());
        TFMM_LAUNCHED();
        // per-item partial sizes reuse the entry-count scratch
        hipLaunchKernelGGL(item_finish_kernel, dim3(grid(T)), dim3(TB), 0, s, T, ne,
                           (const uint32_t*)t.it_q0.as<uint32_t>(), (const int32_t*)t.it_leaf.as<int32_t>(),
                           t.nd_count.as<int32_t>(), t.it_q1.as<uint32_t>(), ec, t.leaf_item0.as<int32_t>());
        TFMM_LAUNCHED();
        t.leaf_nitems.ensure(ctx, (size_t)(nn + 1) * 4);
        hipLaunchKernelGGL(item_count_kernel, dim3(grid(T)), dim3(TB), 0, s, T, (const int32_t*)t.it_leaf.as<int32_t>(),
                           (const int32_t*)t.leaf_item0.as<int32_t>(), t.leaf_nitems.as<int32_t>());
        TFMM_LAUNCHED();
        t.scratch.ensure(ctx, scan_scratch_bytes(T) + 256);
        exclusive_scan_u32(ec, t.it_pbase.as<uint32_t>(), T, t.scratch.p, tot2, s);
        t.n_partial = read_back(ctx, tot2, s);
    }
    t.walk_valid = true;
    t.walk_theta = theta;
}

}  // namespace tfmm
