// Near field (P2P): exact softened pair accelerations between the particles
// of every near pair of leaves, both directions, self pairs included (the
// gradient of Eq. jia with -(r^2 + eps^2)^(-1/2)).
//
// One wavefront (= one workgroup) owns one target leaf.  A chunk of nt <= 64
// target particles is laid out over the lanes as G groups of L lanes, each
// lane holding R consecutive targets (L = ceil(nt / R), G = floor(64 / L));
// group g takes every G-th staged source (the stage keeps each group's sources
// contiguous, so its loop count is uniform).  R in 1..4 is chosen per chunk to
// keep the most lanes busy (R = 1 with G replicas for small leaves, R > 1 for
// leaves of 33..64 particles), and a staged source is reused for R targets.
// Source leaves are staged into an LDS chunk already expressed in the target
// leaf's frame: the leaf-to-leaf offset Z_B - Z_A is applied in FP64 and the
// result rounded once (FP32 in the mixed path), so the inner loop is a uniform
// stream of LDS broadcasts and FMAs.  Each chunk's partial sums go into FP64
// per-lane accumulators; the groups are summed through LDS at the end.
// A leaf's list is cut into work items of bounded source count (a leaf in a
// sparse halo can be near almost every particle); every item writes its own
// partial sums and a second kernel adds a leaf's items in order.
#include <algorithm>

#include "common.h"

namespace tfmm {
namespace {

constexpr int CH = 256;   // staged source particles per chunk
static_assert(CH + kWave <= 1040, "the staging's multiply-shift division needs positions below 1040");
constexpr int UNR = 4;    // inner-loop unroll

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt_refined(x); }

template <typename T>
__device__ __forceinline__ T far_away();
template <> __device__ __forceinline__ float far_away<float>() { return 1.0e18f; }
template <> __device__ __forceinline__ double far_away<double>() { return 1.0e100; }

// POT: also the potential -m_b (r^2 + eps^2)^(-1/2) into ph.
template <typename T, bool SAFE, bool POT>
__device__ __forceinline__ void interact(const typename Vec4<T>::type& s, T tx, T ty, T tz, T eps2, T& ax,
                                         T& ay, T& az, T& ph) {
    const T dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
    const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
    const T ri = rsqrt_t(r2);
    const T mri = s.w * ri;
    T w = mri * (ri * ri);
    if (SAFE) w = (r2 > T(0)) ? w : T(0);
    ax = fma(w, dx, ax);
    ay = fma(w, dy, ay);
    az = fma(w, dz, az);
    if constexpr (POT) ph -= (SAFE && !(r2 > T(0))) ? T(0) : mri;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

constexpr int RMAX = 4;  // most targets per lane

// Lane layout of a target chunk: the R in 1..RMAX that keeps the most lanes
// busy (useful fraction nt * G / (64 * R)); ties go to the smaller R.
__device__ __forceinline__ void chunk_layout(int nt, int& R, int& L, int& G) {
    R = 1;
    L = nt;
    G = kWave / nt;
#pragma unroll
    for (int r = 2; r <= RMAX; ++r) {
        const int l = (nt + r - 1) / r;
        const int g = kWave / l;
        if (g * R > G * r) {  // nt g / r > nt G / R
            R = r;
            L = l;
            G = g;
        }
    }
}

// Interactions of one staged chunk for a lane's R targets: the ng sources its
// group owns, stored contiguously from src (the loop count is the same for
// every lane, so the loop runs on scalar registers).
template <typename T, bool SAFE, bool POT, int R>
__device__ __forceinline__ void consume(const typename Vec4<T>::type* src, int ng, const T* tx, const T* ty,
                                        const T* tz, T eps2, T* sx, T* sy, T* sz, T* sp) {
    constexpr int U = (R >= 4) ? 1 : 4 / R;
    const int nmain = ng / U * U;
    int i = 0;
    for (; i < nmain; i += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const typename Vec4<T>::type v = src[i + u];
#pragma unroll
            for (int r = 0; r < R; ++r)
                interact<T, SAFE, POT>(v, tx[r], ty[r], tz[r], eps2, sx[r], sy[r], sz[r], sp[r]);
        }
    }
    for (; i < ng; ++i) {
        const typename Vec4<T>::type v = src[i];
#pragma unroll
        for (int r = 0; r < R; ++r) interact<T, SAFE, POT>(v, tx[r], ty[r], tz[r], eps2, sx[r], sy[r], sz[r], sp[r]);
    }
}

// One staged chunk for a lane's R targets: FP32 (or FP64) partial sums of the
// chunk, then added to the lane's FP64 accumulators (inactive lanes add zeros).
template <typename T, bool SAFE, bool POT, int R>
__device__ __forceinline__ void chunk(bool act, const typename Vec4<T>::type* src, int ng, const T* tx,
                                      const T* ty, const T* tz, T eps2, double* ax, double* ay, double* az,
                                      double* ap) {
    T sx[R], sy[R], sz[R], sp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sx[r] = sy[r] = sz[r] = sp[r] = T(0);
    if (act) consume<T, SAFE, POT, R>(src, ng, tx, ty, tz, eps2, sx, sy, sz, sp);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ax[r] += (double)sx[r];
        ay[r] += (double)sy[r];
        az[r] += (double)sz[r];
        if constexpr (POT) ap[r] += (double)sp[r];
    }
}

// POT: the near-field potential too (-sum m_b (r^2 + eps^2)^(-1/2), the
// particle's own term included when eps > 0; the caller removes it).
template <typename T, bool SAFE, bool POT>
__global__ __launch_bounds__(kWave) void p2p_kernel(const int32_t* __restrict__ it_leaf,
                                                    const uint32_t* __restrict__ it_q0,
                                                    const uint32_t* __restrict__ it_q1,
                                                    const uint32_t* __restrict__ it_pbase,
                                                    const int32_t* __restrict__ first,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ src,
                                                    const double4* __restrict__ Z,
                                                    const typename Vec4<T>::type* __restrict__ P, T eps2,
                                                    const int32_t* __restrict__ leaf_nitems,
                                                    double* __restrict__ partial, double* __restrict__ near,
                                                    double* __restrict__ partial_pot,
                                                    double* __restrict__ near_pot) {
    using V4 = typename Vec4<T>::type;
    constexpr int SPL = CH / kWave;  // staged sources per lane per chunk
    __shared__ V4 stage[CH + 2 * kWave];
    __shared__ int e_start[kWave];
    __shared__ int e_first[kWave];
    __shared__ double e_off[3][kWave];
    __shared__ double red[POT ? 4 : 3][kWave];
    const int lane = threadIdx.x;
    // work items (in target leaf order) in chunks of 32 per XCD
    const uint32_t blk = xcd_block<32>(blockIdx.x, gridDim.x);
    const int32_t A = it_leaf[blk];
    const int32_t fa = first[A], na = count[A];
    const double4 za = Z[A];
    const uint32_t q0 = it_q0[blk], q1 = it_q1[blk];
    // a leaf served by one item writes the result, otherwise its own partial slot
    const bool whole = leaf_nitems[A] == 1;
    double* out = whole ? near + 3 * (int64_t)fa : partial + 3 * (int64_t)it_pbase[blk];
    double* pout = nullptr;
    if constexpr (POT) pout = whole ? near_pot + fa : partial_pot + it_pbase[blk];
    V4 pad;
    pad.x = far_away<T>();
    pad.y = far_away<T>();
    pad.z = far_away<T>();
    pad.w = T(0);

    for (int32_t tc = 0; tc < na; tc += kWave) {
        const int nt = (na - tc) < kWave ? (na - tc) : kWave;
        int R, L, G;
        chunk_layout(nt, R, L, G);
        const int l = lane % L;
        const int g = lane / L;
        const bool act = g < G;
        // the lane's targets l R + r; slots past nt repeat a valid target and are dropped
        T tx[RMAX], ty[RMAX], tz[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            int ti = l * R + r;
            ti = ti < nt ? ti : nt - 1;
            const V4 me = P[fa + tc + ti];
            tx[r] = me.x;
            ty[r] = me.y;
            tz[r] = me.z;
        }
        double ax[RMAX], ay[RMAX], az[RMAX], ap[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) ax[r] = ay[r] = az[r] = ap[r] = 0.0;

        for (uint32_t qb = q0; qb < q1; qb += kWave) {
            // one list entry per lane: source leaf, its range and its offset
            const int ne = (int)((q1 - qb) < (uint32_t)kWave ? (q1 - qb) : (uint32_t)kWave);
            int nb = 0;
            if (lane < ne) {
                const int32_t B = src[qb + lane];
                const double4 zb = Z[B];
                nb = count[B];
                e_first[lane] = first[B];
                e_off[0][lane] = zb.x - za.x;
                e_off[1][lane] = zb.y - za.y;
                e_off[2][lane] = zb.z - za.z;
            }
            const int incl = wave_incl_scan(nb);
            const int total = __shfl(incl, kWave - 1, kWave);
            e_start[lane] = (lane < ne) ? incl - nb : 0x7fffffff;
            __syncthreads();

            for (int c0 = 0; c0 < total; c0 += CH) {
                const int cnt = (total - c0) < CH ? (total - c0) : CH;
                // stage: lane takes the consecutive sources c0 + SPL lane + k; the
                // entry of the first by binary search, then at most one step per
                // source (every entry holds at least one source)
                int idx[SPL], ent[SPL];
                {
                    const int s0 = c0 + SPL * lane;
                    int lo = 0;
#pragma unroll
                    for (int st = kWave / 2; st > 0; st >>= 1)
                        if (e_start[lo + st] <= s0) lo += st;
#pragma unroll
                    for (int k = 0; k < SPL; ++k) {
                        const int sidx = s0 + k;
                        if (k > 0 && lo + 1 < kWave && e_start[lo + 1] <= sidx) ++lo;
                        ent[k] = lo;
                        idx[k] = e_first[lo] + (sidx - e_start[lo]);
                    }
                }
                V4 v[SPL];
#pragma unroll
                for (int k = 0; k < SPL; ++k)
                    if (SPL * lane + k < cnt) v[k] = P[idx[k]];
                // the chunk padded to a multiple of G; group g owns sources
                // g, g + G, ..., stored contiguously at g * gs (gs odd, so the
                // groups' reads of one step fall in distinct LDS banks)
                const int cp = (cnt + G - 1) / G * G;
                const int ng = __builtin_amdgcn_readfirstlane(cp / G);  // the same on every lane
                const int gs = ng | 1;
                // c / G for c < CH + kWave as (c * gm) >> 16, gm = ceil(2^16 / G): exact
                // while c * (gm G - 2^16) < 2^16, i.e. for every c below 1040
                const uint32_t gm = (uint32_t)__builtin_amdgcn_readfirstlane((65536 + G - 1) / G);
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    const int c = SPL * lane + k;
                    if (c < cnt) {
                        V4 w;
                        w.x = (T)((double)v[k].x + e_off[0][ent[k]]);
                        w.y = (T)((double)v[k].y + e_off[1][ent[k]]);
                        w.z = (T)((double)v[k].z + e_off[2][ent[k]]);
                        w.w = v[k].w;
                        const int q = (int)(((uint32_t)c * gm) >> 16);
                        stage[(c - q * G) * gs + q] = w;
                    }
                }
                if (cnt + lane < cp) {
                    const int c = cnt + lane;
                    const int q = (int)(((uint32_t)c * gm) >> 16);
                    stage[(c - q * G) * gs + q] = pad;
                }
                __syncthreads();
                const V4* src = stage + g * gs;
                switch (R) {
                    case 1: chunk<T, SAFE, POT, 1>(act, src, ng, tx, ty, tz, eps2, ax, ay, az, ap); break;
                    case 2: chunk<T, SAFE, POT, 2>(act, src, ng, tx, ty, tz, eps2, ax, ay, az, ap); break;
                    case 3: chunk<T, SAFE, POT, 3>(act, src, ng, tx, ty, tz, eps2, ax, ay, az, ap); break;
                    default: chunk<T, SAFE, POT, 4>(act, src, ng, tx, ty, tz, eps2, ax, ay, az, ap); break;
                }
                __syncthreads();
            }
        }

        // target t = l R + r sits in slot r of lanes l, l + L, ..., one per
        // group; slot by slot, through LDS
        const int tl = lane / R, tr = lane % R;
        double fx = 0.0, fy = 0.0, fz = 0.0, fp = 0.0;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < R) {
                red[0][lane] = ax[r];
                red[1][lane] = ay[r];
                red[2][lane] = az[r];
                if constexpr (POT) red[POT ? 3 : 0][lane] = ap[r];
                __syncthreads();
                if (lane < nt && tr == r) {
                    for (int q = 0; q < G; ++q) {
                        fx += red[0][q * L + tl];
                        fy += red[1][q * L + tl];
                        fz += red[2][q * L + tl];
                        if constexpr (POT) fp += red[POT ? 3 : 0][q * L + tl];
                    }
                }
                __syncthreads();
            }
        }
        if (lane < nt) {
            const int64_t j = (int64_t)(tc + lane);
            out[3 * j] = fx;
            out[3 * j + 1] = fy;
            out[3 * j + 2] = fz;
            if constexpr (POT) pout[j] = fp;
        }
    }
}

// Leaves served by several items (listed in multi_leaf, in any order): one
// wavefront per such leaf adds the items' partial sums in item order.  The
// grid is an upper bound of the list length; the surplus wavefronts exit.
template <bool POT>
__global__ __launch_bounds__(kWave) void p2p_reduce_kernel(const int32_t* __restrict__ multi_leaf,
                                                           const uint32_t* __restrict__ multi_count,
                                                           const int32_t* __restrict__ leaf_item0,
                                                           const int32_t* __restrict__ leaf_nitems,
                                                           const int32_t* __restrict__ first,
                                                           const int32_t* __restrict__ count,
                                                           const uint32_t* __restrict__ it_pbase,
                                                           const double* __restrict__ partial,
                                                           double* __restrict__ near,
                                                           const double* __restrict__ partial_pot,
                                                           double* __restrict__ near_pot) {
    if (blockIdx.x >= *multi_count) return;
    const int32_t L = multi_leaf[blockIdx.x];
    const int32_t ni = leaf_nitems[L], i0 = leaf_item0[L];
    const int32_t fa = first[L], na = count[L];
    constexpr int B = 8;  // items whose rows are loaded together (sums stay in item order)
    for (int32_t r = threadIdx.x; r < na; r += kWave) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
        for (int32_t i = 0; i < ni; i += B) {
            int64_t row[B];
#pragma unroll
            for (int u = 0; u < B; ++u) row[u] = i + u < ni ? (int64_t)it_pbase[i0 + i + u] + r : 0;
            double v[B][4];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                if (i + u < ni) {
                    const double* p = partial + 3 * row[u];
                    v[u][0] = p[0];
                    v[u][1] = p[1];
                    v[u][2] = p[2];
                    if constexpr (POT) v[u][3] = partial_pot[row[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                if (i + u < ni) {
                    sx += v[u][0];
                    sy += v[u][1];
                    sz += v[u][2];
                    if constexpr (POT) sp += v[u][3];
                }
            }
        }
        near[3 * (int64_t)(fa + r)] = sx;
        near[3 * (int64_t)(fa + r) + 1] = sy;
        near[3 * (int64_t)(fa + r) + 2] = sz;
        if constexpr (POT) near_pot[fa + r] = sp;
    }
}

template <typename T, bool POT>
void launch(Tree& t, double eps2, hipStream_t s) {
    using V4 = typename Vec4<T>::type;
    const int64_t ni = t.n_items;
    if (ni <= 0) return;
    const dim3 g((unsigned)ni);
    double* ppot = POT ? t.partial_pot.as<double>() : nullptr;
    double* npot = POT ? t.near_pot.as<double>() : nullptr;
    if (eps2 > 0.0)
        hipLaunchKernelGGL((p2p_kernel<T, false, POT>), g, dim3(kWave), 0, s, t.it_leaf.as<int32_t>(),
                           t.it_q0.as<uint32_t>(), t.it_q1.as<uint32_t>(), t.it_pbase.as<uint32_t>(),
                           t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(), t.p2p_src.as<int32_t>(),
                           t.nd_Z.as<double4>(), t.src4.as<V4>(), (T)eps2, t.leaf_nitems.as<int32_t>(),
                           t.partial.as<double>(), t.near3.as<double>(), ppot, npot);
    else
        hipLaunchKernelGGL((p2p_kernel<T, true, POT>), g, dim3(kWave), 0, s, t.it_leaf.as<int32_t>(),
                           t.it_q0.as<uint32_t>(), t.it_q1.as<uint32_t>(), t.it_pbase.as<uint32_t>(),
                           t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(), t.p2p_src.as<int32_t>(),
                           t.nd_Z.as<double4>(), t.src4.as<V4>(), (T)eps2, t.leaf_nitems.as<int32_t>(),
                           t.partial.as<double>(), t.near3.as<double>(), ppot, npot);
    TFMM_LAUNCHED();
}

template <bool POT>
void launch_reduce(Tree& t, hipStream_t s) {
    const int64_t ni = t.n_items;
    if (ni <= 0) return;
    double* ppot = POT ? t.partial_pot.as<double>() : nullptr;
    double* npot = POT ? t.near_pot.as<double>() : nullptr;
    // every leaf has at least one item, so at most n_items - n_leaves leaves have several
    const int64_t nmulti = ni - t.n_leaves;
    if (nmulti > 0) {
        hipLaunchKernelGGL((p2p_reduce_kernel<POT>), dim3((unsigned)nmulti), dim3(kWave), 0, s,
                           t.multi_leaf.as<int32_t>(), t.multi_count, t.leaf_item0.as<int32_t>(),
                           t.leaf_nitems.as<int32_t>(), t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(),
                           t.it_pbase.as<uint32_t>(), t.partial.as<double>(), t.near3.as<double>(),
                           (const double*)ppot, npot);
        TFMM_LAUNCHED();
    }
}

}  // namespace

// The partial sums of leaves whose near list was cut into several items
// (after run_p2p on the same stream).
void run_p2p_reduce(Tree& t, bool with_pot, hipStream_t s) {
    if (with_pot) launch_reduce<true>(t, s);
    else launch_reduce<false>(t, s);
}

void run_p2p(Tree& t, int precision, double eps2, bool with_pot, hipStream_t s) {
    t.near3.ensure(t.ctx, (size_t)t.n * 24);
    t.partial.ensure(t.ctx, (size_t)std::max<int64_t>(t.n_partial, 1) * 24);
    if (with_pot) {
        t.near_pot.ensure(t.ctx, (size_t)t.n * 8);
        t.partial_pot.ensure(t.ctx, (size_t)std::max<int64_t>(t.n_partial, 1) * 8);
        if (precision == TFMM_MIXED32) launch<float, true>(t, eps2, s);
        else launch<double, true>(t, eps2, s);
    } else {
        if (precision == TFMM_MIXED32) launch<float, false>(t, eps2, s);
        else launch<double, false>(t, eps2, s);
    }
}

}  // namespace tfmm
