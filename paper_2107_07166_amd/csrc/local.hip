// Downward pass in FP64: local expansions moved to the leaves (L2L) and
// evaluated at the particles (L2P) -- the paper's step (ii), Sec. 2: the
// Taylor expansion from each node's centre of mass to the particle positions.
//
// A local expansion is a polynomial about its node's centre, so moving it to
// a descendant's centre is an exact re-expansion.  Up to p = 4 each leaf
// gathers the M2L results of itself and of all its ancestors, each shifted
// directly from the ancestor's centre to the leaf's (the composition of the
// level-by-level shifts, in one pass); from p = 5 the shifts run level by
// level (below):
//   standard   : L_leaf = sum_A shift(L_A, d_A),  d_A = Z_leaf - Z_A;
//   conserving : P_leaf = sum_A shift(P_A, d_A),
//                Q'_e,leaf = sum_A shift(Q'_e,A - d_A,e P_A, d_A)
// (the vector field -x_e P(x) + Q'_e(x) re-expanded about the new centre).
// L2P then evaluates a_e = -sum_j L_{j+e} x^j / j!  or  -x_e P(x) + Q'_e(x)
// at x = X_a - Z_leaf and writes F_a = G m_a (near + far) in the caller's
// particle order.
#include <algorithm>

#include "common.h"
#include "expansions_gen.h"

namespace tfmm {
namespace {

constexpr int LB = 128;

// Orders whose downward pass runs level by level (each node shifted once, one
// launch per level) instead of by direct ancestor-to-leaf shifts (one launch,
// every ancestor shifted once per leaf).  On the 2^22-particle disk at p = 6
// the level-by-level pass takes 0.19 / 0.43 ms (standard / conserving)
// against 0.24 / 0.76 ms; on 2^20 Plummer particles at p = 4 it is slower
// (0.086 / 0.073 against 0.026 / 0.065 ms), the launches outweighing the
// cheaper shifts.
constexpr int kL2LByLevelP = 5;

template <int P>
__global__ __launch_bounds__(LB) void l2l_std_kernel(int64_t n_leaves, const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ parent,
                                                     const double4* __restrict__ Z,
                                                     const uint32_t* __restrict__ m2l_off,
                                                     const double* __restrict__ loc,
                                                     double* __restrict__ loc_leaf) {
    using E = Expansion<P>;
    constexpr int NC = E::NC;
    const int64_t i = (int64_t)blockIdx.x * LB + threadIdx.x;
    if (i >= n_leaves) return;
    const int32_t leaf = leaves[i];
    const double4 zl = Z[leaf];
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    for (int32_t A = leaf; A >= 0; A = parent[A]) {
        if (m2l_off[A + 1] == m2l_off[A]) continue;
        const double4 za = Z[A];
        E::shift_std(loc + (int64_t)A * NC, zl.x - za.x, zl.y - za.y, zl.z - za.z, acc);
    }
    double* out = loc_leaf + (int64_t)leaf * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = acc[k];
}

// Conserving: thread (leaf, part); part 0 -> P, part e+1 -> Q'_e.
template <int P>
__global__ __launch_bounds__(LB) void l2l_cons_kernel(int64_t n_leaves, const int32_t* __restrict__ leaves,
                                                      const int32_t* __restrict__ parent,
                                                      const double4* __restrict__ Z,
                                                      const uint32_t* __restrict__ m2l_off,
                                                      const double* __restrict__ loc,
                                                      double* __restrict__ loc_leaf) {
    constexpr int NC1 = Expansion<P>::NC1;
    constexpr int NLOC = 4 * NC1;
    const int64_t t = (int64_t)blockIdx.x * LB + threadIdx.x;
    const int64_t i = t >> 2;
    const int part = (int)(t & 3);
    if (i >= n_leaves) return;
    const int32_t leaf = leaves[i];
    const double4 zl = Z[leaf];
    double acc[NC1];
#pragma unroll
    for (int k = 0; k < NC1; ++k) acc[k] = 0.0;
    for (int32_t A = leaf; A >= 0; A = parent[A]) {
        if (m2l_off[A + 1] == m2l_off[A]) continue;
        const double4 za = Z[A];
        const double d[3] = {zl.x - za.x, zl.y - za.y, zl.z - za.z};
        const double* la = loc + (int64_t)A * NLOC;
        if constexpr (P == 1) {
            if (part == 0) acc[0] += la[0];
            else acc[0] += la[part] - d[part - 1] * la[0];
        } else {
            using E1 = Expansion<P - 1>;
            if (part == 0) {
                E1::shift_std(la, d[0], d[1], d[2], acc);
            } else {
                // the shift is linear: shift(Q'_e) - d_e shift(P) = shift(Q'_e - d_e P)
                const double de = d[part - 1];
                double v[NC1];
#pragma unroll
                for (int k = 0; k < NC1; ++k) v[k] = fma(-de, la[k], la[part * NC1 + k]);
                E1::shift_std(v, d[0], d[1], d[2], acc);
            }
        }
    }
    double* out = loc_leaf + (int64_t)leaf * NLOC + part * NC1;
#pragma unroll
    for (int k = 0; k < NC1; ++k) out[k] = acc[k];
}

// Level-by-level downward pass: a node's local expansion is its own M2L
// result plus its parent's expansion shifted to its centre, one launch per
// level (the top levels, at most kTopNodes nodes, in one block).  has[i] is 1
// when node i or one of its ancestors has a non-empty far list; only such
// nodes' expansions are written, and every leaf's (zeros if none).  Each node
// is shifted once, instead of every ancestor once per leaf.
//   standard   : L_i = L_own + shift(L_parent, d),  d = Z_i - Z_parent;
//   conserving : P_i = P_own + shift(P_parent, d),
//                Q'_e,i = Q'_e,own + shift(Q'_e,parent - d_e P_parent, d).
// Thread (node, part): part 0 only for the standard variant; parts 0..3
// (P, Q'_x, Q'_y, Q'_z) for the conserving one.
template <int P, int VAR>
__device__ __forceinline__ void l2l_node(int32_t i, int part, const int32_t* __restrict__ parent,
                                         const int32_t* __restrict__ nchild, const double4* __restrict__ Z,
                                         const uint32_t* __restrict__ m2l_off, const double* __restrict__ loc,
                                         double* __restrict__ acc_out, uint8_t* __restrict__ has) {
    constexpr bool CONS = VAR == TFMM_CONSERVING;
    constexpr int NP = CONS ? Expansion<P>::NC1 : Expansion<P>::NC;  // coefficients per part
    constexpr int NLOC = CONS ? 4 * NP : NP;
    const bool own = m2l_off[i + 1] > m2l_off[i];
    const int32_t par = parent[i];
    const bool inherit = par >= 0 && has[par] != 0;
    double* out = acc_out + (int64_t)i * NLOC + part * NP;
    if (!own && !inherit) {
        if (part == 0) has[i] = 0;
        if (nchild[i] == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) out[k] = 0.0;
        }
        return;
    }
    double acc[NP];
    if (own) {
        const double* lo = loc + (int64_t)i * NLOC + part * NP;
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = lo[k];
    } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = 0.0;
    }
    if (inherit) {
        const double4 zi = Z[i], zp = Z[par];
        const double d[3] = {zi.x - zp.x, zi.y - zp.y, zi.z - zp.z};
        const double* la = acc_out + (int64_t)par * NLOC;
        if constexpr (!CONS) {
            Expansion<P>::shift_std(la, d[0], d[1], d[2], acc);
        } else if constexpr (P == 1) {
            if (part == 0) acc[0] += la[0];
            else acc[0] += la[part] - d[part - 1] * la[0];
        } else {
            using E1 = Expansion<P - 1>;
            if (part == 0) {
                E1::shift_std(la, d[0], d[1], d[2], acc);
            } else {
                const double de = d[part - 1];
                double v[NP];
#pragma unroll
                for (int k = 0; k < NP; ++k) v[k] = fma(-de, la[k], la[part * NP + k]);
                E1::shift_std(v, d[0], d[1], d[2], acc);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) out[k] = acc[k];
    if (part == 0) has[i] = 1;
}

template <int P, int VAR>
__global__ __launch_bounds__(LB) void l2l_level_kernel(int32_t b, int32_t e, const int32_t* __restrict__ parent,
                                                       const int32_t* __restrict__ nchild,
                                                       const double4* __restrict__ Z,
                                                       const uint32_t* __restrict__ m2l_off,
                                                       const double* __restrict__ loc, double* __restrict__ acc_out,
                                                       uint8_t* __restrict__ has) {
    constexpr int PARTS = VAR == TFMM_CONSERVING ? 4 : 1;
    const int64_t t = (int64_t)blockIdx.x * LB + threadIdx.x;
    const int64_t i = b + t / PARTS;
    if (i >= e) return;
    l2l_node<P, VAR>((int32_t)i, (int)(t % PARTS), parent, nchild, Z, m2l_off, loc, acc_out, has);
}

struct LevelRange {
    int32_t b[kLevels + 2];
};

// The top levels in one block, level after level.
template <int P, int VAR>
__global__ __launch_bounds__(LB) void l2l_top_kernel(LevelRange lv, int top, const int32_t* __restrict__ parent,
                                                     const int32_t* __restrict__ nchild,
                                                     const double4* __restrict__ Z,
                                                     const uint32_t* __restrict__ m2l_off,
                                                     const double* __restrict__ loc, double* __restrict__ acc_out,
                                                     uint8_t* __restrict__ has) {
    constexpr int PARTS = VAR == TFMM_CONSERVING ? 4 : 1;
    for (int L = 0; L <= top; ++L) {
        const int64_t cnt = (int64_t)(lv.b[L + 1] - lv.b[L]) * PARTS;
        for (int64_t t = threadIdx.x; t < cnt; t += LB)
            l2l_node<P, VAR>(lv.b[L] + (int32_t)(t / PARTS), (int)(t % PARTS), parent, nchild, Z, m2l_off, loc,
                             acc_out, has);
        __syncthreads();
    }
}

template <int P, int VAR>
void l2l_levels(Tree& t, hipStream_t s) {
    constexpr int PARTS = VAR == TFMM_CONSERVING ? 4 : 1;
    constexpr int64_t kTopNodes = LB;
    t.loc_has.ensure(t.ctx, (size_t)std::max<int64_t>(t.n_nodes, 1));
    int top = -1;
    while (top + 1 <= t.max_level && t.level_begin[(size_t)top + 2] <= kTopNodes) ++top;
    if (top >= 0) {
        LevelRange lv{};
        for (int L = 0; L <= top + 1; ++L) lv.b[L] = (int32_t)t.level_begin[L];
        hipLaunchKernelGGL((l2l_top_kernel<P, VAR>), dim3(1), dim3(LB), 0, s, lv, top, t.nd_parent.as<int32_t>(),
                           t.nd_nchild.as<int32_t>(), t.nd_Z.as<double4>(), t.m2l_off.as<uint32_t>(),
                           t.loc.as<double>(), t.loc_leaf.as<double>(), t.loc_has.as<uint8_t>());
        TFMM_LAUNCHED();
    }
    for (int L = top + 1; L <= t.max_level; ++L) {
        const int32_t b = (int32_t)t.level_begin[L], e = (int32_t)t.level_begin[L + 1];
        if (e <= b) continue;
        hipLaunchKernelGGL((l2l_level_kernel<P, VAR>), dim3((unsigned)cdiv((int64_t)(e - b) * PARTS, LB)), dim3(LB),
                           0, s, b, e, t.nd_parent.as<int32_t>(), t.nd_nchild.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.m2l_off.as<uint32_t>(), t.loc.as<double>(), t.loc_leaf.as<double>(),
                           t.loc_has.as<uint8_t>());
        TFMM_LAUNCHED();
    }
}

// Far-field acceleration at every particle (sorted order) from its leaf's
// locals, into far3 (three values per particle).  It runs on the tree's
// second stream right after L2L, beside the near field.
template <int P, int VAR>
__global__ __launch_bounds__(LB) void l2p_far_kernel(int64_t n, const double4* __restrict__ Xm,
                                                     const int32_t* __restrict__ leaf_of,
                                                     const double4* __restrict__ Z,
                                                     const double* __restrict__ loc_leaf,
                                                     double* __restrict__ far3) {
    using E = Expansion<P>;
    const int64_t j = (int64_t)blockIdx.x * LB + threadIdx.x;
    if (j >= n) return;
    const int32_t leaf = leaf_of[j];
    const double4 x = Xm[j];
    const double4 z = Z[leaf];
    const double dx = x.x - z.x, dy = x.y - z.y, dz = x.z - z.z;
    double a[3];
    if constexpr (VAR == TFMM_CONSERVING) {
        constexpr int NC1 = E::NC1;
        const double* l = loc_leaf + (int64_t)leaf * 4 * NC1;
        E::l2p_cons(l, l + NC1, dx, dy, dz, a);
    } else {
        E::l2p_std(loc_leaf + (int64_t)leaf * E::NC, dx, dy, dz, a);
    }
    far3[3 * j] = a[0];
    far3[3 * j + 1] = a[1];
    far3[3 * j + 2] = a[2];
}

// The same for the conserving locals from order 6 (224 or more coefficients
// per leaf), where loading them per thread is bound by the address units
// (each lane fetches the whole set although the lanes of a leaf read the
// same words).  A block's particles are consecutive in sorted order, so they
// belong to a few consecutive leaves: the block copies their locals into LDS
// once (coalesced) and every thread reads its leaf's coefficients from there.
// At most 8 leaves and 32 KB of coefficients per round; blocks spanning more
// leaves take several rounds.  On the 2^22-particle disk (p = 6) this took
// the kernel from 0.36 to 0.22 ms with the same forces bit for bit (16 slots
// per round: 0.25 ms, the staging area then limiting the kernel to fewer
// waves); at lower orders and for the standard locals (fewer coefficients,
// and the staged kernel holds more registers) it was slower.
constexpr int kL2pSlots = 8;

template <int P, int VAR>
__device__ __forceinline__ void l2p_eval(const double* __restrict__ l, double dx, double dy, double dz, double* a) {
    using E = Expansion<P>;
    if constexpr (VAR == TFMM_CONSERVING) E::l2p_cons(l, l + E::NC1, dx, dy, dz, a);
    else E::l2p_std(l, dx, dy, dz, a);
}

template <int P, int VAR>
__global__ __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(P == 6 ? 4 : 1)))
void l2p_far_staged_kernel(int64_t n, const double4* __restrict__ Xm, const int32_t* __restrict__ leaf_of,
                           const double4* __restrict__ Z, const double* __restrict__ loc_leaf,
                           double* __restrict__ far3) {
    using E = Expansion<P>;
    constexpr int NL = VAR == TFMM_CONSERVING ? 4 * E::NC1 : E::NC;  // coefficients per leaf
    constexpr int STRIDE = NL | 1;  // odd: the slots' words fall in different banks
    constexpr int SLOTS = 4096 / STRIDE < kL2pSlots ? 4096 / STRIDE : kL2pSlots;
    static_assert(SLOTS >= 1, "one leaf's locals fit the staging area");
    __shared__ double cs[SLOTS * STRIDE];
    __shared__ int32_t slot_leaf[SLOTS];
    __shared__ int wave_flags[LB / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t j0 = (int64_t)blockIdx.x * LB;
    const int64_t j = j0 + tid;
    const bool live = j < n;
    const int32_t leaf = live ? leaf_of[j] : -1;
    // a new leaf starts at j when its leaf differs from j - 1's (or j is the block's first)
    const bool start = live && (tid == 0 || leaf_of[j - 1] != leaf);
    const unsigned long long bal = __ballot(start);
    if (lane == 0) wave_flags[wv] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wave_flags[w];
    int nslots = 0;
    for (int w = 0; w < LB / kWave; ++w) nslots += wave_flags[w];
    const unsigned long long below = lane == 0 ? 0ull : (bal << (kWave - lane));
    // slot of this thread's leaf: the leaf starts counted up to and including j
    const int slot = before + __popcll(below) + (start ? 1 : 0) - 1;
    // rounds of SLOTS leaves (one round unless the leaves are tiny)
    const double4 x = live ? Xm[j] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double4 z = live ? Z[leaf] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double dx = x.x - z.x, dy = x.y - z.y, dz = x.z - z.z;
    for (int base = 0; base < nslots; base += SLOTS) {
        const int staged = nslots - base < SLOTS ? nslots - base : SLOTS;
        const bool mine = live && slot >= base && slot < base + SLOTS;
        if (start && mine) slot_leaf[slot - base] = leaf;
        __syncthreads();
        for (int idx = tid; idx < staged * NL; idx += LB) {
            const int sl = idx / NL, k = idx - sl * NL;
            cs[sl * STRIDE + k] = loc_leaf[(int64_t)slot_leaf[sl] * NL + k];
        }
        __syncthreads();
        if (mine) {
            double a[3];
            l2p_eval<P, VAR>(cs + (slot - base) * STRIDE, dx, dy, dz, a);
            far3[3 * j] = a[0];
            far3[3 * j + 1] = a[1];
            far3[3 * j + 2] = a[2];
        }
        __syncthreads();
    }
}

// The force G m (near + far) of every particle, into its caller-order slot.
__global__ __launch_bounds__(LB) void force_combine_kernel(int64_t n, const double4* __restrict__ Xm,
                                                           const int32_t* __restrict__ perm,
                                                           const double* __restrict__ near,
                                                           const double* __restrict__ far3, double G,
                                                           double* __restrict__ force) {
    const int64_t j = (int64_t)blockIdx.x * LB + threadIdx.x;
    if (j >= n) return;
    const double s = G * Xm[j].w;
    const int64_t o = perm[j];
    force[3 * o] = s * (near[3 * j] + far3[3 * j]);
    force[3 * o + 1] = s * (near[3 * j + 1] + far3[3 * j + 1]);
    force[3 * o + 2] = s * (near[3 * j + 2] + far3[3 * j + 2]);
}

// Potential output: phi_a = sum_{|j| <= p} L_j x^j / j! (standard locals with
// L_0, of the same node pairs) + the near-field sum, less the particle's own
// term -m_a / eps that the near-field kernel includes when eps > 0 (removed
// in the precision it was added in); pot[a] = G phi_a in caller order.
template <int P, typename TS>
__global__ __launch_bounds__(LB) void l2p_pot_kernel(int64_t n, const double4* __restrict__ Xm,
                                                     const int32_t* __restrict__ leaf_of,
                                                     const int32_t* __restrict__ perm,
                                                     const double4* __restrict__ Z,
                                                     const double* __restrict__ loc_leaf,
                                                     const double* __restrict__ near_pot, double eps2, double G,
                                                     double* __restrict__ pot) {
    using E = Expansion<P>;
    const int64_t j = (int64_t)blockIdx.x * LB + threadIdx.x;
    if (j >= n) return;
    const int32_t leaf = leaf_of[j];
    const double4 x = Xm[j];
    const double4 z = Z[leaf];
    double phi = E::l2p_pot(loc_leaf + (int64_t)leaf * E::NC, x.x - z.x, x.y - z.y, x.z - z.z) + near_pot[j];
    if (eps2 > 0.0) {
        if constexpr (sizeof(TS) == 4) phi += (double)((float)x.w * __builtin_amdgcn_rsqf((float)eps2));
        else phi += x.w * rsqrt_refined(eps2);
    }
    pot[perm[j]] = G * phi;
}

template <int P>
void potential_down(Tree& t, int precision, double eps2, double G, double* pot, hipStream_t s) {
    const int64_t nl = t.n_leaves, n = t.n;
    t.loc_pot_leaf.ensure(t.ctx, (size_t)t.n_nodes * Expansion<P>::NC * 8);
    hipLaunchKernelGGL(l2l_std_kernel<P>, dim3((unsigned)cdiv(nl, LB)), dim3(LB), 0, s, nl, t.leaves.as<int32_t>(),
                       t.nd_parent.as<int32_t>(), t.nd_Z.as<double4>(), t.m2l_off.as<uint32_t>(),
                       t.loc_pot.as<double>(), t.loc_pot_leaf.as<double>());
    TFMM_LAUNCHED();
    if (precision == TFMM_MIXED32)
        hipLaunchKernelGGL((l2p_pot_kernel<P, float>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.perm.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_pot_leaf.as<double>(), t.near_pot.as<double>(), eps2, G, pot);
    else
        hipLaunchKernelGGL((l2p_pot_kernel<P, double>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.perm.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_pot_leaf.as<double>(), t.near_pot.as<double>(), eps2, G, pot);
    TFMM_LAUNCHED();
}

template <int P>
void l2l_dispatch(Tree& t, int variant, hipStream_t s) {
    const int64_t nl = t.n_leaves;
    if constexpr (P >= kL2LByLevelP) {
        if (variant == TFMM_CONSERVING) l2l_levels<P, TFMM_CONSERVING>(t, s);
        else l2l_levels<P, TFMM_STANDARD>(t, s);
        return;
    }
    if (variant == TFMM_CONSERVING)
        hipLaunchKernelGGL(l2l_cons_kernel<P>, dim3((unsigned)cdiv(nl * 4, LB)), dim3(LB), 0, s, nl,
                           t.leaves.as<int32_t>(), t.nd_parent.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.m2l_off.as<uint32_t>(), t.loc.as<double>(), t.loc_leaf.as<double>());
    else
        hipLaunchKernelGGL(l2l_std_kernel<P>, dim3((unsigned)cdiv(nl, LB)), dim3(LB), 0, s, nl,
                           t.leaves.as<int32_t>(), t.nd_parent.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.m2l_off.as<uint32_t>(), t.loc.as<double>(), t.loc_leaf.as<double>());
    TFMM_LAUNCHED();
}

template <int P>
void l2p_far_dispatch(Tree& t, int variant, hipStream_t s) {
    const int64_t n = t.n;
    if constexpr (P >= 6) {
        if (variant == TFMM_CONSERVING) {
            hipLaunchKernelGGL((l2p_far_staged_kernel<P, TFMM_CONSERVING>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0,
                               s, n, t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.nd_Z.as<double4>(),
                               t.loc_leaf.as<double>(), t.far3.as<double>());
            TFMM_LAUNCHED();
            return;
        }
    }
    if (variant == TFMM_CONSERVING)
        hipLaunchKernelGGL((l2p_far_kernel<P, TFMM_CONSERVING>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_leaf.as<double>(), t.far3.as<double>());
    else
        hipLaunchKernelGGL((l2p_far_kernel<P, TFMM_STANDARD>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_leaf.as<double>(), t.far3.as<double>());
    TFMM_LAUNCHED();
}

}  // namespace

void run_l2l(Tree& t, int p, int variant, hipStream_t s) {
    const int nloc = n_local(p, variant);
    t.loc_leaf.ensure(t.ctx, (size_t)t.n_nodes * nloc * 8);
    switch (p) {
        case 1: l2l_dispatch<1>(t, variant, s); break;
        case 2: l2l_dispatch<2>(t, variant, s); break;
        case 3: l2l_dispatch<3>(t, variant, s); break;
        case 4: l2l_dispatch<4>(t, variant, s); break;
        case 5: l2l_dispatch<5>(t, variant, s); break;
        case 6: l2l_dispatch<6>(t, variant, s); break;
        case 7: l2l_dispatch<7>(t, variant, s); break;
        case 8: l2l_dispatch<8>(t, variant, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

// L2L of the potential locals (t.loc_pot) and the potential at every particle.
void run_potential_down(Tree& t, int p, int precision, double eps2, double G, double* pot, hipStream_t s) {
    switch (p) {
        case 1: potential_down<1>(t, precision, eps2, G, pot, s); break;
        case 2: potential_down<2>(t, precision, eps2, G, pot, s); break;
        case 3: potential_down<3>(t, precision, eps2, G, pot, s); break;
        case 4: potential_down<4>(t, precision, eps2, G, pot, s); break;
        case 5: potential_down<5>(t, precision, eps2, G, pot, s); break;
        case 6: potential_down<6>(t, precision, eps2, G, pot, s); break;
        case 7: potential_down<7>(t, precision, eps2, G, pot, s); break;
        case 8: potential_down<8>(t, precision, eps2, G, pot, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

void run_l2p_far(Tree& t, int p, int variant, hipStream_t s) {
    t.far3.ensure(t.ctx, (size_t)t.n * 24);
    switch (p) {
        case 1: l2p_far_dispatch<1>(t, variant, s); break;
        case 2: l2p_far_dispatch<2>(t, variant, s); break;
        case 3: l2p_far_dispatch<3>(t, variant, s); break;
        case 4: l2p_far_dispatch<4>(t, variant, s); break;
        case 5: l2p_far_dispatch<5>(t, variant, s); break;
        case 6: l2p_far_dispatch<6>(t, variant, s); break;
        case 7: l2p_far_dispatch<7>(t, variant, s); break;
        case 8: l2p_far_dispatch<8>(t, variant, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

void run_force_combine(Tree& t, double G, double* force, hipStream_t s) {
    const int64_t n = t.n;
    hipLaunchKernelGGL(force_combine_kernel, dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n, t.Xm.as<double4>(),
                       t.perm.as<int32_t>(), t.near3.as<double>(), t.far3.as<double>(), G, force);
    TFMM_LAUNCHED();
}

}  // namespace tfmm
