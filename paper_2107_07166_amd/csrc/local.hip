// Downward pass in FP64: local expansions moved to the leaves (L2L) and
// evaluated at the particles (L2P) -- the paper's step (ii), Sec. 2: the
// Taylor expansion from each node's centre of mass to the particle positions.
//
// A local expansion is a polynomial about its node's centre, so moving it to
// a descendant's centre is an exact re-expansion.  Each leaf gathers the M2L
// results of itself and of all its ancestors, each shifted directly from the
// ancestor's centre to the leaf's (the composition of the level-by-level
// shifts, in one pass):
//   standard   : L_leaf = sum_A shift(L_A, d_A),  d_A = Z_leaf - Z_A;
//   conserving : P_leaf = sum_A shift(P_A, d_A),
//                Q'_e,leaf = sum_A shift(Q'_e,A - d_A,e P_A, d_A)
// (the vector field -x_e P(x) + Q'_e(x) re-expanded about the new centre).
// L2P then evaluates a_e = -sum_j L_{j+e} x^j / j!  or  -x_e P(x) + Q'_e(x)
// at x = X_a - Z_leaf and writes F_a = G m_a (near + far) in the caller's
// particle order.
#include "common.h"
#include "expansions_gen.h"

namespace tfmm {
namespace {

constexpr int LB = 128;

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

template <int P, int VAR>
__global__ __launch_bounds__(LB) void l2p_kernel(int64_t n, const double4* __restrict__ Xm,
                                                 const int32_t* __restrict__ leaf_of,
                                                 const int32_t* __restrict__ perm,
                                                 const double4* __restrict__ Z,
                                                 const double* __restrict__ loc_leaf,
                                                 const double* __restrict__ near, double G,
                                                 double* __restrict__ force) {
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
    const double s = G * x.w;
    const int64_t o = perm[j];
    force[3 * o] = s * (near[3 * j] + a[0]);
    force[3 * o + 1] = s * (near[3 * j + 1] + a[1]);
    force[3 * o + 2] = s * (near[3 * j + 2] + a[2]);
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
void l2p_dispatch(Tree& t, int variant, double G, double* force, hipStream_t s) {
    const int64_t n = t.n;
    if (variant == TFMM_CONSERVING)
        hipLaunchKernelGGL((l2p_kernel<P, TFMM_CONSERVING>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.perm.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_leaf.as<double>(), t.near3.as<double>(), G, force);
    else
        hipLaunchKernelGGL((l2p_kernel<P, TFMM_STANDARD>), dim3((unsigned)cdiv(n, LB)), dim3(LB), 0, s, n,
                           t.Xm.as<double4>(), t.leaf_of.as<int32_t>(), t.perm.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.loc_leaf.as<double>(), t.near3.as<double>(), G, force);
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

void run_l2p(Tree& t, int p, int variant, double G, double* force, hipStream_t s) {
    switch (p) {
        case 1: l2p_dispatch<1>(t, variant, G, force, s); break;
        case 2: l2p_dispatch<2>(t, variant, G, force, s); break;
        case 3: l2p_dispatch<3>(t, variant, G, force, s); break;
        case 4: l2p_dispatch<4>(t, variant, G, force, s); break;
        case 5: l2p_dispatch<5>(t, variant, G, force, s); break;
        case 6: l2p_dispatch<6>(t, variant, G, force, s); break;
        case 7: l2p_dispatch<7>(t, variant, G, force, s); break;
        case 8: l2p_dispatch<8>(t, variant, G, force, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

}  // namespace tfmm
