// Multipole moments of every node in FP64 (the paper's step (i), Sec. 2).
//
// Raw Cartesian moments about the node's centre of mass, M_k = sum_b m_b y_b^k
// with y_b = Y_b - Z_B and |k| <= p (the monopole, quadrupole, octopole, ...
// of Eqs. quad_mom, octo_mom, hexa_mom before their traces are removed; with
// a softened kernel the traces matter), are stored in the form the M2L
// kernels contract with:
//     W_k = (-1)^|k| M_k / k! = sum_b m_b (-y_b)^k / k!.
// Leaves sum over their particles (P2M).  Inner nodes shift their children
// exactly (M2M): with y' = y + d_c, d_c = Z_c - Z_P,
//     W_k(P) = sum_c sum_{i + j = k} W_i(c) (-d_c)^j / j!.
// FP64 throughout; an FP32 copy feeds the mixed-precision M2L.
#include "common.h"
#include "expansions_gen.h"

namespace tfmm {
namespace {

constexpr int TB = 128;

template <int P>
__global__ __launch_bounds__(TB) void p2m_kernel(int64_t n_leaves, const int32_t* __restrict__ leaves,
                                                 const int32_t* __restrict__ first,
                                                 const int32_t* __restrict__ count,
                                                 const double4* __restrict__ Xm, const double4* __restrict__ Z,
                                                 double* __restrict__ W64, float* __restrict__ W32) {
    using E = Expansion<P>;
    constexpr int NC = E::NC;
    constexpr int NCP = (NC + 3) / 4 * 4;
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n_leaves) return;
    const int32_t node = leaves[i];
    const double4 z = Z[node];
    double w[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) w[k] = 0.0;
    const int32_t s0 = first[node], s1 = s0 + count[node];
    for (int32_t s = s0; s < s1; s += 4) {
        double4 p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (s + u < s1) p[u] = Xm[s + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (s + u < s1) E::p2m(p[u].w, z.x - p[u].x, z.y - p[u].y, z.z - p[u].z, w);
    }
    double* o64 = W64 + (int64_t)node * NCP;
    float* o32 = W32 + (int64_t)node * NCP;
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
        const double v = k < NC ? w[k] : 0.0;
        o64[k] = v;
        o32[k] = (float)v;
    }
}

template <int P>
__global__ __launch_bounds__(TB) void m2m_kernel(int32_t lb, int32_t le, const int32_t* __restrict__ child_first,
                                                 const int32_t* __restrict__ nchild,
                                                 const double4* __restrict__ Z, double* __restrict__ W64,
                                                 float* __restrict__ W32) {
    using E = Expansion<P>;
    constexpr int NC = E::NC;
    constexpr int NCP = (NC + 3) / 4 * 4;
    const int32_t node = lb + (int32_t)(blockIdx.x * TB + threadIdx.x);
    if (node >= le) return;
    const int32_t nc = nchild[node];
    if (nc == 0) return;  // leaves: P2M
    const double4 z = Z[node];
    double w[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) w[k] = 0.0;
    const int32_t c0 = child_first[node];
    for (int32_t c = c0; c < c0 + nc; ++c) {
        const double4 zc = Z[c];
        E::m2m(W64 + (int64_t)c * NCP, z.x - zc.x, z.y - zc.y, z.z - zc.z, w);
    }
    double* o64 = W64 + (int64_t)node * NCP;
    float* o32 = W32 + (int64_t)node * NCP;
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
        const double v = k < NC ? w[k] : 0.0;
        o64[k] = v;
        o32[k] = (float)v;
    }
}

template <int P>
void run(Tree& t, hipStream_t s) {
    hipLaunchKernelGGL(p2m_kernel<P>, dim3((unsigned)cdiv(t.n_leaves, TB)), dim3(TB), 0, s, t.n_leaves,
                       t.leaves.as<int32_t>(), t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(),
                       t.Xm.as<double4>(), t.nd_Z.as<double4>(), t.W64.as<double>(), t.W32.as<float>());
    TFMM_LAUNCHED();
    for (int L = t.max_level - 1; L >= 0; --L) {
        const int32_t b = (int32_t)t.level_begin[L], e = (int32_t)t.level_begin[L + 1];
        if (e <= b) continue;
        hipLaunchKernelGGL(m2m_kernel<P>, dim3((unsigned)cdiv(e - b, TB)), dim3(TB), 0, s, b, e,
                           t.nd_child_first.as<int32_t>(), t.nd_nchild.as<int32_t>(), t.nd_Z.as<double4>(),
                           t.W64.as<double>(), t.W32.as<float>());
        TFMM_LAUNCHED();
    }
}

}  // namespace

void compute_moments(Tree& t, int p, hipStream_t s) {
    if (t.mom_p == p) return;
    const int NCP = (int)round_up(c_le(p), 4);
    const int64_t nn = t.n_nodes;
    t.W64.ensure(t.ctx, (size_t)nn * NCP * 8);
    t.W32.ensure(t.ctx, (size_t)nn * NCP * 4);
    switch (p) {
        case 1: run<1>(t, s); break;
        case 2: run<2>(t, s); break;
        case 3: run<3>(t, s); break;
        case 4: run<4>(t, s); break;
        case 5: run<5>(t, s); break;
        case 6: run<6>(t, s); break;
        case 7: run<7>(t, s); break;
        case 8: run<8>(t, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
    t.mom_p = p;
}

}  // namespace tfmm
