// Multipole moments of every node in FP64 (the paper's step (i), Sec. 2).
//
// Raw Cartesian moments about the node's centre of mass,
//     M_k = sum_b m_b y_b^k,  y_b = Y_b - Z_B,  |k| <= p,
// (the monopole, quadrupole, octopole, ... of Eqs. quad_mom, octo_mom,
// hexa_mom before their traces are removed; with a softened kernel the traces
// matter).  Leaves sum over their particles (P2M); inner nodes shift their
// children's moments exactly (M2M):
//     M_k(P) = sum_c sum_{i <= k} C(k, i) M_i(c) d_c^(k - i),  d_c = Z_c - Z_P.
// The M2L kernels read W_k = (-1)^|k| M_k / k! (FP64 and an FP32 copy).
#include "common.h"

namespace tfmm {
namespace {

constexpr int TB = 256;

__device__ __forceinline__ int cle(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }

__device__ __forceinline__ int midx(int kx, int ky, int kz) {
    const int n = kx + ky + kz, a = ky + kz;
    return cle(n - 1) + a * (a + 1) / 2 + kz;
}

__device__ __forceinline__ void mdecode(int k, int& kx, int& ky, int& kz) {
    int n = 0;
    while (cle(n) <= k) ++n;
    int r = k - cle(n - 1);
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= r) ++a;
    kz = r - a * (a + 1) / 2;
    ky = a - kz;
    kx = n - a;
}

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

__device__ __forceinline__ double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

__device__ __forceinline__ double fact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

__global__ __launch_bounds__(TB) void moments_level_kernel(int NC, int NCP, int32_t lb, int32_t le,
                                                           const int32_t* __restrict__ first,
                                                           const int32_t* __restrict__ count,
                                                           const int32_t* __restrict__ child_first,
                                                           const int32_t* __restrict__ nchild,
                                                           const double4* __restrict__ Xm,
                                                           const double4* __restrict__ Z,
                                                           double* __restrict__ mom, double* __restrict__ W64,
                                                           float* __restrict__ W32) {
    const int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x;
    const int32_t node = lb + (int32_t)(t / NCP);
    const int k = (int)(t % NCP);
    if (node >= le) return;
    if (k >= NC) {
        W64[(int64_t)node * NCP + k] = 0.0;
        W32[(int64_t)node * NCP + k] = 0.0f;
        return;
    }
    int kx, ky, kz;
    mdecode(k, kx, ky, kz);
    const double4 z = Z[node];
    double acc = 0.0;
    const int32_t nc = nchild[node];
    if (nc == 0) {
        const int32_t s0 = first[node], s1 = s0 + count[node];
        for (int32_t s = s0; s < s1; ++s) {
            const double4 p = Xm[s];
            acc += p.w * ipow(p.x - z.x, kx) * ipow(p.y - z.y, ky) * ipow(p.z - z.z, kz);
        }
    } else {
        const int32_t c0 = child_first[node];
        for (int32_t c = c0; c < c0 + nc; ++c) {
            const double4 zc = Z[c];
            const double dx = zc.x - z.x, dy = zc.y - z.y, dz = zc.z - z.z;
            const double* mc = mom + (int64_t)c * NC;
            for (int ix = 0; ix <= kx; ++ix) {
                const double bx = binom(kx, ix) * ipow(dx, kx - ix);
                for (int iy = 0; iy <= ky; ++iy) {
                    const double by = bx * binom(ky, iy) * ipow(dy, ky - iy);
                    for (int iz = 0; iz <= kz; ++iz)
                        acc += by * binom(kz, iz) * ipow(dz, kz - iz) * mc[midx(ix, iy, iz)];
                }
            }
        }
    }
    mom[(int64_t)node * NC + k] = acc;
    const int n = kx + ky + kz;
    const double w = ((n & 1) ? -acc : acc) / (fact(kx) * fact(ky) * fact(kz));
    W64[(int64_t)node * NCP + k] = w;
    W32[(int64_t)node * NCP + k] = (float)w;
}

}  // namespace

void compute_moments(Tree& t, int p, hipStream_t s) {
    if (t.mom_p == p) return;
    const int NC = c_le(p);
    const int NCP = (int)round_up(NC, 4);
    const int64_t nn = t.n_nodes;
    t.mom.ensure(t.ctx, (size_t)nn * NC * 8);
    t.W64.ensure(t.ctx, (size_t)nn * NCP * 8);
    t.W32.ensure(t.ctx, (size_t)nn * NCP * 4);
    for (int L = t.max_level; L >= 0; --L) {
        const int32_t b = (int32_t)t.level_begin[L], e = (int32_t)t.level_begin[L + 1];
        if (e <= b) continue;
        const int64_t work = (int64_t)(e - b) * NCP;
        hipLaunchKernelGGL(moments_level_kernel, dim3((unsigned)cdiv(work, TB)), dim3(TB), 0, s, NC, NCP, b, e,
                           t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(), t.nd_child_first.as<int32_t>(),
                           t.nd_nchild.as<int32_t>(), t.Xm.as<double4>(), t.nd_Z.as<double4>(), t.mom.as<double>(),
                           t.W64.as<double>(), t.W32.as<float>());
        TFMM_LAUNCHED();
    }
    t.mom_p = p;
}

}  // namespace tfmm
