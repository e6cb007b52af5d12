// Near field (P2P): exact softened pair accelerations between the particles
// of every near pair of leaves, both directions, self pairs included (the
// gradient of Eq. jia with -(r^2 + eps^2)^(-1/2)).
//
// One wavefront owns one target leaf.  Its nt <= 64 targets sit on NT = the
// next power of two >= nt lanes, replicated G = 64 / NT times; replica g
// takes every G-th source particle, so small leaves still fill the wave, and
// the replicas are summed by a butterfly at the end.  Coordinates are relative
// to each particle's own leaf centre of mass (FP32 in the mixed path), the
// leaf-to-leaf offset Z_B - Z_A is formed in FP64 and rounded once per source
// leaf, and each source leaf's FP32 partial sum is added into an FP64
// accumulator.
#include "common.h"

namespace tfmm {
namespace {

constexpr int PB = 256;  // 4 waves per block, one target leaf per wave

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) {
    // v_rsq_f64 seed (about 2^-23 relative) refined by two Newton steps.
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    return y;
}

template <typename T, bool SAFE>
__global__ __launch_bounds__(PB) void p2p_kernel(int64_t n_leaves, const int32_t* __restrict__ leaves,
                                                 const int32_t* __restrict__ first,
                                                 const int32_t* __restrict__ count,
                                                 const uint32_t* __restrict__ off,
                                                 const int32_t* __restrict__ src,
                                                 const double4* __restrict__ Z,
                                                 const typename Vec4<T>::type* __restrict__ P, T eps2,
                                                 double* __restrict__ near) {
    using V4 = typename Vec4<T>::type;
    const int64_t wave = ((int64_t)blockIdx.x * PB + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (wave >= n_leaves) return;
    const int32_t A = leaves[wave];
    const int32_t fa = first[A], na = count[A];
    const double4 za = Z[A];
    const uint32_t q0 = off[A], q1 = off[A + 1];
    for (int32_t tc = 0; tc < na; tc += kWave) {
        const int nt = (na - tc) < kWave ? (na - tc) : kWave;
        int lg = 0;
        while ((1 << lg) < nt) ++lg;
        const int NT = 1 << lg;
        const int G = kWave >> lg;
        const int tl = lane & (NT - 1);
        const int g = lane >> lg;
        const bool act = tl < nt;
        V4 me;
        if (act) me = P[fa + tc + tl];
        else { me.x = T(0); me.y = T(0); me.z = T(0); me.w = T(0); }
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (uint32_t q = q0; q < q1; ++q) {
            const int32_t B = src[q];
            const int32_t fb = first[B], nb = count[B];
            const double4 zb = Z[B];
            const T tx = me.x - (T)(zb.x - za.x);
            const T ty = me.y - (T)(zb.y - za.y);
            const T tz = me.z - (T)(zb.z - za.z);
            T sx = T(0), sy = T(0), sz = T(0);
            if (act) {
                for (int k = g; k < nb; k += G) {
                    const V4 sp = P[fb + k];
                    const T dx = sp.x - tx, dy = sp.y - ty, dz = sp.z - tz;
                    const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                    const T ri = rsqrt_t(r2);
                    T w = sp.w * ri * (ri * ri);
                    if (SAFE) w = (r2 > T(0)) ? w : T(0);
                    sx = fma(w, dx, sx);
                    sy = fma(w, dy, sy);
                    sz = fma(w, dz, sz);
                }
            }
            ax += (double)sx;
            ay += (double)sy;
            az += (double)sz;
        }
        for (int o = NT; o < kWave; o <<= 1) {
            ax += __shfl_xor(ax, o, kWave);
            ay += __shfl_xor(ay, o, kWave);
            az += __shfl_xor(az, o, kWave);
        }
        if (act && g == 0) {
            const int64_t j = (int64_t)(fa + tc + tl);
            near[3 * j] = ax;
            near[3 * j + 1] = ay;
            near[3 * j + 2] = az;
        }
    }
}

template <typename T>
void launch(Tree& t, double eps2, hipStream_t s) {
    using V4 = typename Vec4<T>::type;
    const int64_t nl = t.n_leaves;
    const dim3 g((unsigned)cdiv(nl * kWave, PB));
    if (eps2 > 0.0)
        hipLaunchKernelGGL((p2p_kernel<T, false>), g, dim3(PB), 0, s, nl, t.leaves.as<int32_t>(),
                           t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(), t.p2p_off.as<uint32_t>(),
                           t.p2p_src.as<int32_t>(), t.nd_Z.as<double4>(), t.src4.as<V4>(), (T)eps2,
                           t.near3.as<double>());
    else
        hipLaunchKernelGGL((p2p_kernel<T, true>), g, dim3(PB), 0, s, nl, t.leaves.as<int32_t>(),
                           t.nd_first.as<int32_t>(), t.nd_count.as<int32_t>(), t.p2p_off.as<uint32_t>(),
                           t.p2p_src.as<int32_t>(), t.nd_Z.as<double4>(), t.src4.as<V4>(), (T)eps2,
                           t.near3.as<double>());
    TFMM_LAUNCHED();
}

}  // namespace

void run_p2p(Tree& t, int precision, double eps2, hipStream_t s) {
    t.near3.ensure(t.ctx, (size_t)t.n * 24);
    if (precision == TFMM_MIXED32) launch<float>(t, eps2, s);
    else launch<double>(t, eps2, s);
}

}  // namespace tfmm
