// Far field, multipole to local (M2L), standard and conserving.
//
// For a far pair of nodes (target A, source B) with R = Z_A - Z_B the kernel
// builds the derivative tensors of the softened kernel at R (generalised D
// tensors of Eqs. D..Dijkl) with the radial recurrence of expansions_gen.h,
// then contracts them with B's moments:
//   standard  : L_j(A) += sum_i D_{i+j}(R) W_i(B)    (Taylor series of Eq. taylor)
//   conserving: P_j(A) += sum_i G_{i+j}(R) W_i(B), Q'_ej(A) += Q_ej - R_e P_j
//               (realigned force, Eq. realign, scalar kept to degree p-1).
//   conserving_r2 (order 2 locals only): the same contraction with G replaced
//               by the scalar of Eq. realign2 / nab-expansion, (R.R + eps^2)
//               ^(-3/2) (1 - R.delta / |R|^2): G_0 = (R.R+eps^2)^(-3/2),
//               G_e = -G_0 R_e / |R|^2 (Eq. aaB0 after the sum over B).
// Each row of 16 lanes owns one target node: its lanes stride over the
// target's source list, each lane accumulating a private local expansion, and
// a DPP reduction across the row produces the node's locals (written once, no
// atomics, fixed order -> reproducible).  Far lists are a few dozen to a few
// hundred sources long; with 32 lanes per target the short lists of the disk
// (75 per node at theta = 0.8) left a third of the lanes idle in their last
// round: 16 lanes took 3-6 % off the evaluation on the disk and the binary and
// changed nothing for the default variants on the Plummer sphere (lists of
// ~400, where 32 lanes are busy; the raised scalar degrees, whose far field
// is not hidden beside the near field, are 6-12 % slower there).
#include "common.h"
#include "expansions_gen.h"

namespace tfmm {
namespace {

constexpr int MB = 256;         // largest block (4 waves); launches may use fewer
// Block size of the force M2L launches.  M2L runs beside the near-field
// kernel (one-wave blocks, most of the device); smaller M2L blocks get a
// larger share of the compute units.  With one-wave blocks the standard far
// field finishes early and the evaluation is 1-6 % faster than with four-wave
// blocks (Plummer sphere, binary, disk), although the near field then runs
// longer beside it; the conserving one, the heavier, needs them to finish
// with the near field at all.
constexpr int kForceBlock = 64;
constexpr int LPT = 16;         // lanes per target node (one DPP row)
constexpr int TPW = kWave / LPT;  // target nodes per wavefront

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// Reductions with DPP lane moves only (no LDS): pairs and quads (quad_perm),
// half rows (row_half_mirror), then rows (row_mirror); every row and bank
// takes part.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(uint32_t)u);
    const int hi = dpp_i<CTRL>((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum over each row of 16 lanes, the result in every lane of the row.
static_assert(LPT == 16, "the reduction sums one DPP row");
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
    v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror
    v += dpp<0x140>(v);  // row_mirror
    return v;
}

// POTL (standard only): also L_0, the potential's constant term.  wstride:
// moments per node in W (the moments may be of a higher order than P; the
// graded order puts the first c(<=P) of them first).
template <int P, int VAR, typename T, bool POTL = false>
__global__ __launch_bounds__(MB) void m2l_kernel(int64_t n_targets,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ src, uint32_t src_mask,
                                                 const double4* __restrict__ Z, const T* __restrict__ W,
                                                 int64_t wstride, double eps2, double* __restrict__ loc) {
    using E = Expansion<P>;
    constexpr int NC = E::NC;
    constexpr int NC1 = E::NC1;
    constexpr int NCP = (NC + 3) / 4 * 4;
    constexpr bool CONS = VAR != TFMM_STANDARD;
    static_assert(VAR != TFMM_CONSERVING_R2 || P == 2, "the r2 locals are of order 2");
    constexpr int NOUT = CONS ? 4 * NC1 : NC;
    // wave index through readfirstlane: the compiler then keeps the target's
    // list bounds in scalar registers
    // target nodes in chunks of 64 blocks per XCD
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(xcd_block<64>(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    if (wave * TPW >= n_targets) return;
    const int row = lane / LPT, sl = lane % LPT;
    const int64_t ti = wave * TPW + row;
    const bool has = ti < n_targets;
    const int32_t A = (int32_t)(has ? ti : wave * TPW);
    const double4 za = Z[A];
    T acc[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) acc[k] = T(0);
    const uint32_t q0 = has ? off[A] : 0u, q1 = has ? off[A + 1] : 0u;
    for (uint32_t q = q0 + sl; q < q1; q += LPT) {
        const int32_t B = (int32_t)(src[q] & src_mask);
        const double4 zb = Z[B];
        const T Rx = (T)(za.x - zb.x), Ry = (T)(za.y - zb.y), Rz = (T)(za.z - zb.z);
        const T s = Rx * Rx + Ry * Ry + Rz * Rz + (T)eps2;
        const T rinv = rsqrt_t(s);
        const T inv_s = rinv * rinv;
        T F[P + 1];
        F[0] = -rinv;
#pragma unroll
        for (int n = 1; n <= P; ++n) F[n] = (T)(-(2 * n - 1)) * F[n - 1] * inv_s;
        T w[NCP];
        const typename Vec4<T>::type* wb = reinterpret_cast<const typename Vec4<T>::type*>(W + (int64_t)B * wstride);
#pragma unroll
        for (int k = 0; k < NCP / 4; ++k) {
            const typename Vec4<T>::type v = wb[k];
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
        if constexpr (VAR == TFMM_CONSERVING_R2) {
            T G[NC1];
            const T rr = Rx * Rx + Ry * Ry + Rz * Rz;
            const T c = -F[1] / rr;
            G[0] = F[1];
            G[1] = Rx * c;
            G[2] = Ry * c;
            G[3] = Rz * c;
            E::m2l_cons(G, w, Rx, Ry, Rz, acc, acc + NC1);
        } else if constexpr (VAR == TFMM_CONSERVING) {
            T G[NC1];
            E::g_derivs(Rx, Ry, Rz, F, G);
            E::m2l_cons(G, w, Rx, Ry, Rz, acc, acc + NC1);
        } else {
            T D[NC];
            E::phi_derivs(Rx, Ry, Rz, F, D);
            E::template m2l_std<T, POTL>(D, w, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < NOUT; ++k) acc[k] = row_sum(acc[k]);
    if (has && q1 > q0 && sl == LPT - 1) {
        double* out = loc + (int64_t)A * NOUT;
#pragma unroll
        for (int k = 0; k < NOUT; ++k) out[k] = (double)acc[k];
    }
}

// Minimum waves per SIMD asked of the compiler for a pass.  The FP32 P pass
// at order 6 (conserving, or the knob with a force of order 5) fits 128
// registers without spills, four waves per SIMD instead of three; on the
// 2^22-particle disk that takes 0.07-0.14 ms off a 4.6-5.0 ms evaluation with
// the same locals bit for bit.  The Q' passes (190 registers) spill 23-29
// registers at three waves and were much slower (evaluation 5.3 against 4.6
// ms); orders 7 and 8 spill over 100 at four.
constexpr int cons_pass_waves(int P, int PS, int MASK, int tsize) {
    return (tsize == 4 && P == 6 && PS >= 5 && MASK == 1) ? 4 : 1;
}

// Conserving M2L for a subset of the output polynomials per launch (bit 0:
// P, bits 1..3: Q'_x,y,z), for orders whose four accumulator sets do not fit
// the registers together: every launch recomputes the g-derivatives of its
// pairs and accumulates popcount(MASK) sets of NC1 locals, each written into
// its slice of the node's 4 NC1 block.
// PS: order of the realigned standard force.  PS == P is the conserving
// variant of order P; PS < P keeps its projection scalar to degree P - 1
// (Knob<PS, P - 1>), with moments and locals of order P.
template <int P, int PS, int MASK, typename T>
__global__ __launch_bounds__(MB) __attribute__((amdgpu_waves_per_eu(cons_pass_waves(P, PS, MASK, sizeof(T)))))
void m2l_cons_pass_kernel(int64_t n_targets, const uint32_t* __restrict__ off,
                          const uint32_t* __restrict__ src, uint32_t src_mask,
                          const double4* __restrict__ Z, const T* __restrict__ W,
                          double eps2, double* __restrict__ loc) {
    using E = Expansion<P>;
    constexpr int NC = E::NC;
    constexpr int NC1 = E::NC1;
    constexpr int NCP = (NC + 3) / 4 * 4;
    constexpr int NPOLY = (MASK & 1) + ((MASK >> 1) & 1) + ((MASK >> 2) & 1) + ((MASK >> 3) & 1);
    // target nodes in chunks of 64 blocks per XCD
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(xcd_block<64>(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    if (wave * TPW >= n_targets) return;
    const int row = lane / LPT, sl = lane % LPT;
    const int64_t ti = wave * TPW + row;
    const bool has = ti < n_targets;
    const int32_t A = (int32_t)(has ? ti : wave * TPW);
    const double4 za = Z[A];
    T acc[NPOLY * NC1];
#pragma unroll
    for (int k = 0; k < NPOLY * NC1; ++k) acc[k] = T(0);
    const uint32_t q0 = has ? off[A] : 0u, q1 = has ? off[A + 1] : 0u;
    for (uint32_t q = q0 + sl; q < q1; q += LPT) {
        const int32_t B = (int32_t)(src[q] & src_mask);
        const double4 zb = Z[B];
        const T Rx = (T)(za.x - zb.x), Ry = (T)(za.y - zb.y), Rz = (T)(za.z - zb.z);
        const T s = Rx * Rx + Ry * Ry + Rz * Rz + (T)eps2;
        const T rinv = rsqrt_t(s);
        const T inv_s = rinv * rinv;
        T F[P + 1];
        F[0] = -rinv;
#pragma unroll
        for (int n = 1; n <= P; ++n) F[n] = (T)(-(2 * n - 1)) * F[n - 1] * inv_s;
        T w[NCP];
        const typename Vec4<T>::type* wb = reinterpret_cast<const typename Vec4<T>::type*>(W + (int64_t)B * NCP);
#pragma unroll
        for (int k = 0; k < NCP / 4; ++k) {
            const typename Vec4<T>::type v = wb[k];
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
        T G[NC1];
        if constexpr (PS == P) {
            E::g_derivs(Rx, Ry, Rz, F, G);
        } else {
            T G0[Expansion<PS>::NC1];
            Expansion<PS>::g_derivs(Rx, Ry, Rz, F, G0);
            Knob<PS, P - 1>::scalar(Rx, Ry, Rz, G0, G);
        }
        int slot = 0;
        if constexpr (MASK & 1) E::cons_p(G, w, acc + NC1 * slot++);
        if constexpr (MASK & 2) E::cons_qx(G, w, Rx, acc + NC1 * slot++);
        if constexpr (MASK & 4) E::cons_qy(G, w, Ry, acc + NC1 * slot++);
        if constexpr (MASK & 8) E::cons_qz(G, w, Rz, acc + NC1 * slot++);
    }
#pragma unroll
    for (int k = 0; k < NPOLY * NC1; ++k) acc[k] = row_sum(acc[k]);
    if (has && q1 > q0 && sl == LPT - 1) {
        double* out = loc + (int64_t)A * (4 * NC1);
        int slot = 0;
#pragma unroll
        for (int poly = 0; poly < 4; ++poly) {
            if (!((MASK >> poly) & 1)) continue;
#pragma unroll
            for (int k = 0; k < NC1; ++k) out[poly * NC1 + k] = (double)acc[slot * NC1 + k];
            ++slot;
        }
    }
}

// From p = 6 the conserving locals are accumulated one polynomial per launch:
// the four accumulator sets together take 486 registers at p = 6 (one wave
// per SIMD), one set 129-190 (two to three waves).  On the 2^22-particle disk
// (p = 6, theta = 0.8) the far field took 4.54 ms in four launches against
// 4.81 ms in two (P with Q'_x, Q'_y with Q'_z; 264 registers) and 4.97 ms in
// one; reading the moments where the contraction uses them instead of into
// registers first was slower in every split.  Computing the g-derivatives once
// per pair and sharing them through LDS (a workgroup of four wavefronts per
// two targets: the first builds the tensors of a block of pairs, then each
// contracts one polynomial; 256 registers with spills, two waves per SIMD)
// gave the same locals bit for bit but took 6.5 ms against 4.5.  At p = 5 the
// fused kernel (285 registers) beats four launches (2.7 against 3.0 ms on 2^20
// Plummer particles).  In FP64 the fused p = 4 kernel also runs at one wave
// per SIMD (256 + 76 registers), yet four launches of 126-136 registers are
// slower there too (4.25 against 3.82-3.87 ms on the same workload), and so
// are two launches of two polynomials (3.84-3.90 against 3.70-3.75 ms).
constexpr int kConsSplitP = 6;

template <int P, int VAR, typename T>
void launch(Tree& t, double eps2, hipStream_t s) {
    const int64_t nt = t.n_nodes;  // every node; nodes with an empty far list write nothing
    if (nt <= 0) return;
    const T* W = (sizeof(T) == 4) ? reinterpret_cast<const T*>(t.W32.p) : reinterpret_cast<const T*>(t.W64.p);
    const int mb = kForceBlock;
    const dim3 grid((unsigned)cdiv(cdiv(nt, TPW) * kWave, mb));
    if constexpr (VAR == TFMM_CONSERVING && P >= kConsSplitP) {
        auto pass = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(mb), 0, s, nt, t.m2l_off.template as<uint32_t>(),
                               t.m2l_src.template as<uint32_t>(), t.m2l_src_mask, t.nd_Z.template as<double4>(), W,
                               eps2, t.loc.template as<double>());
            TFMM_LAUNCHED();
        };
        pass(m2l_cons_pass_kernel<P, P, 0x1, T>);
        pass(m2l_cons_pass_kernel<P, P, 0x2, T>);
        pass(m2l_cons_pass_kernel<P, P, 0x4, T>);
        pass(m2l_cons_pass_kernel<P, P, 0x8, T>);
    } else {
        hipLaunchKernelGGL((m2l_kernel<P, VAR, T>), grid, dim3(mb), 0, s, nt,
                           t.m2l_off.as<uint32_t>(), t.m2l_src.as<uint32_t>(), t.m2l_src_mask, t.nd_Z.as<double4>(), W,
                           (int64_t)round_up(c_le(P), 4), eps2, t.loc.as<double>());
        TFMM_LAUNCHED();
    }
}

// The conserving far field of force order PS with the projection scalar kept
// to degree K > PS - 1: locals of order K + 1 (split by polynomial from order
// kConsSplitP, like the conserving variant).
template <int PS, int K, typename T>
void launch_knob(Tree& t, double eps2, hipStream_t s) {
    constexpr int P = K + 1;
    const int64_t nt = t.n_nodes;
    if (nt <= 0) return;
    const T* W = (sizeof(T) == 4) ? reinterpret_cast<const T*>(t.W32.p) : reinterpret_cast<const T*>(t.W64.p);
    const int mb = kForceBlock;
    const dim3 grid((unsigned)cdiv(cdiv(nt, TPW) * kWave, mb));
    auto pass = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(mb), 0, s, nt, t.m2l_off.template as<uint32_t>(),
                           t.m2l_src.template as<uint32_t>(), t.m2l_src_mask, t.nd_Z.template as<double4>(), W, eps2,
                           t.loc.template as<double>());
        TFMM_LAUNCHED();
    };
    if constexpr (P >= kConsSplitP) {
        pass(m2l_cons_pass_kernel<P, PS, 0x1, T>);
        pass(m2l_cons_pass_kernel<P, PS, 0x2, T>);
        pass(m2l_cons_pass_kernel<P, PS, 0x4, T>);
        pass(m2l_cons_pass_kernel<P, PS, 0x8, T>);
    } else {
        pass(m2l_cons_pass_kernel<P, PS, 0xF, T>);
    }
}

template <int PS, int K>
void dispatch_knob(Tree& t, int precision, double eps2, hipStream_t s) {
    if (precision == TFMM_MIXED32) launch_knob<PS, K, float>(t, eps2, s);
    else launch_knob<PS, K, double>(t, eps2, s);
}

template <int P>
void dispatch_var(Tree& t, int variant, int precision, double eps2, hipStream_t s) {
    if (variant == TFMM_CONSERVING_R2) {
        if constexpr (P == 2) {
            if (precision == TFMM_MIXED32) launch<P, TFMM_CONSERVING_R2, float>(t, eps2, s);
            else launch<P, TFMM_CONSERVING_R2, double>(t, eps2, s);
        } else {
            fail(TFMM_EINVAL, "conserving_r2 locals are of order 2");
        }
    } else if (variant == TFMM_CONSERVING) {
        if (precision == TFMM_MIXED32) launch<P, TFMM_CONSERVING, float>(t, eps2, s);
        else launch<P, TFMM_CONSERVING, double>(t, eps2, s);
    } else {
        if (precision == TFMM_MIXED32) launch<P, TFMM_STANDARD, float>(t, eps2, s);
        else launch<P, TFMM_STANDARD, double>(t, eps2, s);
    }
}

template <int P, typename T>
void launch_pot(Tree& t, int mom_p, double eps2, hipStream_t s) {
    const int64_t nt = t.n_nodes;
    if (nt <= 0) return;
    const T* W = (sizeof(T) == 4) ? reinterpret_cast<const T*>(t.W32.p) : reinterpret_cast<const T*>(t.W64.p);
    const dim3 grid((unsigned)cdiv(cdiv(nt, TPW) * kWave, MB));
    hipLaunchKernelGGL((m2l_kernel<P, TFMM_STANDARD, T, true>), grid, dim3(MB), 0, s, nt, t.m2l_off.as<uint32_t>(),
                       t.m2l_src.as<uint32_t>(), t.m2l_src_mask, t.nd_Z.as<double4>(), W,
                       (int64_t)round_up(c_le(mom_p), 4), eps2, t.loc_pot.as<double>());
    TFMM_LAUNCHED();
}

template <int P>
void dispatch_pot(Tree& t, int mom_p, int precision, double eps2, hipStream_t s) {
    if (precision == TFMM_MIXED32) launch_pot<P, float>(t, mom_p, eps2, s);
    else launch_pot<P, double>(t, mom_p, eps2, s);
}

}  // namespace

// Standard locals with their constant term (the far-field potential of
// Eq. taylor truncated at degree p) into t.loc_pot, for every variant; the
// moments on the device are of order mom_p >= p.
void run_m2l_pot(Tree& t, int p, int mom_p, int precision, double eps2, hipStream_t s) {
    const int64_t tot = t.n_nodes * (int64_t)c_le(p);
    // no clearing: a node's locals are written whole when its far list is not
    // empty, and the downward pass reads only such nodes
    t.loc_pot.ensure(t.ctx, (size_t)tot * 8);
    switch (p) {
        case 1: dispatch_pot<1>(t, mom_p, precision, eps2, s); break;
        case 2: dispatch_pot<2>(t, mom_p, precision, eps2, s); break;
        case 3: dispatch_pot<3>(t, mom_p, precision, eps2, s); break;
        case 4: dispatch_pot<4>(t, mom_p, precision, eps2, s); break;
        case 5: dispatch_pot<5>(t, mom_p, precision, eps2, s); break;
        case 6: dispatch_pot<6>(t, mom_p, precision, eps2, s); break;
        case 7: dispatch_pot<7>(t, mom_p, precision, eps2, s); break;
        case 8: dispatch_pot<8>(t, mom_p, precision, eps2, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

void run_m2l(Tree& t, int p, int variant, int precision, double eps2, hipStream_t s, int kdeg) {
    const bool knob = variant == TFMM_CONSERVING && kdeg > p - 1;
    const int nloc = knob ? n_local(kdeg + 1, variant) : n_local(p, variant);
    const int64_t tot = t.n_nodes * (int64_t)nloc;
    // no clearing: a node's locals are written whole when its far list is not
    // empty, and the downward pass reads only such nodes
    t.loc.ensure(t.ctx, (size_t)tot * 8);
    if (knob) {
        switch (p * 16 + kdeg) {
            case 1 * 16 + 1: dispatch_knob<1, 1>(t, precision, eps2, s); break;
            case 1 * 16 + 2: dispatch_knob<1, 2>(t, precision, eps2, s); break;
            case 2 * 16 + 2: dispatch_knob<2, 2>(t, precision, eps2, s); break;
            case 2 * 16 + 3: dispatch_knob<2, 3>(t, precision, eps2, s); break;
            case 3 * 16 + 3: dispatch_knob<3, 3>(t, precision, eps2, s); break;
            case 3 * 16 + 4: dispatch_knob<3, 4>(t, precision, eps2, s); break;
            case 4 * 16 + 4: dispatch_knob<4, 4>(t, precision, eps2, s); break;
            case 4 * 16 + 5: dispatch_knob<4, 5>(t, precision, eps2, s); break;
            case 5 * 16 + 5: dispatch_knob<5, 5>(t, precision, eps2, s); break;
            case 5 * 16 + 6: dispatch_knob<5, 6>(t, precision, eps2, s); break;
            case 6 * 16 + 6: dispatch_knob<6, 6>(t, precision, eps2, s); break;
            default: fail(TFMM_EINVAL, "scalar_degree must satisfy p-1 <= K <= min(p+1, 6)");
        }
        return;
    }
    switch (p) {
        case 1: dispatch_var<1>(t, variant, precision, eps2, s); break;
        case 2: dispatch_var<2>(t, variant, precision, eps2, s); break;
        case 3: dispatch_var<3>(t, variant, precision, eps2, s); break;
        case 4: dispatch_var<4>(t, variant, precision, eps2, s); break;
        case 5: dispatch_var<5>(t, variant, precision, eps2, s); break;
        case 6: dispatch_var<6>(t, variant, precision, eps2, s); break;
        case 7: dispatch_var<7>(t, variant, precision, eps2, s); break;
        case 8: dispatch_var<8>(t, variant, precision, eps2, s); break;
        default: fail(TFMM_EINVAL, "p must be in 1..8");
    }
}

}  // namespace tfmm
