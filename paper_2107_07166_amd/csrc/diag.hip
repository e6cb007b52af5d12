// Momentum diagnostics in FP64: the net force of Eq. netforce and the net
// torque of Eq. total_torque summed over every particle, taken about the
// system's centre of mass, plus linear and angular momentum.  Fixed grid,
// fixed per-thread strides and fixed tree reductions: bitwise reproducible.
#include <mutex>

#include "common.h"

namespace tfmm {
namespace {

constexpr int DB = 256;
constexpr int DG = 512;
constexpr int N1 = 4;   // m, m x, m y, m z
constexpr int N2 = 16;  // F(3) |F| rxF(3) |r||F| P(3) L(3)
// Scratch of one evaluation: per-block partial sums of both passes, the two
// pass totals, then the 20 output values.
constexpr int kScratchDoubles = DG * (N1 + N2) + N1 + N2;
constexpr int kOut = 20;

// Scratch of the allocation-free entry point (tfmm_momentum_diagnostics_noalloc),
// one copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address of each GPU's copy is looked up once
// per device with hipGetSymbolAddress (diag_scratch_init) and used instead.
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

template <int NV>
__device__ void block_reduce(double (&v)[NV], double* sh) {
    for (int k = 0; k < NV; ++k) sh[k * DB + threadIdx.x] = v[k];
    __syncthreads();
    for (int s = DB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < NV; ++k) sh[k * DB + threadIdx.x] += sh[k * DB + threadIdx.x + s];
        __syncthreads();
    }
}

__global__ __launch_bounds__(DB) void diag_pass1(int64_t n, const double* __restrict__ pos,
                                                 const double* __restrict__ mass, double* __restrict__ part) {
    __shared__ double sh[N1 * DB];
    double v[N1] = {0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x; i < n; i += (int64_t)DB * DG) {
        const double m = mass[i];
        v[0] += m;
        v[1] += m * pos[3 * i];
        v[2] += m * pos[3 * i + 1];
        v[3] += m * pos[3 * i + 2];
    }
    block_reduce<N1>(v, sh);
    if (threadIdx.x < N1) part[blockIdx.x * N1 + threadIdx.x] = sh[threadIdx.x * DB];
}

template <int NV>
__global__ __launch_bounds__(DB) void diag_final(const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[NV * DB];
    double v[NV];
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < DG; b += DB)
        for (int k = 0; k < NV; ++k) v[k] += part[b * NV + k];
    block_reduce<NV>(v, sh);
    if (threadIdx.x < NV) out[threadIdx.x] = sh[threadIdx.x * DB];
}

__global__ __launch_bounds__(DB) void diag_pass2(int64_t n, const double* __restrict__ pos,
                                                 const double* __restrict__ vel, const double* __restrict__ mass,
                                                 const double* __restrict__ force, const double* __restrict__ tot1,
                                                 double* __restrict__ part) {
    __shared__ double sh[N2 * DB];
    const double M = tot1[0];
    const double cx = tot1[1] / M, cy = tot1[2] / M, cz = tot1[3] / M;
    double v[N2];
    for (int k = 0; k < N2; ++k) v[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x; i < n; i += (int64_t)DB * DG) {
        const double fx = force[3 * i], fy = force[3 * i + 1], fz = force[3 * i + 2];
        const double rx = pos[3 * i] - cx, ry = pos[3 * i + 1] - cy, rz = pos[3 * i + 2] - cz;
        const double fn = sqrt(fx * fx + fy * fy + fz * fz);
        const double rn = sqrt(rx * rx + ry * ry + rz * rz);
        v[0] += fx;
        v[1] += fy;
        v[2] += fz;
        v[3] += fn;
        v[4] += ry * fz - rz * fy;
        v[5] += rz * fx - rx * fz;
        v[6] += rx * fy - ry * fx;
        v[7] += rn * fn;
        if (vel) {
            const double m = mass[i];
            const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
            v[8] += m * vx;
            v[9] += m * vy;
            v[10] += m * vz;
            v[11] += m * (ry * vz - rz * vy);
            v[12] += m * (rz * vx - rx * vz);
            v[13] += m * (rx * vy - ry * vx);
        }
    }
    block_reduce<N2>(v, sh);
    if (threadIdx.x < N2) part[blockIdx.x * N2 + threadIdx.x] = sh[threadIdx.x * DB];
}

// The 20 output values from the two pass totals (layout of
// tfmm_momentum_diagnostics).  One thread.
__global__ void diag_finish(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double M = a[0];  // a: m, mx, my, mz; b: pass 2
    for (int d = 0; d < 3; ++d) {
        out[d] = b[d];
        out[4 + d] = b[4 + d];
        out[8 + d] = b[8 + d];
        out[11 + d] = b[11 + d];
        out[15 + d] = a[1 + d] / M;
    }
    out[3] = b[3];
    out[7] = b[7];
    out[14] = M;
    const double fs = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double ts = sqrt(b[4] * b[4] + b[5] * b[5] + b[6] * b[6]);
    out[18] = b[3] > 0 ? fs / b[3] : 0.0;
    out[19] = b[7] > 0 ? ts / b[7] : 0.0;
}

// Every kernel writes each scratch value it later reads (fixed grid of DG
// blocks), so nothing has to start at zero.  buf: kScratchDoubles doubles;
// out: 20 doubles (device).
void launch_diagnostics(int64_t n, const double* pos, const double* vel, const double* mass, const double* force,
                        double* buf, double* out, hipStream_t s) {
    double* p1 = buf;
    double* p2 = p1 + DG * N1;
    double* t1 = p2 + DG * N2;
    double* t2 = t1 + N1;
    hipLaunchKernelGGL(diag_pass1, dim3(DG), dim3(DB), 0, s, n, pos, mass, p1);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(diag_final<N1>, dim3(1), dim3(DB), 0, s, (const double*)p1, t1);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(diag_pass2, dim3(DG), dim3(DB), 0, s, n, pos, vel, mass, force, (const double*)t1, p2);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(diag_final<N2>, dim3(1), dim3(DB), 0, s, (const double*)p2, t2);
    TFMM_LAUNCHED();
    hipLaunchKernelGGL(diag_finish, dim3(1), dim3(kWave), 0, s, (const double*)t1, (const double*)t2, out);
    TFMM_LAUNCHED();
}

}  // namespace

void run_diagnostics(int64_t n, const double* pos, const double* vel, const double* mass, const double* force,
                     double* out, Ctx* ctx, hipStream_t s) {
    DevBuf buf;
    buf.ensure(ctx, (size_t)(kScratchDoubles + kOut) * 8);
    double* dev_out = buf.as<double>() + kScratchDoubles;
    launch_diagnostics(n, pos, vel, mass, force, buf.as<double>(), dev_out, s);
    TFMM_HIP(hipMemcpyAsync(ctx->pinned, dev_out, kOut * sizeof(double), hipMemcpyDeviceToHost, s));
    TFMM_HIP(hipStreamSynchronize(s));
    std::memcpy(out, ctx->pinned, kOut * sizeof(double));
}

// Looks up the device address of this GPU's copy of `scratch` (the device
// must be current); once per device, at context creation.
void diag_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) fail(TFMM_EINVAL, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return;
    void* ptr = nullptr;
    TFMM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(TFMM_EDEVICE, "hipGetSymbolAddress returned no address for the diagnostics scratch");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
}

// Allocation-free diagnostics: the same kernels as run_diagnostics on the
// device's static scratch, results written to out (device, 20 doubles); no
// synchronisation, no allocation, no memset.
void run_diagnostics_noalloc(int64_t n, const double* pos, const double* vel, const double* mass,
                             const double* force, double* out, int device, hipStream_t s) {
    double* buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (device >= 0 && device < kMaxDevices) buf = g_scratch_ptr[device];
    }
    if (!buf) fail(TFMM_ESTATE, "the diagnostics scratch of this device was not set up (no context created on it)");
    launch_diagnostics(n, pos, vel, mass, force, buf, out, s);
}

}  // namespace tfmm
