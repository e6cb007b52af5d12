// Kick-drift-kick leapfrog on state resident in device memory (FP64).
//
// The paper evolves a self-gravitating star with FMM gravity (Sec. 4) and
// reads off the angular momentum over time; here the gravity-only analogue:
//   v += (F / m) dt/2;  x += v dt;  F = F(x);  v += (F / m) dt/2.
// Both the kick and the drift are exact elementwise updates in FP64; the
// tree is rebuilt from the drifted positions before every force evaluation.
#include "common.h"

namespace tfmm {
namespace {

constexpr int KB = 256;

__global__ __launch_bounds__(KB) void kick_kernel(int64_t n, double* __restrict__ vel,
                                                  const double* __restrict__ force,
                                                  const double* __restrict__ mass, double h) {
    const int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    const double s = h / mass[i];
    vel[3 * i] += force[3 * i] * s;
    vel[3 * i + 1] += force[3 * i + 1] * s;
    vel[3 * i + 2] += force[3 * i + 2] * s;
}

__global__ __launch_bounds__(KB) void drift_kernel(int64_t n, double* __restrict__ pos,
                                                   const double* __restrict__ vel, double dt) {
    const int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i >= 3 * n) return;
    pos[i] += vel[i] * dt;
}

}  // namespace

void run_kick(int64_t n, double* vel, const double* force, const double* mass, double h, hipStream_t s) {
    hipLaunchKernelGGL(kick_kernel, dim3((unsigned)cdiv(n, KB)), dim3(KB), 0, s, n, vel, force, mass, h);
    TFMM_LAUNCHED();
}

void run_drift(int64_t n, double* pos, const double* vel, double dt, hipStream_t s) {
    hipLaunchKernelGGL(drift_kernel, dim3((unsigned)cdiv(3 * n, KB)), dim3(KB), 0, s, n, pos, vel, dt);
    TFMM_LAUNCHED();
}

}  // namespace tfmm
