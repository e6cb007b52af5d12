// Small device-to-host read-backs on the critical path (tree header, walk
// state, list totals).
//
// A one-block kernel queued on the producer's stream copies the words into a
// pinned, device-coherent mailbox together with the context's device error
// word, fences at system scope and then publishes a sequence number; the host
// spins on that number.  This replaces a runtime copy plus a stream
// synchronisation (two copy kernels and the runtime's wake-up latency) by one
// tiny kernel and a poll.  A wait that lasts longer than kSpinNs falls back to
// a blocking stream synchronisation, which also surfaces any device error.
#include <immintrin.h>

#include <chrono>

#include "common.h"

namespace tfmm {
namespace {

constexpr int kBoxBlock = 256;
constexpr int64_t kSpinNs = 20'000'000;  // 20 ms of polling, then block

__global__ __launch_bounds__(kBoxBlock) void mailbox_kernel(const uint32_t* __restrict__ src, int nwords,
                                                            const uint32_t* __restrict__ err,
                                                            uint32_t* __restrict__ box, uint32_t seq) {
    for (int i = threadIdx.x; i < nwords; i += kBoxBlock) box[kBoxHeaderWords + i] = src[i];
    if (threadIdx.x == 0) box[1] = *err;
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(box, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

void read_back_bytes(Ctx* ctx, const void* dev, size_t bytes, void* out, bool check_err, hipStream_t s) {
    if (bytes % 4 != 0 || bytes > kBoxPayload) fail(TFMM_EINVAL, "read-back size");
    uint32_t* box = ctx->mbox;
    uint32_t seq = ++ctx->mbox_seq;
    if (seq == 0u) seq = ++ctx->mbox_seq;  // 0 is the mailbox's initial value
    hipLaunchKernelGGL(mailbox_kernel, dim3(1), dim3(kBoxBlock), 0, s, static_cast<const uint32_t*>(dev),
                       (int)(bytes / 4), (const uint32_t*)ctx->dev_err, ctx->mbox_dev, seq);
    TFMM_LAUNCHED();
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 1; __atomic_load_n(box, __ATOMIC_ACQUIRE) != seq; ++k) {
        _mm_pause();
        if ((k & 1023u) == 0u &&
            std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count() >
                kSpinNs) {
            TFMM_HIP(hipStreamSynchronize(s));
            if (__atomic_load_n(box, __ATOMIC_ACQUIRE) != seq)
                fail(TFMM_EDEVICE, "a read-back did not arrive after its stream completed");
            break;
        }
    }
    std::memcpy(out, box + kBoxHeaderWords, bytes);
    if (check_err && box[1] != 0u)
        fail(TFMM_EDEVICE, "a device-side wait ran past its bound (internal error); results are invalid");
}

}  // namespace tfmm
