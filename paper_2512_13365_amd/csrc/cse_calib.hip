// cse_calib.hip -- microbenchmarks of the two on-chip rates the step kernels
// are bounded by: the issue rate of 32-bit integer VALU instructions and the
// LDS read bandwidth.  The benchmark runs them to state measured peaks beside
// the ones derived from the unit counts and clock, and a counter run over
// them calibrates how VALU-busy figures are read from SQ counters (the
// instruction count of each launch is known exactly).
//
// valu: every lane runs 8 independent chains of v_add_u32 written as inline
// assembly (register operands only), 16 per chain per iteration: 128 VALU
// instructions per wave and iteration, none dependent on the one before it.
// lds:  every lane reads 16 B per ds_read_b128 from a 64 KiB shared array,
// consecutive lanes consecutive 16 B (no bank conflicts), 8 reads per
// iteration.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;
constexpr int kChains = 8;
constexpr int kUnroll = 16;
constexpr int kLdsWords = 4096;  // uint4 entries: 64 KiB
constexpr int kLdsReads = 8;

__global__ __launch_bounds__(kBlock) void calib_valu_kernel(uint32_t* out, int iters) {
    uint32_t x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * (c + 1) + blockIdx.x;
    const uint32_t k = 0x9E3779B9u + blockIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(k));
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= x[c];
    if (r == 0x7FFFFFFFu) out[blockIdx.x] = r;  // keeps the chains alive; never true in practice
}

__global__ __launch_bounds__(kBlock) void calib_lds_kernel(uint32_t* out, int iters) {
    __shared__ uint4 buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kBlock) buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint32_t acc0 = 0, acc1 = 0;
    int base = threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kLdsReads; ++u) {
            const uint4 v = buf[(base + u * kBlock) & (kLdsWords - 1)];
            acc0 = acc0 ^ v.x ^ v.y;  // two three-input xors per read
            acc1 = acc1 ^ v.z ^ v.w;
        }
        base = (base + kLdsReads * kBlock) & (kLdsWords - 1);
    }
    if ((acc0 ^ acc1) == 0x7FFFFFFFu) out[blockIdx.x] = acc0;
}

}  // namespace

extern "C" {

// kind 0: VALU, 1: LDS.  Launches `blocks` workgroups of 256 lanes for
// `iters` iterations on the default stream, times it with HIP events
// (*ms), and reports the work: VALU instructions per wave (kind 0) or LDS
// bytes read in all (kind 1) in *work.  Returns 0, or the HIP error code.
int cse_calib_run(int kind, int blocks, int iters, float* ms, double* work) {
    if (kind < 0 || kind > 1 || blocks < 1 || iters < 1 || !ms || !work) return (int)hipErrorInvalidValue;
    uint32_t* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&out, sizeof(uint32_t) * (size_t)blocks);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        // One warm-up launch, then the timed one.
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            if (rep == 1) e = hipEventRecord(e0, nullptr);
            if (kind == 0)
                hipLaunchKernelGGL(calib_valu_kernel, dim3(blocks), dim3(kBlock), 0, nullptr, out, iters);
            else
                hipLaunchKernelGGL(calib_lds_kernel, dim3(blocks), dim3(kBlock), 0, nullptr, out, iters);
            if (e == hipSuccess) e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (kind == 0)
        *work = (double)iters * kChains * kUnroll;
    else
        *work = (double)blocks * kBlock * (double)iters * kLdsReads * 16.0;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return (int)e;
}

}  // extern "C"
