// Throughput of the FP64 arithmetic pipes of this GPU: chains of 16x16x4 and
// 4x4x4 (four blocks) FP64 matrix-core products and of FP64 vector FMAs, four
// or eight independent accumulators per lane, operands in registers only.
// The caller times each kind with events on `stream` and divides the flops it
// issued by the time.  Each lane writes one result to out[global thread id],
// so `out` holds nblocks * 256 doubles.  Part of the measuring library
// (libhbmprobe.so), not of the operator.  The kernels carry no launch bounds:
// with a 256-thread bound the compiler moved the MFMA accumulators between
// VGPRs and AGPRs in every iteration, which measures those moves instead.
// (The FP64 MFMA on gfx950 accumulates in VGPRs.)
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kRateThreads = 256;

__global__ void k_rate_mfma16(double *out, int iters, double a0, double b0)
{
    d4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
    const double a = a0 + threadIdx.x * 1e-9, b = b0 - threadIdx.x * 1e-9;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
    }
    out[(int64_t)blockIdx.x * kRateThreads + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

__global__ void k_rate_mfma4(double *out, int iters, double a0, double b0)
{
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    const double a = a0 + threadIdx.x * 1e-9, b = b0 - threadIdx.x * 1e-9;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c3, 0, 0, 0);
    }
    out[(int64_t)blockIdx.x * kRateThreads + threadIdx.x] = c0 + c1 + c2 + c3;
}

__global__ void k_rate_fma(double *out, int iters, double a0, double b0)
{
    double c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = threadIdx.x + j;
    const double a = a0 + threadIdx.x * 1e-9;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = __builtin_fma(c[j], a, b0);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += c[j];
    out[(int64_t)blockIdx.x * kRateThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// kind: 0 16x16x4 FP64 MFMA, 1 4x4x4 FP64 MFMA (four blocks), 2 v_fma_f64.  Flops one 64-lane
// wavefront issues per iteration: 4 * 2048, 4 * 512 and 8 * 128.  Returns the hipError_t of the
// launch.
int fp64_rate(int kind, double *out, int nblocks, int iters, void *stream)
{
    if (!out || nblocks <= 0 || iters <= 0 || kind < 0 || kind > 2) return (int)hipErrorInvalidValue;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto k = kind == 0 ? k_rate_mfma16 : kind == 1 ? k_rate_mfma4 : k_rate_fma;
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(kRateThreads), 0, s, out, iters, 1.0, 0.5);
    return (int)hipGetLastError();
}

double fp64_rate_flops_per_wave_iter(int kind)
{
    return kind == 0 ? 4.0 * 2 * 16 * 16 * 4 : kind == 1 ? 4.0 * 2 * 4 * 4 * 4 * 4 : 8.0 * 2 * 64;
}

}  // extern "C"
