// Vector kernels for the Krylov solver and the tuner (blas.hip).
#pragma once

#include "mfhex_internal.h"

namespace mfhex {

constexpr int kRedBlocks = 1024;  // fixed reduction grid (deterministic sums)
constexpr int kRedThreads = 256;

// Device scalar slots of the solver.
enum : int {
    kScRR = 0,      // r.r of the current residual
    kScRRNew = 1,   // r.r after the last update
    kScPAp = 2,     // p.Ap
    kScAlpha = 3,
    kScBeta = 4,
    kScBB = 5,      // b.b
    kScRRTrue = 6,  // ||b - A x||^2 in FP64
    kScFlag = 7,    // 1 after a breakdown / non-finite value
    kScTmp = 8,
    kScRRPrev = 9,  // r.r before the last beta update
    kScRZ = 10,     // r.z of the current residual (Jacobi-preconditioned CG)
    kScRZPrev = 11, // r.z before the last beta update
    kScRZTmp = 12,
    kNumSc = 16
};
enum : int { kFinStore = 0, kFinAlpha = 1, kFinBeta = 2, kFinAlphaPre = 3, kFinBetaPre = 4 };

// prec arguments are MFHEX_F64 / MFHEX_F32.
hipError_t launch_dot(const void *a, int pa, const void *b, int pb, int64_t n, double *partial, hipStream_t s);
// kFinStore: sc[k] = sum; kFinAlpha: pAp, alpha = rr / pAp (flag on pAp <= 0);
// kFinBeta: rr_new, beta = rr_new / rr, rr = rr_new, hist[k] = sqrt(rr_new).
// Preconditioned forms: kFinAlphaPre: alpha = rz / pAp; kFinBetaPre: the
// partials hold r.r then r.z (2 kRedBlocks): rr = rr_new, beta = rz_new / rz,
// rz = rz_new, hist[k] = sqrt(rr_new).
hipError_t launch_finalize(const double *partial, double *sc, int op, int k, double *hist, int hist_len,
                           hipStream_t s);
hipError_t launch_update_xr(double *x, void *r, const void *p, const void *Ap, int prec, const double *sc, int64_t n,
                            double *partial, hipStream_t s);
hipError_t launch_update_p(const void *r, void *p, int prec, const double *sc, int64_t n, hipStream_t s);
// x += alpha p; r -= alpha Ap; z = dinv r; partials of r.r and r.z (2 kRedBlocks).
hipError_t launch_update_xrz(double *x, void *r, const void *p, const void *Ap, const void *dinv, void *z, int prec,
                             const double *sc, int64_t n, double *partial, hipStream_t s);
// z = dinv r; partials of r.z (kRedBlocks).
hipError_t launch_precond(const void *r, const void *dinv, void *z, int prec, int64_t n, double *partial,
                          hipStream_t s);
// dinv64 = 1 / d where d > 0, else 0 (masked nodes); dinv32 = fp32(dinv64).
hipError_t launch_jacobi_inverse(const double *d, double *dinv64, float *dinv32, int64_t n, hipStream_t s);
hipError_t launch_residual(const double *b, const double *Ax, double *r64, float *r32, int64_t n, double *partial,
                           hipStream_t s);
hipError_t launch_copy(const void *src, int ps, void *dst, int pd, int64_t n, hipStream_t s);
// bytes (a multiple of 4) of zeros at p, by a kernel (graph-capture safe, unlike a runtime memset).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_fill_uniform(double *x, int64_t n, uint64_t seed, hipStream_t s);
// out2[0] = max |a - b| (inf if a has a NaN), out2[1] = max |b|; partial holds 2*kRedBlocks doubles.
hipError_t launch_relmaxdiff(const void *a, const void *b, int64_t n, int prec, double *partial, double *out2,
                             hipStream_t s);

}  // namespace mfhex
