// p-multigrid kernels (mg.hip) and the hierarchy attached to an operator (mg.cpp).
#pragma once

#include <vector>

#include "mfhex_internal.h"

struct mfhex_op_s;

namespace mfhex {

// y_fine += P x_coarse (dir = 0) or y_coarse += P^T r_fine (dir = 1) for levels of order
// pf (fine) and pc (coarse) on the same nex x ney x nez mesh.  I1: device [pf+1][pc+1] in the
// vectors' precision prec (MFHEX_F64 / MFHEX_F32).
struct TransferLaunch {
    int pf, pc, dir, prec;
    int32_t nex, ney, nez;
    const int32_t *off_f, *off_c;  // element restrictions of the two levels
    const void *I1;
    const void *src;
    void *dst;
    hipStream_t stream;
};
hipError_t launch_transfer(const TransferLaunch &t);

// Chebyshev smoother vector steps (n entries):
//   init:  x = 0 (when zero_x), r = dinv (b - Ax) (Ax may be null: r = dinv b), d = r / theta
//   step:  x += d; r -= dinv Ad; d = cd d + cr r
//   last:  x += d
//   resid: r = b - Ax
// (all vectors in precision prec)
hipError_t launch_cheb_init(const void *b, const void *Ax, const void *dinv, void *x, void *r, void *d,
                            double inv_theta, bool zero_x, int prec, int64_t n, hipStream_t s);
hipError_t launch_cheb_step(void *x, void *d, void *r, const void *Ad, const void *dinv, double cd, double cr,
                            bool last, int prec, int64_t n, hipStream_t s);
hipError_t launch_mg_residual(const void *b, const void *Ax, void *r, int prec, int64_t n, hipStream_t s);
// v *= (dinv > 0) and, with scale != 0, v *= scale.
hipError_t launch_mask_scale(double *v, const double *dinv, double scale, int64_t n, hipStream_t s);
// out = dinv * a (elementwise).
hipError_t launch_scale_by(const double *a, const double *dinv, double *out, int64_t n, hipStream_t s);
// partial sums of sum_i v_i^2 / dinv_i over dinv_i > 0 (v^T D v).
hipError_t launch_dot_dinv(const double *v, const double *dinv, int64_t n, double *partial, hipStream_t s);

struct MgLevel {
    mfhex_op_s *op = nullptr;  // level operator (level 0: the caller's, not owned)
    int p = 0;
    int64_t n = 0;
    double lam = 0.0;          // power-method estimate of lambda_max(D^-1 A)
    double *dinv64 = nullptr;  // FP64 inverse diagonal (set-up and FP64 cycles)
    // vectors in the cycle precision (FP64 or FP32): inverse diagonal, level right-hand side and
    // solution (the fine level's come from the caller in an FP64 cycle; in an FP32 cycle they hold
    // the caller's vectors rounded), Chebyshev work
    void *dinv = nullptr, *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *ad = nullptr;
    void *I1 = nullptr;        // interpolation from level l+1 to this level, [p+1][p_{l+1}+1]
};

struct MgHierarchy {
    std::vector<MgLevel> lv;
    int degree = 3, coarse_degree = 8, power_iters = 15;
    int prec = MFHEX_F64;       // precision of the V-cycle
    double lo = 0.25, hi = 1.1;
    double *partial = nullptr;  // reduction scratch (2 kRedBlocks doubles)
};

// Orders of the levels: p, floor(p/2), ..., 1 (at most max_levels when > 0).
std::vector<int> mg_orders(int p, int max_levels);

}  // namespace mfhex
