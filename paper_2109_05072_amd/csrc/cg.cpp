// Conjugate-gradient drivers on the matrix-free operator (host loop, device scalars).
//
// FP64 mode: unpreconditioned Hestenes-Stiefel CG (the solver Sec. 1 pairs with
// sum-factorized operator evaluation; the benchmarks of Sec. 2 run it
// unpreconditioned).  One iteration is apply, dot, fused x/r update with the
// new residual norm, and the direction update; alpha and beta never leave the
// GPU.  The host reads the scalars back every `check_every` iterations.  When
// the recursive residual reaches the tolerance, the true residual b - A x is
// computed; the solve stops only if it meets the tolerance too, and otherwise
// continues from it.
//
// Mixed mode (reliable updates): the operator, r, p and Ap are FP32 (FP32
// geometric factors and accumulation), x stays FP64 and every dot product
// accumulates in FP64.  When the recursive residual has dropped by
// replace_delta since the last replacement, every replace_every iterations,
// or when it claims convergence, the residual is replaced by the FP64 true
// residual r = fp32(b - A64 x) and beta is recomputed from it; convergence is
// only accepted on that true residual.  If three replacements in a row fail
// to lower the true residual, the solve continues in FP64.
//
// Jacobi preconditioning (either mode): z = D^-1 r with D the operator
// diagonal (mfhex_diagonal, inverted once per solve; 0 at masked nodes),
// alpha = r.z / p.Ap, beta = (r.z)_new / (r.z)_old, p = z + beta p; the
// update kernel forms z and both r.r and r.z in the same pass, and every
// residual replacement recomputes z and r.z.  Convergence is still measured
// on ||r||.  (Sec. 1: CG with preconditioners on sum-factorized operators;
// Sec. 2, Nek5000/RS: Jacobi smoothing.)
#include <algorithm>
#include <chrono>
#include <cmath>

#include "blas.h"
#include "op.h"

namespace mfhex {

namespace {

struct Ctx {
    mfhex_op op;
    hipStream_t s;
    int64_t n;
    double *r64, *p64, *ap64, *partial, *sc, *hist;
    float *r32, *p32, *ap32;
    bool pre;  // preconditioned (Jacobi or multigrid)
    bool mg;   // multigrid V-cycle as the preconditioner
    double *z64, *dinv64;
    float *z32, *dinv32;
};

#define TRY(expr)                         \
    do {                                  \
        const int c_ = (expr);            \
        if (c_ != MFHEX_OK) return c_;    \
    } while (0)
#define HIP(expr, what) TRY(check_hip(ctx.op, (expr), what))

// Read n scalars from device slot 0.. into the pinned host buffer and wait.
int read_scalars(Ctx &ctx)
{
    HIP(hipMemcpyAsync(ctx.op->pinned, ctx.sc, kNumSc * sizeof(double), hipMemcpyDeviceToHost, ctx.s), "read scalars");
    HIP(hipStreamSynchronize(ctx.s), "hipStreamSynchronize");
    return MFHEX_OK;
}

int dot_store(Ctx &ctx, const void *a, int pa, const void *b, int pb, int slot)
{
    HIP(launch_dot(a, pa, b, pb, ctx.n, ctx.partial, ctx.s), "dot kernel");
    HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, slot, nullptr, 0, ctx.s), "finalize kernel");
    return MFHEX_OK;
}

// z = M^-1 r (Jacobi: dinv r; multigrid: one V-cycle, FP64) and r.z into sc[slot].
int precond_store(Ctx &ctx, int prec, const void *r, void *z, int slot)
{
    if (ctx.mg) {
        TRY(mg_vcycle(ctx.op, static_cast<const double *>(r), static_cast<double *>(z), ctx.s));
        HIP(launch_dot(r, MFHEX_F64, z, MFHEX_F64, ctx.n, ctx.partial, ctx.s), "dot kernel");
    } else {
        const void *dinv = prec == MFHEX_F64 ? (const void *)ctx.dinv64 : (const void *)ctx.dinv32;
        HIP(launch_precond(r, dinv, z, prec, ctx.n, ctx.partial, ctx.s), "preconditioner kernel");
    }
    HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, slot, nullptr, 0, ctx.s), "finalize kernel");
    return MFHEX_OK;
}

// ||b - A x||^2 in FP64 into sc[kScRRTrue]; r64 / r32 receive the residual when non-null.
int true_residual(Ctx &ctx, const double *b, const double *x, double *r64, float *r32)
{
    TRY(apply_impl(ctx.op, MFHEX_F64, 1, x, ctx.ap64, ctx.s, true, -1));
    HIP(launch_residual(b, ctx.ap64, r64, r32, ctx.n, ctx.partial, ctx.s), "residual kernel");
    HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, kScRRTrue, nullptr, 0, ctx.s), "finalize kernel");
    return MFHEX_OK;
}

// FP64 CG from the current x (x0_is_zero: from 0).  k0: iterations already
// done (history offset).  Returns the status; *iters counts all iterations.
int cg64(Ctx &ctx, const double *b, double *x, const mfhex_cg_opts &o, bool x0_zero, int k0, int *iters, double bnorm)
{
    const int64_t n = ctx.n;
    if (x0_zero) {
        HIP(hipMemsetAsync(x, 0, n * sizeof(double), ctx.s), "hipMemsetAsync");
        HIP(launch_residual(b, nullptr, ctx.r64, nullptr, n, ctx.partial, ctx.s), "residual kernel");
        HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, kScRR, nullptr, 0, ctx.s), "finalize kernel");
    } else {
        TRY(true_residual(ctx, b, x, ctx.r64, nullptr));
        HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, kScRR, nullptr, 0, ctx.s), "finalize kernel");
    }
    if (ctx.pre) TRY(precond_store(ctx, MFHEX_F64, ctx.r64, ctx.z64, kScRZ));
    double *const zr = ctx.pre ? ctx.z64 : ctx.r64;  // search directions come from z (= r unpreconditioned)
    HIP(launch_copy(zr, MFHEX_F64, ctx.p64, MFHEX_F64, n, ctx.s), "copy kernel");
    const bool exact = o.max_iters_exact != 0;
    const int every = std::max(1, o.check_every);
    int k = k0;
    int status = MFHEX_ERR_NOCONV;
    while (k < o.maxit) {
        TRY(apply_impl(ctx.op, MFHEX_F64, 1, ctx.p64, ctx.ap64, ctx.s, true, -1));
        HIP(launch_dot(ctx.p64, MFHEX_F64, ctx.ap64, MFHEX_F64, n, ctx.partial, ctx.s), "dot kernel");
        HIP(launch_finalize(ctx.partial, ctx.sc, ctx.pre ? kFinAlphaPre : kFinAlpha, 0, nullptr, 0, ctx.s),
            "finalize kernel");
        if (ctx.mg) {
            // r.r from the update, then z = V(r) and r.z into the second half of the partials
            HIP(launch_update_xr(x, ctx.r64, ctx.p64, ctx.ap64, MFHEX_F64, ctx.sc, n, ctx.partial, ctx.s),
                "update kernel");
            TRY(mg_vcycle(ctx.op, ctx.r64, ctx.z64, ctx.s));
            HIP(launch_dot(ctx.r64, MFHEX_F64, ctx.z64, MFHEX_F64, n, ctx.partial + kRedBlocks, ctx.s), "dot kernel");
        } else if (ctx.pre)
            HIP(launch_update_xrz(x, ctx.r64, ctx.p64, ctx.ap64, ctx.dinv64, ctx.z64, MFHEX_F64, ctx.sc, n, ctx.partial,
                                  ctx.s),
                "update kernel");
        else
            HIP(launch_update_xr(x, ctx.r64, ctx.p64, ctx.ap64, MFHEX_F64, ctx.sc, n, ctx.partial, ctx.s),
                "update kernel");
        ++k;
        HIP(launch_finalize(ctx.partial, ctx.sc, ctx.pre ? kFinBetaPre : kFinBeta, k, ctx.hist, kHist, ctx.s),
            "finalize kernel");
        if (!exact && (k % every == 0 || k == o.maxit)) {
            TRY(read_scalars(ctx));
            const double *h = ctx.op->pinned;
            if (h[kScFlag] != 0.0) {
                status = MFHEX_ERR_BREAKDOWN;
                break;
            }
            if (std::sqrt(h[kScRRNew]) <= o.rtol * bnorm) {
                // the recursive residual claims convergence: accept only on the true residual,
                // otherwise continue from the true residual (beta from it, direction kept)
                const double rr_old = h[kScRRPrev], rz_old = h[kScRZPrev];
                TRY(true_residual(ctx, b, x, ctx.r64, nullptr));
                if (ctx.pre) TRY(precond_store(ctx, MFHEX_F64, ctx.r64, ctx.z64, kScRZTmp));
                TRY(read_scalars(ctx));
                double *hp = ctx.op->pinned;
                if (std::sqrt(hp[kScRRTrue]) <= o.rtol * bnorm) {
                    status = MFHEX_OK;
                    break;
                }
                hp[kScRR] = hp[kScRRTrue];
                if (ctx.pre) {
                    hp[kScRZ] = hp[kScRZTmp];
                    hp[kScBeta] = hp[kScRZTmp] / rz_old;
                } else {
                    hp[kScBeta] = hp[kScRRTrue] / rr_old;
                }
                HIP(hipMemcpyAsync(ctx.sc + kScRR, hp + kScRR, sizeof(double), hipMemcpyHostToDevice, ctx.s),
                    "write scalar");
                HIP(hipMemcpyAsync(ctx.sc + kScBeta, hp + kScBeta, sizeof(double), hipMemcpyHostToDevice, ctx.s),
                    "write scalar");
                HIP(hipMemcpyAsync(ctx.sc + kScRZ, hp + kScRZ, sizeof(double), hipMemcpyHostToDevice, ctx.s),
                    "write scalar");
                HIP(hipStreamSynchronize(ctx.s), "hipStreamSynchronize");
            }
        }
        HIP(launch_update_p(zr, ctx.p64, MFHEX_F64, ctx.sc, n, ctx.s), "update kernel");
    }
    if (exact) {
        TRY(read_scalars(ctx));
        status = ctx.op->pinned[kScFlag] != 0.0 ? MFHEX_ERR_BREAKDOWN : MFHEX_OK;
    }
    *iters = k;
    return status;
}

}  // namespace

int cg_solve(mfhex_op op, const double *b, double *x, void *work, const mfhex_cg_opts *o, mfhex_cg_stats *st,
             double *rhist, hipStream_t s)
{
    if (!op) return set_error(nullptr, MFHEX_ERR_ARG, "null handle");
    if (!b || !x || !work || !o) return set_error(op, MFHEX_ERR_ARG, "null argument");
    if (op->d.ncomp != 1) return set_error(op, MFHEX_ERR_UNSUPPORTED, "CG solves one component (ncomp = 1)");
    if (o->maxit < 0 || !(o->rtol >= 0.0)) return set_error(op, MFHEX_ERR_ARG, "bad maxit or rtol");
    if (o->mode != MFHEX_CG_F64 && o->mode != MFHEX_CG_MIXED) return set_error(op, MFHEX_ERR_ARG, "bad CG mode");
    if (o->precond != MFHEX_PRECOND_NONE && o->precond != MFHEX_PRECOND_JACOBI && o->precond != MFHEX_PRECOND_MG)
        return set_error(op, MFHEX_ERR_ARG, "bad preconditioner");
    if (o->precond == MFHEX_PRECOND_MG && !op->mg)
        return set_error(op, MFHEX_ERR_STATE, "multigrid preconditioner needs mfhex_mg_setup");
    if (o->precond == MFHEX_PRECOND_MG && o->mode != MFHEX_CG_F64)
        return set_error(op, MFHEX_ERR_UNSUPPORTED, "multigrid preconditioning runs in FP64 mode");
    if (o->mode == MFHEX_CG_MIXED && !op->q32)
        return set_error(op, MFHEX_ERR_STATE, "mixed CG needs an operator created with MFHEX_FLAG_F32");
    if (o->mode == MFHEX_CG_MIXED && op->d.variable_kappa)
        return set_error(op, MFHEX_ERR_UNSUPPORTED, "mixed CG with a variable coefficient is not built");
    if ((uintptr_t)work & 255) return set_error(op, MFHEX_ERR_ARG, "work area must be 256-byte aligned");
    const auto t0 = std::chrono::steady_clock::now();
    const CgLayout L = cg_layout(op->N);
    char *w = static_cast<char *>(work);
    Ctx ctx{op, s, op->N,
            reinterpret_cast<double *>(w + L.r64), reinterpret_cast<double *>(w + L.p64),
            reinterpret_cast<double *>(w + L.ap64), reinterpret_cast<double *>(w + L.partial),
            reinterpret_cast<double *>(w + L.sc), reinterpret_cast<double *>(w + L.hist),
            reinterpret_cast<float *>(w + L.r32), reinterpret_cast<float *>(w + L.p32),
            reinterpret_cast<float *>(w + L.ap32), o->precond != MFHEX_PRECOND_NONE, o->precond == MFHEX_PRECOND_MG,
            reinterpret_cast<double *>(w + L.z64), reinterpret_cast<double *>(w + L.dinv64),
            reinterpret_cast<float *>(w + L.z32), reinterpret_cast<float *>(w + L.dinv32)};
    HIP(hipMemsetAsync(ctx.sc, 0, kNumSc * sizeof(double), s), "hipMemsetAsync");
    if (ctx.pre && !ctx.mg) {
        // operator diagonal into dinv64, inverted in place (FP32 copy for mixed mode)
        TRY(diagonal_impl(op, ctx.dinv64, s));
        HIP(launch_jacobi_inverse(ctx.dinv64, ctx.dinv64, ctx.dinv32, op->N, s), "inverse kernel");
    }
    TRY(dot_store(ctx, b, MFHEX_F64, b, MFHEX_F64, kScBB));
    TRY(read_scalars(ctx));
    const double bnorm = std::sqrt(op->pinned[kScBB]);
    mfhex_cg_stats out{};
    int status = MFHEX_OK;
    int iters = 0;
    if (!std::isfinite(bnorm)) return set_error(op, MFHEX_ERR_BREAKDOWN, "right-hand side is not finite");
    if (bnorm == 0.0) {
        HIP(hipMemsetAsync(x, 0, op->N * sizeof(double), s), "hipMemsetAsync");
        HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (rhist) rhist[0] = 0.0;
        if (st) *st = out;
        return MFHEX_OK;
    }
    double r0 = bnorm;
    if (o->mode == MFHEX_CG_F64) {
        status = cg64(ctx, b, x, *o, o->x0_is_zero != 0, 0, &iters, bnorm);
    } else {
        const int64_t n = op->N;
        if (o->x0_is_zero) {
            HIP(hipMemsetAsync(x, 0, n * sizeof(double), s), "hipMemsetAsync");
            HIP(launch_residual(b, nullptr, nullptr, ctx.r32, n, ctx.partial, s), "residual kernel");
            HIP(launch_finalize(ctx.partial, ctx.sc, kFinStore, kScRRTrue, nullptr, 0, s), "finalize kernel");
        } else {
            TRY(true_residual(ctx, b, x, nullptr, ctx.r32));
        }
        TRY(dot_store(ctx, ctx.r32, MFHEX_F32, ctx.r32, MFHEX_F32, kScRR));
        if (ctx.pre) TRY(precond_store(ctx, MFHEX_F32, ctx.r32, ctx.z32, kScRZ));
        float *const zr = ctx.pre ? ctx.z32 : ctx.r32;
        HIP(launch_copy(zr, MFHEX_F32, ctx.p32, MFHEX_F32, n, s), "copy kernel");
        TRY(read_scalars(ctx));
        double last_true = std::sqrt(op->pinned[kScRRTrue]);
        r0 = last_true;
        double best_true = last_true;
        int stalls = 0, since = 0;
        const int every = std::max(1, o->check_every);
        const int repl_every = o->replace_every > 0 ? o->replace_every : 100;
        const double delta = o->replace_delta > 0.0 ? o->replace_delta : 0.1;
        status = MFHEX_ERR_NOCONV;
        bool fallback = false;
        while (iters < o->maxit) {
            TRY(apply_impl(op, MFHEX_F32, 1, ctx.p32, ctx.ap32, s, true, -1));
            HIP(launch_dot(ctx.p32, MFHEX_F32, ctx.ap32, MFHEX_F32, n, ctx.partial, s), "dot kernel");
            HIP(launch_finalize(ctx.partial, ctx.sc, ctx.pre ? kFinAlphaPre : kFinAlpha, 0, nullptr, 0, s),
                "finalize kernel");
            if (ctx.pre)
                HIP(launch_update_xrz(x, ctx.r32, ctx.p32, ctx.ap32, ctx.dinv32, ctx.z32, MFHEX_F32, ctx.sc, n,
                                      ctx.partial, s),
                    "update kernel");
            else
                HIP(launch_update_xr(x, ctx.r32, ctx.p32, ctx.ap32, MFHEX_F32, ctx.sc, n, ctx.partial, s),
                    "update kernel");
            ++iters;
            ++since;
            HIP(launch_finalize(ctx.partial, ctx.sc, ctx.pre ? kFinBetaPre : kFinBeta, iters, ctx.hist, kHist, s),
                "finalize kernel");
            if (iters % every == 0 || iters == o->maxit) {
                TRY(read_scalars(ctx));
                const double *h = op->pinned;
                if (h[kScFlag] != 0.0) {
                    fallback = true;
                    break;
                }
                const double rec = std::sqrt(h[kScRRNew]);
                if (rec <= delta * last_true || since >= repl_every || rec <= o->rtol * bnorm) {
                    // residual replacement with the FP64 true residual; beta from the new r
                    const double rr_old = h[kScRRPrev], rz_old = h[kScRZPrev];
                    TRY(true_residual(ctx, b, x, nullptr, ctx.r32));
                    TRY(dot_store(ctx, ctx.r32, MFHEX_F32, ctx.r32, MFHEX_F32, kScTmp));
                    if (ctx.pre) TRY(precond_store(ctx, MFHEX_F32, ctx.r32, ctx.z32, kScRZTmp));
                    TRY(read_scalars(ctx));
                    ++out.replacements;
                    since = 0;
                    const double tr = std::sqrt(op->pinned[kScRRTrue]);
                    if (tr <= o->rtol * bnorm) {
                        status = MFHEX_OK;
                        break;
                    }
                    if (tr >= best_true) {
                        if (++stalls >= 3) {
                            fallback = true;
                            break;
                        }
                    } else {
                        stalls = 0;
                        best_true = tr;
                    }
                    last_true = tr;
                    // beta = (r_new . r_new) / (r_prev . r_prev), rr = r_new . r_new
                    // (preconditioned: beta from r.z, rz = r_new . z_new)
                    op->pinned[kScRR] = op->pinned[kScTmp];
                    if (ctx.pre) {
                        op->pinned[kScRZ] = op->pinned[kScRZTmp];
                        op->pinned[kScBeta] = op->pinned[kScRZTmp] / rz_old;
                    } else {
                        op->pinned[kScBeta] = op->pinned[kScTmp] / rr_old;
                    }
                    HIP(hipMemcpyAsync(ctx.sc + kScRR, op->pinned + kScRR, sizeof(double), hipMemcpyHostToDevice, s),
                        "write scalar");
                    HIP(hipMemcpyAsync(ctx.sc + kScBeta, op->pinned + kScBeta, sizeof(double), hipMemcpyHostToDevice, s),
                        "write scalar");
                    HIP(hipMemcpyAsync(ctx.sc + kScRZ, op->pinned + kScRZ, sizeof(double), hipMemcpyHostToDevice, s),
                        "write scalar");
                    HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
                }
            }
            HIP(launch_update_p(zr, ctx.p32, MFHEX_F32, ctx.sc, n, s), "update kernel");
        }
        if (fallback && iters < o->maxit) {
            out.fell_back_to_f64 = 1;
            HIP(hipMemsetAsync(ctx.sc + kScFlag, 0, sizeof(double), s), "hipMemsetAsync");
            int it2 = iters;
            status = cg64(ctx, b, x, *o, false, iters, &it2, bnorm);
            iters = it2;
        } else if (fallback) {
            status = MFHEX_ERR_BREAKDOWN;
        }
    }
    // final FP64 true residual and recursive estimate
    TRY(true_residual(ctx, b, x, nullptr, nullptr));
    TRY(read_scalars(ctx));
    out.iters = iters;
    out.rel_resid_true = std::sqrt(op->pinned[kScRRTrue]) / bnorm;
    out.rel_resid_rec = std::sqrt(op->pinned[kScRR]) / bnorm;
    if (rhist) {
        const int nh = std::min(iters, kHist - 1);
        rhist[0] = r0;
        if (nh > 0)
            HIP(hipMemcpy(rhist + 1, ctx.hist + 1, nh * sizeof(double), hipMemcpyDeviceToHost), "copy history");
    }
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = out;
    if (status == MFHEX_ERR_NOCONV) set_error(op, status, "CG reached maxit");
    if (status == MFHEX_ERR_BREAKDOWN) set_error(op, status, "CG breakdown");
    return status;
}

}  // namespace mfhex
