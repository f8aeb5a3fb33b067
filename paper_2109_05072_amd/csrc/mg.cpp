// p-multigrid preconditioner: hierarchy set-up and the V-cycle (host loop, device kernels).
//
// Levels p, floor(p/2), ..., 1 on the fine operator's mesh with the same
// quadrature family and mask (Sec. 1: high-order codes precondition with
// p-multigrid).  Each level smooths with Chebyshev iteration on D^-1 A over
// [lo, hi] x lambda, D the operator diagonal (mfhex_diagonal) and lambda a
// power-method estimate of the top eigenvalue of D^-1 A (Sec. 2,
// Nek5000/RS: Chebyshev-accelerated Jacobi smoothing).  V-cycle on level l
// for A_l x = b_l from x = 0:
//     x = S(b, 0); r = b - A x; b_{l+1} = P^T r; x_{l+1} = V(b_{l+1});
//     x += P x_{l+1}; x = S(b, x)
// with S the degree-k Chebyshev smoother; the coarsest level is smoothed
// only (degree k_coarse).  Equal pre- and post-smoothers and R = P^T make
// the V-cycle a symmetric positive definite preconditioner for CG.
#include <cmath>
#include <memory>
#include <string>

#include "blas.h"
#include "mg.h"
#include "op.h"

namespace mfhex {

std::vector<int> mg_orders(int p, int max_levels)
{
    std::vector<int> o{p};
    while (o.back() > 1 && (max_levels <= 0 || (int)o.size() < max_levels)) o.push_back(std::max(1, o.back() / 2));
    return o;
}

namespace {

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

mfhex_desc level_desc(const mfhex_desc &fine, int p, int prec)
{
    mfhex_desc d = fine;
    d.p = p;
    d.q = fine.quad == MFHEX_GAUSS ? p + 2 : p + 1;
    d.flags = prec == MFHEX_F32 ? MFHEX_FLAG_F32 : 0u;
    d.variable_kappa = 0;
    d.ncomp = 1;
    return d;
}

int64_t n_nodes(const mfhex_desc &d)
{
    return (int64_t)(d.p * (int64_t)d.nex + 1) * (d.p * (int64_t)d.ney + 1) * (d.p * (int64_t)d.nez + 1);
}

struct Opts {
    int degree, coarse_degree, power_iters, max_levels, prec;
    double lo, hi;
};

Opts resolve(const mfhex_mg_opts *o)
{
    Opts r{3, 8, 15, 0, MFHEX_F64, 0.25, 1.1};
    if (o) {
        r.prec = o->precision;
        if (o->degree > 0) r.degree = o->degree;
        if (o->coarse_degree > 0) r.coarse_degree = o->coarse_degree;
        if (o->power_iters > 0) r.power_iters = o->power_iters;
        if (o->max_levels > 0) r.max_levels = o->max_levels;
        if (o->lo > 0.0) r.lo = o->lo;
        if (o->hi > 0.0) r.hi = o->hi;
    }
    return r;
}

size_t elem_bytes(int prec) { return prec == MFHEX_F32 ? sizeof(float) : sizeof(double); }

// Work-buffer layout: per coarse level an operator workspace; per level the FP64 inverse
// diagonal and the cycle vectors (FP64 cycle: r, d, ad, and b, x below the fine level, the
// inverse diagonal being the FP64 one; FP32 cycle: dinv, r, d, ad, b, x on every level); the
// interpolation matrices in the cycle precision; the reduction scratch; and for an FP32 cycle
// two FP64 fine-level vectors for the power method.
struct MgLayout {
    std::vector<size_t> ws, ws_bytes, dinv64, vec, mat;
    size_t partial = 0, power = 0, total = 0;
};

MgLayout mg_layout(const mfhex_desc &fine, const std::vector<int> &orders, int prec)
{
    MgLayout L;
    size_t o = 0;
    const int nl = (int)orders.size();
    const size_t eb = elem_bytes(prec);
    L.ws.assign(nl, 0);
    L.ws_bytes.assign(nl, 0);
    L.dinv64.assign(nl, 0);
    L.vec.assign(nl, 0);
    L.mat.assign(nl, 0);
    for (int l = 1; l < nl; ++l) {
        const mfhex_desc d = level_desc(fine, orders[l], prec);
        const int64_t E = (int64_t)d.nex * d.ney * d.nez;
        L.ws[l] = o;
        L.ws_bytes[l] = workspace_layout(d, E, d.p + 1, d.q).total;
        o += al(L.ws_bytes[l]);
    }
    for (int l = 0; l < nl; ++l) {
        const int64_t n = n_nodes(level_desc(fine, orders[l], prec));
        L.dinv64[l] = o;
        o += al(n * sizeof(double));
        L.vec[l] = o;
        o += (prec == MFHEX_F32 ? 6 : l == 0 ? 3 : 5) * al(n * eb);
    }
    for (int l = 0; l + 1 < nl; ++l) {
        L.mat[l] = o;
        o += al((size_t)(orders[l] + 1) * (orders[l + 1] + 1) * eb);
    }
    L.partial = o;
    o += al(2 * kRedBlocks * sizeof(double));
    if (prec == MFHEX_F32) {
        L.power = o;
        o += 2 * al(n_nodes(fine) * sizeof(double));
    }
    L.total = o;
    return L;
}

// Lagrange basis on `xc` (nc nodes) evaluated at `xf` (nf points): M[f][c], product formula.
std::vector<double> interp_matrix(const double *xc, int nc, const double *xf, int nf)
{
    std::vector<double> M((size_t)nf * nc);
    for (int f = 0; f < nf; ++f)
        for (int c = 0; c < nc; ++c) {
            double v = 1.0;
            for (int m = 0; m < nc; ++m)
                if (m != c) v *= (xf[f] - xc[m]) / (xc[c] - xc[m]);
            M[(size_t)f * nc + c] = v;
        }
    return M;
}

#define TRY(expr)                         \
    do {                                  \
        const int c_ = (expr);            \
        if (c_ != MFHEX_OK) return c_;    \
    } while (0)

double read_dot(mfhex_op op, double *partial, hipStream_t s, int *err)
{
    *err = check_hip(op, launch_finalize(partial, partial + kRedBlocks, kFinStore, 0, nullptr, 0, s), "finalize");
    if (*err) return 0.0;
    double h = 0.0;
    *err = check_hip(op, hipMemcpyAsync(&h, partial + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (!*err) *err = check_hip(op, hipStreamSynchronize(s), "sync");
    return h;
}

// Power method on D^-1 A (FP64) from the counter-based uniform vector (seed), masked; v, av:
// FP64 work vectors of L.n entries.
int power_lambda(mfhex_op fine, MgLevel &L, double *v, double *av, double *partial, int iters, hipStream_t s)
{
    const int64_t n = L.n;
    int e = 0;
    TRY(check_hip(fine, launch_fill_uniform(v, n, 2024, s), "fill"));
    TRY(check_hip(fine, launch_mask_scale(v, L.dinv64, 0.0, n, s), "mask"));
    TRY(check_hip(fine, launch_dot(v, MFHEX_F64, v, MFHEX_F64, n, partial, s), "dot"));
    double nv = read_dot(fine, partial, s, &e);
    if (e) return e;
    TRY(check_hip(fine, launch_mask_scale(v, L.dinv64, 1.0 / std::sqrt(nv), n, s), "scale"));
    double lam = 0.0;
    for (int k = 0; k < iters; ++k) {
        TRY(apply_impl(L.op, MFHEX_F64, 1, v, av, s, true, -1));
        TRY(check_hip(fine, launch_dot(v, MFHEX_F64, av, MFHEX_F64, n, partial, s), "dot"));
        const double vav = read_dot(fine, partial, s, &e);
        if (e) return e;
        TRY(check_hip(fine, launch_dot_dinv(v, L.dinv64, n, partial, s), "dot"));
        const double vdv = read_dot(fine, partial, s, &e);
        if (e) return e;
        lam = vav / vdv;
        TRY(check_hip(fine, launch_scale_by(av, L.dinv64, v, n, s), "scale"));  // v = dinv A v
        TRY(check_hip(fine, launch_dot(v, MFHEX_F64, v, MFHEX_F64, n, partial, s), "dot"));
        nv = read_dot(fine, partial, s, &e);
        if (e) return e;
        TRY(check_hip(fine, launch_mask_scale(v, L.dinv64, 1.0 / std::sqrt(nv), n, s), "scale"));
    }
    if (!(lam > 0.0) || !std::isfinite(lam)) return set_error(fine, MFHEX_ERR_BREAKDOWN, "power method failed");
    L.lam = lam;
    return MFHEX_OK;
}

// Degree-k Chebyshev smoother on level L: x <- S(b, x) (x = 0 when zero_x), vectors in the
// cycle precision; the recurrence coefficients are formed in FP64 on the host.
int chebyshev(mfhex_op fine, const MgHierarchy &h, const MgLevel &L, const void *b, void *x, int degree,
              bool zero_x, hipStream_t s)
{
    const double lo = h.lo * L.lam, hi = h.hi * L.lam;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    if (!zero_x) TRY(apply_impl(L.op, h.prec, 1, x, L.ad, s, true, -1));
    TRY(check_hip(fine,
                  launch_cheb_init(b, zero_x ? nullptr : L.ad, L.dinv, x, L.r, L.d, 1.0 / theta, zero_x, h.prec,
                                   L.n, s),
                  "chebyshev kernel"));
    double rho = 1.0 / sigma;
    for (int k = 0; k < degree; ++k) {
        const bool last = k == degree - 1;
        double cd = 0.0, cr = 0.0;
        if (!last) {
            TRY(apply_impl(L.op, h.prec, 1, L.d, L.ad, s, true, -1));
            const double rho_new = 1.0 / (2.0 * sigma - rho);
            cd = rho_new * rho;
            cr = 2.0 * rho_new / delta;
            rho = rho_new;
        }
        TRY(check_hip(fine, launch_cheb_step(x, L.d, L.r, L.ad, L.dinv, cd, cr, last, h.prec, L.n, s),
                      "chebyshev kernel"));
    }
    return MFHEX_OK;
}

int transfer(mfhex_op fine, const MgHierarchy &h, const MgLevel &F, const MgLevel &Cl, int dir, const void *src,
             void *dst, hipStream_t s)
{
    TransferLaunch t{};
    t.pf = F.p;
    t.pc = Cl.p;
    t.dir = dir;
    t.prec = h.prec;
    t.nex = fine->d.nex;
    t.ney = fine->d.ney;
    t.nez = fine->d.nez;
    t.off_f = F.op->offsets;
    t.off_c = Cl.op->offsets;
    t.I1 = F.I1;
    t.src = src;
    t.dst = dst;
    t.stream = s;
    return check_hip(fine, launch_transfer(t), "transfer kernel");
}

int vcycle(mfhex_op fine, MgHierarchy &h, int l, const void *b, void *x, hipStream_t s)
{
    MgLevel &L = h.lv[l];
    if (l + 1 == (int)h.lv.size()) return chebyshev(fine, h, L, b, x, h.coarse_degree, true, s);
    TRY(chebyshev(fine, h, L, b, x, h.degree, true, s));
    TRY(apply_impl(L.op, h.prec, 1, x, L.ad, s, true, -1));
    TRY(check_hip(fine, launch_mg_residual(b, L.ad, L.r, h.prec, L.n, s), "residual kernel"));
    MgLevel &Cl = h.lv[l + 1];
    TRY(check_hip(fine, launch_zero(Cl.b, Cl.n * elem_bytes(h.prec), s), "zero fill"));
    TRY(transfer(fine, h, L, Cl, 1, L.r, Cl.b, s));
    TRY(vcycle(fine, h, l + 1, Cl.b, Cl.x, s));
    TRY(transfer(fine, h, L, Cl, 0, Cl.x, x, s));
    return chebyshev(fine, h, L, b, x, h.degree, false, s);
}

}  // namespace

int mg_vcycle(mfhex_op op, const double *r, double *z, hipStream_t s)
{
    if (!op) return set_error(nullptr, MFHEX_ERR_ARG, "null handle");
    if (!op->mg) return set_error(op, MFHEX_ERR_STATE, "no multigrid hierarchy (mfhex_mg_setup)");
    if (!r || !z) return set_error(op, MFHEX_ERR_ARG, "null vector");
    MgHierarchy &h = *op->mg;
    if (h.prec != MFHEX_F32) return vcycle(op, h, 0, r, z, s);
    MgLevel &L0 = h.lv[0];
    TRY(check_hip(op, launch_copy(r, MFHEX_F64, L0.b, MFHEX_F32, L0.n, s), "copy kernel"));
    TRY(vcycle(op, h, 0, L0.b, L0.x, s));
    return check_hip(op, launch_copy(L0.x, MFHEX_F32, z, MFHEX_F64, L0.n, s), "copy kernel");
}

void mg_release(mfhex_op op)
{
    if (!op || !op->mg) return;
    for (size_t l = 1; l < op->mg->lv.size(); ++l) mfhex_destroy(op->mg->lv[l].op);
    op->mg.reset();
}

}  // namespace mfhex

using namespace mfhex;

extern "C" {

int mfhex_mg_query(const mfhex_desc *fine, const mfhex_mg_opts *opts, size_t *work_bytes, int32_t *nlevels)
{
    mfhex_sizes sz;
    const int c = mfhex_query(fine, &sz);
    if (c) return c;
    if (fine->kind != MFHEX_DIFFUSION || fine->variable_kappa || fine->ncomp != 1 || (fine->flags & MFHEX_FLAG_OTF)) {
        return fail_global(MFHEX_ERR_UNSUPPORTED,
                           "multigrid: scalar diffusion with stored geometric factors and constant kappa only");
    }
    const Opts o = resolve(opts);
    if (o.prec != MFHEX_F64 && o.prec != MFHEX_F32) return fail_global(MFHEX_ERR_ARG, "multigrid: bad precision");
    if (o.prec == MFHEX_F32 && !(fine->flags & MFHEX_FLAG_F32))
        return fail_global(MFHEX_ERR_ARG, "multigrid: an FP32 cycle needs an operator created with MFHEX_FLAG_F32");
    const std::vector<int> orders = mg_orders(fine->p, o.max_levels);
    if (work_bytes) *work_bytes = mg_layout(*fine, orders, o.prec).total;
    if (nlevels) *nlevels = (int32_t)orders.size();
    return MFHEX_OK;
}

int mfhex_mg_setup(mfhex_op op, const mfhex_desc *fine, const mfhex_mg_opts *opts, void *work_dev, size_t work_bytes,
                   void *stream)
{
    if (!op) return fail_global(MFHEX_ERR_ARG, "null handle");
    size_t need = 0;
    int32_t nl = 0;
    int c = mfhex_mg_query(fine, opts, &need, &nl);
    if (c) return set_error(op, c, mfhex_last_error(nullptr));
    if (fine->p != op->d.p || fine->q != op->d.q || fine->nex != op->d.nex || fine->ney != op->d.ney ||
        fine->nez != op->d.nez || fine->quad != op->d.quad || fine->dirichlet != op->d.dirichlet ||
        fine->kind != op->d.kind || fine->flags != op->d.flags)
        return set_error(op, MFHEX_ERR_ARG, "description does not match the operator");
    if (!work_dev || ((uintptr_t)work_dev & 255) || work_bytes < need)
        return set_error(op, MFHEX_ERR_ARG, "multigrid work area missing, misaligned or too small (mfhex_mg_query)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    mg_release(op);
    const Opts o = resolve(opts);
    const std::vector<int> orders = mg_orders(fine->p, o.max_levels);
    const MgLayout L = mg_layout(*fine, orders, o.prec);
    const size_t eb = elem_bytes(o.prec);
    char *w = static_cast<char *>(work_dev);
    auto h = std::make_unique<MgHierarchy>();
    h->prec = o.prec;
    h->degree = o.degree;
    h->coarse_degree = o.coarse_degree;
    h->power_iters = o.power_iters;
    h->lo = o.lo;
    h->hi = o.hi;
    h->partial = reinterpret_cast<double *>(w + L.partial);
    h->lv.resize(orders.size());
    auto cleanup = [&](int code) {
        for (size_t l = 1; l < h->lv.size(); ++l) mfhex_destroy(h->lv[l].op);
        return code;
    };
    for (size_t l = 0; l < orders.size(); ++l) {
        MgLevel &lv = h->lv[l];
        const mfhex_desc d = level_desc(*fine, orders[l], o.prec);
        lv.p = orders[l];
        lv.n = n_nodes(d);
        if (l == 0) {
            lv.op = op;
        } else if ((c = mfhex_create(&d, w + L.ws[l], L.ws_bytes[l], stream, &lv.op))) {
            lv.op = nullptr;
            return cleanup(set_error(op, c, std::string("coarse level: ") + mfhex_last_error(nullptr)));
        }
        const size_t vb = al(lv.n * eb);
        char *v = w + L.vec[l];
        lv.dinv64 = reinterpret_cast<double *>(w + L.dinv64[l]);
        int k = 0;
        lv.dinv = o.prec == MFHEX_F32 ? static_cast<void *>(v + vb * k++) : lv.dinv64;
        lv.r = v + vb * k++;
        lv.d = v + vb * k++;
        lv.ad = v + vb * k++;
        if (l > 0 || o.prec == MFHEX_F32) {
            lv.b = v + vb * k++;
            lv.x = v + vb * k++;
        }
        if ((c = diagonal_impl(lv.op, lv.dinv64, s))) return cleanup(set_error(op, c, lv.op->err));
        float *dinv32 = o.prec == MFHEX_F32 ? static_cast<float *>(lv.dinv) : nullptr;
        if ((c = check_hip(op, launch_jacobi_inverse(lv.dinv64, lv.dinv64, dinv32, lv.n, s), "inverse kernel")))
            return cleanup(c);
        double *pv = static_cast<double *>(lv.r), *pav = static_cast<double *>(lv.ad);
        if (o.prec == MFHEX_F32) {
            pv = reinterpret_cast<double *>(w + L.power);
            pav = reinterpret_cast<double *>(w + L.power + al(n_nodes(*fine) * sizeof(double)));
        }
        if ((c = power_lambda(op, lv, pv, pav, h->partial, h->power_iters, s))) return cleanup(c);
    }
    for (size_t l = 0; l + 1 < orders.size(); ++l) {
        Basis1D bf, bc;
        std::string e;
        build_basis(orders[l], orders[l] + 1, MFHEX_GLL, &bf, &e);
        build_basis(orders[l + 1], orders[l + 1] + 1, MFHEX_GLL, &bc, &e);
        const std::vector<double> M = interp_matrix(bc.nodes, orders[l + 1] + 1, bf.nodes, orders[l] + 1);
        const std::vector<float> M32(M.begin(), M.end());
        h->lv[l].I1 = w + L.mat[l];
        const void *src = o.prec == MFHEX_F32 ? static_cast<const void *>(M32.data()) : M.data();
        if ((c = check_hip(op, hipMemcpy(h->lv[l].I1, src, M.size() * eb, hipMemcpyHostToDevice),
                           "copy interpolation")))
            return cleanup(c);
    }
    if ((c = check_hip(op, hipStreamSynchronize(s), "hipStreamSynchronize"))) return cleanup(c);
    op->mg = std::move(h);
    return MFHEX_OK;
}

int mfhex_mg_apply(mfhex_op op, const double *r_dev, double *z_dev, void *stream)
{
    return mg_vcycle(op, r_dev, z_dev, static_cast<hipStream_t>(stream));
}

int mfhex_mg_level(mfhex_op op, int level, int32_t *p, int64_t *n_nodes_out, double *lambda_max)
{
    if (!op) return fail_global(MFHEX_ERR_ARG, "null handle");
    if (!op->mg) return set_error(op, MFHEX_ERR_STATE, "no multigrid hierarchy (mfhex_mg_setup)");
    if (level < 0 || level >= (int)op->mg->lv.size()) return set_error(op, MFHEX_ERR_ARG, "no such level");
    const MgLevel &L = op->mg->lv[level];
    if (p) *p = L.p;
    if (n_nodes_out) *n_nodes_out = L.n;
    if (lambda_max) *lambda_max = L.lam;
    return MFHEX_OK;
}

}  // extern "C"
