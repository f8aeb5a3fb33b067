// C ABI of libmfhex: validation, workspace layout, operator setup and the
// apply entry points.  Kernels live in the *.hip files; this file only checks
// arguments, carves the caller's workspace and enqueues work on the caller's
// stream.
#include <climits>
#include <cstdlib>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "blas.h"
#include "op.h"

using namespace mfhex;

namespace {

thread_local std::string g_err;  // last failure of a call that had no handle

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

int fail(int code, const std::string &m)
{
    g_err = m;
    return code;
}

int validate(const mfhex_desc *d, Basis1D *basis)
{
    if (!d) return fail(MFHEX_ERR_ARG, "null description");
    if (d->nex < 1 || d->ney < 1 || d->nez < 1) return fail(MFHEX_ERR_ARG, "nex, ney, nez must be >= 1");
    if (d->p < 1 || d->p > 8) return fail(MFHEX_ERR_UNSUPPORTED, "order p must be in [1, 8]");
    if (d->kind != MFHEX_MASS && d->kind != MFHEX_DIFFUSION) return fail(MFHEX_ERR_ARG, "kind must be mass or diffusion");
    if (d->ncomp != 1 && d->ncomp != 3) return fail(MFHEX_ERR_ARG, "ncomp must be 1 or 3");
    if (d->dirichlet != 0 && d->dirichlet != 1) return fail(MFHEX_ERR_ARG, "dirichlet must be 0 or 1");
    if (d->variable_kappa != 0 && d->variable_kappa != 1) return fail(MFHEX_ERR_ARG, "variable_kappa must be 0 or 1");
    if (d->variable_kappa && d->kind != MFHEX_DIFFUSION)
        return fail(MFHEX_ERR_ARG, "a variable coefficient needs a diffusion operator");
    if (d->flags & ~(MFHEX_FLAG_F32 | MFHEX_FLAG_RHS | MFHEX_FLAG_OTF | MFHEX_FLAG_DETERMINISTIC))
        return fail(MFHEX_ERR_ARG, "unknown flag bits");
    if ((d->flags & MFHEX_FLAG_OTF) &&
        (d->kind != MFHEX_DIFFUSION || d->variable_kappa || (d->flags & MFHEX_FLAG_F32)))
        return fail(MFHEX_ERR_UNSUPPORTED, "in-kernel geometric factors: FP64 diffusion with constant kappa only");
    if (!d->vertex_xyz) return fail(MFHEX_ERR_ARG, "vertex_xyz is null");
    const int64_t N = (int64_t)(d->p * (int64_t)d->nex + 1) * (d->p * (int64_t)d->ney + 1) * (d->p * (int64_t)d->nez + 1);
    if (N >= INT32_MAX) return fail(MFHEX_ERR_UNSUPPORTED, "more than 2^31-1 nodes (int32 restriction offsets)");
    std::string e;
    const int c = build_basis(d->p, d->q, d->quad, basis, &e);
    if (c != MFHEX_OK) return fail(c, e);
    return MFHEX_OK;
}

}  // namespace

namespace mfhex {

int fail_global(int code, const std::string &msg) { return fail(code, msg); }

}  // namespace mfhex

namespace mfhex {

Layout workspace_layout(const mfhex_desc &d, int64_t E, int P, int Q)
{
    const int g = d.kind == MFHEX_DIFFUSION ? kQdDiff : 1;
    const int64_t nv = (int64_t)(d.nex + 1) * (d.ney + 1) * (d.nez + 1);
    const size_t Q3 = (size_t)Q * Q * Q, P3 = (size_t)P * P * P;
    Layout L;
    size_t o = 0;
    L.vert = o;
    o += al(nv * 3 * sizeof(double));
    L.offsets = o;
    o += al(E * P3 * sizeof(int32_t));
    L.q64 = SIZE_MAX;
    if (!(d.flags & MFHEX_FLAG_OTF)) {
        L.q64 = o;
        o += al(E * g * Q3 * sizeof(double));
    }
    L.q32 = SIZE_MAX;
    if (d.flags & MFHEX_FLAG_F32) {
        L.q32 = o;
        o += al(E * g * Q3 * sizeof(float));
    }
    L.kappa = SIZE_MAX;
    if (d.variable_kappa) {
        L.kappa = o;
        o += al(E * Q3 * sizeof(double));
    }
    L.wdet = SIZE_MAX;
    if ((d.flags & MFHEX_FLAG_RHS) && d.kind == MFHEX_DIFFUSION) {
        L.wdet = o;
        o += al(E * Q3 * sizeof(double));
    }
    L.ebuf = SIZE_MAX;
    if (d.flags & MFHEX_FLAG_DETERMINISTIC) {
        L.ebuf = o;
        o += al(E * P3 * d.ncomp * sizeof(double));
    }
    L.basis = o;
    o += al(basis_len(P, Q) * (sizeof(double) + sizeof(float)) + 256);
    L.bad = o;
    o += 256;
    L.total = o;
    return L;
}

CgLayout cg_layout(int64_t n)
{
    CgLayout L;
    size_t o = 0;
    L.r64 = o;
    o += al(n * 8);
    L.p64 = o;
    o += al(n * 8);
    L.ap64 = o;
    o += al(n * 8);
    L.r32 = o;
    o += al(n * 4);
    L.p32 = o;
    o += al(n * 4);
    L.ap32 = o;
    o += al(n * 4);
    L.partial = o;
    o += al(2 * kRedBlocks * 8);
    L.sc = o;
    o += al(kNumSc * 8);
    L.hist = o;
    o += al(kHist * 8);
    L.z64 = o;
    o += al(n * 8);
    L.dinv64 = o;
    o += al(n * 8);
    L.z32 = o;
    o += al(n * 4);
    L.dinv32 = o;
    o += al(n * 4);
    L.total = o;
    return L;
}

int set_error(mfhex_op op, int code, const std::string &msg)
{
    if (op) op->err = msg;
    else g_err = msg;
    return code;
}

int check_hip(mfhex_op op, hipError_t e, const char *what)
{
    if (e == hipSuccess) return MFHEX_OK;
    return set_error(op, MFHEX_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int mode_of(const mfhex_op_s &op) { return op.d.kind == MFHEX_DIFFUSION ? kDiff : kMass; }

bool valid_variant(const mfhex_op_s &op, int prec, int variant)
{
    if ((prec != MFHEX_F64 && prec != MFHEX_F32) || variant < 0 || variant >= kNumVariants) return false;
    if (variant_vc(variant) > 1 && op.d.variable_kappa) return false;
    const bool otf = (op.d.flags & MFHEX_FLAG_OTF) != 0;
    if (otf && variant_vc(variant) > 1) return false;  // in-kernel factors: single-vector variants
    // the factored-gradient kernel: diffusion with Gauss points and stored factors
    if (variant_gf(variant) && (mode_of(op) != kDiff || op.basis.colloc || otf)) return false;
    // the matrix-core gradient: collocated FP64 diffusion with stored factors
    if (variant_mx(variant) && (mode_of(op) != kDiff || !op.basis.colloc || otf || prec != MFHEX_F64)) return false;
    return apply_lds(op.P, op.Q, mode_of(op), prec == MFHEX_F32 ? 4 : 8, variant, otf) <= kMaxLds;
}

int default_variant(const mfhex_op_s &op, int prec, int nvec)
{
    // one vector: the measured single-vector best for this operator and q;
    // several: the largest chunk that fits the LDS budget and does not exceed
    // the vector count
    if (nvec <= 1) {
        const int v = (mode_of(op) == kMass            ? kDefVariantMass
                       : prec == MFHEX_F32 ? kDefVariantDiff32
                                           : kDefVariantDiff)[op.Q - 2];
        return valid_variant(op, prec, v) ? v : 0;
    }
    // (with the scatter staging that several chunks need, the chunk must still leave room for two
    // thread groups per compute unit)
    const int eb = prec == MFHEX_F32 ? 4 : 8;
    for (int v = 8; v >= 5; --v) {  // the multi-vector chunk variants
        if (variant_vc(v) > nvec || !valid_variant(op, prec, v)) continue;
        const bool stage = nvec > variant_vc(v);
        if (apply_lds(op.P, op.Q, mode_of(op), eb, v, false, stage) <= kLdsTwoGroups) return v;
    }
    for (int v = 8; v >= 5; --v)
        if (variant_vc(v) <= nvec && valid_variant(op, prec, v)) return v;
    return 0;
}

// Pipeline depth: the mass kernel chains the measured best number of element
// groups per thread group; the diffusion kernel takes one.
int default_chain(const mfhex_op_s &op) { return mode_of(op) == kMass ? kDefChainMass[op.Q - 2] : 1; }

LaunchCfg config_for(const mfhex_op_s &op, int prec, int nvec)
{
    auto it = op.config.find({prec, nvec});
    if (it != op.config.end()) return it->second;
    LaunchCfg c;
    c.variant = default_variant(op, prec, nvec);
    c.chain = default_chain(op);
    return c;
}

hipError_t launch_apply(const ApplyLaunch &a)
{
    switch (a.P - 1) {
    case 1: return launch_apply_p1(a);
    case 2: return launch_apply_p2(a);
    case 3: return launch_apply_p3(a);
    case 4: return launch_apply_p4(a);
    case 5: return launch_apply_p5(a);
    case 6: return launch_apply_p6(a);
    case 7: return launch_apply_p7(a);
    case 8: return launch_apply_p8(a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kgrad(const KgradLaunch &a)
{
    switch (a.P - 1) {
    case 1: return launch_kgrad_p1(a);
    case 2: return launch_kgrad_p2(a);
    case 3: return launch_kgrad_p3(a);
    case 4: return launch_kgrad_p4(a);
    case 5: return launch_kgrad_p5(a);
    case 6: return launch_kgrad_p6(a);
    case 7: return launch_kgrad_p7(a);
    case 8: return launch_kgrad_p8(a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_diag(const DiagLaunch &a)
{
    switch (a.P - 1) {
    case 1: return launch_diag_p1(a);
    case 2: return launch_diag_p2(a);
    case 3: return launch_diag_p3(a);
    case 4: return launch_diag_p4(a);
    case 5: return launch_diag_p5(a);
    case 6: return launch_diag_p6(a);
    case 7: return launch_diag_p7(a);
    case 8: return launch_diag_p8(a);
    default: return hipErrorInvalidValue;
    }
}

static OpView view_of(const mfhex_op_s &op, int prec)
{
    OpView v;
    v.nelem = op.E;
    v.nex = op.d.nex;
    v.ney = op.d.ney;
    v.nez = op.d.nez;
    v.p = op.d.p;
    v.q = op.d.q;
    v.nnodes = op.N;
    v.offsets = op.offsets;
    v.qdata = prec == MFHEX_F32 ? (const void *)op.q32 : (const void *)op.q64;
    v.kappa = op.kappa;
    return v;
}

int apply_impl(mfhex_op op, int prec, int nrhs, const void *x, void *y, hipStream_t s, bool zero, int variant, int chain,
               void *ebuf_in)
{
    if (!op) return set_error(nullptr, MFHEX_ERR_ARG, "null handle");
    if (prec != MFHEX_F64 && prec != MFHEX_F32) return set_error(op, MFHEX_ERR_ARG, "prec must be F64 or F32");
    if (nrhs < 1 || nrhs > 4096) return set_error(op, MFHEX_ERR_ARG, "nrhs must be in [1, 4096]");
    if (!x || !y) return set_error(op, MFHEX_ERR_ARG, "null vector");
    if (prec == MFHEX_F32 && !op->q32)
        return set_error(op, MFHEX_ERR_STATE, "FP32 apply needs an operator created with MFHEX_FLAG_F32");
    if (prec == MFHEX_F32 && op->d.variable_kappa)
        return set_error(op, MFHEX_ERR_UNSUPPORTED, "variable coefficient is FP64 only");
    if (op->d.variable_kappa && !op->kappa_set) return set_error(op, MFHEX_ERR_STATE, "kappa not set");
    const int nvec = nrhs * op->d.ncomp;
    const size_t bytes = (size_t)op->N * nvec * (prec == MFHEX_F32 ? 4 : 8);
    const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y;
    if (xa < ya + bytes && ya < xa + bytes) return set_error(op, MFHEX_ERR_ARG, "x and y overlap");
    void *const ebuf = ebuf_in ? ebuf_in : op->ebuf;
    if (ebuf && nrhs != 1)
        return set_error(op, MFHEX_ERR_UNSUPPORTED, "deterministic operators apply one right-hand side at a time");
    const LaunchCfg cfg = config_for(*op, prec, nvec);
    const int var = variant >= 0 ? variant : cfg.variant;
    if (!valid_variant(*op, prec, var)) return set_error(op, MFHEX_ERR_ARG, "invalid launch variant");
    const int nchain = chain > 0 ? chain : cfg.chain;
    if (nchain > kMaxChain || (nchain > 1 && mode_of(*op) != kMass))
        return set_error(op, MFHEX_ERR_ARG, "invalid pipeline depth");
    if (zero && !ebuf) {
        const int c = check_hip(op, launch_zero(y, bytes, s), "zero fill");
        if (c) return c;
    }
    ApplyLaunch a{};
    a.v = view_of(*op, prec);
    a.P = op->P;
    a.colloc = op->basis.colloc;
    a.basis_dev = prec == MFHEX_F32 ? (const void *)op->basis32 : (const void *)op->basis64;
    a.prec = prec;
    a.mode = mode_of(*op);
    a.vark = op->d.variable_kappa;
    a.nvec = nvec;
    a.variant = var;
    a.chain = nchain;
    a.otf = (op->d.flags & MFHEX_FLAG_OTF) != 0;
    a.vert = op->vert;
    a.x = x;
    a.y = y;
    a.wdet = nullptr;
    a.ebuf = ebuf;
    a.stream = s;
    const int c = check_hip(op, launch_apply(a), "apply kernel launch");
    if (c || !ebuf) return c;
    // deterministic operators: element values in the element buffer, summed per node in a fixed order
    GeomLaunch g{op->d.nex, op->d.ney, op->d.nez, op->d.p, op->d.q, op->vert, &op->basis, s};
    return check_hip(op, launch_det_assemble(g, op->d.dirichlet, nvec, prec, ebuf, y, !zero),
                     "assembly kernel launch");
}

int diagonal_impl(mfhex_op op, double *d, hipStream_t s)
{
    if (!op) return set_error(nullptr, MFHEX_ERR_ARG, "null handle");
    if (!d) return set_error(op, MFHEX_ERR_ARG, "null output");
    if (op->d.variable_kappa && !op->kappa_set) return set_error(op, MFHEX_ERR_STATE, "kappa not set");
    if (!op->q64) return set_error(op, MFHEX_ERR_UNSUPPORTED, "the diagonal needs stored geometric factors");
    int c = check_hip(op, launch_zero(d, op->N * sizeof(double), s), "zero fill");
    if (c) return c;
    DiagLaunch a{};
    a.v = view_of(*op, MFHEX_F64);
    a.P = op->P;
    a.colloc = op->basis.colloc;
    a.mode = mode_of(*op);
    a.vark = op->d.variable_kappa;
    a.basis_dev = op->basis64;
    a.d = d;
    a.stream = s;
    return check_hip(op, launch_diag(a), "diagonal kernel launch");
}

}  // namespace mfhex

// ---------------------------------------------------------------------------

extern "C" {

int mfhex_query(const mfhex_desc *d, mfhex_sizes *out)
{
    Basis1D b;
    const int c = validate(d, &b);
    if (c) return c;
    if (!out) return fail(MFHEX_ERR_ARG, "null output");
    const int P = d->p + 1, Q = d->q;
    out->n_elem = (int64_t)d->nex * d->ney * d->nez;
    out->n_nodes = (int64_t)(d->p * (int64_t)d->nex + 1) * (d->p * (int64_t)d->ney + 1) * (d->p * (int64_t)d->nez + 1);
    out->n_qpts = out->n_elem * Q * Q * Q;
    out->workspace_bytes = workspace_layout(*d, out->n_elem, P, Q).total;
    out->cg_work_bytes = cg_layout(out->n_nodes).total;
    return MFHEX_OK;
}

int mfhex_create(const mfhex_desc *d, void *workspace_dev, size_t workspace_bytes, void *stream, mfhex_op *out)
{
    if (!out) return fail(MFHEX_ERR_ARG, "null output handle");
    *out = nullptr;
    Basis1D b;
    int c = validate(d, &b);
    if (c) return c;
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255)) return fail(MFHEX_ERR_ARG, "workspace must be 256-byte aligned");
    mfhex_op op = new mfhex_op_s();
    op->d = *d;
    op->d.vertex_xyz = nullptr;
    op->basis = b;
    op->P = d->p + 1;
    op->Q = d->q;
    op->g = d->kind == MFHEX_DIFFUSION ? kQdDiff : 1;
    op->E = (int64_t)d->nex * d->ney * d->nez;
    op->N = (int64_t)(d->p * (int64_t)d->nex + 1) * (d->p * (int64_t)d->ney + 1) * (d->p * (int64_t)d->nez + 1);
    op->NQ = op->E * op->Q * op->Q * op->Q;
    const Layout L = workspace_layout(*d, op->E, op->P, op->Q);
    if (workspace_bytes < L.total) {
        delete op;
        return fail(MFHEX_ERR_ARG, "workspace too small (see mfhex_query)");
    }
    char *ws = static_cast<char *>(workspace_dev);
    op->vert = reinterpret_cast<double *>(ws + L.vert);
    op->offsets = reinterpret_cast<int32_t *>(ws + L.offsets);
    op->q64 = L.q64 == SIZE_MAX ? nullptr : reinterpret_cast<double *>(ws + L.q64);
    op->q32 = L.q32 == SIZE_MAX ? nullptr : reinterpret_cast<float *>(ws + L.q32);
    op->kappa = L.kappa == SIZE_MAX ? nullptr : reinterpret_cast<double *>(ws + L.kappa);
    op->wdet = L.wdet == SIZE_MAX ? nullptr : reinterpret_cast<double *>(ws + L.wdet);
    op->ebuf = L.ebuf == SIZE_MAX ? nullptr : static_cast<void *>(ws + L.ebuf);
    op->bad = reinterpret_cast<int32_t *>(ws + L.bad);
    op->basis64 = reinterpret_cast<double *>(ws + L.basis);
    op->basis32 = reinterpret_cast<float *>(ws + L.basis + ((basis_len(op->P, op->Q) * sizeof(double) + 255) & ~size_t(255)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto bail = [&](int code) {
        // queued copies read host memory that the caller may free after the return
        (void)hipStreamSynchronize(s);
        g_err = op->err;
        if (op->pinned) (void)hipHostFree(op->pinned);
        delete op;
        return code;
    };
    if ((c = check_hip(op, hipGetDevice(&op->device), "hipGetDevice"))) return bail(c);
    if ((c = check_hip(op, hipHostMalloc((void **)&op->pinned, 64 * sizeof(double)), "hipHostMalloc"))) return bail(c);
    const int64_t nv = (int64_t)(d->nex + 1) * (d->ney + 1) * (d->nez + 1);
    if ((c = check_hip(op, hipMemcpyAsync(op->vert, d->vertex_xyz, nv * 3 * sizeof(double), hipMemcpyHostToDevice, s),
                       "copy vertices")))
        return bail(c);
    if ((c = check_hip(op, hipMemsetAsync(op->bad, 0, 256, s), "hipMemsetAsync"))) return bail(c);
    {
        // device basis block: B [Q][P], B^T [P][Q], D [Q][Q], D^T [Q][Q]
        const int P = op->P, Q = op->Q;
        std::vector<double> h(basis_len(P, Q));
        std::vector<float> h32(basis_len(P, Q));
        for (int a = 0; a < Q; ++a)
            for (int i = 0; i < P; ++i) {
                h[a * P + i] = b.B[a * P + i];
                h[Q * P + i * Q + a] = b.B[a * P + i];
            }
        for (int a = 0; a < Q; ++a)
            for (int k = 0; k < Q; ++k) {
                h[2 * Q * P + a * Q + k] = b.D[a * Q + k];
                h[2 * Q * P + Q * Q + k * Q + a] = b.D[a * Q + k];
            }
        // folded (even-odd) rows of a NO x NI row-major matrix at `m` into `f`
        auto fold = [](const double *m, int NO, int NI, double *f) {
            const int H = NI / 2;
            for (int o = 0; o < (NO + 1) / 2; ++o) {
                for (int i = 0; i < H; ++i) {
                    f[o * NI + i] = 0.5 * (m[o * NI + i] + m[o * NI + NI - 1 - i]);
                    f[o * NI + H + i] = 0.5 * (m[o * NI + i] - m[o * NI + NI - 1 - i]);
                }
                if (NI & 1) f[o * NI + 2 * H] = m[o * NI + H];
            }
        };
        fold(&h[basis_b(P, Q)], Q, P, &h[basis_bf(P, Q)]);
        fold(&h[basis_bt(P, Q)], P, Q, &h[basis_btf(P, Q)]);
        fold(&h[basis_d(P, Q)], Q, Q, &h[basis_df(P, Q)]);
        fold(&h[basis_dt(P, Q)], Q, Q, &h[basis_dtf(P, Q)]);
        for (int a = 0; a < Q; ++a) {
            h[basis_xq(P, Q) + a] = b.xq[a];
            h[basis_wq(P, Q) + a] = b.wq[a];
        }
        {
            // the basis derivative at the points, G[a][i] = l_i'(x_a), and its transpose, folded
            std::vector<double> g(Q * P), gt(P * Q);
            for (int a = 0; a < Q; ++a)
                for (int i = 0; i < P; ++i) g[a * P + i] = gt[i * Q + a] = b.Gn[a * P + i];
            fold(g.data(), Q, P, &h[basis_gf(P, Q)]);
            fold(gt.data(), P, Q, &h[basis_gtf(P, Q)]);
        }
        for (size_t i = 0; i < h.size(); ++i) h32[i] = (float)h[i];
        if ((c = check_hip(op, hipMemcpy(op->basis64, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
                           "copy basis")))
            return bail(c);
        if ((c = check_hip(op, hipMemcpy(op->basis32, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice),
                           "copy basis")))
            return bail(c);
    }
    GeomLaunch g{d->nex, d->ney, d->nez, d->p, d->q, op->vert, &op->basis, s};
    if ((c = check_hip(op, launch_offsets(g, d->dirichlet, op->offsets), "offsets kernel"))) return bail(c);
    if ((c = check_hip(op, launch_qdata(g, d->kind, op->q64, op->q32, op->wdet, op->bad), "qdata kernel")))
        return bail(c);
    if (op->kappa) {
        if ((c = check_hip(op, hipMemsetAsync(op->kappa, 0, op->NQ * sizeof(double), s), "hipMemsetAsync")))
            return bail(c);
    }
    int32_t bad = 0;
    if ((c = check_hip(op, hipMemcpyAsync(&bad, op->bad, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy flag")))
        return bail(c);
    if ((c = check_hip(op, hipStreamSynchronize(s), "hipStreamSynchronize"))) return bail(c);
    if (bad) {
        op->err = "mesh has an element with detJ <= 0 at a quadrature point";
        return bail(MFHEX_ERR_MESH);
    }
    load_tune_cache(op);
    *out = op;
    return MFHEX_OK;
}

int mfhex_destroy(mfhex_op op)
{
    if (!op) return MFHEX_OK;
    mg_release(op);
    if (op->pinned) (void)hipHostFree(op->pinned);
    delete op;
    return MFHEX_OK;
}

int mfhex_set_kappa(mfhex_op op, const double *kappa_dev, void *stream)
{
    if (!op) return fail(MFHEX_ERR_ARG, "null handle");
    if (!op->d.variable_kappa || !op->kappa) return set_error(op, MFHEX_ERR_STATE, "operator has no variable coefficient");
    if (!kappa_dev) return set_error(op, MFHEX_ERR_ARG, "null kappa");
    const int c = check_hip(op, hipMemcpyAsync(op->kappa, kappa_dev, op->NQ * sizeof(double), hipMemcpyDeviceToDevice,
                                               static_cast<hipStream_t>(stream)),
                            "copy kappa");
    if (c) return c;
    op->kappa_set = true;
    return MFHEX_OK;
}

int mfhex_apply(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream)
{
    return apply_impl(op, prec, nrhs, x_dev, y_dev, static_cast<hipStream_t>(stream), true, -1);
}

int mfhex_apply_add(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream)
{
    return apply_impl(op, prec, nrhs, x_dev, y_dev, static_cast<hipStream_t>(stream), false, -1);
}

int mfhex_apply_adjoint(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream)
{
    // The mass and diffusion operators (and M A M) are symmetric.
    return apply_impl(op, prec, nrhs, x_dev, y_dev, static_cast<hipStream_t>(stream), true, -1);
}

int mfhex_kappa_grad(mfhex_op op, const double *u_dev, const double *r_dev, double *g_dev, void *stream)
{
    if (!op) return fail(MFHEX_ERR_ARG, "null handle");
    if (op->d.kind != MFHEX_DIFFUSION) return set_error(op, MFHEX_ERR_STATE, "coefficient gradient needs a diffusion operator");
    if (op->d.ncomp != 1) return set_error(op, MFHEX_ERR_UNSUPPORTED, "coefficient gradient needs ncomp = 1");
    if (!op->q64) return set_error(op, MFHEX_ERR_UNSUPPORTED, "coefficient gradient needs stored geometric factors");
    if (!u_dev || !r_dev || !g_dev) return set_error(op, MFHEX_ERR_ARG, "null vector");
    KgradLaunch a{};
    a.v = view_of(*op, MFHEX_F64);
    a.P = op->P;
    a.colloc = op->basis.colloc;
    a.basis_dev = op->basis64;
    a.u = u_dev;
    a.r = r_dev;
    a.g = g_dev;
    a.stream = static_cast<hipStream_t>(stream);
    return check_hip(op, launch_kgrad(a), "coefficient gradient kernel launch");
}

int mfhex_diagonal(mfhex_op op, double *diag_dev, void *stream)
{
    return diagonal_impl(op, diag_dev, static_cast<hipStream_t>(stream));
}

int mfhex_qpoint_coords(mfhex_op op, double *xyz_dev, void *stream)
{
    if (!op) return fail(MFHEX_ERR_ARG, "null handle");
    if (!xyz_dev) return set_error(op, MFHEX_ERR_ARG, "null output");
    GeomLaunch g{op->d.nex, op->d.ney, op->d.nez, op->d.p, op->d.q, op->vert, &op->basis, static_cast<hipStream_t>(stream)};
    return check_hip(op, launch_qpoint_coords(g, xyz_dev), "coordinates kernel");
}

int mfhex_node_coords(mfhex_op op, double *xyz_dev, void *stream)
{
    if (!op) return fail(MFHEX_ERR_ARG, "null handle");
    if (!xyz_dev) return set_error(op, MFHEX_ERR_ARG, "null output");
    GeomLaunch g{op->d.nex, op->d.ney, op->d.nez, op->d.p, op->d.q, op->vert, &op->basis, static_cast<hipStream_t>(stream)};
    return check_hip(op, launch_node_coords(g, xyz_dev), "coordinates kernel");
}

int mfhex_rhs(mfhex_op op, const double *f_dev, double *b_dev, void *stream)
{
    if (!op) return fail(MFHEX_ERR_ARG, "null handle");
    if (!f_dev || !b_dev) return set_error(op, MFHEX_ERR_ARG, "null vector");
    const double *wdet = op->d.kind == MFHEX_MASS ? op->q64 : op->wdet;
    if (!wdet) return set_error(op, MFHEX_ERR_STATE, "load vector needs a mass operator or MFHEX_FLAG_RHS");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int c = check_hip(op, launch_zero(b_dev, op->N * sizeof(double), s), "zero fill");
    if (c) return c;
    ApplyLaunch a{};
    a.v = view_of(*op, MFHEX_F64);
    a.P = op->P;
    a.colloc = op->basis.colloc;
    a.basis_dev = op->basis64;
    a.prec = MFHEX_F64;
    a.mode = kRhs;
    a.vark = 0;
    a.nvec = 1;
    a.variant = 0;
    a.x = f_dev;
    a.y = b_dev;
    a.wdet = wdet;
    a.stream = s;
    return check_hip(op, launch_apply(a), "load vector kernel launch");
}

int mfhex_cg(mfhex_op op, const double *b_dev, double *x_dev, void *cg_work_dev, const mfhex_cg_opts *opts,
             mfhex_cg_stats *stats, double *rhist, void *stream)
{
    return cg_solve(op, b_dev, x_dev, cg_work_dev, opts, stats, rhist, static_cast<hipStream_t>(stream));
}

int mfhex_tune(mfhex_op op, int prec, int nrhs, void *scratch_dev, const char *cache_path, void *stream)
{
    return tune(op, prec, nrhs, scratch_dev, cache_path, static_cast<hipStream_t>(stream));
}

int mfhex_get_config(mfhex_op op, int prec, int nrhs, int32_t *variant, int32_t *elems_per_group,
                     int32_t *threads_per_group, int32_t *groups_per_block)
{
    if (!op || nrhs < 1) return fail(MFHEX_ERR_ARG, "bad argument");
    const LaunchCfg c = config_for(*op, prec, nrhs * op->d.ncomp);
    if (variant) *variant = c.variant;
    if (elems_per_group) *elems_per_group = variant_g(op->Q, c.variant, mode_of(*op));
    if (threads_per_group) *threads_per_group = variant_nt(op->Q, c.variant);
    if (groups_per_block) *groups_per_block = c.chain;
    return MFHEX_OK;
}

int mfhex_set_config(mfhex_op op, int prec, int nrhs, int32_t variant, int32_t groups_per_block)
{
    if (!op || nrhs < 1) return fail(MFHEX_ERR_ARG, "bad argument");
    if (!valid_variant(*op, prec, variant)) return set_error(op, MFHEX_ERR_ARG, "invalid launch variant");
    const int chain = groups_per_block > 0 ? groups_per_block : default_chain(*op);
    if (groups_per_block < 0 || chain > kMaxChain || (chain > 1 && mode_of(*op) != kMass))
        return set_error(op, MFHEX_ERR_ARG, "invalid pipeline depth");
    LaunchCfg c;
    c.variant = variant;
    c.chain = chain;
    op->config[{prec, nrhs * op->d.ncomp}] = c;
    return MFHEX_OK;
}

const char *mfhex_strerror(int code)
{
    switch (code) {
    case MFHEX_OK: return "ok";
    case MFHEX_ERR_ARG: return "invalid argument";
    case MFHEX_ERR_UNSUPPORTED: return "unsupported configuration";
    case MFHEX_ERR_HIP: return "HIP runtime error";
    case MFHEX_ERR_MESH: return "inverted or degenerate element (detJ <= 0)";
    case MFHEX_ERR_NOCONV: return "CG did not converge within maxit";
    case MFHEX_ERR_BREAKDOWN: return "CG breakdown (p^T A p <= 0 or non-finite)";
    case MFHEX_ERR_STATE: return "call not valid for this operator state";
    default: return "unknown status";
    }
}

const char *mfhex_last_error(mfhex_op op) { return op ? op->err.c_str() : g_err.c_str(); }

int mfhex_basis_1d(int p, int q, int quad, double *nodes, double *xq, double *wq, double *B, double *D)
{
    Basis1D b;
    std::string e;
    const int c = build_basis(p, q, quad, &b, &e);
    if (c) return fail(c, e);
    for (int i = 0; i < b.P; ++i)
        if (nodes) nodes[i] = b.nodes[i];
    for (int a = 0; a < b.Q; ++a) {
        if (xq) xq[a] = b.xq[a];
        if (wq) wq[a] = b.wq[a];
        for (int i = 0; i < b.P; ++i)
            if (B) B[a * b.P + i] = b.B[a * b.P + i];
        for (int k = 0; k < b.Q; ++k)
            if (D) D[a * b.Q + k] = b.D[a * b.Q + k];
    }
    return MFHEX_OK;
}

const char *mfhex_version(void) { return "mfhex 0.1 (gfx950)"; }

}  // extern "C"
