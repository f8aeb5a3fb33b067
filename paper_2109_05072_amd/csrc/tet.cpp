// Tetrahedral P_p diffusion operator: host set-up and C ABI.
//
// Sec. 2.1 (libCEED) and Sec. 2.2 (its MAGMA backend) apply a non-tensor basis through its full
// matrices: the interpolation / gradient matrix of one element (all points by
// all basis functions) times the element values of every element, one matrix
// product C = A B with A the basis matrix and B one column per element.  Here
// the gradient matrices G_d (d = 1..3) multiply 16 elements at a time on the
// FP64 matrix cores, the pointwise 3x3 factor acts on the products in
// registers, and the transposed products go back to the nodes.
//
// Mesh: every hexahedron of the structured box is split into the 6 Kuhn
// tetrahedra around its main diagonal (tetrahedron t, an axis permutation pi,
// has the cube corners 0, e_pi0, e_pi0 + e_pi1, (1,1,1)); each is affine on
// the physical positions of those corners.  Its P_p nodes, equispaced in
// barycentric coordinates, are points of the hexahedral lattice of spacing
// h/p, numbered as in the hexahedral operator.
// Basis: Lagrange on those nodes in Silvester's product form
//   phi_n(lambda) = prod_i R_{n_i}(p lambda_i),  R_k(z) = prod_{j<k} (z-j)/(k-j).
// Rule: the collapsed (conical product) rule, q points per direction:
// Gauss-Legendre in a, Gauss-Jacobi (1-s) in b and (1-s)^2 in c, mapped to
// xi = (a (1-b)(1-c), b (1-c), c); exact to degree 2q-1.  The Gauss-Jacobi
// points are the eigenvalues of the Jacobi matrix of P^(alpha,0) (Sturm
// bisection), the weights the closed form
//   w_j = 2^(alpha+1) Gamma(n+alpha+1) Gamma(n+1) / (Gamma(n+alpha+1) n!)
//         / ((1 - x_j^2) P_n'(x_j)^2)  (beta = 0).
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "blas.h"
#include "op.h"
#include "tet.h"

struct mfhex_tet_s {
    mfhex_tet_desc d{};
    mfhex::tet::Dims D{};
    int64_t E = 0, ngroups = 0, N = 0;
    double *afrag = nullptr, *bfrag = nullptr, *qdata = nullptr;
    int32_t *offsets = nullptr;
    const int32_t *lattice = nullptr;
};

namespace mfhex {
namespace tet {
namespace {

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// Eigenvalues of the symmetric tridiagonal matrix (diagonal a, off-diagonal b[1..m-1]) inside
// (-1, 1), ascending, by Sturm-sequence bisection.
void tridiag_eigs(const std::vector<double> &a, const std::vector<double> &b, double *lam)
{
    const int m = (int)a.size();
    auto count = [&](double x) {
        int c = 0;
        double d = a[0] - x;
        if (d < 0) ++c;
        for (int k = 1; k < m; ++k) {
            if (d == 0.0) d = 1e-300;
            d = a[k] - x - b[k] * b[k] / d;
            if (d < 0) ++c;
        }
        return c;
    };
    for (int j = 0; j < m; ++j) {
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (count(mid) > j) hi = mid;
            else lo = mid;
        }
        lam[j] = 0.5 * (lo + hi);
    }
}

// Jacobi polynomial P_n^(alpha,beta)(x) by its three-term recurrence.
double jacobi_poly(int n, double al_, double be, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * (al_ - be + (al_ + be + 2.0) * x);
    for (int k = 2; k <= n; ++k) {
        const double s = 2.0 * k + al_ + be;
        const double a1 = 2.0 * k * (k + al_ + be) * (s - 2.0);
        const double a2 = (s - 1.0) * (al_ * al_ - be * be);
        const double a3 = (s - 2.0) * (s - 1.0) * s;
        const double a4 = 2.0 * (k + al_ - 1.0) * (k + be - 1.0) * s;
        const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// n-point Gauss-Jacobi rule for int_0^1 f(s) (1-s)^alpha ds (beta = 0).
void gauss_jacobi_01(int n, int alpha, double *s, double *w)
{
    const double A = alpha;
    std::vector<double> a(n), b(n, 0.0), x(n);
    // Jacobi matrix of P^(A,0): diagonal -A^2 / (t (t+2)) with t = 2k + A (first row -A / (A+2)),
    // off-diagonal sqrt(4 k^2 (k+A)^2 / (t^2 (t+1)(t-1)))
    for (int k = 0; k < n; ++k) {
        const double t = 2.0 * k + A;
        a[k] = k == 0 ? -A / (A + 2.0) : -A * A / (t * (t + 2.0));
        if (k >= 1) {
            const double kk = k;
            b[k] = std::sqrt(4.0 * kk * (kk + A) * kk * (kk + A) / (t * t * (t + 1.0) * (t - 1.0)));
        }
    }
    tridiag_eigs(a, b, x.data());
    // Gamma(n+alpha+1) Gamma(n+1) / (Gamma(n+alpha+1) n!) = 1 for beta = 0
    for (int j = 0; j < n; ++j) {
        const double dp = 0.5 * (n + A + 1.0) * jacobi_poly(n - 1, A + 1.0, 1.0, x[j]);
        const double wj = std::pow(2.0, A + 1.0) / ((1.0 - x[j] * x[j]) * dp * dp);
        s[j] = 0.5 * (1.0 + x[j]);
        w[j] = wj / std::pow(2.0, A + 1.0);
    }
}

struct Rule {
    std::vector<double> xi, w;  // [Q][3], [Q]
};

Rule tet_rule(int q)
{
    std::vector<double> a(q), wa(q), b(q), wb(q), c(q), wc(q);
    gauss_jacobi_01(q, 0, a.data(), wa.data());
    gauss_jacobi_01(q, 1, b.data(), wb.data());
    gauss_jacobi_01(q, 2, c.data(), wc.data());
    Rule R;
    for (int k = 0; k < q; ++k)
        for (int j = 0; j < q; ++j)
            for (int i = 0; i < q; ++i) {
                R.xi.push_back(a[i] * (1.0 - b[j]) * (1.0 - c[k]));
                R.xi.push_back(b[j] * (1.0 - c[k]));
                R.xi.push_back(c[k]);
                R.w.push_back(wa[i] * wb[j] * wc[k]);
            }
    return R;
}

// Barycentric multi-indices (n1, n2, n3) of the basis functions (n0 = p - n1 - n2 - n3).
std::vector<int> lattice(int p)
{
    std::vector<int> L;
    for (int n3 = 0; n3 <= p; ++n3)
        for (int n2 = 0; n2 <= p - n3; ++n2)
            for (int n1 = 0; n1 <= p - n3 - n2; ++n1) {
                L.push_back(n1);
                L.push_back(n2);
                L.push_back(n3);
                L.push_back(0);
            }
    return L;
}

// R_k(z) and R_k'(z).
void silvester(int k, double z, double &r, double &dr)
{
    r = 1.0;
    dr = 0.0;
    for (int j = 0; j < k; ++j) {
        const double f = (z - j) / (k - j);
        dr = dr * f + r / (k - j);
        r *= f;
    }
}

// Values B [M][P] and reference gradients G [3][M][P] at points xi [M][3].
void eval_basis(int p, const double *xi, int M, double *B, double *G)
{
    const std::vector<int> L = lattice(p);
    const int P = n_basis(p);
    for (int m = 0; m < M; ++m) {
        const double lam[4] = {1.0 - xi[3 * m] - xi[3 * m + 1] - xi[3 * m + 2], xi[3 * m], xi[3 * m + 1],
                               xi[3 * m + 2]};
        for (int n = 0; n < P; ++n) {
            const int k[4] = {p - L[4 * n] - L[4 * n + 1] - L[4 * n + 2], L[4 * n], L[4 * n + 1], L[4 * n + 2]};
            double r[4], dr[4];
            for (int i = 0; i < 4; ++i) silvester(k[i], p * lam[i], r[i], dr[i]);
            double dl[4];
            for (int i = 0; i < 4; ++i) {
                dl[i] = p * dr[i];
                for (int j = 0; j < 4; ++j)
                    if (j != i) dl[i] *= r[j];
            }
            if (B) B[(size_t)m * P + n] = r[0] * r[1] * r[2] * r[3];
            for (int d = 0; d < 3; ++d) G[((size_t)d * M + m) * P + n] = dl[d + 1] - dl[0];
        }
    }
}

struct Layout {
    size_t afrag, bfrag, lattice, wq, vert, bad, offsets, qdata, total;
};

Layout layout(const mfhex_tet_desc &d, const Dims &D, int64_t ngroups)
{
    Layout L{};
    size_t o = 0;
    L.afrag = o;
    o += al(afrag_len(D) * 8);
    L.bfrag = o;
    o += al(bfrag_len(D) * 8);
    L.lattice = o;
    o += al((size_t)D.P * 4 * 4);
    L.wq = o;
    o += al((size_t)D.Q * 8);
    L.vert = o;
    o += al((size_t)(d.nex + 1) * (d.ney + 1) * (d.nez + 1) * 3 * 8);
    L.bad = o;
    o += 256;
    L.offsets = o;
    if (!pair_groups(D.p)) o += al((size_t)ngroups * D.P * kGroup * 4);
    L.qdata = o;
    o += al((size_t)ngroups * D.Q * 6 * kGroup * 8);
    L.total = o;
    return L;
}

// Element groups: 16 consecutive elements, or (low orders) the two x-adjacent hexahedra of a pair.
int64_t n_groups(const mfhex_tet_desc &d)
{
    if (pair_groups(d.p)) return (int64_t)((d.nex + 1) / 2) * d.ney * d.nez;
    return (6LL * d.nex * d.ney * d.nez + kGroup - 1) / kGroup;
}

int validate(const mfhex_tet_desc *d)
{
    if (!d) return fail_global(MFHEX_ERR_ARG, "null description");
    if (d->p < 1 || d->p > kMaxP) return fail_global(MFHEX_ERR_UNSUPPORTED, "tetrahedral operator: p must be 1..6");
    if (d->q != d->p && d->q != d->p + 1)
        return fail_global(MFHEX_ERR_UNSUPPORTED, "tetrahedral operator: q must be p or p+1");
    if (d->nex < 1 || d->ney < 1 || d->nez < 1) return fail_global(MFHEX_ERR_ARG, "empty mesh");
    const int64_t E = 6LL * d->nex * d->ney * d->nez;
    const int64_t N = (int64_t)(d->p * (int64_t)d->nex + 1) * (d->p * (int64_t)d->ney + 1) * (d->p * (int64_t)d->nez + 1);
    if (N >= (1LL << 31) || E >= (1LL << 31) / kGroup)
        return fail_global(MFHEX_ERR_UNSUPPORTED, "tetrahedral operator: node or element count too large");
    if (!d->vertex_xyz) return fail_global(MFHEX_ERR_ARG, "null vertex array");
    return MFHEX_OK;
}

}  // namespace
}  // namespace tet
}  // namespace mfhex

using namespace mfhex;
using namespace mfhex::tet;

extern "C" {

int mfhex_tet_query(const mfhex_tet_desc *d, mfhex_tet_sizes *out)
{
    int c = validate(d);
    if (c) return c;
    if (!out) return fail_global(MFHEX_ERR_ARG, "null output");
    const Dims D = dims(d->p, d->q);
    const int64_t E = 6LL * d->nex * d->ney * d->nez, G = n_groups(*d);
    out->n_nodes = (int64_t)(d->p * (int64_t)d->nex + 1) * (d->p * (int64_t)d->ney + 1) * (d->p * (int64_t)d->nez + 1);
    out->n_elem = E;
    out->n_qpts = E * D.Q;
    out->n_basis = D.P;
    out->n_points = D.Q;
    out->workspace_bytes = layout(*d, D, G).total;
    return MFHEX_OK;
}

int mfhex_tet_basis(int p, int q, double *xi, double *w, double *B, double *G)
{
    if (p < 1 || p > tet::kMaxP || q < 1 || q > tet::kMaxP + 2) return fail_global(MFHEX_ERR_ARG, "bad p or q");
    const Rule R = tet_rule(q);
    const int Q = q * q * q;
    if (xi) std::memcpy(xi, R.xi.data(), sizeof(double) * 3 * Q);
    if (w) std::memcpy(w, R.w.data(), sizeof(double) * Q);
    if (G || B) {
        std::vector<double> g((size_t)3 * Q * n_basis(p));
        eval_basis(p, R.xi.data(), Q, B, g.data());
        if (G) std::memcpy(G, g.data(), g.size() * sizeof(double));
    }
    return MFHEX_OK;
}

int mfhex_tet_create(const mfhex_tet_desc *d, void *workspace_dev, size_t workspace_bytes, void *stream,
                     mfhex_tet *out)
{
    mfhex_tet_sizes sz;
    int c = mfhex_tet_query(d, &sz);
    if (c) return c;
    if (!out) return fail_global(MFHEX_ERR_ARG, "null output handle");
    *out = nullptr;
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255) || workspace_bytes < sz.workspace_bytes)
        return fail_global(MFHEX_ERR_ARG, "workspace missing, misaligned or too small (mfhex_tet_query)");
    auto op = std::make_unique<mfhex_tet_s>();
    op->d = *d;
    op->d.vertex_xyz = nullptr;
    op->D = dims(d->p, d->q);
    op->E = sz.n_elem;
    op->N = sz.n_nodes;
    op->ngroups = n_groups(*d);
    const Dims &D = op->D;
    const tet::Layout L = layout(*d, D, op->ngroups);
    char *w = static_cast<char *>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // on a failure after copies were queued, wait for them: their host sources are locals
    auto drain = [&](int code) {
        (void)hipStreamSynchronize(s);
        return code;
    };

    // gradient matrices G_d [Q][P] at the rule's points, as matrix-core fragments
    const Rule R = tet_rule(d->q);
    std::vector<double> g((size_t)3 * D.Q * D.P);
    eval_basis(d->p, R.xi.data(), D.Q, nullptr, g.data());
    auto G = [&](int dd, int k, int n) { return (k < D.Q && n < D.P) ? g[((size_t)dd * D.Q + k) * D.P + n] : 0.0; };
    std::vector<double> af(afrag_len(D)), bf(bfrag_len(D));
    for (int b = 0; b < D.Qp / 16; ++b)
        for (int dd = 0; dd < 3; ++dd) {
            for (int st = 0; st < D.Pk / 4; ++st)
                for (int l = 0; l < 64; ++l)
                    af[(((size_t)b * 3 + dd) * (D.Pk / 4) + st) * 64 + l] = G(dd, 16 * b + l % 16, 4 * st + l / 16);
            for (int r = 0; r < 4; ++r)
                for (int t = 0; t < D.Pn / 16; ++t)
                    for (int l = 0; l < 64; ++l)
                        bf[((((size_t)b * 3 + dd) * 4 + r) * (D.Pn / 16) + t) * 64 + l] =
                            G(dd, 16 * b + 4 * r + l / 16, 16 * t + l % 16);
        }
    const std::vector<int> lat = lattice(d->p);
    const size_t nv = (size_t)(d->nex + 1) * (d->ney + 1) * (d->nez + 1) * 3;
    op->afrag = reinterpret_cast<double *>(w + L.afrag);
    op->bfrag = reinterpret_cast<double *>(w + L.bfrag);
    op->offsets = pair_groups(d->p) ? nullptr : reinterpret_cast<int32_t *>(w + L.offsets);
    op->lattice = reinterpret_cast<const int32_t *>(w + L.lattice);
    op->qdata = reinterpret_cast<double *>(w + L.qdata);
    int *bad = reinterpret_cast<int *>(w + L.bad);
    if ((c = check_hip(nullptr, hipMemcpyAsync(op->afrag, af.data(), af.size() * 8, hipMemcpyHostToDevice, s), "copy")) ||
        (c = check_hip(nullptr, hipMemcpyAsync(op->bfrag, bf.data(), bf.size() * 8, hipMemcpyHostToDevice, s), "copy")) ||
        (c = check_hip(nullptr, hipMemcpyAsync(w + L.lattice, lat.data(), lat.size() * 4, hipMemcpyHostToDevice, s),
                       "copy")) ||
        (c = check_hip(nullptr, hipMemcpyAsync(w + L.wq, R.w.data(), R.w.size() * 8, hipMemcpyHostToDevice, s), "copy")) ||
        (c = check_hip(nullptr, hipMemcpyAsync(w + L.vert, d->vertex_xyz, nv * 8, hipMemcpyHostToDevice, s), "copy")) ||
        (c = check_hip(nullptr, hipMemsetAsync(bad, 0, sizeof(int), s), "hipMemsetAsync")))
        return drain(c);
    TetSetupLaunch S{};
    S.p = d->p;
    S.q = d->q;
    S.nex = d->nex;
    S.ney = d->ney;
    S.nez = d->nez;
    S.dirichlet = d->dirichlet;
    S.nelem = op->E;
    S.ngroups = op->ngroups;
    S.vert = reinterpret_cast<const double *>(w + L.vert);
    S.lattice = reinterpret_cast<const int32_t *>(w + L.lattice);
    S.wq = reinterpret_cast<const double *>(w + L.wq);
    S.offsets = op->offsets;
    S.qdata = op->qdata;
    S.bad = bad;
    S.stream = s;
    if ((c = check_hip(nullptr, launch_tet_setup(S), "tetrahedral set-up kernel"))) return drain(c);
    int hbad = 0;
    if ((c = check_hip(nullptr, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s), "copy")) ||
        (c = check_hip(nullptr, hipStreamSynchronize(s), "hipStreamSynchronize")))
        return c;
    if (hbad) return fail_global(MFHEX_ERR_MESH, "degenerate tetrahedron (det J = 0)");
    *out = op.release();
    return MFHEX_OK;
}

int mfhex_tet_apply(mfhex_tet op, const double *x_dev, double *y_dev, void *stream)
{
    if (!op) return fail_global(MFHEX_ERR_ARG, "null handle");
    if (!x_dev || !y_dev) return fail_global(MFHEX_ERR_ARG, "null vector");
    const uintptr_t xa = (uintptr_t)x_dev, ya = (uintptr_t)y_dev, bytes = (uintptr_t)op->N * sizeof(double);
    if (xa < ya + bytes && ya < xa + bytes) return fail_global(MFHEX_ERR_ARG, "x and y overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int c = check_hip(nullptr, launch_zero(y_dev, (size_t)op->N * sizeof(double), s), "zero fill");
    if (c) return c;
    TetLaunch a{};
    a.p = op->D.p;
    a.q = op->D.q;
    a.nex = op->d.nex;
    a.ney = op->d.ney;
    a.nez = op->d.nez;
    a.dirichlet = op->d.dirichlet;
    a.lattice = op->lattice;
    a.nelem = op->E;
    a.ngroups = op->ngroups;
    a.afrag = op->afrag;
    a.bfrag = op->bfrag;
    a.offsets = op->offsets;
    a.qdata = op->qdata;
    a.x = x_dev;
    a.y = y_dev;
    a.stream = s;
    return check_hip(nullptr, launch_tet_apply(a), "tetrahedral apply kernel");
}

int mfhex_tet_destroy(mfhex_tet op)
{
    delete op;
    return MFHEX_OK;
}

}  // extern "C"
