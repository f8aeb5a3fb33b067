// 1D bases of the tensor-product element (host setup, FP64).
//
// Nodes: Gauss-Lobatto-Legendre points on [-1,1] (the Q_p basis of Sec. 1).
// Quadrature: Gauss-Legendre with q = p+2 points, or Gauss-Lobatto with
// q = p+1 points collocated with the nodes.
//
// Rules are the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// orthogonal family (Golub-Welsch), found by Sturm-sequence bisection:
//   Gauss, n points: Legendre recurrence, off-diagonal k / sqrt(4k^2 - 1);
//   Lobatto, n points: -1, +1 and the n-2 zeros of the Jacobi polynomial
//   P^{(1,1)}_{n-2} (the zeros of P_{n-1}'), off-diagonal
//   sqrt(k (k+2) / ((2k+1)(2k+3))).
// Weights from the closed forms 2 / ((1-x^2) P_n'(x)^2) (Gauss) and
// 2 / (n (n-1) P_{n-1}(x)^2) (Lobatto).  Lagrange polynomials, their
// derivatives and the collocation differentiation matrices use the
// barycentric form.
#include <cmath>
#include <cstring>

#include "mfhex_internal.h"

namespace mfhex {

namespace {

// Number of eigenvalues below x of the tridiagonal matrix with zero
// diagonal and off-diagonal off[0..m-2] (LDL^T pivots of T - x I).
int sturm_count(const double *off, int m, double x)
{
    int cnt = 0;
    double d = -x;
    if (d < 0) ++cnt;
    for (int k = 1; k < m; ++k) {
        if (d == 0.0) d = 1e-300;
        d = -x - off[k - 1] * off[k - 1] / d;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// All m eigenvalues (ascending, inside (-1,1)) by bisection.
void tridiag_eigs(const double *off, int m, double *lam)
{
    for (int j = 0; j < m; ++j) {
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(off, m, mid) > j) hi = mid;
            else lo = mid;
        }
        lam[j] = 0.5 * (lo + hi);
    }
}

// Legendre P_n(x) and P_n'(x) (for |x| < 1 the derivative uses
// (1 - x^2) P_n' = n (P_{n-1} - x P_n)).
void legendre(int n, double x, double *pn, double *dpn)
{
    double pm1 = 0.0, p0 = 1.0;
    for (int k = 0; k < n; ++k) {
        const double p1 = ((2 * k + 1) * x * p0 - k * pm1) / (k + 1);
        pm1 = p0;
        p0 = p1;
    }
    *pn = p0;
    *dpn = (n == 0) ? 0.0 : n * (pm1 - x * p0) / (1.0 - x * x);
}

void bary_weights(const double *x, int n, double *lam)
{
    for (int j = 0; j < n; ++j) {
        double pr = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) pr *= (x[j] - x[k]);
        lam[j] = 1.0 / pr;
    }
}

// Values and derivatives at z of the n Lagrange polynomials through x.
void bary_eval(const double *x, const double *lam, int n, double z, double *l, double *dl)
{
    for (int j = 0; j < n; ++j)
        if (z == x[j]) {
            // z is node j: Kronecker values, derivatives = row j of the
            // differentiation matrix.
            double s = 0.0;
            for (int k = 0; k < n; ++k) {
                l[k] = (k == j) ? 1.0 : 0.0;
                if (k != j) {
                    dl[k] = (lam[k] / lam[j]) / (x[j] - x[k]);
                    s += dl[k];
                }
            }
            dl[j] = -s;
            return;
        }
    double den = 0.0;
    for (int k = 0; k < n; ++k) den += lam[k] / (z - x[k]);
    for (int j = 0; j < n; ++j) {
        l[j] = (lam[j] / (z - x[j])) / den;
        double s = 0.0;
        for (int k = 0; k < n; ++k)
            if (k != j) s += 1.0 / (z - x[k]);
        dl[j] = l[j] * s;
    }
}

}  // namespace

int gauss_rule(int n, double *x, double *w)
{
    if (n < 1 || n > 32) return MFHEX_ERR_ARG;
    double off[32];
    for (int k = 1; k < n; ++k) off[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    tridiag_eigs(off, n, x);
    for (int j = 0; j < n; ++j) {
        double pn, dpn;
        legendre(n, x[j], &pn, &dpn);
        w[j] = 2.0 / ((1.0 - x[j] * x[j]) * dpn * dpn);
    }
    return MFHEX_OK;
}

int lobatto_rule(int n, double *x, double *w)
{
    if (n < 2 || n > 32) return MFHEX_ERR_ARG;
    const int m = n - 2;
    double off[32];
    for (int k = 1; k < m; ++k) off[k - 1] = std::sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)));
    x[0] = -1.0;
    x[n - 1] = 1.0;
    if (m > 0) tridiag_eigs(off, m, x + 1);
    for (int j = 0; j < n; ++j) {
        double pn, dpn;
        legendre(n - 1, x[j], &pn, &dpn);
        w[j] = 2.0 / (n * (n - 1.0) * pn * pn);
    }
    return MFHEX_OK;
}

int build_basis(int p, int q, int quad, Basis1D *out, std::string *err)
{
    std::memset(out, 0, sizeof(*out));
    const int P = p + 1;
    if (p < 1 || P > kMaxP) {
        if (err) *err = "order p must be in [1, 8]";
        return MFHEX_ERR_UNSUPPORTED;
    }
    if (quad == MFHEX_GAUSS && q != p + 2) {
        if (err) *err = "Gauss quadrature is built for q = p + 2 only";
        return MFHEX_ERR_UNSUPPORTED;
    }
    if (quad == MFHEX_GLL && q != p + 1) {
        if (err) *err = "Gauss-Lobatto quadrature must be collocated: q = p + 1";
        return MFHEX_ERR_ARG;
    }
    if (quad != MFHEX_GAUSS && quad != MFHEX_GLL) {
        if (err) *err = "unknown quadrature rule";
        return MFHEX_ERR_ARG;
    }
    const int Q = q;
    out->P = P;
    out->Q = Q;
    out->colloc = (quad == MFHEX_GLL);
    double wn[kMaxP];
    lobatto_rule(P, out->nodes, wn);
    if (quad == MFHEX_GAUSS) gauss_rule(Q, out->xq, out->wq);
    else lobatto_rule(Q, out->xq, out->wq);

    double lamn[kMaxP], lamq[kMaxQ], l[kMaxQ], dl[kMaxQ];
    bary_weights(out->nodes, P, lamn);
    bary_weights(out->xq, Q, lamq);
    for (int a = 0; a < Q; ++a) {
        bary_eval(out->nodes, lamn, P, out->xq[a], l, dl);
        for (int i = 0; i < P; ++i) {
            out->B[a * P + i] = l[i];
            out->Gn[a * P + i] = dl[i];
        }
        bary_eval(out->xq, lamq, Q, out->xq[a], l, dl);
        for (int b = 0; b < Q; ++b) out->D[a * Q + b] = dl[b];
    }
    return MFHEX_OK;
}

}  // namespace mfhex
