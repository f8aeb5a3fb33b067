/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the matrix-free hexahedral
 * continuous-Galerkin operators (mass and diffusion) and the CG solve on them.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * source with the GPU library: it has its own Legendre recurrences, its own
 * Lagrange polynomials (product formula), its own trilinear geometry and NO
 * sum factorization -- every element operator is evaluated from dense
 * tabulations of the tensor basis, i.e. straight from the definition
 *
 *     y = M ( sum_e R_e^T A^e R_e ) M x,     A^e = Dhat^T G^e Dhat,
 *
 * (Sec. 2, the operator-level form A_L = block-diag(A^e) with A^e = D^T G^e D
 * and six symmetric geometric factors G_rr ... G_tt), where R_e is the element
 * restriction and M the Dirichlet mask.  The basis is the tensor Lagrange
 * basis Q_p on Gauss-Lobatto points on [-1,1]^3 (Sec. 1).
 *
 * Readings of points the paper leaves open (they are listed in the design
 * notes): Gauss-Legendre quadrature with q = p+2 points per direction for the
 * mass / stiffness problems, Gauss-Lobatto with q = p+1 (collocated with the
 * nodes) for the collocated stiffness problem; a trilinear element map from
 * the 8 vertices of each hexahedron; homogeneous Dirichlet on all six faces
 * applied as M A M; lexicographic numbering, x fastest.
 *
 * Floating point: compiled with -O2 -ffp-contract=off, never -ffast-math.
 * Results are deterministic and independent of the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_MEM (-2)
#define ORC_ERR_BREAKDOWN (-3)
#define ORC_ERR_NOCONV (-4)

#define ORC_GAUSS 0
#define ORC_GLL 1
#define ORC_MASS 1
#define ORC_DIFFUSION 2

typedef struct {
    int32_t nex, ney, nez; /* elements per direction                        */
    int32_t p;             /* polynomial order, nodes per direction P = p+1  */
    int32_t q;             /* quadrature points per direction               */
    int32_t quad;          /* ORC_GAUSS or ORC_GLL                           */
    int32_t kind;          /* ORC_MASS or ORC_DIFFUSION                      */
    int32_t dirichlet;     /* 1: homogeneous Dirichlet on all faces          */
    const double *vert;    /* [(nex+1)(ney+1)(nez+1)][3], x fastest          */
    const double *kappa;   /* NULL or [E][q^3] per-point diffusion coeff.    */
} orc_prob;

/* ------------------------------------------------------------------------- */
/* 1D: Legendre polynomials, Gauss and Gauss-Lobatto rules, Lagrange basis   */
/* ------------------------------------------------------------------------- */

/* P_n(x) by the Bonnet three-term recurrence; also returns P_{n-1}(x). */
static void legendre_pair(int n, double x, double *pn, double *pnm1)
{
    double a = 1.0, b = x; /* P_0, P_1 */
    if (n == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
        a = b;
        b = c;
    }
    *pn = b;
    *pnm1 = a;
}

/* Gauss-Legendre: the q roots of P_q, ascending; w = 2 / ((1-x^2) P_q'(x)^2). */
int orc_gauss(int q, double *x, double *w)
{
    if (q < 1 || q > 64) return ORC_ERR_ARG;
    for (int j = 0; j < q; ++j) {
        double t = -cos(M_PI * (j + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pn, pm;
            legendre_pair(q, t, &pn, &pm);
            dp = q * (pm - t * pn) / (1.0 - t * t); /* (1-x^2)P' = n(P_{n-1} - x P_n) */
            double dt = pn / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double pn, pm;
        legendre_pair(q, t, &pn, &pm);
        dp = q * (pm - t * pn) / (1.0 - t * t);
        x[j] = t;
        w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    return ORC_OK;
}

/* Gauss-Lobatto-Legendre: -1, the p-1 roots of P_p', +1 (the roots of
 * (1-x^2) P_p'); w = 2 / (p (p+1) P_p(x)^2).  Newton on f = (1-x^2) P_p',
 * whose derivative is -p(p+1) P_p by the Legendre differential equation. */
int orc_gll(int p, double *x, double *w)
{
    if (p < 1 || p > 64) return ORC_ERR_ARG;
    x[0] = -1.0;
    x[p] = 1.0;
    for (int j = 1; j < p; ++j) {
        double t = -cos(M_PI * j / p);
        for (int it = 0; it < 100; ++it) {
            double pn, pm;
            legendre_pair(p, t, &pn, &pm);
            double f = p * (pm - t * pn);          /* (1-t^2) P_p'(t) */
            double dt = f / (-p * (p + 1.0) * pn); /* f / f'          */
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[j] = t;
    }
    for (int j = 0; j <= p; ++j) {
        double pn, pm;
        legendre_pair(p, x[j], &pn, &pm);
        w[j] = 2.0 / (p * (p + 1.0) * pn * pn);
    }
    return ORC_OK;
}

/* Lagrange basis on nodes xi[0..P-1] evaluated at points xq[0..Q-1] by the
 * product formula: B[k][j] = l_j(xq_k), G[k][j] = l_j'(xq_k). */
void orc_lagrange(int P, const double *xi, int Q, const double *xq, double *B, double *G)
{
    for (int k = 0; k < Q; ++k) {
        double x = xq[k];
        for (int j = 0; j < P; ++j) {
            double v = 1.0;
            for (int m = 0; m < P; ++m)
                if (m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
            double d = 0.0;
            for (int l = 0; l < P; ++l) {
                if (l == j) continue;
                double t = 1.0 / (xi[j] - xi[l]);
                for (int m = 0; m < P; ++m)
                    if (m != j && m != l) t *= (x - xi[m]) / (xi[j] - xi[m]);
                d += t;
            }
            B[k * P + j] = v;
            G[k * P + j] = d;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Dense tensor tabulation (no sum factorization)                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int P, Q, P3, Q3;
    double *xq, *wq;    /* 1D quadrature (Q)                               */
    double *w3;         /* tensor weights (Q3)                              */
    double *phi;        /* [Q3][P3]  phi_n(xi_pt)                           */
    double *dphi;       /* [3][Q3][P3] reference gradient of phi_n at pt    */
    double *rq;         /* [Q3][3] reference coordinates of the points      */
} orc_tab;

static void tab_free(orc_tab *t)
{
    free(t->xq); free(t->wq); free(t->w3); free(t->phi); free(t->dphi); free(t->rq);
    memset(t, 0, sizeof(*t));
}

static int tab_build(const orc_prob *pr, orc_tab *t)
{
    memset(t, 0, sizeof(*t));
    int P = pr->p + 1, Q = pr->q;
    t->P = P; t->Q = Q; t->P3 = P * P * P; t->Q3 = Q * Q * Q;
    double xi[65], wi[65];
    double *B = malloc(sizeof(double) * Q * P), *G = malloc(sizeof(double) * Q * P);
    t->xq = malloc(sizeof(double) * Q);
    t->wq = malloc(sizeof(double) * Q);
    t->w3 = malloc(sizeof(double) * t->Q3);
    t->phi = malloc(sizeof(double) * (size_t)t->Q3 * t->P3);
    t->dphi = malloc(sizeof(double) * 3 * (size_t)t->Q3 * t->P3);
    t->rq = malloc(sizeof(double) * 3 * t->Q3);
    if (!B || !G || !t->xq || !t->wq || !t->w3 || !t->phi || !t->dphi || !t->rq) {
        free(B); free(G); tab_free(t); return ORC_ERR_MEM;
    }
    orc_gll(pr->p, xi, wi); /* nodes: Gauss-Lobatto points (Sec. 1) */
    if (pr->quad == ORC_GAUSS) orc_gauss(Q, t->xq, t->wq);
    else orc_gll(Q - 1, t->xq, t->wq);
    orc_lagrange(P, xi, Q, t->xq, B, G);
    for (int c = 0; c < Q; ++c)
        for (int b = 0; b < Q; ++b)
            for (int a = 0; a < Q; ++a) {
                int pt = a + Q * (b + Q * c);
                t->w3[pt] = t->wq[a] * t->wq[b] * t->wq[c];
                t->rq[3 * pt + 0] = t->xq[a];
                t->rq[3 * pt + 1] = t->xq[b];
                t->rq[3 * pt + 2] = t->xq[c];
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j)
                        for (int i = 0; i < P; ++i) {
                            int n = i + P * (j + P * k);
                            size_t o = (size_t)pt * t->P3 + n;
                            t->phi[o] = B[a * P + i] * B[b * P + j] * B[c * P + k];
                            t->dphi[o] = G[a * P + i] * B[b * P + j] * B[c * P + k];
                            t->dphi[(size_t)t->Q3 * t->P3 + o] = B[a * P + i] * G[b * P + j] * B[c * P + k];
                            t->dphi[2 * (size_t)t->Q3 * t->P3 + o] = B[a * P + i] * B[b * P + j] * G[c * P + k];
                        }
            }
    free(B); free(G);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Mesh: numbering, restriction, trilinear geometry                          */
/* ------------------------------------------------------------------------- */

static int64_t n_nodes(const orc_prob *pr)
{
    return (int64_t)(pr->p * pr->nex + 1) * (pr->p * pr->ney + 1) * (pr->p * pr->nez + 1);
}

/* Global node ids of element e's P^3 nodes (local order i + P(j + P k)); a
 * masked (Dirichlet boundary) node is returned as -1 when mask != 0. */
static void elem_nodes(const orc_prob *pr, int64_t e, int mask, int64_t *gid)
{
    int p = pr->p, P = p + 1;
    int64_t ex = e % pr->nex, ey = (e / pr->nex) % pr->ney, ez = e / ((int64_t)pr->nex * pr->ney);
    int64_t nx = (int64_t)p * pr->nex + 1, ny = (int64_t)p * pr->ney + 1;
    int64_t lx = nx - 1, ly = ny - 1, lz = (int64_t)p * pr->nez;
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                int64_t I = p * ex + i, J = p * ey + j, K = p * ez + k;
                int64_t g = I + nx * (J + ny * K);
                int bnd = (I == 0 || I == lx || J == 0 || J == ly || K == 0 || K == lz);
                gid[i + P * (j + P * k)] = (mask && bnd) ? -1 : g;
            }
}

/* The 8 vertex coordinates of element e, ordered dx + 2 dy + 4 dz. */
static void elem_vertices(const orc_prob *pr, int64_t e, double X[8][3])
{
    int64_t ex = e % pr->nex, ey = (e / pr->nex) % pr->ney, ez = e / ((int64_t)pr->nex * pr->ney);
    int64_t vx = pr->nex + 1, vy = pr->ney + 1;
    for (int v = 0; v < 8; ++v) {
        int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
        int64_t id = (ex + dx) + vx * ((ey + dy) + vy * (ez + dz));
        for (int d = 0; d < 3; ++d) X[v][d] = pr->vert[3 * id + d];
    }
}

/* Trilinear map at reference point r: physical position x and Jacobian
 * J[i][j] = d x_i / d r_j. */
static void trilinear(double X[8][3], const double r[3], double x[3], double J[3][3])
{
    for (int i = 0; i < 3; ++i) {
        x[i] = 0.0;
        for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
    }
    for (int v = 0; v < 8; ++v) {
        double s[3], h[3];
        for (int d = 0; d < 3; ++d) {
            s[d] = ((v >> d) & 1) ? 1.0 : -1.0;
            h[d] = 0.5 * (1.0 + s[d] * r[d]);
        }
        double N = h[0] * h[1] * h[2];
        double dN[3] = {0.5 * s[0] * h[1] * h[2], 0.5 * s[1] * h[0] * h[2], 0.5 * s[2] * h[0] * h[1]};
        for (int i = 0; i < 3; ++i) {
            x[i] += N * X[v][i];
            for (int j = 0; j < 3; ++j) J[i][j] += dN[j] * X[v][i];
        }
    }
}

/* Adjugate (transposed cofactor matrix) and determinant. */
static double adjugate(double J[3][3], double A[3][3])
{
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
}

/* Pointwise data of element e at tabulated point pt: w*detJ (mass) and the
 * symmetric diffusion tensor D = w adj(J) adj(J)^T / detJ (Sec. 2: the
 * geometric factors G^e); kappa is NOT included.  Returns detJ. */
static double point_data(const orc_tab *t, double X[8][3], int pt, double *wdet, double D[3][3])
{
    double x[3], J[3][3], A[3][3];
    trilinear(X, &t->rq[3 * pt], x, J);
    double det = adjugate(J, A);
    double w = t->w3[pt];
    *wdet = w * det;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * A[j][k];
            D[i][j] = w * s / det;
        }
    return det;
}

static int check_prob(const orc_prob *pr)
{
    if (!pr || !pr->vert) return ORC_ERR_ARG;
    if (pr->nex < 1 || pr->ney < 1 || pr->nez < 1) return ORC_ERR_ARG;
    if (pr->p < 1 || pr->p > 16 || pr->q < 1 || pr->q > 24) return ORC_ERR_ARG;
    if (pr->quad != ORC_GAUSS && pr->quad != ORC_GLL) return ORC_ERR_ARG;
    if (pr->quad == ORC_GLL && pr->q < 2) return ORC_ERR_ARG;
    if (pr->kind != ORC_MASS && pr->kind != ORC_DIFFUSION) return ORC_ERR_ARG;
    return ORC_OK;
}

int64_t orc_num_nodes(const orc_prob *pr) { return check_prob(pr) ? -1 : n_nodes(pr); }

/* ------------------------------------------------------------------------- */
/* Element-level dense operators                                             */
/* ------------------------------------------------------------------------- */

/* y_e = A^e u_e for one element with the dense tabulation; u_e, y_e are P^3
 * long, y_e is overwritten.  kappa_e may be NULL (kappa = 1). */
static void elem_apply(const orc_prob *pr, const orc_tab *t, double X[8][3], const double *kappa_e,
                       const double *ue, double *ye)
{
    const int P3 = t->P3, Q3 = t->Q3;
    const size_t S = (size_t)Q3 * P3;
    for (int n = 0; n < P3; ++n) ye[n] = 0.0;
    for (int pt = 0; pt < Q3; ++pt) {
        double wdet, D[3][3];
        point_data(t, X, pt, &wdet, D);
        double kap = kappa_e ? kappa_e[pt] : 1.0;
        if (pr->kind == ORC_MASS) {
            const double *ph = &t->phi[(size_t)pt * P3];
            double u = 0.0;
            for (int n = 0; n < P3; ++n) u += ph[n] * ue[n];
            double v = wdet * u;
            for (int n = 0; n < P3; ++n) ye[n] += ph[n] * v;
        } else {
            const double *g0 = &t->dphi[(size_t)pt * P3];
            const double *g1 = g0 + S, *g2 = g0 + 2 * S;
            double gu[3] = {0.0, 0.0, 0.0};
            for (int n = 0; n < P3; ++n) {
                gu[0] += g0[n] * ue[n];
                gu[1] += g1[n] * ue[n];
                gu[2] += g2[n] * ue[n];
            }
            double v[3];
            for (int i = 0; i < 3; ++i)
                v[i] = kap * (D[i][0] * gu[0] + D[i][1] * gu[1] + D[i][2] * gu[2]);
            for (int n = 0; n < P3; ++n) ye[n] += g0[n] * v[0] + g1[n] * v[1] + g2[n] * v[2];
        }
    }
}

/* Dense element matrix A^e (P^3 x P^3, row-major), no mask.  kappa from the
 * problem when present. */
int orc_element_matrix(const orc_prob *pr, int64_t e, double *Ae)
{
    if (check_prob(pr)) return ORC_ERR_ARG;
    int64_t E = (int64_t)pr->nex * pr->ney * pr->nez;
    if (e < 0 || e >= E) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    const int P3 = t.P3, Q3 = t.Q3;
    const size_t S = (size_t)Q3 * P3;
    double X[8][3];
    elem_vertices(pr, e, X);
    memset(Ae, 0, sizeof(double) * (size_t)P3 * P3);
    for (int pt = 0; pt < Q3; ++pt) {
        double wdet, D[3][3];
        point_data(&t, X, pt, &wdet, D);
        double kap = pr->kappa ? pr->kappa[e * Q3 + pt] : 1.0;
        for (int n = 0; n < P3; ++n)
            for (int m = 0; m < P3; ++m) {
                size_t on = (size_t)pt * P3 + n, om = (size_t)pt * P3 + m;
                double s;
                if (pr->kind == ORC_MASS) {
                    s = t.phi[on] * wdet * t.phi[om];
                } else {
                    s = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            s += t.dphi[a * S + on] * kap * D[a][b] * t.dphi[b * S + om];
                }
                Ae[(size_t)n * P3 + m] += s;
            }
    }
    tab_free(&t);
    return ORC_OK;
}

/* Global node ids of element e (length P^3); -1 for masked nodes when the
 * problem is Dirichlet.  Lets the test harness assemble sparse matrices. */
int orc_element_nodes(const orc_prob *pr, int64_t e, int64_t *gid)
{
    if (check_prob(pr)) return ORC_ERR_ARG;
    elem_nodes(pr, e, pr->dirichlet, gid);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Global matrix-free apply  y = M (sum_e R_e^T A^e R_e) M x                 */
/* ------------------------------------------------------------------------- */

/* x, y: [N][nvec] row-major; the operator acts on each of the nvec columns
 * independently.  Elements are processed in z-layers: all even layers in
 * parallel, then all odd layers (layers of one parity share no node), each
 * layer sequentially in element order, so the summation order at every node
 * is fixed and independent of the thread count. */
int orc_apply(const orc_prob *pr, int nvec, const double *x, double *y, int nthreads)
{
    if (check_prob(pr) || nvec < 1 || !x || !y) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    const int64_t N = n_nodes(pr);
    const int P3 = t.P3, Q3 = t.Q3;
    memset(y, 0, sizeof(double) * (size_t)N * nvec);
    int err = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel
        {
            int64_t *gid = malloc(sizeof(int64_t) * P3);
            double *ue = malloc(sizeof(double) * P3), *ye = malloc(sizeof(double) * P3);
            if (!gid || !ue || !ye) {
#pragma omp atomic write
                err = ORC_ERR_MEM;
            } else {
#pragma omp for schedule(dynamic, 1)
                for (int ez = parity; ez < pr->nez; ez += 2) {
                    for (int64_t el = 0; el < (int64_t)pr->nex * pr->ney; ++el) {
                        int64_t e = el + (int64_t)pr->nex * pr->ney * ez;
                        double X[8][3];
                        elem_vertices(pr, e, X);
                        elem_nodes(pr, e, pr->dirichlet, gid);
                        const double *ke = pr->kappa ? pr->kappa + e * Q3 : NULL;
                        for (int v = 0; v < nvec; ++v) {
                            for (int n = 0; n < P3; ++n) ue[n] = gid[n] < 0 ? 0.0 : x[gid[n] * nvec + v];
                            elem_apply(pr, &t, X, ke, ue, ye);
                            for (int n = 0; n < P3; ++n)
                                if (gid[n] >= 0) y[gid[n] * nvec + v] += ye[n];
                        }
                    }
                }
            }
            free(gid); free(ue); free(ye);
        }
    }
    tab_free(&t);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Setup-type outputs used to build inputs and checks                        */
/* ------------------------------------------------------------------------- */

/* Physical coordinates [E][Q^3][3] and detJ [E][Q^3] of every quadrature
 * point (either output may be NULL). */
int orc_qpoint_geometry(const orc_prob *pr, double *xyz, double *detj)
{
    if (check_prob(pr)) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    int64_t E = (int64_t)pr->nex * pr->ney * pr->nez;
    for (int64_t e = 0; e < E; ++e) {
        double X[8][3];
        elem_vertices(pr, e, X);
        for (int pt = 0; pt < t.Q3; ++pt) {
            double x[3], J[3][3], A[3][3];
            trilinear(X, &t.rq[3 * pt], x, J);
            double det = adjugate(J, A);
            if (xyz) for (int d = 0; d < 3; ++d) xyz[(e * t.Q3 + pt) * 3 + d] = x[d];
            if (detj) detj[e * t.Q3 + pt] = det;
        }
    }
    tab_free(&t);
    return ORC_OK;
}

/* Physical coordinates [N][3] of the global nodes (Gauss-Lobatto points
 * pushed through the trilinear map of the lowest-numbered owning element). */
int orc_node_coords(const orc_prob *pr, double *xyz)
{
    if (check_prob(pr)) return ORC_ERR_ARG;
    int p = pr->p, P = p + 1;
    double xi[65], wi[65];
    orc_gll(p, xi, wi);
    int64_t nx = (int64_t)p * pr->nex + 1, ny = (int64_t)p * pr->ney + 1, nz = (int64_t)p * pr->nez + 1;
    for (int64_t K = 0; K < nz; ++K)
        for (int64_t J = 0; J < ny; ++J)
            for (int64_t I = 0; I < nx; ++I) {
                int64_t ex = I / p, ey = J / p, ez = K / p;
                if (ex == pr->nex) ex--;
                if (ey == pr->ney) ey--;
                if (ez == pr->nez) ez--;
                int i = (int)(I - p * ex), j = (int)(J - p * ey), k = (int)(K - p * ez);
                double X[8][3], r[3] = {xi[i], xi[j], xi[k]}, x[3], Jm[3][3];
                elem_vertices(pr, ex + pr->nex * (ey + pr->ney * ez), X);
                trilinear(X, r, x, Jm);
                int64_t g = I + nx * (J + ny * K);
                for (int d = 0; d < 3; ++d) xyz[3 * g + d] = x[d];
            }
    (void)P;
    return ORC_OK;
}

/* Load vector b_n = sum_e sum_pt w detJ f(pt) phi_n(pt), masked when the
 * problem is Dirichlet.  f is given per quadrature point, [E][Q^3]. */
int orc_rhs(const orc_prob *pr, const double *fq, double *b)
{
    if (check_prob(pr)) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    const int64_t N = n_nodes(pr), E = (int64_t)pr->nex * pr->ney * pr->nez;
    const int P3 = t.P3, Q3 = t.Q3;
    int64_t *gid = malloc(sizeof(int64_t) * P3);
    memset(b, 0, sizeof(double) * N);
    for (int64_t e = 0; e < E; ++e) {
        double X[8][3];
        elem_vertices(pr, e, X);
        elem_nodes(pr, e, pr->dirichlet, gid);
        for (int pt = 0; pt < Q3; ++pt) {
            double wdet, D[3][3];
            point_data(&t, X, pt, &wdet, D);
            double v = wdet * fq[e * Q3 + pt];
            for (int n = 0; n < P3; ++n)
                if (gid[n] >= 0) b[gid[n]] += t.phi[(size_t)pt * P3 + n] * v;
        }
    }
    free(gid);
    tab_free(&t);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Gradient of a misfit with respect to the per-point coefficient kappa      */
/* ------------------------------------------------------------------------- */

/* For y = M A(kappa) M u, the derivative of r^T y with respect to kappa at
 * point pt of element e is (Dhat M r)_pt^T D_pt (Dhat M u)_pt, with D the
 * kappa-free diffusion tensor.  g: [E][Q^3]. */
int orc_kappa_grad(const orc_prob *pr, const double *u, const double *r, double *g)
{
    if (check_prob(pr) || pr->kind != ORC_DIFFUSION) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    const int64_t E = (int64_t)pr->nex * pr->ney * pr->nez;
    const int P3 = t.P3, Q3 = t.Q3;
    const size_t S = (size_t)Q3 * P3;
    int64_t *gid = malloc(sizeof(int64_t) * P3);
    double *ue = malloc(sizeof(double) * P3), *re = malloc(sizeof(double) * P3);
    for (int64_t e = 0; e < E; ++e) {
        double X[8][3];
        elem_vertices(pr, e, X);
        elem_nodes(pr, e, pr->dirichlet, gid);
        for (int n = 0; n < P3; ++n) {
            ue[n] = gid[n] < 0 ? 0.0 : u[gid[n]];
            re[n] = gid[n] < 0 ? 0.0 : r[gid[n]];
        }
        for (int pt = 0; pt < Q3; ++pt) {
            double wdet, D[3][3];
            point_data(&t, X, pt, &wdet, D);
            double gu[3] = {0, 0, 0}, gr[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a) {
                const double *ga = &t.dphi[a * S + (size_t)pt * P3];
                for (int n = 0; n < P3; ++n) {
                    gu[a] += ga[n] * ue[n];
                    gr[a] += ga[n] * re[n];
                }
            }
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += gr[a] * D[a][b] * gu[b];
            g[e * Q3 + pt] = s;
        }
    }
    free(gid); free(ue); free(re);
    tab_free(&t);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Unpreconditioned conjugate gradients (Hestenes-Stiefel), x0 = 0           */
/* ------------------------------------------------------------------------- */

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Runs until ||r_k|| <= rtol ||b|| or maxit iterations.  rhist (length
 * maxit+1, may be NULL) receives ||r_k||_2 for k = 0.. iterations done.
 * *iters gets the number of iterations performed. */
int orc_cg(const orc_prob *pr, const double *b, double *x, int maxit, double rtol, double *rhist,
           int *iters, int nthreads)
{
    if (check_prob(pr) || maxit < 0) return ORC_ERR_ARG;
    const int64_t N = n_nodes(pr);
    double *r = malloc(sizeof(double) * N), *p = malloc(sizeof(double) * N), *Ap = malloc(sizeof(double) * N);
    if (!r || !p || !Ap) { free(r); free(p); free(Ap); return ORC_ERR_MEM; }
    for (int64_t i = 0; i < N; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double rr = dot(N, r, r), bn = sqrt(rr);
    if (rhist) rhist[0] = bn;
    int k = 0, status = ORC_OK;
    if (bn == 0.0) { *iters = 0; free(r); free(p); free(Ap); return ORC_OK; }
    status = ORC_ERR_NOCONV;
    while (k < maxit) {
        int e = orc_apply(pr, 1, p, Ap, nthreads);
        if (e) { status = e; break; }
        double pAp = dot(N, p, Ap);
        if (!(pAp > 0.0)) { status = ORC_ERR_BREAKDOWN; break; }
        double alpha = rr / pAp;
        for (int64_t i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = dot(N, r, r);
        ++k;
        if (rhist) rhist[k] = sqrt(rr_new);
        if (sqrt(rr_new) <= rtol * bn) { status = ORC_OK; break; }
        double beta = rr_new / rr;
        for (int64_t i = 0; i < N; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    *iters = k;
    free(r); free(p); free(Ap);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Operator diagonal and Jacobi-preconditioned CG                            */
/* ------------------------------------------------------------------------- */

/* d = diag( M (sum_e R_e^T A^e R_e) M ): every element adds the diagonal of
 * its element matrix at its nodes, masked nodes stay 0.  The element
 * diagonal comes straight from the dense tabulation:
 *     (A^e)_nn = sum_pt kappa dphi_n(pt)^T D(pt) dphi_n(pt)   (diffusion),
 *     (A^e)_nn = sum_pt w detJ phi_n(pt)^2                     (mass).
 * Elements are visited in order, so the sums are deterministic. */
int orc_diagonal(const orc_prob *pr, double *d)
{
    if (check_prob(pr) || !d) return ORC_ERR_ARG;
    orc_tab t;
    if (tab_build(pr, &t)) return ORC_ERR_MEM;
    const int P3 = t.P3, Q3 = t.Q3;
    const size_t S = (size_t)Q3 * P3;
    const int64_t N = n_nodes(pr), E = (int64_t)pr->nex * pr->ney * pr->nez;
    int64_t *gid = malloc(sizeof(int64_t) * P3);
    double *de = malloc(sizeof(double) * P3);
    if (!gid || !de) { free(gid); free(de); tab_free(&t); return ORC_ERR_MEM; }
    for (int64_t i = 0; i < N; ++i) d[i] = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        double X[8][3];
        elem_vertices(pr, e, X);
        elem_nodes(pr, e, pr->dirichlet, gid);
        for (int n = 0; n < P3; ++n) de[n] = 0.0;
        for (int pt = 0; pt < Q3; ++pt) {
            double wdet, D[3][3];
            point_data(&t, X, pt, &wdet, D);
            double kap = pr->kappa ? pr->kappa[e * Q3 + pt] : 1.0;
            for (int n = 0; n < P3; ++n) {
                size_t on = (size_t)pt * P3 + n;
                if (pr->kind == ORC_MASS) {
                    de[n] += wdet * t.phi[on] * t.phi[on];
                } else {
                    double g[3] = {t.dphi[on], t.dphi[S + on], t.dphi[2 * S + on]};
                    double s = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) s += g[a] * D[a][b] * g[b];
                    de[n] += kap * s;
                }
            }
        }
        for (int n = 0; n < P3; ++n)
            if (gid[n] >= 0) d[gid[n]] += de[n];
    }
    free(gid); free(de); tab_free(&t);
    return ORC_OK;
}

/* Jacobi-preconditioned CG in textbook form, x0 = 0:
 *     z = Dinv r,  alpha = r.z / p.Ap,  x += alpha p,  r -= alpha Ap,
 *     z = Dinv r,  beta = (r.z)_new / (r.z)_old,  p = z + beta p,
 * stopping on the unpreconditioned residual ||r|| <= rtol ||b|| exactly like
 * orc_cg; rhist[k] = ||r_k||.  dinv: inverse of the operator diagonal (0 at
 * masked nodes).  Sec. 1 pairs CG with preconditioners on top of
 * sum-factorized operator evaluation; Jacobi (diagonal) scaling is the
 * smoother the Nek5000/RS solvers of Sec. 2 accelerate with Chebyshev. */
int orc_pcg(const orc_prob *pr, const double *b, const double *dinv, double *x, int maxit, double rtol,
            double *rhist, int *iters, int nthreads)
{
    if (check_prob(pr) || maxit < 0 || !dinv) return ORC_ERR_ARG;
    const int64_t N = n_nodes(pr);
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *Ap = malloc(sizeof(double) * N);
    if (!r || !z || !p || !Ap) { free(r); free(z); free(p); free(Ap); return ORC_ERR_MEM; }
    for (int64_t i = 0; i < N; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double rz = dot(N, r, z), bn = sqrt(dot(N, r, r));
    if (rhist) rhist[0] = bn;
    int k = 0, status = ORC_OK;
    if (bn == 0.0) { *iters = 0; free(r); free(z); free(p); free(Ap); return ORC_OK; }
    status = ORC_ERR_NOCONV;
    while (k < maxit) {
        int e = orc_apply(pr, 1, p, Ap, nthreads);
        if (e) { status = e; break; }
        double pAp = dot(N, p, Ap);
        if (!(pAp > 0.0)) { status = ORC_ERR_BREAKDOWN; break; }
        double alpha = rz / pAp;
        for (int64_t i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rn = sqrt(dot(N, r, r));
        ++k;
        if (rhist) rhist[k] = rn;
        if (rn <= rtol * bn) { status = ORC_OK; break; }
        for (int64_t i = 0; i < N; ++i) z[i] = dinv[i] * r[i];
        double rz_new = dot(N, r, z);
        double beta = rz_new / rz;
        for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    *iters = k;
    free(r); free(z); free(p); free(Ap);
    return status;
}
