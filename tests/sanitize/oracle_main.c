/* Driver that runs every entry point of the FP64 oracle on tiny perturbed
 * meshes, built with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: the oracle is compiled into this program as one unit).
 * Besides the sanitizers' own checks it verifies a few facts the method fixes,
 * so that a run that silently skipped work would fail:
 *   mass: 1^T M 1 = volume of the unit cube;
 *   diffusion: A applied to an affine field vanishes at interior nodes;
 *   symmetry u.Av = v.Au; CG reaches its tolerance; the diagonal is positive
 *   at interior nodes; the load vector of f = 1 sums to the volume.
 * Exit status 0 and "sanitize oracle: OK" on success. */
#include "../../oracle/oracle.c"

#include <stdio.h>

static uint64_t lcg = 2109u;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "FAIL: " __VA_ARGS__);         \
            fprintf(stderr, "\n");                         \
            ++fails;                                       \
        }                                                  \
    } while (0)

int main(void)
{
    const int nex = 2, ney = 2, nez = 1;
    const int nv = (nex + 1) * (ney + 1) * (nez + 1);
    double vert[(2 + 1) * (2 + 1) * (1 + 1) * 3];
    for (int k = 0; k <= nez; ++k)
        for (int j = 0; j <= ney; ++j)
            for (int i = 0; i <= nex; ++i) {
                double *v = vert + 3 * (i + (nex + 1) * (j + (ney + 1) * k));
                v[0] = (double)i / nex;
                v[1] = (double)j / ney;
                v[2] = (double)k / nez;
                if (i > 0 && i < nex && j > 0 && j < ney) { /* interior in x, y: perturb */
                    v[0] += (urand() - 0.5) * 0.2 / nex;
                    v[1] += (urand() - 0.5) * 0.2 / ney;
                }
            }
    (void)nv;
    for (int p = 1; p <= 4; ++p) {
        for (int kind = ORC_MASS; kind <= ORC_DIFFUSION; ++kind) {
            for (int quad = ORC_GAUSS; quad <= ORC_GLL; ++quad) {
                if (kind == ORC_MASS && quad == ORC_GLL) continue;
                const int q = quad == ORC_GAUSS ? p + 2 : p + 1;
                for (int dir = 0; dir <= 1; ++dir) {
                    if (kind == ORC_MASS && dir) continue;
                    orc_prob pr = {nex, ney, nez, p, q, quad, kind, dir, vert, NULL};
                    const int64_t n = n_nodes(&pr), E = (int64_t)nex * ney * nez;
                    const int Q3 = q * q * q, P = p + 1;
                    double *x = calloc(n, 8), *y = calloc(n, 8), *u = calloc(n, 8), *v = calloc(n, 8);
                    double *Au = calloc(n, 8), *Av = calloc(n, 8), *xyz = calloc(3 * n, 8), *d = calloc(n, 8);
                    double *qx = calloc(3 * E * Q3, 8), *dj = calloc(E * Q3, 8), *fq = calloc(E * Q3, 8);
                    double *g = calloc(E * Q3, 8), *Ae = calloc((size_t)P * P * P * P * P * P, 8);
                    double *hist = calloc(2001, 8), *dinv = calloc(n, 8);
                    int64_t *gid = calloc((size_t)P * P * P, 8);
                    int it = 0;
                    CHECK(orc_node_coords(&pr, xyz) == ORC_OK, "node coords");
                    CHECK(orc_qpoint_geometry(&pr, qx, dj) == ORC_OK, "qpoint geometry");
                    for (int64_t e = 0; e < E; ++e) {
                        CHECK(orc_element_matrix(&pr, e, Ae) == ORC_OK, "element matrix");
                        CHECK(orc_element_nodes(&pr, e, gid) == ORC_OK, "element nodes");
                    }
                    for (int64_t i = 0; i < n; ++i) {
                        u[i] = 2 * urand() - 1;
                        v[i] = 2 * urand() - 1;
                    }
                    CHECK(orc_apply(&pr, 1, u, Au, 1) == ORC_OK, "apply u");
                    CHECK(orc_apply(&pr, 1, v, Av, 1) == ORC_OK, "apply v");
                    double uAv = 0, vAu = 0, s = 0;
                    for (int64_t i = 0; i < n; ++i) {
                        uAv += u[i] * Av[i];
                        vAu += v[i] * Au[i];
                        s += fabs(u[i] * Av[i]);
                    }
                    CHECK(fabs(uAv - vAu) <= 1e-13 * s, "symmetry p=%d kind=%d quad=%d", p, kind, quad);
                    if (kind == ORC_MASS) {
                        for (int64_t i = 0; i < n; ++i) x[i] = 1.0;
                        CHECK(orc_apply(&pr, 1, x, y, 1) == ORC_OK, "apply 1");
                        double vol = 0;
                        for (int64_t i = 0; i < n; ++i) vol += y[i];
                        CHECK(fabs(vol - 1.0) <= 1e-13, "mass volume p=%d: %.17g", p, vol);
                        for (int64_t i = 0; i < E * Q3; ++i) fq[i] = 1.0;
                        CHECK(orc_rhs(&pr, fq, y) == ORC_OK, "rhs");
                        vol = 0;
                        for (int64_t i = 0; i < n; ++i) vol += y[i];
                        CHECK(fabs(vol - 1.0) <= 1e-13, "load vector of 1 p=%d: %.17g", p, vol);
                    } else {
                        /* affine field a + b.x: A of it vanishes at interior nodes (Gauss always; GLL p >= 2) */
                        if (!(quad == ORC_GLL && p < 2)) {
                            for (int64_t i = 0; i < n; ++i) x[i] = 0.3 + xyz[3 * i] - 2 * xyz[3 * i + 1] + 0.5 * xyz[3 * i + 2];
                            orc_prob pn = pr;
                            pn.dirichlet = 0;
                            CHECK(orc_apply(&pn, 1, x, y, 1) == ORC_OK, "apply affine");
                            const int n1 = p * nex + 1, n2 = p * ney + 1, n3 = p * nez + 1;
                            double mx = 0;
                            for (int64_t i = 0; i < n; ++i) {
                                const int ix = i % n1, iy = (i / n1) % n2, iz = i / (n1 * n2);
                                if (ix > 0 && ix < n1 - 1 && iy > 0 && iy < n2 - 1 && iz > 0 && iz < n3 - 1)
                                    mx = fmax(mx, fabs(y[i]));
                            }
                            CHECK(mx <= 1e-12, "affine nullity p=%d quad=%d: %.3g", p, quad, mx);
                        }
                        for (int64_t i = 0; i < E * Q3; ++i) g[i] = 0;
                        CHECK(orc_kappa_grad(&pr, u, v, g) == ORC_OK, "kappa grad");
                        CHECK(orc_diagonal(&pr, d) == ORC_OK, "diagonal");
                        if (dir) {
                            for (int64_t i = 0; i < n; ++i) x[i] = 2 * urand() - 1;
                            double *b = calloc(n, 8);
                            CHECK(orc_apply(&pr, 1, x, b, 1) == ORC_OK, "apply rhs");
                            int code = orc_cg(&pr, b, y, 2000, 1e-10, hist, &it, 1);
                            CHECK(code == ORC_OK, "cg p=%d quad=%d code %d after %d", p, quad, code, it);
                            for (int64_t i = 0; i < n; ++i) dinv[i] = d[i] > 0 ? 1.0 / d[i] : 0.0;
                            code = orc_pcg(&pr, b, dinv, y, 2000, 1e-10, hist, &it, 1);
                            CHECK(code == ORC_OK, "pcg p=%d quad=%d code %d after %d", p, quad, code, it);
                            free(b);
                        }
                    }
                    free(x); free(y); free(u); free(v); free(Au); free(Av); free(xyz); free(d);
                    free(qx); free(dj); free(fq); free(g); free(Ae); free(hist); free(dinv); free(gid);
                }
            }
        }
    }
    /* the 1D rules and Lagrange tables at every size the operators use */
    for (int n = 1; n <= 12; ++n) {
        double xq[16], wq[16], xi[16], wi[16], B[256], G[256];
        CHECK(orc_gauss(n, xq, wq) == ORC_OK, "gauss %d", n);
        if (n >= 2) {
            CHECK(orc_gll(n - 1, xi, wi) == ORC_OK, "gll %d", n);
            orc_lagrange(n, xi, n, xq, B, G);
        }
        double sw = 0;
        for (int i = 0; i < n; ++i) sw += wq[i];
        CHECK(fabs(sw - 2.0) <= 1e-14, "gauss weights %d", n);
    }
    if (fails) {
        fprintf(stderr, "sanitize oracle: %d failures\n", fails);
        return 1;
    }
    printf("sanitize oracle: OK\n");
    return 0;
}
