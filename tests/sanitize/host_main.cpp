// Driver for the library's host set-up code built with AddressSanitizer and
// UndefinedBehaviorSanitizer: the 1D Gauss / Gauss-Lobatto rules and the
// interpolation and derivative matrices (basis.cpp), and the tetrahedral rule
// and basis tables (tet.cpp), at every order the operators accept.  The
// device entry points of tet.cpp are linked against stubs that report
// failure (no GPU is involved; none of them is called).  Besides the
// sanitizers' checks it verifies facts the mathematics fixes: weights sum to
// the reference volume, exactness on monomials, rows of B sum to 1 and rows
// of D to 0, B reproduces x and D maps x to 1, the tetrahedral basis is a
// partition of unity.  Exit status 0 and "sanitize host: OK" on success.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2109_05072_amd/csrc/blas.h"
#include "../../paper_2109_05072_amd/csrc/mfhex_internal.h"
#include "../../paper_2109_05072_amd/csrc/op.h"
#include "../../paper_2109_05072_amd/csrc/tet.h"

// ---- stubs for what the set-up code links against but these checks never call ----
namespace mfhex {
hipError_t launch_zero(void *, size_t, hipStream_t) { return hipErrorNotSupported; }
int check_hip(mfhex_op, hipError_t e, const char *) { return e == hipSuccess ? MFHEX_OK : MFHEX_ERR_HIP; }
int fail_global(int code, const std::string &) { return code; }
namespace tet {
hipError_t launch_tet_setup(const TetSetupLaunch &) { return hipErrorNotSupported; }
hipError_t launch_tet_apply(const TetLaunch &) { return hipErrorNotSupported; }
}  // namespace tet
}  // namespace mfhex
extern "C" {
hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipMemsetAsync(void *, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNotSupported; }
}

static int fails = 0;
#define CHECK(cond, ...)                           \
    do {                                           \
        if (!(cond)) {                             \
            std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
            std::fprintf(stderr, "\n");            \
            ++fails;                               \
        }                                          \
    } while (0)

int main()
{
    using namespace mfhex;
    // 1D rules: weights sum to 2, exact to degree 2n-1 (Gauss) / 2n-3 (Lobatto)
    for (int n = 1; n <= kMaxQ + 2; ++n) {
        double x[16], w[16];
        CHECK(gauss_rule(n, x, w) == 0, "gauss_rule %d", n);
        for (int k = 0; k <= 2 * n - 1; ++k) {
            double s = 0;
            for (int i = 0; i < n; ++i) s += w[i] * std::pow(x[i], k);
            const double exact = (k % 2) ? 0.0 : 2.0 / (k + 1);
            CHECK(std::fabs(s - exact) <= 1e-13, "gauss %d degree %d: %.17g", n, k, s);
        }
        if (n >= 2) {
            CHECK(lobatto_rule(n, x, w) == 0, "lobatto_rule %d", n);
            for (int k = 0; k <= 2 * n - 3; ++k) {
                double s = 0;
                for (int i = 0; i < n; ++i) s += w[i] * std::pow(x[i], k);
                const double exact = (k % 2) ? 0.0 : 2.0 / (k + 1);
                CHECK(std::fabs(s - exact) <= 1e-13, "lobatto %d degree %d: %.17g", n, k, s);
            }
        }
    }
    // operator bases: B rows sum to 1, D rows to 0, B x_nodes = x_points, D x_points = 1
    for (int p = 1; p <= 8; ++p) {
        for (int quad = MFHEX_GAUSS; quad <= MFHEX_GLL; ++quad) {
            const int q = quad == MFHEX_GAUSS ? p + 2 : p + 1;
            Basis1D b;
            std::string err;
            CHECK(build_basis(p, q, quad, &b, &err) == 0, "build_basis p=%d quad=%d: %s", p, quad, err.c_str());
            const int P = b.P, Q = b.Q;
            for (int a = 0; a < Q; ++a) {
                double sb = 0, sx = 0, sd = 0, sdx = 0;
                for (int i = 0; i < P; ++i) {
                    sb += b.B[a * P + i];
                    sx += b.B[a * P + i] * b.nodes[i];
                }
                for (int c = 0; c < Q; ++c) {
                    sd += b.D[a * Q + c];
                    sdx += b.D[a * Q + c] * b.xq[c];
                }
                CHECK(std::fabs(sb - 1) <= 1e-13 && std::fabs(sx - b.xq[a]) <= 1e-13, "B p=%d quad=%d row %d", p, quad, a);
                CHECK(std::fabs(sd) <= 1e-11 && std::fabs(sdx - 1) <= 1e-11, "D p=%d quad=%d row %d", p, quad, a);
            }
        }
        std::string err;
        Basis1D bad;
        CHECK(build_basis(p, p + 3, MFHEX_GLL, &bad, &err) != 0, "GLL with q != p+1 accepted at p=%d", p);
    }
    // tetrahedral rule and basis: weights sum to 1/6, partition of unity, gradients sum to 0
    for (int p = 1; p <= tet::kMaxP; ++p) {
        for (int q = p; q <= p + 1; ++q) {
            const int P = tet::n_basis(p), Q3 = q * q * q;
            std::vector<double> xi(3 * Q3), w(Q3), B((size_t)Q3 * P), G(3 * (size_t)Q3 * P);
            CHECK(mfhex_tet_basis(p, q, xi.data(), w.data(), B.data(), G.data()) == MFHEX_OK, "tet_basis %d %d", p, q);
            double sw = 0;
            for (int k = 0; k < Q3; ++k) {
                sw += w[k];
                CHECK(xi[3 * k] >= 0 && xi[3 * k + 1] >= 0 && xi[3 * k + 2] >= 0 &&
                          xi[3 * k] + xi[3 * k + 1] + xi[3 * k + 2] <= 1 + 1e-14,
                      "tet point %d outside p=%d q=%d", k, p, q);
                double sb = 0, sg[3] = {0, 0, 0};
                for (int n = 0; n < P; ++n) {
                    sb += B[(size_t)k * P + n];
                    for (int d = 0; d < 3; ++d) sg[d] += G[((size_t)d * Q3 + k) * P + n];
                }
                CHECK(std::fabs(sb - 1) <= 1e-12, "tet partition of unity p=%d q=%d pt %d", p, q, k);
                for (int d = 0; d < 3; ++d) CHECK(std::fabs(sg[d]) <= 1e-10, "tet gradient sum p=%d q=%d", p, q);
            }
            CHECK(std::fabs(sw - 1.0 / 6.0) <= 1e-14, "tet weights p=%d q=%d: %.17g", p, q, sw);
        }
        CHECK(mfhex_tet_basis(p, tet::kMaxP + 3, nullptr, nullptr, nullptr, nullptr) != MFHEX_OK, "tet q > 8 accepted");
    }
    std::vector<double> vert(3 * 27, 0.0);
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                double *v = &vert[3 * (i + 3 * (j + 3 * k))];
                v[0] = i / 2.0, v[1] = j / 2.0, v[2] = k / 2.0;
            }
    mfhex_tet_desc d{2, 2, 2, 3, 3, 1, vert.data()};
    mfhex_tet_sizes sz{};
    CHECK(mfhex_tet_query(&d, &sz) == MFHEX_OK && sz.n_nodes == 7 * 7 * 7 && sz.n_elem == 48, "tet_query");
    if (fails) {
        std::fprintf(stderr, "sanitize host: %d failures\n", fails);
        return 1;
    }
    std::printf("sanitize host: OK\n");
    return 0;
}
