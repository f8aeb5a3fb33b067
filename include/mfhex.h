/*
 * mfhex.h -- matrix-free high-order hexahedral operators on AMD MI355X (gfx950).
 *
 * C ABI of libmfhex.so.  The library applies the continuous-Galerkin mass and
 * diffusion operators of tensor-product Q_p elements (Lagrange basis on
 * Gauss-Lobatto points, reference element [-1,1]^3; Sec. 1) on structured
 * hexahedral meshes, in the matrix-free factored form A^e = D^T G^e D with
 * the six symmetric geometric factors G_rr ... G_tt stored per quadrature
 * point (Sec. 2), by sum factorization, and solves with unpreconditioned CG.
 * Benchmark problems (Sec. 1): mass = BP1, stiffness = BP3, collocated
 * stiffness (Gauss-Lobatto quadrature at the nodes) = BP5; BP6 = BP5 with
 * three components.
 *
 * Conventions shared by every call:
 *   - Every function returns int: MFHEX_OK (0) or a negative MFHEX_ERR_*.
 *     Nothing aborts or throws; mfhex_last_error() gives a message.
 *   - "_dev" pointers are device (HBM) pointers owned by the CALLER; the
 *     library never allocates or frees device memory (its only device
 *     storage is the fixed array of mfhex_apply_static, part of the loaded
 *     code object).  Host pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     apply / apply_add / apply_adjoint / kappa_grad / diagonal / rhs /
 *     *_coords / mg_apply / tet_apply enqueue kernels only (outputs are
 *     cleared by a fill kernel, never by a runtime memset; no allocation and
 *     no host synchronization), so they may be recorded into a graph by
 *     stream capture.  create, cg, tune and mg_setup synchronize the stream
 *     and must not be captured.
 *   - Node numbering: global node (I,J,K), I in [0, p*nex], is
 *     I + (p*nex+1)*(J + (p*ney+1)*K).  Element (ex,ey,ez) is
 *     ex + nex*(ey + ney*ez).  Quadrature point (a,b,c) of an element is
 *     a + q*(b + q*c).
 *   - Multi-vectors are row-major [n_nodes][nrhs][ncomp]: the nvec =
 *     nrhs*ncomp values of a node are contiguous.  The operator acts on each
 *     of the nvec columns independently (BP6 = three uncoupled components).
 *   - With dirichlet = 1 the operator is M A M, M the 0/1 mask of interior
 *     nodes: boundary entries of the input are ignored and those of the
 *     output are zero.
 *   - One handle must not be used from two host threads at once; distinct
 *     handles are independent.
 */
#ifndef MFHEX_H
#define MFHEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
    MFHEX_OK = 0,
    MFHEX_ERR_ARG = -1,         /* invalid argument or size                      */
    MFHEX_ERR_UNSUPPORTED = -2, /* valid but not built (e.g. p > 8)              */
    MFHEX_ERR_HIP = -3,         /* a HIP runtime call failed                     */
    MFHEX_ERR_MESH = -4,        /* an element has detJ <= 0 somewhere            */
    MFHEX_ERR_NOCONV = -5,      /* CG reached maxit; x and stats are valid       */
    MFHEX_ERR_BREAKDOWN = -6,   /* CG: p^T A p <= 0 or a non-finite value        */
    MFHEX_ERR_STATE = -7        /* call not valid for this handle (e.g. no kappa) */
};

enum { MFHEX_MASS = 1, MFHEX_DIFFUSION = 2 };      /* operator kind       */
enum { MFHEX_GAUSS = 0, MFHEX_GLL = 1 };           /* quadrature rule     */
enum { MFHEX_F64 = 0, MFHEX_F32 = 1 };             /* arithmetic / data   */
enum { MFHEX_CG_F64 = 0, MFHEX_CG_MIXED = 1 };     /* solver mode         */
enum { MFHEX_PRECOND_NONE = 0, MFHEX_PRECOND_JACOBI = 1, MFHEX_PRECOND_MG = 2 }; /* CG preconditioner */

/* desc.flags bits */
#define MFHEX_FLAG_F32 1u  /* also build FP32 quadrature data (for prec = MFHEX_F32) */
#define MFHEX_FLAG_RHS 2u  /* keep w*detJ per point for mfhex_rhs on a diffusion op  */
#define MFHEX_FLAG_OTF 4u  /* diffusion, FP64, constant kappa: no stored geometric factors; the apply
                            * evaluates w adj(J) adj(J)^T / detJ at every point from the element's 8
                            * vertices (the factors equal the stored ones up to rounding).  The
                            * workspace then holds no factor array; mfhex_diagonal (and so the
                            * Jacobi-preconditioned CG) is not available on such an operator. */
#define MFHEX_FLAG_DETERMINISTIC 8u /* results that do not depend on the order in which element groups run
                            * (a reference for checks of the atomic path, e.g. run-to-run spread): the
                            * apply stores every element's values (plain stores) in a workspace buffer
                            * of n_elem (p+1)^3 ncomp FP64 values, and a second kernel sums each node's
                            * (up to 8) element values in increasing element order.  The paper's
                            * operator is the same (E->L scatter-add, Sec. 2, A_L = sum R^T A^e R);
                            * only the summation order is fixed.  One right-hand side per apply
                            * (nrhs = 1, else MFHEX_ERR_UNSUPPORTED); the load vector keeps atomics. */

/* Operator description.
 *   p in [1,8].  quad = MFHEX_GAUSS needs q = p+2 (mass and stiffness);
 *   quad = MFHEX_GLL needs q = p+1 (collocated with the nodes).
 *   kind: MFHEX_MASS (pointwise w*detJ) or MFHEX_DIFFUSION (pointwise
 *   w adj(J) adj(J)^T / detJ, Sec. 2).  ncomp in {1,3}.
 *   variable_kappa = 1 (diffusion, FP64 only): a per-point coefficient
 *   set by mfhex_set_kappa multiplies the geometric factors.
 *   vertex_xyz: HOST array [(nex+1)(ney+1)(nez+1)][3] of FP64 vertex
 *   coordinates, x fastest; each hexahedron is the trilinear image of
 *   [-1,1]^3 through its 8 vertices.  Copied into the workspace by create. */
typedef struct {
    int32_t nex, ney, nez;
    int32_t p, q, quad, kind, ncomp, dirichlet, variable_kappa;
    uint32_t flags;
    const double *vertex_xyz;
} mfhex_desc;

/* Sizes derived from a description (filled by mfhex_query). */
typedef struct {
    int64_t n_nodes;        /* nodes per component, (p nex+1)(p ney+1)(p nez+1)     */
    int64_t n_elem;         /* nex ney nez                                         */
    int64_t n_qpts;         /* n_elem * q^3                                        */
    size_t workspace_bytes; /* device workspace for mfhex_create                   */
    size_t cg_work_bytes;   /* device work area for mfhex_cg (per solve, nrhs = 1) */
} mfhex_sizes;

typedef struct mfhex_op_s *mfhex_op; /* opaque; library-owned host state only */

/* Validate `d` and compute sizes.  No device work.  The paper defines no
 * such call: it sizes the caller-owned storage of the operator (element
 * restriction, the geometric factors of Sec. 2 per point, the 1D bases of
 * Sec. 1), in the spirit of the caller-managed arrays of the libCEED
 * interface (Sec. 2.1).  Errors: MFHEX_ERR_ARG for a null pointer or a
 * description out of range, MFHEX_ERR_UNSUPPORTED for p > 8. */
int mfhex_query(const mfhex_desc *d, mfhex_sizes *out);

/* Set up an operator: 1D bases on the host, element restriction (int32
 * offsets, Dirichlet nodes encoded negative) copied into the workspace,
 * quadrature data built on the GPU from the vertices (Sec. 2, the geometric
 * factors G^e).  workspace_dev: caller-owned device buffer of at least
 * sizes.workspace_bytes, 256-byte aligned, which must outlive the handle.
 * Synchronizes `stream`.  Returns MFHEX_ERR_MESH if any point has
 * detJ <= 0.  On error *out is NULL. */
int mfhex_create(const mfhex_desc *d, void *workspace_dev, size_t workspace_bytes, void *stream,
                 mfhex_op *out);

/* Release the handle's host state.  Device memory stays with the caller. */
int mfhex_destroy(mfhex_op op);

/* Per-point coefficient kappa for a variable_kappa operator: device FP64
 * [n_elem][q^3], copied into the workspace (asynchronous).  The paper is
 * silent on coefficients; this is the reading used for the differentiable
 * form: kappa multiplies the six geometric factors of Sec. 2 at each point,
 * so A(kappa) stays symmetric and is linear in kappa.  MFHEX_ERR_STATE on an
 * operator created without variable_kappa. */
int mfhex_set_kappa(mfhex_op op, const double *kappa_dev, void *stream);

/* y = A x for nvec = nrhs*ncomp columns, x and y device arrays of
 * n_nodes*nvec FP64 (prec = MFHEX_F64) or FP32 (prec = MFHEX_F32, needs
 * MFHEX_FLAG_F32; FP32 data and accumulation throughout).  y is fully
 * overwritten.  x and y must not overlap.  Asynchronous.  (Sec. 2: the
 * operator-level kernel w_L = A_L u_L, restriction, basis contractions,
 * pointwise geometric factors and the transposes fused in one kernel.) */
int mfhex_apply(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream);

/* y += A x (no zero fill of y); otherwise as mfhex_apply. */
int mfhex_apply_add(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream);

/* y = A^T x.  The operators are symmetric, so this is the same action; it is
 * the backward of mfhex_apply with respect to its input.  The paper defines
 * no adjoint; since A^e = D^T G^e D (Sec. 2) with G^e symmetric, A^T = A,
 * and this call runs the apply kernel.  Same arguments, layout and errors as
 * mfhex_apply. */
int mfhex_apply_adjoint(mfhex_op op, int prec, int nrhs, const void *x_dev, void *y_dev, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): y = A x for one
 * right-hand side (nvec = ncomp), in the deterministic form of
 * MFHEX_FLAG_DETERMINISTIC (element values stored, then summed per node in
 * increasing element order), on any operator, with or without that flag.
 * The element values live in a device array the library owns: one copy per
 * GPU, mfhex_apply_static_max_bytes() = 64 MiB, held until the process
 * ends.  The operator needs n_elem (p+1)^3 ncomp values of that buffer (8
 * bytes each for MFHEX_F64, 4 for MFHEX_F32); above the maximum the call
 * returns MFHEX_ERR_ARG and launches nothing.  The operator's device must be
 * current (MFHEX_ERR_STATE otherwise); the first call on a device looks up
 * that device's copy of the array.  No allocation, no host synchronization:
 * it enqueues the apply and assembly kernels on `stream`.  Every call on one
 * GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (two streams, two host threads) race; calls ordered on one stream do not.
 * x, y and prec as in mfhex_apply (y fully overwritten); the result equals
 * mfhex_apply on an operator created with MFHEX_FLAG_DETERMINISTIC. */
int mfhex_apply_static(mfhex_op op, int prec, const void *x_dev, void *y_dev, void *stream);
size_t mfhex_apply_static_max_bytes(void);

/* Gradient of s = r^T (M A(kappa) M) u with respect to the per-point
 * coefficient (the paper defines none; with A^e = D^T (kappa G0^e) D of
 * Sec. 2, s is linear in each kappa_pt, and its derivative is the pointwise
 * product below): g[e][pt] = (Dhat M r)_pt^T G0_pt (Dhat M u)_pt, G0 the
 * kappa-free geometric factors.  u, r: device FP64 [n_nodes] (ncomp = 1);
 * g: device FP64 [n_elem][q^3], overwritten.  Diffusion operators with
 * stored geometric factors only (MFHEX_ERR_UNSUPPORTED with MFHEX_FLAG_OTF).
 * For a loss L(y), r = dL/dy gives dL/dkappa.  Asynchronous. */
int mfhex_kappa_grad(mfhex_op op, const double *u_dev, const double *r_dev, double *g_dev, void *stream);

/* Diagonal of the assembled operator M (sum_e R_e^T A^e R_e) M, device FP64
 * [n_nodes], overwritten (0 at masked nodes; with ncomp = 3 it is the
 * diagonal of each component's block).  Evaluated matrix-free: each
 * element's diagonal is a sum of transposed interpolations of its point
 * factors with squared or mixed 1D matrices (the sum factorization of
 * Sec. 1 and the operator form A^e = Dhat^T G^e Dhat of Sec. 2), added with
 * atomics.  The Jacobi preconditioner of mfhex_cg uses it.  Variable
 * coefficient operators need mfhex_set_kappa first.  Asynchronous. */
int mfhex_diagonal(mfhex_op op, double *diag_dev, void *stream);

/* Physical coordinates of the quadrature points, device FP64
 * [n_elem][q^3][3], and of the nodes, device FP64 [n_nodes][3] (for
 * evaluating coefficients, forcings and nodal fields).  Asynchronous. */
int mfhex_qpoint_coords(mfhex_op op, double *xyz_dev, void *stream);
int mfhex_node_coords(mfhex_op op, double *xyz_dev, void *stream);

/* Load vector b_n = sum over points of w detJ f phi_n (masked when
 * dirichlet), f given per point as device FP64 [n_elem][q^3]; b: device
 * FP64 [n_nodes], overwritten.  Mass operators, or diffusion operators
 * created with MFHEX_FLAG_RHS.  Asynchronous. */
int mfhex_rhs(mfhex_op op, const double *f_dev, double *b_dev, void *stream);

/* CG options.
 *   mode MFHEX_CG_F64: unpreconditioned Hestenes-Stiefel CG in FP64.
 *   mode MFHEX_CG_MIXED: FP32 operator and FP32 r, p, Ap; FP64 x and all dot
 *     products; the residual is replaced by the FP64 true residual
 *     fp32(b - A64 x) whenever the recursive residual has fallen by
 *     replace_delta since the last replacement, or every replace_every
 *     iterations (needs MFHEX_FLAG_F32).
 *   Stops when ||r||_2 <= rtol ||b||_2; in mixed mode only on the FP64 true
 *   residual.  maxit bounds the iterations.  check_every: iterations
 *   between host convergence checks (one stream sync each).  x0_is_zero = 0
 *   starts from the given x.  max_iters_exact = 1 runs exactly maxit
 *   iterations without convergence checks (FP64 mode; returns MFHEX_OK).
 *   precond MFHEX_PRECOND_JACOBI: Jacobi-preconditioned CG in either mode,
 *   z = D^-1 r with D = mfhex_diagonal (computed and inverted at the start of
 *   every solve; 0 at masked nodes), alpha = r.z / p.Ap, beta from r.z; the
 *   stopping test stays on ||r||.  precond MFHEX_PRECOND_MG: one p-multigrid
 *   V-cycle per iteration (mfhex_mg_setup first; FP64 mode only).  pad_ must be 0. */
typedef struct {
    int32_t maxit, check_every, mode, replace_every, x0_is_zero, max_iters_exact, precond, pad_;
    double rtol, replace_delta;
} mfhex_cg_opts;

typedef struct {
    int32_t iters, replacements, fell_back_to_f64, pad_;
    double rel_resid_true; /* ||b - A x|| / ||b|| in FP64 at exit          */
    double rel_resid_rec;  /* recursive residual estimate at exit          */
    double seconds;        /* wall time from first launch to exit          */
} mfhex_cg_stats;

/* Solve A x = b.  b, x: device FP64 [n_nodes] (ncomp = 1).  cg_work_dev:
 * caller-owned device buffer of sizes.cg_work_bytes.  rhist (may be NULL):
 * HOST array of maxit+1 doubles receiving ||r_0|| and then ||r_k||
 * (recursive) after each iteration; entries past 8191 iterations are not
 * written.  Synchronizes
 * `stream`.  Returns MFHEX_OK on convergence, MFHEX_ERR_NOCONV at maxit,
 * MFHEX_ERR_BREAKDOWN on p^T A p <= 0 / non-finite values.  (Sec. 1: CG
 * on the sum-factorized operator; Sec. 2: the benchmarks run it
 * unpreconditioned; Jacobi scaling is the smoother of the Nek5000/RS
 * solvers of Sec. 2.) */
int mfhex_cg(mfhex_op op, const double *b_dev, double *x_dev, void *cg_work_dev, const mfhex_cg_opts *opts,
             mfhex_cg_stats *stats, double *rhist, void *stream);

/* p-multigrid preconditioner (Sec. 1: p-multigrid in high-order codes;
 * Sec. 2, Nek5000/RS: Chebyshev-accelerated Jacobi smoothing).  Levels p,
 * floor(p/2), ..., 1 on the operator's mesh (same quadrature family and
 * mask); prolongation = the coarse field at the fine nodes, restriction its
 * transpose; on every level a Chebyshev smoother on D^-1 A (D =
 * mfhex_diagonal) over [lo, hi] x lambda, lambda from power_iters steps of
 * the power method (start vector: SplitMix64 uniform, seed 2024, masked; the
 * generalized Rayleigh quotient of the last iterate); V-cycle: pre-smooth
 * from 0 (degree), restrict, recurse, prolong and add, post-smooth (degree);
 * the coarsest level is smoothed only (coarse_degree).  Fields left 0 take
 * the defaults degree 3, coarse_degree 8, power_iters 15, all levels,
 * lo 0.25, hi 1.1.  Scalar diffusion with stored factors and constant kappa
 * only.  precision: MFHEX_F64 (default) or MFHEX_F32, the arithmetic of the
 * V-cycle (level operators, smoothers, transfers; needs an operator created
 * with MFHEX_FLAG_F32); set-up (diagonals, power method) is FP64 either way
 * and mfhex_mg_apply takes and returns FP64 vectors. */
typedef struct {
    int32_t degree, coarse_degree, power_iters, max_levels;
    int32_t precision, pad_;
    double lo, hi;
} mfhex_mg_opts;

/* Device work-area size (bytes, 256-byte aligned buffer) and level count for
 * a hierarchy on an operator of description `fine` (opts may be NULL). */
int mfhex_mg_query(const mfhex_desc *fine, const mfhex_mg_opts *opts, size_t *work_bytes, int32_t *nlevels);

/* Build the hierarchy and attach it to `op` (created from `fine`, whose
 * vertex pointer is read again for the coarse levels).  work_dev:
 * caller-owned device buffer of mfhex_mg_query's size; it holds the coarse
 * operators, level vectors and transfer matrices and must outlive `op`
 * (mfhex_destroy releases the coarse handles).  Synchronizes `stream`. */
int mfhex_mg_setup(mfhex_op op, const mfhex_desc *fine, const mfhex_mg_opts *opts, void *work_dev, size_t work_bytes,
                   void *stream);

/* z = M^-1 r: one V-cycle.  r, z: device FP64 [n_nodes], distinct.  Asynchronous. */
int mfhex_mg_apply(mfhex_op op, const double *r_dev, double *z_dev, void *stream);

/* Order, node count and lambda_max(D^-1 A) estimate of level `level` (0 = finest). */
int mfhex_mg_level(mfhex_op op, int level, int32_t *p, int64_t *n_nodes, double *lambda_max);

/* Autotune the apply for (prec, nrhs) -- the counterpart of the offline
 * benchmark sweep that selects the best routine and batch size for the
 * non-tensor products in MAGMA (Sec. 2.2), run here on the caller's own
 * operator: time every launch variant of the
 * fused kernel (elements per thread group, threads per group; for the mass
 * operator also pipeline depths 1, 2 and 4) on this operator, reject any whose
 * result differs from the default configuration by more than 1e-13 (relative,
 * max norm; 1e-5 for FP32), time the others in three interleaved rounds of ten
 * applies, keep the one with the smallest median for this handle and append
 * "<arch> kind quad p nvec prec variant depth" to the text cache
 * at cache_path (NULL: no file); handles created later read the file named by
 * the environment variable MFHEX_TUNE_CACHE.  scratch_dev: caller-owned
 * device buffer of at least MFHEX_TUNE_SCRATCH(n_nodes * nvec) bytes
 * (256-byte aligned).  Synchronizes `stream`. */
#define MFHEX_TUNE_SCRATCH(len) (3 * ((((size_t)(len)) * 8 + 255) & ~(size_t)255) + 32768)
int mfhex_tune(mfhex_op op, int prec, int nrhs, void *scratch_dev, const char *cache_path, void *stream);

/* (Companions of mfhex_tune, the selection layer of Sec. 2.2.)
 * Launch configuration the apply uses now for (prec, nrhs): the variant, the
 * elements per thread group and threads per group it stands for, and the
 * pipeline depth (element groups one thread group works through in turn,
 * loading the next group's data while it computes the current one; always 1
 * for diffusion).  Outputs may be NULL. */
int mfhex_get_config(mfhex_op op, int prec, int nrhs, int32_t *variant, int32_t *elems_per_group,
                     int32_t *threads_per_group, int32_t *groups_per_block);

/* Force the launch configuration for (prec, nrhs): variant 0 .. 16 (5 .. 8
 * carry 2, 4, 8, 16 vectors of a multi-vector together; 9 .. 14 are the
 * factored-gradient diffusion kernel for Gauss points, which forms the
 * gradient with the basis derivative at the points in three contraction
 * stages instead of six; 15 and 16 carry 4 and 8 vectors with the gradient
 * contractions on the FP64 matrix cores, collocated FP64 diffusion only) and
 * pipeline depth
 * groups_per_block (0: the operator's default, measured per order for mass
 * and 1 for diffusion; mass accepts 1 .. 64, diffusion only 1).
 * MFHEX_ERR_ARG if out of range. */
int mfhex_set_config(mfhex_op op, int prec, int nrhs, int32_t variant, int32_t groups_per_block);

/* Static message for a status code; message of the last failure on a
 * handle (NULL op: last failure of a call that had no handle yet). */
const char *mfhex_strerror(int code);
const char *mfhex_last_error(mfhex_op op);

/* The 1D data an operator of order p with rule (q, quad) uses, computed on
 * the host (no device work): Gauss-Lobatto nodes [p+1], quadrature points and
 * weights [q], interpolation B [q][p+1] (B[a][i] = l_i(x_a)) and the
 * collocated derivative on the points D [q][q].  Any output may be NULL.
 * (Sec. 1: Lagrange basis on Gauss-Lobatto points; Sec. 2: the dense 1D
 * derivative matrix of the tensor contractions.) */
int mfhex_basis_1d(int p, int q, int quad, double *nodes, double *xq, double *wq, double *B, double *D);

/* ---- Tetrahedral P_p diffusion: the non-tensor basis as a matrix product ----
 * Sec. 2.1 (libCEED) and Sec. 2.2 (MAGMA, its non-tensor backend): a non-tensor basis
 * is applied through its full matrices, the gradient matrix of one element
 * (all quadrature points by all basis functions) times one column per
 * element, i.e. one matrix product for all elements (batched along the
 * elements).  Here 16 elements at a time go through the FP64 matrix cores,
 * with the pointwise 3x3 factor applied to the products in registers and
 * the transposed product back to the nodes in the same kernel.
 *
 * Mesh: the structured box of mfhex_desc (same vertex array, x fastest),
 * every hexahedron split into the 6 Kuhn tetrahedra around its main
 * diagonal, each affine on its 4 corner vertices.  Element e = 6 cube + t,
 * cube = ex + nex (ey + ney ez).  Basis: Lagrange P_p (p = 1..6) on
 * equispaced barycentric nodes; these are the points of the lattice of
 * spacing h/p, so a vector has (p nex + 1)(p ney + 1)(p nez + 1) entries,
 * numbered as in the hexahedral operator (x fastest).  Rule: collapsed
 * Gauss-Jacobi, q points per direction (q = p or p+1; q = p integrates the
 * stiffness of an affine element exactly), Q = q^3 points per element.
 * y = A x with A = sum_e P_e^T K_e P_e, K_e the element stiffness; with
 * dirichlet = 1 the box-boundary nodes are masked (y = 0 there, x ignored). */
typedef struct mfhex_tet_s *mfhex_tet;

typedef struct {
    int32_t nex, ney, nez, p, q, dirichlet;
    const double *vertex_xyz; /* HOST [(nex+1)(ney+1)(nez+1)][3]; read during mfhex_tet_create only */
} mfhex_tet_desc;

typedef struct {
    int64_t n_nodes, n_elem, n_qpts;
    size_t workspace_bytes; /* device bytes the caller provides (256-byte aligned) */
    int32_t n_basis, n_points;  /* per element: (p+1)(p+2)(p+3)/6 and q^3 */
} mfhex_tet_sizes;

/* Sizes of an operator (host only).  ERR_UNSUPPORTED for p outside 1..6 or
 * q not in {p, p+1}. */
int mfhex_tet_query(const mfhex_tet_desc *d, mfhex_tet_sizes *out);

/* Build the operator in the caller's workspace (basis-gradient fragments,
 * element restriction, per-point factors w |det J| J^-1 J^-T).  Synchronizes
 * `stream`; ERR_MESH for a degenerate tetrahedron.  The workspace must
 * outlive the handle; the library owns only host metadata. */
int mfhex_tet_create(const mfhex_tet_desc *d, void *workspace_dev, size_t workspace_bytes, void *stream,
                     mfhex_tet *out);

/* y = A x, FP64 device vectors [n_nodes] that must not overlap (else
 * MFHEX_ERR_ARG).  Asynchronous on `stream` (y is zeroed first, then summed
 * with atomics). */
int mfhex_tet_apply(mfhex_tet op, const double *x_dev, double *y_dev, void *stream);

int mfhex_tet_destroy(mfhex_tet op);

/* The library's reference tables (host only, no device work): rule points
 * xi [q^3][3] and weights w [q^3] on the tetrahedron {xi >= 0, sum xi <= 1},
 * basis values B [q^3][P] and reference gradients G [3][q^3][P] at the points,
 * basis functions ordered by (n3, n2, n1) with n1 fastest, n the barycentric
 * multi-index of the node.  Any output may be NULL.  Errors of the mfhex_tet
 * calls are read with mfhex_last_error(NULL). */
int mfhex_tet_basis(int p, int q, double *xi, double *w, double *B, double *G);

/* Library version string. */
const char *mfhex_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MFHEX_H */
