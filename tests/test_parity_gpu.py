"""GPU parity: the HIP library, called through its C ABI, against the FP64 CPU
oracle on the same seeded inputs.

Tolerances (max-norm relative, ||y_gpu - y_orc||_inf / ||y_orc||_inf):
  FP64 apply / load vector / coefficient gradient: 1e-12 (the stated target);
  FP32 apply: 2e-5 (unit roundoff 6e-8 times the ~(3(p+q)+15)-term chains of
  the contractions, with margin).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def build(mf, nex, ney, nez, p, kind="diffusion", quad="gauss", dirichlet=True, ncomp=1, vark=False, f32=False,
          rhs=False, perturb=0.1, otf=False, det=False):
    vert = synth.mesh_vertices(nex, ney, nez, perturb)
    op = mf.Operator(nex, ney, nez, p, vert, kind=kind, quad=quad, ncomp=ncomp, dirichlet=dirichlet,
                     variable_kappa=vark, f32=f32, rhs=rhs, otf=otf, deterministic=det)
    q = p + 2 if quad == "gauss" else p + 1
    pr = oracle.Problem(nex, ney, nez, p, q, oracle.GAUSS if quad == "gauss" else oracle.GLL,
                        oracle.DIFFUSION if kind == "diffusion" else oracle.MASS, int(dirichlet), vert)
    return op, pr


def interior_mask(pr):
    nx, ny, nz = pr.p * pr.nex + 1, pr.p * pr.ney + 1, pr.p * pr.nez + 1
    I = np.arange(pr.n_nodes)
    ix, iy, iz = I % nx, (I // nx) % ny, I // (nx * ny)
    return ((ix > 0) & (ix < nx - 1) & (iy > 0) & (iy < ny - 1) & (iz > 0) & (iz < nz - 1)).astype(float)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def valid_variants(op, dtype=torch.float64, nrhs=1):
    """Launch variants the operator accepts (some exceed the LDS budget at high order)."""
    from paper_2109_05072_amd import _lib as L
    out = []
    for v in range(17):
        try:
            op.set_config(v, dtype, nrhs)
            out.append(v)
        except L.MFHexError:
            pass
    return out


# --- apply parity across orders, rules, masks ------------------------------------------------

@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("kind,quad", [("diffusion", "gauss"), ("diffusion", "gll"), ("mass", "gauss")])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_apply_fp64_matches_oracle(gpu_lib, p, kind, quad, dirichlet):
    _say("apply64", p, kind, quad, dirichlet)
    op, pr = build(gpu_lib, 5, 3, 2, p, kind, quad, dirichlet)
    x = synth.uniform_vector(pr.n_nodes)
    yo = oracle.apply(pr, x)
    y = host(op.apply(dev(x)))
    assert relerr(y, yo) <= TOL64
    # mass: thread groups that pipeline 1, 2, 3 or 7 element groups (30 elements:
    # the last thread group of the odd depths gets a ragged share)
    depths = (1, 2, 3, 7) if kind == "mass" else (0,)
    for v in valid_variants(op):
        for d in depths:
            op.set_config(v, groups_per_block=d)
            _say("apply64 variant", v, op.get_config())
            y2 = host(op.apply(dev(x)))
            assert relerr(y2, yo) <= TOL64


def _pq_id(p, quad="gauss"):
    return f"p{p}-q{p + 2 if quad == 'gauss' else p + 1}"


@pytest.mark.parametrize("p", range(1, 9), ids=[_pq_id(p) for p in range(1, 9)])
@pytest.mark.parametrize("kind,quad", [("diffusion", "gauss"), ("diffusion", "gll"), ("mass", "gauss")])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_apply_fp32_matches_oracle(gpu_lib, p, kind, quad, dirichlet):
    # the FP32 operator of mixed-precision CG: default launch and every FP32 launch variant the
    # tuner may pick (the two-element FP32 defaults at q = 7 and 8 included), ragged element groups
    _say("apply32", p, kind, quad, dirichlet)
    op, pr = build(gpu_lib, 5, 3, 2, p, kind, quad, dirichlet, f32=True)
    x = synth.uniform_vector(pr.n_nodes)
    yo = oracle.apply(pr, x)
    _say("apply32 default", op.get_config(torch.float32))
    y = host(op.apply(dev(x, torch.float32)))
    assert relerr(y, yo) <= TOL32
    variants = valid_variants(op, torch.float32)
    assert 0 in variants
    for v in variants:
        op.set_config(v, torch.float32)
        _say("apply32 variant", v, op.get_config(torch.float32))
        assert relerr(host(op.apply(dev(x, torch.float32))), yo) <= TOL32


@pytest.mark.parametrize("p", [5, 6, 7], ids=["p5-q7-default", "p6-q8-default-two-element", "p7-q9-default"])
def test_fp32_default_launch_at_mixed_cg_orders(gpu_lib, p):
    # the FP32 launch defaults of their own (five-element groups at q = 7, two-element groups at
    # q = 8, the FP64 choice at q = 9) on a mesh whose element rows leave a ragged last group (7 =
    # 5 + 2 = 3 x 2 + 1), against the oracle and against the FP64 apply rounded to FP32 accuracy
    op, pr = build(gpu_lib, 7, 3, 3, p, "diffusion", "gauss", True, f32=True)
    cfg = op.get_config(torch.float32)
    _say("fp32 default", p, cfg)
    if p in (5, 6):
        assert cfg[1] == {5: 5, 6: 2}[p], cfg
    x = synth.uniform_vector(pr.n_nodes, seed=9)
    yo = oracle.apply(pr, x)
    y32 = host(op.apply(dev(x, torch.float32)))
    y64 = host(op.apply(dev(x)))
    print("fp32 default", p, cfg, "err vs oracle", relerr(y32, yo))
    assert relerr(y32, yo) <= TOL32
    assert relerr(y64, yo) <= TOL64


@pytest.mark.parametrize("p,ncomp,nrhs", [(2, 3, 1), (3, 1, 4), (5, 3, 2), (8, 1, 3), (4, 3, 8)])
@pytest.mark.parametrize("quad", ["gauss", "gll"])
def test_multivector_matches_oracle_and_looped(gpu_lib, p, ncomp, nrhs, quad):
    _say("multivector", p, ncomp, nrhs, quad)
    op, pr = build(gpu_lib, 3, 3, 2, p, "diffusion", quad, True, ncomp=ncomp)
    nvec = ncomp * nrhs
    x = synth.uniform_vector(pr.n_nodes, nvec=nvec)
    yo = oracle.apply(pr, x)
    y = host(op.apply(dev(x)))
    assert relerr(y, yo) <= TOL64
    # every launch variant, including chunks of 2/4/8 vectors that do not divide nvec
    for v in valid_variants(op, nrhs=nrhs):
        op.set_config(v, nrhs=nrhs)
        _say("multivector variant", v, op.get_config(nrhs=nrhs))
        assert relerr(host(op.apply(dev(x))), yo) <= TOL64
    # one launch for all vectors == separate single-vector launches
    if ncomp == 1:
        single, _ = build(gpu_lib, 3, 3, 2, p, "diffusion", quad, True)
        for v in range(nvec):
            yv = host(single.apply(dev(x[:, v].copy())))
            assert relerr(y[:, v], yv) <= 1e-14


@pytest.mark.parametrize("p,ncomp,nrhs", [(2, 3, 2), (4, 1, 5), (7, 3, 1)])
def test_mass_multivector_pipeline_matches_oracle(gpu_lib, p, ncomp, nrhs):
    """Chunks of vectors and pipelined element groups together: the next work
    item is either the next chunk of the same group or the next group."""
    _say("mass multivector", p, ncomp, nrhs)
    op, pr = build(gpu_lib, 3, 2, 3, p, "mass", "gauss", False, ncomp=ncomp)
    nvec = ncomp * nrhs
    x = synth.uniform_vector(pr.n_nodes, nvec=nvec)
    yo = oracle.apply(pr, x)
    for v in valid_variants(op, nrhs=nrhs):
        for d in (1, 2, 5):
            op.set_config(v, nrhs=nrhs, groups_per_block=d)
            _say("mass multivector config", op.get_config(nrhs=nrhs))
            assert relerr(host(op.apply(dev(x))), yo) <= TOL64


def test_pipeline_depth_configuration(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    diff, _ = build(gpu_lib, 2, 2, 2, 3, "diffusion", "gauss")
    mass, _ = build(gpu_lib, 2, 2, 2, 3, "mass", "gauss", False)
    assert diff.get_config()[3] == 1
    d0 = mass.get_config()[3]
    assert 1 <= d0 <= 64
    diff.set_config(0, groups_per_block=1)
    for bad in (2, 65, -1):
        with pytest.raises(L.MFHexError):
            diff.set_config(0, groups_per_block=bad)
    for bad in (65, -1):
        with pytest.raises(L.MFHexError):
            mass.set_config(0, groups_per_block=bad)
    mass.set_config(1, groups_per_block=64)
    assert mass.get_config()[0] == 1 and mass.get_config()[3] == 64
    mass.set_config(1, groups_per_block=0)
    assert mass.get_config()[3] == d0


def test_apply_add_accumulates(gpu_lib):
    op, pr = build(gpu_lib, 3, 2, 2, 3)
    x = synth.uniform_vector(pr.n_nodes)
    y0 = synth.uniform_vector(pr.n_nodes, seed=3)
    y = dev(y0)
    op.apply_add(dev(x), y)
    assert relerr(host(y) - y0, oracle.apply(pr, x)) <= TOL64


def test_adjoint_is_the_apply(gpu_lib):
    op, pr = build(gpu_lib, 3, 2, 2, 4)
    u = synth.uniform_vector(pr.n_nodes, seed=1)
    v = synth.uniform_vector(pr.n_nodes, seed=2)
    Au = host(op.apply(dev(u)))
    ATv = host(op.apply_adjoint(dev(v)))
    assert abs(v @ Au - u @ ATv) <= 1e-13 * np.linalg.norm(v) * np.linalg.norm(Au)


# --- setup outputs --------------------------------------------------------------------------

@pytest.mark.parametrize("p,quad", [(2, "gauss"), (5, "gll")])
def test_coordinates_match_oracle(gpu_lib, p, quad):
    op, pr = build(gpu_lib, 3, 2, 4, p, "diffusion", quad)
    xq, _ = oracle.qpoint_geometry(pr)
    assert np.abs(host(op.qpoint_coords()) - xq).max() <= 1e-15
    assert np.abs(host(op.node_coords()) - oracle.node_coords(pr)).max() <= 1e-15


@pytest.mark.parametrize("p,kind", [(2, "mass"), (4, "diffusion"), (7, "diffusion")])
def test_load_vector_matches_oracle(gpu_lib, p, kind):
    op, pr = build(gpu_lib, 3, 3, 2, p, kind, "gauss", dirichlet=(kind == "diffusion"), rhs=True)
    f = synth.sin_forcing(host(op.qpoint_coords()))
    fo = synth.sin_forcing(oracle.qpoint_geometry(pr)[0])
    b = host(op.rhs(dev(f)))
    assert relerr(b, oracle.rhs(pr, fo)) <= TOL64


# --- invariants on the GPU at larger sizes -------------------------------------------------

@pytest.mark.parametrize("p", [1, 3, 6])
def test_gpu_invariants(gpu_lib, p):
    ne = max(2, 24 // p)
    opm, _ = build(gpu_lib, ne, ne, ne, p, "mass", "gauss", dirichlet=False)
    one = torch.ones(opm.n_nodes, dtype=torch.float64, device="cuda")
    assert abs(float(one @ opm.apply(one)) - 1.0) < 1e-12
    opd, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", dirichlet=False)
    X = opd.node_coords()
    u = 0.4 + X @ torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    y = host(opd.apply(u.contiguous()))
    n = p * ne + 1
    I = np.arange(opd.n_nodes)
    ix, iy, iz = I % n, (I // n) % n, I // (n * n)
    inner = (ix > 0) & (ix < n - 1) & (iy > 0) & (iy < n - 1) & (iz > 0) & (iz < n - 1)
    assert np.abs(y[inner]).max() <= 1e-12 * np.abs(y).max()


def test_run_to_run_spread(gpu_lib):
    op, pr = build(gpu_lib, 8, 8, 8, 3)
    x = dev(synth.uniform_vector(pr.n_nodes))
    ys = [host(op.apply(x)) for _ in range(5)]
    spread = max(relerr(y, ys[0]) for y in ys)
    print("run-to-run spread", spread)
    assert spread <= 1e-14


# --- deterministic (atomic-free) scatter: the reference for the atomic path ---------------------

@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 8])
@pytest.mark.parametrize("kind,quad,ncomp", [("diffusion", "gauss", 1), ("diffusion", "gll", 3), ("mass", "gauss", 1)])
def test_deterministic_scatter_matches_atomic_and_oracle(gpu_lib, p, kind, quad, ncomp):
    _say("det", p, kind, quad, ncomp)
    dirichlet = kind == "diffusion"
    op, pr = build(gpu_lib, 5, 3, 2, p, kind, quad, dirichlet, ncomp=ncomp, f32=True, det=True)
    ref, _ = build(gpu_lib, 5, 3, 2, p, kind, quad, dirichlet, ncomp=ncomp, f32=True)
    x = synth.uniform_vector(pr.n_nodes, nvec=ncomp) if ncomp > 1 else synth.uniform_vector(pr.n_nodes)
    yo = oracle.apply(pr, x)
    for v in valid_variants(op):
        op.set_config(v)
        ref.set_config(v)
        _say("det variant", v, op.get_config())
        yd = host(op.apply(dev(x)))
        assert relerr(yd, yo) <= TOL64
        assert relerr(yd, host(ref.apply(dev(x)))) <= 1e-14
        if dirichlet:
            assert np.all(yd.reshape(pr.n_nodes, -1)[interior_mask(pr) == 0] == 0.0)
    # FP32 and y += A x
    y32 = host(op.apply(dev(x, torch.float32)))
    assert relerr(y32, yo) <= TOL32
    y0 = synth.uniform_vector(pr.n_nodes * ncomp, seed=8).reshape(x.shape)
    yt = dev(y0)
    op.apply_add(dev(x), yt)
    assert relerr(host(yt), y0 + yo) <= TOL64
    # one right-hand side per apply
    from paper_2109_05072_amd import _lib as L
    with pytest.raises(L.MFHexError) as ei:
        op.apply(dev(np.stack([x, x], axis=1) if ncomp == 1 else np.concatenate([x, x], axis=1)))
    assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED


def test_deterministic_scatter_is_bitwise_reproducible(gpu_lib):
    # the atomic path differs from run to run in the last bits; the deterministic path not at all, and
    # agrees with the atomic path to rounding (about 2.6e5 nodes, several hundred element groups per XCD)
    op, pr = build(gpu_lib, 21, 21, 21, 3, det=True)
    ref, _ = build(gpu_lib, 21, 21, 21, 3)
    x = dev(synth.uniform_vector(pr.n_nodes))
    yd = [host(op.apply(x)) for _ in range(4)]
    ya = [host(ref.apply(x)) for _ in range(4)]
    print("det runs identical:", all(np.array_equal(y, yd[0]) for y in yd),
          "atomic spread", max(relerr(y, ya[0]) for y in ya), "det vs atomic", relerr(yd[0], ya[0]))
    assert all(np.array_equal(y, yd[0]) for y in yd)
    assert relerr(yd[0], ya[0]) <= 1e-14
    # CG on the deterministic operator: the whole residual history repeats exactly
    b = dev(synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr))
    h = [op.cg(b, maxit=40, rtol=0.0, exact_iters=True).history for _ in range(2)]
    assert np.array_equal(h[0], h[1])


# --- autotuner ------------------------------------------------------------------------------

@pytest.mark.parametrize("p,quad,nrhs", [(3, "gauss", 1), (8, "gauss", 1), (5, "gll", 4)])
def test_every_launch_configuration_agrees(gpu_lib, p, quad, nrhs):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 4, 3, 3, p, "diffusion", quad)
    x = dev(synth.uniform_vector(pr.n_nodes, nvec=nrhs))
    ref = host(op.apply(x))
    vs = valid_variants(op, nrhs=nrhs)
    assert 0 in vs
    for v in vs:
        op.set_config(v, nrhs=nrhs)
        assert relerr(host(op.apply(x)), ref) <= 1e-13
    with pytest.raises(L.MFHexError):
        op.set_config(17, nrhs=nrhs)  # one past the last variant
    best = op.tune(nrhs=nrhs)
    assert best[0] in vs and best[3] == 1
    assert relerr(host(op.apply(x)), ref) <= 1e-13


def test_tuner_picks_a_mass_pipeline_depth(gpu_lib, tmp_path):
    op, pr = build(gpu_lib, 4, 4, 3, 4, "mass", "gauss", False)
    x = dev(synth.uniform_vector(pr.n_nodes))
    ref = host(op.apply(x))
    cache = tmp_path / "tune.txt"
    best = op.tune(cache_path=str(cache))
    assert best[3] in (1, 2, 4)
    assert relerr(host(op.apply(x)), ref) <= 1e-13
    fields = cache.read_text().split()
    assert len(fields) == 8 and int(fields[6]) == best[0] and int(fields[7]) == best[3]


# --- coefficient gradient -------------------------------------------------------------------

@pytest.mark.parametrize("p,quad", [(2, "gauss"), (4, "gauss"), (3, "gll")])
def test_variable_kappa_apply_and_gradient_match_oracle(gpu_lib, p, quad):
    op, pr = build(gpu_lib, 3, 3, 2, p, "diffusion", quad, True, vark=True)
    kap = synth.kappa_field(host(op.qpoint_coords()))
    kapo = synth.kappa_field(oracle.qpoint_geometry(pr)[0])
    pr = pr.with_(kappa=kapo)
    op.set_kappa(dev(kap))
    u = synth.uniform_vector(pr.n_nodes, seed=1)
    r = synth.uniform_vector(pr.n_nodes, seed=2)
    assert relerr(host(op.apply(dev(u))), oracle.apply(pr, u)) <= TOL64
    g = host(op.kappa_grad(dev(u), dev(r)))
    assert relerr(g, oracle.kappa_grad(pr, u, r)) <= TOL64


def test_autograd_gradients_vs_finite_differences_and_oracle(gpu_lib):
    from paper_2109_05072_amd.autograd import diffusion
    op, pr = build(gpu_lib, 3, 2, 2, 2, "diffusion", "gauss", True, vark=True)
    kap = dev(synth.kappa_field(host(op.qpoint_coords())))
    n = pr.n_nodes
    u = dev(synth.uniform_vector(n, seed=1)).requires_grad_(True)
    f = dev(synth.uniform_vector(n, seed=2))
    k = kap.clone().requires_grad_(True)

    def loss(uu, kk):
        r = diffusion(uu, kk, op) - f
        return 0.5 * (r * r).sum()

    Lv = loss(u, k)
    gu, gk = torch.autograd.grad(Lv, [u, k])
    rng = np.random.default_rng(synth.SEED_DIR)
    with torch.no_grad():
        for _ in range(4):
            d = dev(rng.standard_normal(kap.shape))
            eps = 1e-2 * float(kap.norm() / d.norm())
            fd = (loss(u, k + eps * d) - loss(u, k - eps * d)) / (2 * eps)
            an = (gk * d).sum()
            assert abs(float(fd - an)) <= 1e-9 * abs(float(an))
            du = dev(rng.standard_normal(n))
            eps = 1e-2 * float(u.norm() / du.norm())
            fd = (loss(u + eps * du, k) - loss(u - eps * du, k)) / (2 * eps)
            an = (gu * du).sum()
            assert abs(float(fd - an)) <= 1e-9 * abs(float(an))
    # against the oracle's gradient (its own coefficient and residual)
    kapo = synth.kappa_field(oracle.qpoint_geometry(pr)[0])
    pro = pr.with_(kappa=kapo)
    uo = host(u.detach())
    r = oracle.apply(pro, uo) - host(f)
    assert relerr(host(gk), oracle.kappa_grad(pro, uo, r)) <= 1e-11
    assert relerr(host(gu), oracle.apply(pro, r)) <= 1e-11


def test_torch_gradcheck_tiny(gpu_lib):
    from paper_2109_05072_amd.autograd import MFHexDiffusion
    op, pr = build(gpu_lib, 2, 1, 1, 1, "diffusion", "gauss", False, vark=True)
    kap = dev(synth.kappa_field(host(op.qpoint_coords()))).requires_grad_(True)
    u = dev(synth.uniform_vector(pr.n_nodes)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: MFHexDiffusion.apply(a, b, op), (u, kap), eps=1e-6, atol=1e-8)


# --- CG -------------------------------------------------------------------------------------

def test_config0_fifty_cg_iterations_match_oracle(gpu_lib):
    # 4x4x4 perturbed mesh, p = 2, Gauss q = 4, Dirichlet, 50 iterations from x0 = 0
    op, pr = build(gpu_lib, 4, 4, 4, 2)
    assert op.n_nodes == 729
    x = synth.uniform_vector(pr.n_nodes)
    assert relerr(host(op.apply(dev(x))), oracle.apply(pr, x)) <= TOL64
    b = synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr)
    xo, ho, it, _ = oracle.cg(pr, b, maxit=50, rtol=0.0)
    assert it == 50
    res = op.cg(dev(b), maxit=50, rtol=0.0, exact_iters=True)
    xg = host(res.x)
    print("config0 x50 rel diff", relerr(xg, xo), "history max rel diff", relerr(res.history, ho))
    assert res.iters == 50
    # the stated FP64 target; the measured agreement is printed above (round-off level, 1e-15)
    assert relerr(xg, xo) <= 1e-12
    assert np.all(np.abs(res.history - ho) <= 1e-12 * ho + 1e-14 * ho[0])


def _masked_rhs(op, pr):
    f = synth.sin_forcing(host(op.qpoint_coords()))
    return op.rhs(dev(f))


@pytest.mark.parametrize("p", [2, 3])
def test_cg_solution_and_mixed_precision(gpu_lib, p):
    ne = 12 if p == 2 else 8
    op, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, f32=True, rhs=True)
    b = _masked_rhs(op, pr)
    r64 = op.cg(b, maxit=5000, rtol=1e-10, mode="f64")
    rmx = op.cg(b, maxit=5000, rtol=1e-10, mode="mixed")
    print("f64", r64.iters, r64.rel_resid_true, r64.seconds, "mixed", rmx.iters, rmx.replacements,
          rmx.rel_resid_true, rmx.seconds, rmx.fell_back_to_f64)
    assert r64.status == 0 and r64.rel_resid_true <= 1e-10
    assert rmx.status == 0 and rmx.rel_resid_true <= 1e-10
    x64, xmx = host(r64.x), host(rmx.x)
    # against the oracle's own solve of its own load vector
    fo = synth.sin_forcing(oracle.qpoint_geometry(pr)[0])
    bo = oracle.rhs(pr, fo)
    assert relerr(host(b), bo) <= TOL64
    xo, _, _, _ = oracle.cg(pr, bo, maxit=5000, rtol=1e-12)
    print("err f64 vs oracle", relerr(x64, xo), "err mixed vs oracle", relerr(xmx, xo))
    assert relerr(x64, xo) <= 1e-7
    assert relerr(xmx, xo) <= 1e-7
    # discretization error against the exact solution is far above the solver error
    ue = synth.sin_solution(host(op.node_coords()))
    assert np.abs(x64 - ue).max() < 1e-2


@pytest.mark.parametrize("p,ne", [(5, 4), (7, 3)], ids=["p5-q7", "p7-q9"])
def test_mixed_cg_at_high_order_matches_oracle(gpu_lib, p, ne):
    # mixed-precision CG at two of the mixed-CG orders (FP32 operator at q = 7 and q = 9): the
    # oracle's own operator confirms the true residual of the GPU solution, and the solution is
    # compared with the oracle's CG solve of the oracle's load vector
    op, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, f32=True, rhs=True)
    b = _masked_rhs(op, pr)
    bo = oracle.rhs(pr, synth.sin_forcing(oracle.qpoint_geometry(pr)[0]))
    assert relerr(host(b), bo) <= TOL64
    rmx = op.cg(b, maxit=20000, rtol=1e-10, mode="mixed")
    r64 = op.cg(b, maxit=20000, rtol=1e-10, mode="f64")
    assert rmx.status == 0 and rmx.rel_resid_true <= 1e-10
    assert r64.status == 0 and r64.rel_resid_true <= 1e-10
    xmx, x64 = host(rmx.x), host(r64.x)
    res_orc = float(np.linalg.norm(bo - oracle.apply(pr, xmx)) / np.linalg.norm(bo))
    xo, _, _, code = oracle.cg(pr, bo, maxit=20000, rtol=1e-13)
    assert code == oracle.OK
    e_mx, e_64 = relerr(xmx, xo), relerr(x64, xo)
    print(f"mixed p={p}: {rmx.iters} it, {rmx.replacements} replacements, fallback {rmx.fell_back_to_f64}, "
          f"true residual (library) {rmx.rel_resid_true:.3e}, (oracle operator) {res_orc:.3e}, "
          f"err vs oracle CG {e_mx:.3e} (FP64 CG {e_64:.3e})", flush=True)
    # the oracle's operator sees the residual the library reports (to rounding of the two applies)
    assert res_orc <= 1.01e-10
    # both solutions sit within the solver tolerance of the oracle's, amplified by the condition
    # number of these small meshes (measured errors are printed above)
    assert e_mx <= 1e-6 and e_64 <= 1e-6


# --- CG status paths --------------------------------------------------------------------------

def test_cg_reports_maxit_as_noconv(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 4, 4, 4, 2, f32=True)
    b = dev(synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr))
    for mode in ("f64", "mixed"):
        res = op.cg(b, maxit=7, rtol=1e-14, mode=mode)
        print("noconv", mode, res.status, res.iters, res.rel_resid_true)
        assert res.status == L.MFHEX_ERR_NOCONV
        assert res.iters == 7
        # x and the statistics stay valid: the reported residual is that of the returned x
        xo = host(res.x)
        true = float(np.linalg.norm(host(b) - oracle.apply(pr, xo)) / np.linalg.norm(host(b)))
        assert abs(true - res.rel_resid_true) <= 1e-8 * true
        assert 1e-14 < res.rel_resid_true < 1.0


def test_cg_non_finite_rhs_is_breakdown(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 3, 3, 3, 2, f32=True)
    bh = synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr)
    bh[pr.n_nodes // 2] = np.nan
    for mode in ("f64", "mixed"):
        with pytest.raises(L.MFHexError) as ei:
            op.cg(dev(bh), maxit=50, rtol=1e-10, mode=mode)
        assert ei.value.code == L.MFHEX_ERR_BREAKDOWN


def test_cg_negative_coefficient_is_breakdown(gpu_lib):
    # kappa < 0 makes the operator negative definite: p^T A p < 0 at the first iteration
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 3, 3, 3, 2, vark=True)
    op.set_kappa(-torch.ones(op.n_elem * op.q ** 3, dtype=torch.float64, device="cuda"))
    b = dev(synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr))
    with pytest.raises(L.MFHexError) as ei:
        op.cg(b, maxit=50, rtol=1e-10)
    assert ei.value.code == L.MFHEX_ERR_BREAKDOWN
    # the same operator with kappa > 0 converges
    op.set_kappa(torch.ones(op.n_elem * op.q ** 3, dtype=torch.float64, device="cuda"))
    assert op.cg(b, maxit=500, rtol=1e-10).status == 0


def test_mixed_cg_falls_back_to_fp64_when_replacements_stall(gpu_lib):
    # a tolerance below FP64 round-off: the true residual stops falling near 1e-16, three residual
    # replacements in a row without progress hand the solve to FP64 CG, which then runs to maxit
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 3, 3, 3, 2, f32=True)
    b = dev(synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr))
    res = op.cg(b, maxit=1500, rtol=1e-17, mode="mixed", replace_every=20)
    print("fallback", res.status, res.iters, res.replacements, res.fell_back_to_f64, res.rel_resid_true)
    assert res.fell_back_to_f64
    assert res.status == L.MFHEX_ERR_NOCONV and res.iters == 1500
    assert res.replacements >= 3
    assert res.rel_resid_true <= 1e-13
    xo, _, _, _ = oracle.cg(pr, host(b), maxit=1500, rtol=1e-14)
    assert relerr(host(res.x), xo) <= 1e-11


# --- geometric factors evaluated in the kernel (no stored factors) ---------------------------

@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("quad", ["gauss", "gll"])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_otf_apply_matches_oracle_and_stored_factors(gpu_lib, p, quad, dirichlet):
    _say("otf", p, quad, dirichlet)
    op, pr = build(gpu_lib, 3, 2, 2, p, "diffusion", quad, dirichlet, otf=True)
    ref, _ = build(gpu_lib, 3, 2, 2, p, "diffusion", quad, dirichlet)
    x = synth.uniform_vector(pr.n_nodes)
    yo = oracle.apply(pr, x)
    ys = host(ref.apply(dev(x)))
    for v in valid_variants(op):
        op.set_config(v)
        ref.set_config(v)
        _say("otf variant", v, op.get_config())
        y = host(op.apply(dev(x)))
        assert relerr(y, yo) <= TOL64
        # same factor expressions as the set-up kernel: equal to the stored-factor apply up to rounding
        assert relerr(y, host(ref.apply(dev(x)))) <= 1e-14
    assert relerr(ys, yo) <= TOL64


def test_otf_workspace_has_no_factor_array_and_rejects_what_needs_one(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 4, 3, 2, 3, "diffusion", "gauss", True, otf=True)
    ref, _ = build(gpu_lib, 4, 3, 2, 3, "diffusion", "gauss", True)
    assert ref.sizes.workspace_bytes - op.sizes.workspace_bytes >= 24 * 6 * 125 * 8
    with pytest.raises(L.MFHexError) as ei:
        op.diagonal()
    assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED
    u = dev(synth.uniform_vector(pr.n_nodes, seed=4))
    with pytest.raises(L.MFHexError) as ei:
        op.kappa_grad(u, u)
    assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED
    for kw in (dict(kind="mass", dirichlet=False), dict(vark=True), dict(f32=True)):
        with pytest.raises(L.MFHexError) as ei:
            build(gpu_lib, 2, 2, 2, 2, otf=True, **kw)
        assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED
    # the solver runs on it (unpreconditioned)
    b = dev(synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr))
    res = op.cg(b, maxit=2000, rtol=1e-10)
    xo, _, _, _ = oracle.cg(pr, host(b), maxit=2000, rtol=1e-12)
    assert res.status == 0 and relerr(host(res.x), xo) <= 1e-7


# --- operator diagonal and Jacobi-preconditioned CG -----------------------------------------

@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("kind,quad", [("diffusion", "gauss"), ("diffusion", "gll"), ("mass", "gauss")])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_diagonal_matches_oracle(gpu_lib, p, kind, quad, dirichlet):
    _say("diagonal", p, kind, quad, dirichlet)
    op, pr = build(gpu_lib, 3, 2, 2, p, kind, quad, dirichlet)
    d = host(op.diagonal())
    assert relerr(d, oracle.diagonal(pr)) <= TOL64
    if dirichlet:
        inner = interior_mask(pr) > 0
        assert np.all(d[~inner] == 0.0) and np.all(d[inner] > 0.0)


@pytest.mark.parametrize("p,quad", [(2, "gauss"), (5, "gauss"), (3, "gll")])
def test_diagonal_variable_kappa_matches_oracle(gpu_lib, p, quad):
    op, pr = build(gpu_lib, 3, 2, 2, p, "diffusion", quad, True, vark=True)
    kap = synth.kappa_field(host(op.qpoint_coords()))
    pr = pr.with_(kappa=synth.kappa_field(oracle.qpoint_geometry(pr)[0]))
    op.set_kappa(dev(kap))
    assert relerr(host(op.diagonal()), oracle.diagonal(pr)) <= TOL64


def test_config0_fifty_pcg_iterations_match_oracle(gpu_lib):
    # config-0 mesh (4x4x4, p = 2, Gauss q = 4, Dirichlet), 50 Jacobi-preconditioned iterations
    op, pr = build(gpu_lib, 4, 4, 4, 2)
    b = synth.uniform_vector(pr.n_nodes, seed=3) * interior_mask(pr)
    dinv = oracle.jacobi_inverse(oracle.diagonal(pr))
    xo, ho, it, _ = oracle.pcg(pr, b, dinv, maxit=50, rtol=0.0)
    assert it == 50
    res = op.cg(dev(b), maxit=50, rtol=0.0, exact_iters=True, precond="jacobi")
    xg = host(res.x)
    print("config0 pcg x50 rel diff", relerr(xg, xo), "history max rel diff", relerr(res.history, ho))
    assert res.iters == 50
    assert relerr(xg, xo) <= 1e-12
    assert np.all(np.abs(res.history - ho) <= 1e-12 * ho + 1e-14 * ho[0])


@pytest.mark.parametrize("p", [2, 3])
def test_pcg_solution_and_mixed_precision(gpu_lib, p):
    ne = 12 if p == 2 else 8
    op, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, f32=True, rhs=True)
    b = _masked_rhs(op, pr)
    r0 = op.cg(b, maxit=5000, rtol=1e-10, mode="f64")
    r64 = op.cg(b, maxit=5000, rtol=1e-10, mode="f64", precond="jacobi")
    rmx = op.cg(b, maxit=5000, rtol=1e-10, mode="mixed", precond="jacobi")
    print("cg", r0.iters, "pcg f64", r64.iters, r64.rel_resid_true, "pcg mixed", rmx.iters, rmx.replacements,
          rmx.rel_resid_true, rmx.fell_back_to_f64)
    assert r64.status == 0 and r64.rel_resid_true <= 1e-10
    assert rmx.status == 0 and rmx.rel_resid_true <= 1e-10
    assert r64.iters <= r0.iters
    bo = oracle.rhs(pr, synth.sin_forcing(oracle.qpoint_geometry(pr)[0]))
    xo, _, _, code = oracle.pcg(pr, bo, oracle.jacobi_inverse(oracle.diagonal(pr)), maxit=5000, rtol=1e-12)
    assert code == oracle.OK
    assert relerr(host(r64.x), xo) <= 1e-7
    assert relerr(host(rmx.x), xo) <= 1e-7


def test_pcg_high_contrast_coefficient(gpu_lib):
    # kappa = 10^(4x): Jacobi removes the coefficient scale, far fewer iterations than plain CG
    op, pr = build(gpu_lib, 6, 6, 6, 2, "diffusion", "gauss", True, vark=True)
    xq = host(op.qpoint_coords())
    kap = 10.0 ** (4.0 * xq[:, :, 0])
    op.set_kappa(dev(kap))
    pr = pr.with_(kappa=10.0 ** (4.0 * oracle.qpoint_geometry(pr)[0].reshape(pr.n_elem, -1, 3)[:, :, 0]))
    b = synth.uniform_vector(pr.n_nodes, seed=4) * interior_mask(pr)
    rc = op.cg(dev(b), maxit=20000, rtol=1e-10)
    rp = op.cg(dev(b), maxit=20000, rtol=1e-10, precond="jacobi")
    print("high contrast: cg", rc.iters, "pcg", rp.iters)
    assert rc.status == 0 and rp.status == 0
    assert rp.iters < 0.5 * rc.iters
    xo, _, _, _ = oracle.pcg(pr, b, oracle.jacobi_inverse(oracle.diagonal(pr)), maxit=20000, rtol=1e-12)
    assert relerr(host(rp.x), xo) <= 1e-7


def test_pcg_rejects_unknown_preconditioner(gpu_lib):
    import ctypes as C
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 2, 2, 2, 2)
    b = dev(synth.uniform_vector(pr.n_nodes) * interior_mask(pr))
    x = torch.zeros_like(b)
    work = torch.empty(int(op.sizes.cg_work_bytes) + 256, dtype=torch.uint8, device="cuda")
    wp = (work.data_ptr() + 255) & ~255
    opts = L.mfhex_cg_opts(maxit=10, check_every=1, mode=L.MFHEX_CG_F64, replace_every=100, x0_is_zero=1,
                           max_iters_exact=0, precond=7, rtol=1e-10, replace_delta=0.1)
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_cg(op.handle, b.data_ptr(), x.data_ptr(), wp, opts, None, torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == L.MFHEX_ERR_ARG


# --- p-multigrid preconditioner -------------------------------------------------------------

@pytest.mark.parametrize("p,quad", [(2, "gauss"), (3, "gauss"), (4, "gauss"), (5, "gauss"), (6, "gauss"),
                                    (7, "gauss"), (8, "gauss"), (4, "gll"), (7, "gll")])
def test_mg_levels_and_vcycle_match_oracle(gpu_lib, p, quad):
    from oracle import multigrid as omg
    _say("mg vcycle", p, quad)
    op, pr = build(gpu_lib, 3, 2, 2, p, "diffusion", quad, True)
    nl = op.mg_setup()
    h = omg.Hierarchy(pr)
    lv = op.mg_levels()
    assert nl == len(lv) == len(h.levels)
    for (pl, nl_nodes, lam), L in zip(lv, h.levels):
        assert pl == L["pr"].p and nl_nodes == L["pr"].n_nodes
        assert abs(lam - L["lam"]) <= 1e-10 * L["lam"]
    r = synth.uniform_vector(pr.n_nodes, seed=5) * interior_mask(pr)
    z = host(op.mg_apply(dev(r)))
    zo = h.vcycle(r)
    print("vcycle rel diff", relerr(z, zo))
    assert relerr(z, zo) <= 1e-9
    # symmetric preconditioner: u.M v == v.M u
    u = synth.uniform_vector(pr.n_nodes, seed=6) * interior_mask(pr)
    zu = host(op.mg_apply(dev(u)))
    assert abs(u @ z - r @ zu) <= 1e-11 * abs(u @ z)


@pytest.mark.parametrize("p,ne", [(3, 8), (5, 5), (8, 3)])
def test_mg_pcg_matches_oracle(gpu_lib, p, ne):
    from oracle import multigrid as omg
    op, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, rhs=True)
    op.mg_setup()
    b = _masked_rhs(op, pr)
    res = op.cg(b, maxit=500, rtol=1e-10, precond="mg")
    rj = op.cg(b, maxit=5000, rtol=1e-10, precond="jacobi")
    bo = oracle.rhs(pr, synth.sin_forcing(oracle.qpoint_geometry(pr)[0]))
    xo, ho, it_o = omg.mg_pcg(omg.Hierarchy(pr), bo, maxit=500, rtol=1e-10)
    print("mg pcg", p, ne, "iters", res.iters, "oracle", it_o, "jacobi", rj.iters)
    assert res.status == 0 and res.rel_resid_true <= 1e-10
    assert abs(res.iters - it_o) <= 2
    assert res.iters < 0.3 * rj.iters
    assert relerr(host(res.x), xo) <= 1e-7


@pytest.mark.parametrize("p,quad", [(2, "gauss"), (3, "gauss"), (5, "gauss"), (8, "gauss"), (6, "gll")])
def test_mg_fp32_vcycle_matches_oracle(gpu_lib, p, quad):
    # FP32 V-cycle against the FP64 oracle cycle: set-up (diagonals, power method) is FP64 in both,
    # so the level eigenvalue estimates agree to FP64 rounding; the cycle is a chain of some forty
    # FP32 operator applies and vector updates, each adding about one unit roundoff (2^-24) of
    # relative error to a result of the same scale, so the cycle is held to 40 x 2^-24.
    from oracle import multigrid as omg
    _say("mg vcycle fp32", p, quad)
    op, pr = build(gpu_lib, 3, 2, 2, p, "diffusion", quad, True, f32=True)
    op.mg_setup(dtype=torch.float32)
    h = omg.Hierarchy(pr)
    for (pl, nl_nodes, lam), L in zip(op.mg_levels(), h.levels):
        assert pl == L["pr"].p and abs(lam - L["lam"]) <= 1e-10 * L["lam"]
    r = synth.uniform_vector(pr.n_nodes, seed=5) * interior_mask(pr)
    z = host(op.mg_apply(dev(r)))
    zo = h.vcycle(r)
    print("fp32 vcycle rel diff", relerr(z, zo))
    assert relerr(z, zo) <= 40 * 2.0 ** -24
    assert np.all(z[interior_mask(pr) == 0] == 0.0)


@pytest.mark.parametrize("p,ne", [(3, 8), (6, 4)])
def test_mg_fp32_pcg_converges_like_fp64(gpu_lib, p, ne):
    # FP64 CG with the FP32 V-cycle as preconditioner reaches the same FP64 residual; the
    # preconditioner is the FP64 one perturbed at FP32 rounding, so the iteration count stays
    # within a few of the oracle's FP64-preconditioned count.
    from oracle import multigrid as omg
    op, pr = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, f32=True, rhs=True)
    op.mg_setup(dtype=torch.float32)
    b = _masked_rhs(op, pr)
    res = op.cg(b, maxit=500, rtol=1e-10, precond="mg")
    bo = oracle.rhs(pr, synth.sin_forcing(oracle.qpoint_geometry(pr)[0]))
    xo, ho, it_o = omg.mg_pcg(omg.Hierarchy(pr), bo, maxit=500, rtol=1e-10)
    print("mg32 pcg", p, ne, "iters", res.iters, "oracle", it_o)
    assert res.status == 0 and res.rel_resid_true <= 1e-10
    assert res.iters <= it_o + 3
    assert relerr(host(res.x), xo) <= 1e-7


def test_mg_rejects_what_it_does_not_support(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, 2, 2, 2, 2)
    b = dev(synth.uniform_vector(pr.n_nodes) * interior_mask(pr))
    with pytest.raises(L.MFHexError) as ei:
        op.cg(b, precond="mg")  # no hierarchy yet
    assert ei.value.code == L.MFHEX_ERR_STATE
    for kw in (dict(kind="mass", dirichlet=False), dict(otf=True), dict(vark=True)):
        o2, _ = build(gpu_lib, 2, 2, 2, 2, **kw)
        with pytest.raises(L.MFHexError) as ei:
            o2.mg_setup()
        assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED
    with pytest.raises(L.MFHexError) as ei:
        op.mg_setup(dtype=torch.float32)  # FP32 cycle on an operator without FP32 data
    assert ei.value.code == L.MFHEX_ERR_ARG
    o3, _ = build(gpu_lib, 2, 2, 2, 3, f32=True)
    o3.mg_setup()
    with pytest.raises(L.MFHexError) as ei:
        o3.cg(dev(synth.uniform_vector(o3.n_nodes) * interior_mask(pr.with_(p=3, q=5))), mode="mixed", precond="mg")
    assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED


# --- error paths -----------------------------------------------------------------------------

def test_error_paths(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    vert = synth.mesh_vertices(3, 3, 3, perturb=0.7)
    with pytest.raises(L.MFHexError) as ei:
        gpu_lib.Operator(3, 3, 3, 2, vert)
    assert ei.value.code == L.MFHEX_ERR_MESH
    op, pr = build(gpu_lib, 2, 2, 2, 2)
    x = dev(synth.uniform_vector(pr.n_nodes))
    with pytest.raises(L.MFHexError) as ei:
        op.apply(x.float())
    assert ei.value.code == L.MFHEX_ERR_STATE
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_apply(op.handle, L.MFHEX_F64, 1, x.data_ptr(), x.data_ptr() + 8, 0)
    assert ei.value.code == L.MFHEX_ERR_ARG
    opk, _ = build(gpu_lib, 2, 2, 2, 2, vark=True)
    with pytest.raises(L.MFHexError) as ei:
        opk.apply(x)
    assert ei.value.code == L.MFHEX_ERR_STATE
    # one element, p = 1, Dirichlet: every node is on the boundary -> y = 0
    op1, pr1 = build(gpu_lib, 1, 1, 1, 1)
    y = host(op1.apply(dev(synth.uniform_vector(pr1.n_nodes))))
    assert np.all(y == 0.0)


# --- full-size, sampled against the oracle one output at a time -----------------------------

def _window_value(vert_full, nex, ney, nez, p, quad, kind, dirichlet, x_full, node):
    """(A x)[node] from the oracle on the <= 2x2x2 elements around the node.  x_full: the host
    vector ([N] or [N][nvec]), or a function returning its rows at given node numbers."""
    nx, ny = p * nex + 1, p * ney + 1
    I, J, K = node % nx, (node // nx) % ny, node // (nx * ny)
    lo, hi = [], []
    for L_, ne in ((I, nex), (J, ney), (K, nez)):
        a = max(0, (L_ - 1) // p) if L_ % p == 0 else L_ // p
        b = min(ne - 1, L_ // p)
        lo.append(a)
        hi.append(b)
    wx, wy, wz = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1
    V = vert_full.reshape(nez + 1, ney + 1, nex + 1, 3)
    wv = V[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2].reshape(-1, 3)
    q = p + 2 if quad == oracle.GAUSS else p + 1
    pr = oracle.Problem(wx, wy, wz, p, q, quad, kind, 0, np.ascontiguousarray(wv))
    lnx, lny, lnz = p * wx + 1, p * wy + 1, p * wz + 1
    gi = np.arange(lnx)[None, None, :] + p * lo[0]
    gj = np.arange(lny)[None, :, None] + p * lo[1]
    gk = np.arange(lnz)[:, None, None] + p * lo[2]
    gid = (gi + nx * (gj + ny * gk)).reshape(-1)
    xw = x_full(gid) if callable(x_full) else x_full[gid].copy()
    if dirichlet:
        Gi, Gj, Gk = gid % nx, (gid // nx) % ny, gid // (nx * ny)
        bnd = (Gi == 0) | (Gi == nx - 1) | (Gj == 0) | (Gj == ny - 1) | (Gk == 0) | (Gk == p * nez)
        xw[bnd] = 0.0
    yw = oracle.apply(pr, xw)
    li = (I - p * lo[0]) + lnx * ((J - p * lo[1]) + lny * (K - p * lo[2]))
    return yw[li]


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("kind", ["diffusion", "mass", "diffusion-otf"])
def test_full_size_sampled_against_oracle(gpu_lib, p, kind):
    """The benchmark's operators (about 1e7 nodes, default launch configuration) sampled node by
    node: random nodes, nodes near corners, and nodes on the x-faces inside and between element
    groups (summed on chip before one atomic)."""
    ne = synth.elems_for_dofs(1e7, p)
    otf = kind == "diffusion-otf"
    kind = "diffusion" if otf else kind
    dirichlet = kind == "diffusion"
    _say("full size", p, kind, otf, ne)
    op, _ = build(gpu_lib, ne, ne, ne, p, kind, "gauss", dirichlet, otf=otf)
    _say("launch", op.get_config())
    vert = synth.mesh_vertices(ne, ne, ne)
    x = synth.uniform_vector(op.n_nodes)
    y = host(op.apply(dev(x)))
    rng = np.random.default_rng(17)
    n = p * ne + 1
    nodes = list(rng.integers(0, op.n_nodes, size=20))
    nodes += [1 + n + n * n, (n - 2) + n * (n - 2) + n * n * (n - 2), p + n * p + n * n * p]  # near corners, vertex
    J = K = 2 * p + 1
    nodes += [m * p + n * (J + n * K) for m in range(1, 10)]  # x-faces of the first element groups of a row
    nodes += [m * p + n * (p * 3 + n * p * 5) for m in range(1, 10)]  # ... on element edges in y and z too
    scale = np.abs(y).max()
    kd = oracle.DIFFUSION if kind == "diffusion" else oracle.MASS
    for node in nodes:
        I, J_, K_ = node % n, (node // n) % n, node // (n * n)
        if dirichlet and (min(I, J_, K_) == 0 or max(I, J_, K_) == n - 1):
            assert y[node] == 0.0
            continue
        yo = _window_value(vert, ne, ne, ne, p, oracle.GAUSS, kd, dirichlet, x, node)
        assert abs(y[node] - yo) <= TOL64 * scale, (node, y[node], yo)


@pytest.mark.parametrize("p,ncomp,nrhs", [(3, 3, 32), (5, 1, 8), (8, 3, 4)])
def test_batched_full_size_sampled_against_oracle(gpu_lib, p, ncomp, nrhs):
    """Collocated BP5 / BP6 at the batched benchmark's size (about 3e7 nodes per field), the default
    launch and every multi-vector variant (the candidates of the tuner), sampled node by node with
    all vectors of each sampled node."""
    ne = synth.elems_for_dofs(3e7, p)
    nvec = ncomp * nrhs
    _say("batched full size", p, ncomp, nrhs, ne)
    op, _ = build(gpu_lib, ne, ne, ne, p, "diffusion", "gll", True, ncomp=ncomp)
    vert = synth.mesh_vertices(ne, ne, ne)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_VEC)
    x = torch.rand(op.n_nodes, nvec, generator=gen, dtype=torch.float64, device="cuda").mul_(2).sub_(1)
    y = torch.empty_like(x)
    n = p * ne + 1
    rng = np.random.default_rng(23)
    nodes = [int(v) for v in rng.integers(0, op.n_nodes, size=12)]
    nodes += [1 + n + n * n, (n - 2) + n * (n - 2) + n * n * (n - 2)]
    nodes += [m * p + n * (2 * p + 1 + n * (2 * p + 1)) for m in range(1, 6)]  # x-faces inside and between groups
    on_bnd = np.array([min(v % n, v // n % n, v // (n * n)) == 0 or max(v % n, v // n % n, v // (n * n)) == n - 1
                       for v in nodes])
    rows = lambda gid: x[torch.from_numpy(gid).to("cuda")].cpu().numpy()
    # Dirichlet rows are exactly zero; the others come from the oracle on the elements around the node
    ref = np.stack([np.zeros(nvec) if b else
                    _window_value(vert, ne, ne, ne, p, oracle.GLL, oracle.DIFFUSION, True, rows, v)
                    for v, b in zip(nodes, on_bnd)])
    idx = torch.tensor(nodes, device="cuda")

    def check(tag):
        op.apply(x, y)
        ys = host(y[idx])
        assert np.all(ys[on_bnd] == 0.0), tag
        scale = y.abs().max().item()
        err = np.abs(ys - ref).max() / scale
        print("batched sampled rel err", p, ncomp, nrhs, tag, err)
        assert err <= TOL64, tag

    _say("launch", op.get_config(nrhs=nrhs))
    check("default")
    for v in [v for v in valid_variants(op, nrhs=nrhs) if v >= 5]:
        op.set_config(v, nrhs=nrhs)
        _say("launch", op.get_config(nrhs=nrhs))
        check(v)


def test_kappa_gradient_full_size(gpu_lib):
    """The adjoint workload at its size (p = 4, Gauss q = 6, about 1e7 nodes): the coefficient
    gradient sampled element by element against the oracle on that element alone (inputs masked
    as in the full operator), and the loss 0.5 ||A(kappa) u - f||^2 differentiated along random
    directions by central differences (exact for a loss quadratic in kappa and in u)."""
    from paper_2109_05072_amd.autograd import diffusion
    p = 4
    ne = synth.elems_for_dofs(1e7, p)
    _say("kappa gradient full size", p, ne)
    op, _ = build(gpu_lib, ne, ne, ne, p, "diffusion", "gauss", True, vark=True)
    vert = synth.mesh_vertices(ne, ne, ne)
    n = p * ne + 1
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_VEC)
    u = torch.rand(op.n_nodes, generator=gen, dtype=torch.float64, device="cuda").mul_(2).sub_(1)
    r = torch.rand(op.n_nodes, generator=gen, dtype=torch.float64, device="cuda").mul_(2).sub_(1)
    g = op.kappa_grad(u, r)
    scale = g.abs().max().item()
    rng = np.random.default_rng(29)
    elems = [int(e) for e in rng.integers(0, op.n_elem, size=16)] + [0, op.n_elem - 1, ne * ne * (ne // 2) + ne // 2]
    V = vert.reshape(ne + 1, ne + 1, ne + 1, 3)
    ii = np.arange(p + 1)
    for e in elems:
        ex, ey, ez = e % ne, (e // ne) % ne, e // (ne * ne)
        pr = oracle.Problem(1, 1, 1, p, p + 2, oracle.GAUSS, oracle.DIFFUSION, 0,
                            np.ascontiguousarray(V[ez:ez + 2, ey:ey + 2, ex:ex + 2].reshape(-1, 3)))
        I = (p * ex + ii)[None, None, :]
        J = (p * ey + ii)[None, :, None]
        K = (p * ez + ii)[:, None, None]
        gid = (I + n * (J + n * K)).reshape(-1)
        bnd = ((I == 0) | (I == n - 1) | (J == 0) | (J == n - 1) | (K == 0) | (K == n - 1)).reshape(-1)
        ids = torch.from_numpy(gid).to("cuda")
        uw, rw = host(u[ids]), host(r[ids])
        uw[bnd] = 0.0
        rw[bnd] = 0.0
        go = oracle.kappa_grad(pr, uw, rw)[0]
        err = np.abs(host(g[e]) - go).max() / scale
        assert err <= TOL64, (e, err)
    # finite differences of the loss along random directions, in kappa and in u
    kap = torch.exp(0.5 * torch.rand(op.n_elem, op.q ** 3, generator=gen, dtype=torch.float64, device="cuda"))
    f = torch.rand(op.n_nodes, generator=gen, dtype=torch.float64, device="cuda")
    uu = u.clone().requires_grad_(True)
    k = kap.clone().requires_grad_(True)

    def loss(a, b):
        res = diffusion(a, b, op) - f
        return 0.5 * (res * res).sum()

    gu, gk = torch.autograd.grad(loss(uu, k), [uu, k])
    with torch.no_grad():
        for _ in range(2):
            d = torch.randn(kap.shape, generator=gen, dtype=torch.float64, device="cuda")
            eps = 1e-2 * float(kap.norm() / d.norm())
            fd = (loss(u, kap + eps * d) - loss(u, kap - eps * d)) / (2 * eps)
            an = (gk * d).sum()
            assert abs(float(fd - an)) <= 1e-9 * abs(float(an))
            du = torch.randn(op.n_nodes, generator=gen, dtype=torch.float64, device="cuda")
            eps = 1e-2 * float(u.norm() / du.norm())
            fd = (loss(u + eps * du, kap) - loss(u - eps * du, kap)) / (2 * eps)
            an = (gu * du).sum()
            assert abs(float(fd - an)) <= 1e-9 * abs(float(an))


# --- graph capture ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["bp3-f64", "bp3-f32", "bp6-gll-p8-4rhs", "bp1-mass", "tet-p4"])
def test_captured_apply_replays_match(gpu_lib, case):
    """The asynchronous applies only enqueue kernels (the output is cleared by a fill kernel, not a
    runtime memset), so a caller can record them into a graph.  The graph is replayed several times
    with eager work and synchronizations between the replays (new input, output set to garbage);
    every replay must match the oracle and an eager apply of the same input."""
    from oracle import tet as otet
    _say("graph", case)
    if case == "tet-p4":
        vert = synth.mesh_vertices(3, 3, 2, 0.1)
        op = gpu_lib.TetOperator(3, 3, 2, 4, vert)
        pr = otet.TetProblem(3, 3, 2, 4, 4, 1, vert)
        n, nvec, dt, tol, ref_of = pr.n_nodes, 1, torch.float64, TOL64, (lambda xh: otet.apply(pr, xh))
    else:
        # p = 4 on 3 x 3 x 2 elements: 1521 nodes, so the output is not a whole number of 16-byte words
        kw = {"bp3-f64": dict(p=4), "bp3-f32": dict(p=4, f32=True),
              "bp6-gll-p8-4rhs": dict(p=8, quad="gll", ncomp=3), "bp1-mass": dict(p=5, kind="mass")}[case]
        p = kw.pop("p")
        op, pr = build(gpu_lib, 3, 3, 2, p, **kw)
        nvec = 12 if case.startswith("bp6") else 1
        n = pr.n_nodes
        dt = torch.float32 if case == "bp3-f32" else torch.float64
        tol = TOL32 if dt == torch.float32 else TOL64
        ref_of = lambda xh: oracle.apply(pr, xh)
    shape = (n, nvec) if nvec > 1 else (n,)
    x = dev(synth.uniform_vector(n, nvec=nvec), dt).reshape(shape).contiguous()
    y = torch.empty_like(x)
    op.apply(x, y)  # eager call first: one-time launch set-up happens outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        op.apply(x, y)
    torch.cuda.synchronize()
    for k in range(4):
        x.copy_(dev(synth.uniform_vector(n, nvec=nvec, seed=100 + k), dt).reshape(shape))
        y.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        yr = host(y)
        assert relerr(yr, ref_of(host(x).astype(np.float64))) <= tol, k
        ye = host(op.apply(x))
        assert relerr(yr, ye) <= (1e-14 if dt == torch.float64 else 1e-6), k
