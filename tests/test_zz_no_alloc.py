"""The allocation-free apply (mfhex_apply_static, element values in the
library's own device buffer) against the deterministic apply of an operator
that owns its element buffer (mfhex_apply with MFHEX_FLAG_DETERMINISTIC), and
against the FP64 oracle, on calls in a row whose inputs shrink (the buffer
keeps the previous call's contents)."""
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


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _ops(mf, n, p, kind, quad, ncomp, f32=True, oracle_too=True):
    vert = synth.mesh_vertices(*n)
    kw = dict(kind=kind, quad=quad, ncomp=ncomp, dirichlet=kind == "diffusion", f32=f32)
    plain = mf.Operator(*n, p, vert, **kw)
    det = mf.Operator(*n, p, vert, deterministic=True, **kw)
    pr = None
    if oracle_too:
        q = p + 2 if quad == "gauss" else p + 1
        pr = oracle.Problem(*n, p, q, oracle.GAUSS if quad == "gauss" else oracle.GLL,
                            oracle.DIFFUSION if kind == "diffusion" else oracle.MASS, int(kind == "diffusion"), vert)
    return plain, det, pr


# larger first, then smaller: the second call reads a buffer that still holds the first call's values
CASES = [((7, 5, 4), 5, "diffusion", "gauss", 1),
         ((3, 2, 2), 2, "diffusion", "gauss", 1),
         ((3, 3, 2), 4, "diffusion", "gll", 3),
         ((2, 2, 1), 3, "mass", "gauss", 1)]


def test_static_apply_matches_deterministic_apply(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    assert L.mfhex_apply_static_max_bytes() == 64 << 20
    for n, p, kind, quad, ncomp in CASES:
        _say("static apply", n, p, kind, quad, ncomp)
        plain, det, pr = _ops(gpu_lib, n, p, kind, quad, ncomp)
        x = synth.uniform_vector(pr.n_nodes, nvec=ncomp, seed=11)
        yo = oracle.apply(pr, x)
        for dtype, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
            xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)
            # garbage in y first: the call must overwrite every entry
            y = torch.full_like(xd, float("nan"))
            plain.apply_static(xd, y)
            ys = _host(y)
            yd = _host(det.apply(xd))
            print(f"  {dtype}: static vs deterministic identical {np.array_equal(ys, yd)}, "
                  f"vs oracle {_relerr(ys, yo):.2e}", flush=True)
            assert np.array_equal(ys, yd)
            assert _relerr(ys, yo) <= tol
            # the deterministic operator may take the static buffer too
            y2 = torch.full_like(xd, float("nan"))
            det.apply_static(xd, y2)
            assert np.array_equal(_host(y2), yd)
        plain.close()
        det.close()


def test_static_apply_rejects_operators_above_the_buffer(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    # mass, p = 8, 24^3 elements: 13824 * 729 element values = 80.6 MB in FP64 (above 64 MiB), 40.3 MB in FP32
    _say("static apply size limit")
    plain, det, _ = _ops(gpu_lib, (24, 24, 24), 8, "mass", "gauss", 1, oracle_too=False)
    x = torch.from_numpy(synth.uniform_vector(plain.n_nodes, seed=5)).cuda()
    y = torch.full_like(x, 7.0)
    with pytest.raises(L.MFHexError) as ei:
        plain.apply_static(x, y)
    assert ei.value.code == L.MFHEX_ERR_ARG
    assert "67108864" in str(ei.value)
    assert bool((y == 7.0).all())  # nothing launched
    x32 = x.float()
    y32 = torch.full_like(x32, float("nan"))
    plain.apply_static(x32, y32)
    assert np.array_equal(_host(y32), _host(det.apply(x32)))
    # after the large FP32 call, a small FP64 call on another operator
    small, sdet, pr = _ops(gpu_lib, (2, 3, 2), 3, "diffusion", "gauss", 1)
    xs = synth.uniform_vector(pr.n_nodes, seed=6)
    ys = _host(small.apply_static(torch.from_numpy(xs).cuda()))
    assert np.array_equal(ys, _host(sdet.apply(torch.from_numpy(xs).cuda())))
    assert _relerr(ys, oracle.apply(pr, xs)) <= TOL64
    for o in (plain, det, small, sdet):
        o.close()
