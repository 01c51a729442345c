"""ifgf_apply_noalloc (workspaces in the library's static per-GPU scratch
array, no allocation) against ifgf_apply on the same plan, through the C ABI:
two calls in a row, the second with a smaller input, to the parity bars."""
import math

import numpy as np
import pytest

from paper_2010_02857_amd import inputs

pytestmark = pytest.mark.gpu


def _rel(x, y):
    x, y = np.asarray(x), np.asarray(y)
    return max(float(np.linalg.norm(x - y) / np.linalg.norm(y)), float(np.max(np.abs(x - y)) / np.max(np.abs(y))))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_apply(prec):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_02857_amd import ifgf
    ifgf.lib()
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    tol = 1e-12 if prec == "fp64" else 1e-5
    # first call: N = 6144 with 4 right-hand sides; second: N = 1536, 1
    for n_face, k, nrhs, seed in ((32, 4.0 * math.pi, 4, 51), (16, 2.0 * math.pi, 1, 52)):
        p = inputs.cube_sphere(n_face)
        print(f"noalloc {prec} N={p.shape[0]} nrhs={nrhs}", flush=True)
        plan = ifgf.Plan(p, k, precision=prec, max_nrhs=16)
        x = torch.from_numpy(inputs.densities(seed, nrhs, p.shape[0])).to(dt).cuda()
        want = plan.apply(x)
        got = torch.full_like(want, float("nan"))
        plan.apply_noalloc(x, got)
        torch.cuda.synchronize()
        got, want = got.cpu().numpy(), want.cpu().numpy()
        assert np.isfinite(got).all()
        assert _rel(got, want) < tol
        assert np.array_equal(got, want)        # same kernels, same order
        assert plan.misses() == 0


def test_noalloc_rejects_oversized_plan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_02857_amd import ifgf
    p = inputs.cube_sphere(128)                 # N = 98304: workspaces beyond 256 MiB at 16 RHS
    plan = ifgf.Plan(p, 16.0 * math.pi, precision="fp64", max_nrhs=16)
    x = torch.zeros((16, p.shape[0]), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(ifgf.IFGFError) as e:
        plan.apply_noalloc(x, out)
    assert e.value.status == 1 and "scratch" in str(e.value)
