"""Parity of the HIP library with the CPU oracle, element by element.

Bars: FP64 path within 1e-12 of the FP64 oracle IFGF; mixed path (FP32
arithmetic, FP64 geometry and phase reduction) within 1e-5 of the oracle run
on the same complex64-rounded inputs, each bar in both the relative l2 norm
and the relative infinity norm max|out - ref| / max|ref| (`par`); both paths
within 1e-3 relative l2 of the direct sum (the paper's eps_M).  Every test also checks that no interpolation query found its
cone missing.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2010_02857_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_02857_amd import ifgf
    ifgf.lib()        # the HIP library must be there: no fallback
    return t


def rel(x, y):
    """Relative l2 error (the paper's eps_M when y is the direct sum)."""
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(np.asarray(y)))


def rel_inf(x, y):
    """max_i |x_i - y_i| / max_i |y_i|: one entry off (a target interpolated
    in the wrong cone) shows at its own size, not diluted by the others."""
    x, y = np.asarray(x), np.asarray(y)
    return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))


def par(x, y):
    """Parity measure: the larger of the relative l2 and the relative
    infinity-norm errors, so each bar holds for both."""
    return max(rel(x, y), rel_inf(x, y))


def dev(torch, a, prec):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def as_c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def make_plan(p, k, prec="fp64", **kw):
    from paper_2010_02857_amd import ifgf
    print(f"plan N={p.shape[0]} k={k:.4g} prec={prec} {kw}", flush=True)
    return ifgf.Plan(p, k, precision=prec, **kw)


# ------------------------------------------------------------- workload 1

@pytest.fixture(scope="module")
def w1():
    w = inputs.WORKLOADS[1]
    p, a = w.points(), w.densities()
    return w, p, a, oracle.ifgf(p, a, w.kappa)["out"], oracle.direct(p, a, w.kappa)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cfg1_matches_oracle(torch, w1, prec):
    w, p, a, ref, direct = w1
    plan = make_plan(p, w.kappa, prec)
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    if prec == "fp64":
        assert par(out, ref) < FP64_TOL
    else:
        assert par(out, oracle.ifgf(p, as_c64(a), w.kappa)["out"]) < MIXED_TOL
    assert rel(out, direct) < 1e-3
    assert plan.misses() == 0


def test_cfg1_repeatable_and_plan_reuse(torch, w1):
    w, p, a, ref, _ = w1
    plan = make_plan(p, w.kappa)
    x = dev(torch, a, "fp64")
    o1 = plan.apply(x).cpu().numpy()
    o2 = plan.apply(x).cpu().numpy()
    assert np.array_equal(o1, o2)          # gather-only kernels: bitwise repeatable


@pytest.mark.parametrize("prec,nrhs", [("fp64", 2), ("fp64", 3), ("fp64", 16), ("fp64", 20), ("mixed", 3),
                                       ("mixed", 5), ("mixed", 16)])
def test_batched_rhs(torch, prec, nrhs):
    """Several density vectors per call (padded to 1/4/16 per pass; more
    than 16 in several passes) equal the oracle vector by vector."""
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(11, nrhs, p.shape[0])
    plan = make_plan(p, k, prec, max_nrhs=32)
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    ref = oracle.ifgf(p, a if prec == "fp64" else as_c64(a), k)["out"]
    for r in range(nrhs):
        assert par(out[r], ref[r]) < (FP64_TOL if prec == "fp64" else MIXED_TOL), r
    assert plan.misses() == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint(torch, w1, prec):
    """Adjoint = the same hierarchy with the conjugated kernel: equals
    conj(IFGF(conj v)) of the oracle, and the exact adjoint to eps."""
    w, p, _, _, _ = w1
    v = inputs.densities(21, 2, p.shape[0])
    plan = make_plan(p, w.kappa, prec)
    out = plan.adjoint(dev(torch, v, prec)).cpu().numpy()
    vv = v if prec == "fp64" else as_c64(v)
    ref = np.conj(oracle.ifgf(p, np.conj(vv), w.kappa)["out"])
    assert par(out, ref) < (FP64_TOL if prec == "fp64" else MIXED_TOL)
    exact = np.conj(oracle.direct(p, np.conj(vv), w.kappa))
    assert rel(out, exact) < 1e-3
    assert plan.misses() == 0


@pytest.mark.parametrize("prec,store", [("fp64", 1), ("fp64", 0), ("mixed", 1), ("mixed", 0)])
def test_grad_targets(torch, w1, prec, store):
    """Target-coordinate gradient sum_r Re(conj(g_r) dI_r/dx) equals the
    oracle's differentiated interpolants, with cone values stored by the
    forward call or recomputed."""
    w, p, a, _, _ = w1
    g = inputs.densities(31, 1, p.shape[0])
    aa, gg = (a, g) if prec == "fp64" else (as_c64(a), as_c64(g))
    r = oracle.ifgf(p, aa, w.kappa, grad=True)
    want = np.einsum("rn,rnc->nc", np.conj(gg), r["grad"]).real
    plan = make_plan(p, w.kappa, prec, store_levels=store)
    x = dev(torch, a, prec)
    plan.apply(x)
    got = plan.grad_targets(x, dev(torch, g, prec)).cpu().numpy()
    assert par(got, want) < (1e-10 if prec == "fp64" else 1e-4)
    exact = np.einsum("rn,rnc->nc", np.conj(gg), oracle.direct_grad(p, aa, w.kappa)).real
    assert rel(got, exact) < 1e-2
    # the stored cone values of the forward call (reused when kept) give the
    # same answer as recomputing them
    got2 = plan.grad_targets(x, dev(torch, g, prec), stored=True).cpu().numpy()
    assert par(got2, got) < 1e-14
    assert plan.misses() == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grad_after_densities_change_in_place(torch, prec):
    """apply(x), then x overwritten in place (same pointer): the gradient
    call recomputes the cone values from the new contents, so it equals the
    gradient of a fresh plan that never saw the old densities."""
    p = inputs.cube_sphere(12)
    k = 3.0 * math.pi
    a_old = inputs.densities(32, 1, p.shape[0])
    a_new = inputs.densities(33, 1, p.shape[0])
    g = dev(torch, inputs.densities(34, 1, p.shape[0]), prec)
    plan = make_plan(p, k, prec, store_levels=1)
    x = dev(torch, a_old, prec)
    plan.apply(x)
    x.copy_(dev(torch, a_new, prec))
    got = plan.grad_targets(x, g).cpu().numpy()
    fresh = make_plan(p, k, prec, store_levels=1).grad_targets(dev(torch, a_new, prec), g).cpu().numpy()
    assert np.array_equal(got, fresh)
    # and it differs from the gradient of the old densities
    old = make_plan(p, k, prec).grad_targets(dev(torch, a_old, prec), g).cpu().numpy()
    assert rel(got, old) > 1e-2


def test_grad_more_than_16_rhs(torch):
    """20 right-hand sides run in passes of 16 and 4; the gradient is the sum
    over all of them and equals the oracle's."""
    p = inputs.cube_sphere(12)
    k = 3.0 * math.pi
    nrhs = 20
    a = inputs.densities(35, nrhs, p.shape[0])
    g = inputs.densities(36, nrhs, p.shape[0])
    plan = make_plan(p, k, "fp64", max_nrhs=32)
    got = plan.grad_targets(dev(torch, a, "fp64"), dev(torch, g, "fp64")).cpu().numpy()
    r = oracle.ifgf(p, a, k, grad=True)
    want = np.einsum("rn,rnc->nc", np.conj(g), r["grad"]).real
    assert par(got, want) < 1e-10
    assert plan.misses() == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lattice_ties_and_poles(torch, prec):
    """17^3 lattice, D = 4: points on box faces, on cone faces (theta = pi/2,
    phi = k pi/2, ...) and on the polar axes of box centres, where phi is
    undefined.  Forward, adjoint and target gradient equal the oracle entry
    by entry (the infinity-norm bar catches a single target in another cone),
    and every gradient entry is finite (the polar-axis reading)."""
    p = inputs.lattice(17)
    n, k = p.shape[0], 8.0
    a = inputs.densities(37, 2, n)
    g = inputs.densities(38, 2, n)
    ac, gc = (a, g) if prec == "fp64" else (as_c64(a), as_c64(g))
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    r = oracle.ifgf(p, ac, k, levels=4, grad=True)
    plan = make_plan(p, k, prec, levels=4)
    x = dev(torch, a, prec)
    out = plan.apply(x).cpu().numpy()
    assert par(out, r["out"]) < tol
    adj = plan.adjoint(dev(torch, g, prec)).cpu().numpy()
    assert par(adj, np.conj(oracle.ifgf(p, np.conj(gc), k, levels=4)["out"])) < tol
    got = plan.grad_targets(x, dev(torch, g, prec)).cpu().numpy()
    assert np.isfinite(got).all()
    want = np.einsum("rn,rnc->nc", np.conj(gc), r["grad"]).real
    assert par(got, want) < (1e-10 if prec == "fp64" else 1e-4)
    assert plan.misses() == 0


@pytest.mark.parametrize("n_src,n_tgt", [(1536, 384), (384, 1536)])
def test_laplace_distinct_targets_adjoint(torch, n_src, n_tgt):
    """k = 0 with distinct targets, more sources than targets and the
    reverse: the adjoint maps [nrhs][n_targets] to [nrhs][n_sources] (the
    direction is explicit, not the sign of k, which is -0.0 here) and equals
    conj(oracle(conj v)) on the combined point set."""
    src = inputs.cube_sphere(int(math.isqrt(n_src // 6)))
    tgt = 1.25 * inputs.cube_sphere(int(math.isqrt(n_tgt // 6)))
    n, m = src.shape[0], tgt.shape[0]
    union = np.concatenate([src, tgt])
    v = inputs.densities(39, 2, m)
    a = inputs.densities(40, 2, n)
    plan = make_plan(src, 0.0, "fp64", targets=tgt)
    adj = plan.adjoint(dev(torch, v, "fp64")).cpu().numpy()
    assert adj.shape == (2, n)
    pad_v = np.concatenate([np.zeros((2, n), complex), v], axis=1)
    assert par(adj, np.conj(oracle.ifgf(union, np.conj(pad_v), 0.0)["out"])[:, :n]) < FP64_TOL
    out = plan.apply(dev(torch, a, "fp64")).cpu().numpy()
    assert out.shape == (2, m)
    pad_a = np.concatenate([a, np.zeros((2, m), complex)], axis=1)
    assert par(out, oracle.ifgf(union, pad_a, 0.0)["out"][:, n:]) < FP64_TOL
    assert plan.misses() == 0


def test_autograd_function(torch, w1):
    """loss = sum |I|^2 through torch.autograd: the density gradient is the
    adjoint applied to 2 I, the coordinate gradient the target gradient."""
    from paper_2010_02857_amd import ifgf
    w, p, a, _, _ = w1
    plan = make_plan(p, w.kappa, "fp64")
    x = dev(torch, a, "fp64").requires_grad_(True)
    t = torch.from_numpy(p).cuda().requires_grad_(True)
    out = ifgf.apply(plan, x, t)
    loss = (out.abs() ** 2).sum()
    loss.backward()
    I = out.detach()
    ga = plan.adjoint(2 * I).cpu().numpy()
    assert par(x.grad.cpu().numpy(), ga) < 1e-14
    gx = plan.grad_targets(x.detach(), 2 * I).cpu().numpy()
    assert par(t.grad.cpu().numpy(), gx) < 1e-14


# ------------------------------------------------------- small and degenerate

@pytest.mark.parametrize("case", ["n2", "n3", "cloud_d2", "cloud_d4", "cloud_d6", "laplace", "deg23", "deg46",
                                  "leaf23", "oblate", "nonuniform"])
def test_small_and_degenerate(torch, case):
    rng = np.random.default_rng(5)
    levels, deg, leaf, k = 0, (3, 5), (1, 2), 7.0
    if case == "n2":
        p = np.array([[0.1, 0.2, 0.3], [0.4, -0.2, 0.1]])
    elif case == "n3":
        p = np.array([[0.1, 0.2, 0.3], [0.4, -0.2, 0.1], [-1.0, 0.5, 0.0]])
        levels = 3
    elif case.startswith("cloud"):
        p = inputs.random_box_points(1500, 9)
        levels = int(case[-1])
        k = 30.0
    elif case == "laplace":
        p = inputs.cube_sphere(16)
        k = 0.0
    elif case == "deg23":
        p, deg = inputs.cube_sphere(16), (2, 3)
    elif case == "deg46":
        p, deg = inputs.cube_sphere(16), (4, 6)
    elif case == "leaf23":
        p, leaf = inputs.cube_sphere(16), (2, 3)
    elif case == "oblate":
        p, k = inputs.cube_sphere(24, 0.25), 6 * math.pi
    else:
        # clustered points: many in a few leaf boxes (ragged box sizes)
        p = np.concatenate([inputs.random_box_points(1200, 3, 0.05), inputs.random_box_points(300, 4, 2.0)])
        k, levels = 20.0, 6
    a = inputs.densities(41, 1, p.shape[0])
    plan = make_plan(p, k, "fp64", levels=levels, degrees=deg, leaf=leaf)
    out = plan.apply(dev(torch, a, "fp64")).cpu().numpy()
    ref = oracle.ifgf(p, a, k, levels=levels, degrees=deg, leaf=leaf)["out"]
    assert par(out, ref) < FP64_TOL
    assert plan.misses() == 0


@pytest.mark.parametrize("deg,prec,nrhs", [((1, 1), "fp64", 1), ((1, 4), "fp64", 4), ((2, 2), "mixed", 1),
                                            ((3, 4), "fp64", 16), ((5, 5), "mixed", 4), ((4, 7), "fp64", 2),
                                            ((8, 8), "fp64", 1), ((6, 3), "mixed", 16)])
def test_run_time_node_counts(torch, deg, prec, nrhs):
    """Node counts without compiled kernels (read at run time, any 1..8 per
    direction): forward, adjoint, target gradient and the no-allocation
    apply against the oracle; the error against the direct sum falls with
    the order (Thm. errorestimatenested)."""
    p = inputs.cube_sphere(14)
    k = 9.0
    a = inputs.densities(61, nrhs, p.shape[0])
    g = inputs.densities(62, nrhs, p.shape[0])
    ac, gc = (a, g) if prec == "fp64" else (as_c64(a), as_c64(g))
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    r = oracle.ifgf(p, ac, k, degrees=deg, grad=True)
    ref_adj = np.conj(oracle.ifgf(p, np.conj(ac), k, degrees=deg)["out"])
    plan = make_plan(p, k, prec, degrees=deg, max_nrhs=16, store_levels=0)
    assert plan.kernel_candidates(nrhs) == {d: ["geometry"] for d in plan.kernel_candidates(nrhs)}
    x = dev(torch, a, prec)
    out = plan.apply(x).cpu().numpy()
    assert par(out, r["out"]) < tol
    assert par(plan.adjoint(x).cpu().numpy(), ref_adj) < tol
    got = plan.grad_targets(x, dev(torch, g, prec)).cpu().numpy()
    want = np.einsum("rn,rnc->nc", np.conj(gc), r["grad"]).real
    assert par(got, want) < (1e-10 if prec == "fp64" else 1e-4)
    y = torch.empty_like(x)
    plan.apply_noalloc(x, y)
    assert par(y.cpu().numpy(), out) < (1e-14 if prec == "fp64" else 1e-6)
    assert plan.misses() == 0
    if deg == (8, 8):
        d = oracle.direct(p, ac, k)
        e88, e46 = rel(out, d), rel(oracle.ifgf(p, ac, k, degrees=(4, 6))["out"], d)
        assert e88 < 1e-5 and e88 < e46 / 10


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp64", 4), ("fp64", 16), ("mixed", 1), ("mixed", 4),
                                       ("mixed", 16)])
def test_without_frame_tables(torch, monkeypatch, prec, nrhs):
    """The kernels that compute the child-to-parent geometry themselves (used
    where the frame tables would not fit) give the same results."""
    monkeypatch.setenv("IFGF_NO_FRAMES", "1")
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(12, nrhs, p.shape[0])
    plan = make_plan(p, k, prec, max_nrhs=16)
    assert sum(plan.stats()["n_frames"]) == 0
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    ref = oracle.ifgf(p, a if prec == "fp64" else as_c64(a), k)["out"]
    assert par(out, ref) < (FP64_TOL if prec == "fp64" else MIXED_TOL)
    adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
    ref_adj = np.conj(oracle.ifgf(p, np.conj(a if prec == "fp64" else as_c64(a)), k)["out"])
    assert par(adj, ref_adj) < (FP64_TOL if prec == "fp64" else MIXED_TOL)
    assert plan.misses() == 0


@pytest.mark.parametrize("nrhs", [1, 4])
def test_box_batched_child_to_parent(torch, monkeypatch, nrhs):
    """Child-to-parent batched over the boxes of a parent cone (forced on at
    every level with frame tables, IFGF_BOX_FILL=0) and switched off
    (IFGF_BOX_FILL=2): both against the oracle, forward and adjoint, on a
    sphere (boxes with missing octants) and a ragged random cloud."""
    for pts, k in ((inputs.cube_sphere(20), 5.0 * math.pi), (inputs.random_box_points(5000, 7), 9.0)):
        a = as_c64(inputs.densities(13, nrhs, pts.shape[0]))
        ref = oracle.ifgf(pts, a, k)["out"]
        ref_adj = np.conj(oracle.ifgf(pts, np.conj(a), k)["out"])
        outs = {}
        for fill in ("0", "2"):
            monkeypatch.setenv("IFGF_BOX_FILL", fill)
            plan = make_plan(pts, k, "mixed", max_nrhs=16)
            outs[fill] = plan.apply(dev(torch, a, "mixed")).cpu().numpy()
            adj = plan.adjoint(dev(torch, a, "mixed")).cpu().numpy()
            assert par(outs[fill], ref) < MIXED_TOL
            assert par(adj, ref_adj) < MIXED_TOL
            assert plan.misses() == 0
        assert par(outs["0"], outs["2"]) < 1e-6
    monkeypatch.delenv("IFGF_BOX_FILL")


def test_autotune_and_kernel_choice(torch):
    """Autotuning picks, per level, one of the child-to-parent variants; the
    tuned plan still matches the oracle and the untuned plan."""
    from paper_2010_02857_amd import ifgf
    p = inputs.cube_sphere(24)
    k = 6.0 * math.pi
    for nrhs in (1, 4, 16):
        a = as_c64(inputs.densities(14, nrhs, p.shape[0]))
        plan = make_plan(p, k, "mixed", max_nrhs=16)
        before = plan.apply(dev(torch, a, "mixed")).cpu().numpy()
        default = plan.kernel_choice(nrhs)
        assert default and all(v in ifgf.Plan.C2P_VARIANTS for v in default.values())
        plan.autotune(nrhs)
        tuned = plan.kernel_choice(nrhs)
        assert set(tuned) == set(default)
        after = plan.apply(dev(torch, a, "mixed")).cpu().numpy()
        ref = oracle.ifgf(p, a, k)["out"]
        assert par(after, ref) < MIXED_TOL
        assert par(after, before) < 1e-6
        assert plan.misses() == 0
    plan64 = make_plan(p, k, "fp64", max_nrhs=4)
    plan64.autotune(4)
    a = inputs.densities(15, 4, p.shape[0])
    assert par(plan64.apply(dev(torch, a, "fp64")).cpu().numpy(), oracle.ifgf(p, a, k)["out"]) < FP64_TOL


@pytest.mark.parametrize("prec,nrhs", [("mixed", 1), ("mixed", 4), ("mixed", 16), ("fp64", 1), ("fp64", 4)])
def test_every_child_to_parent_variant(torch, prec, nrhs):
    """Each child-to-parent kernel variant, forced at every level where it
    applies, matches the oracle (forward and adjoint)."""
    from paper_2010_02857_amd import ifgf
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(17, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    ref = oracle.ifgf(p, ac, k)["out"]
    ref_adj = np.conj(oracle.ifgf(p, np.conj(ac), k)["out"])
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    plan = make_plan(p, k, prec, max_nrhs=16)
    cand = plan.kernel_candidates(nrhs)
    assert cand
    tested = set()
    for name in ifgf.Plan.C2P_VARIANTS:
        levels = {d: name for d, names in cand.items() if name in names}
        if not levels:
            continue
        print(f"variant {name} at levels {sorted(levels)}", flush=True)
        plan.set_kernel_choice(nrhs, {d: None for d in cand})
        plan.set_kernel_choice(nrhs, levels)
        assert all(plan.kernel_choice(nrhs)[d] == name for d in levels)
        out = plan.apply(dev(torch, a, prec)).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
        assert par(out, ref) < tol, name
        assert par(adj, ref_adj) < tol, name
        tested.add(name)
    assert plan.misses() == 0
    assert {"geometry", "frames"} <= tested
    with pytest.raises(ifgf.IFGFError):
        plan.set_kernel_choice(nrhs, {2: "geometry"})


@pytest.mark.parametrize("nrhs", [1, 4, 16])
def test_fp64_box_kernel_layouts(torch, monkeypatch, nrhs):
    """The FP64 box kernel forced at every level where it applies, in its
    compact LDS layout (seven wavefronts per CU, taken where frames touch at
    most 24 child cones) and in the padded one (IFGF_BOXACC_COMPACT=0):
    forward and adjoint match the oracle, and the two layouts agree."""
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(19, nrhs, p.shape[0])
    ref = oracle.ifgf(p, a, k)["out"]
    ref_adj = np.conj(oracle.ifgf(p, np.conj(a), k)["out"])
    plan = make_plan(p, k, "fp64", max_nrhs=16)
    cand = plan.kernel_candidates(nrhs)
    levels = {d: "box_acc" for d, names in cand.items() if "box_acc" in names}
    assert levels
    plan.set_kernel_choice(nrhs, levels)
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("IFGF_BOXACC_COMPACT", flag)
        print(f"box kernel compact={flag} at levels {sorted(levels)}", flush=True)
        out = plan.apply(dev(torch, a, "fp64")).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, "fp64")).cpu().numpy()
        assert par(out, ref) < FP64_TOL
        assert par(adj, ref_adj) < FP64_TOL
        outs.append(out)
    assert par(outs[0], outs[1]) < 1e-14
    assert plan.misses() == 0
    monkeypatch.delenv("IFGF_BOXACC_COMPACT")


@pytest.mark.parametrize("prec,nrhs,store", [("mixed", 1, 0), ("mixed", 1, 1), ("fp64", 1, 0), ("mixed", 16, 0),
                                              ("fp64", 4, 1)])
def test_side_stream_matches_one_stream(torch, prec, nrhs, store, monkeypatch):
    """The near field and the cousin evaluations on the plan's second stream,
    ordered by events against the chain of child-to-parent steps (whose
    output buffer held level d + 1 with two ping-pong buffers, store = 0; a
    buffer per level with store = 1), give bitwise the one-stream results:
    forward, adjoint and target gradient, launched back to back with no
    synchronisation in between."""
    p = inputs.cube_sphere(64)                     # N = 24576, D = 7
    n = p.shape[0]
    k = 16.0 * math.pi
    plan = make_plan(p, k, prec, max_nrhs=16, store_levels=store)
    x = dev(torch, inputs.densities(5, nrhs, n), prec)
    g = dev(torch, inputs.densities(6, nrhs, n), prec)
    res = {}
    for side in ("0", "1"):
        monkeypatch.setenv("IFGF_SIDE_STREAM", side)
        outs = [plan.apply(x), plan.apply(x, adjoint=True), plan.grad_targets(x, g), plan.apply(x)]
        torch.cuda.synchronize()
        res[side] = [o.cpu() for o in outs]
    for a, b in zip(res["0"], res["1"]):
        assert torch.equal(a, b)
    assert torch.equal(res["1"][0], res["1"][3])
    assert plan.misses() == 0


@pytest.mark.parametrize("prec,nrhs", [("mixed", 1), ("mixed", 16), ("fp64", 4)])
def test_graph_replay(torch, prec, nrhs):
    """use_graph: the first apply captures a graph, later ones replay it.
    Every replay, with new densities written into the same buffer and eager
    work and synchronisations in between, equals the eagerly launched
    result; forward and adjoint, before and after autotuning."""
    p = inputs.cube_sphere(16)
    k = 4.0 * math.pi
    eager = make_plan(p, k, prec, max_nrhs=16)
    graph = make_plan(p, k, prec, max_nrhs=16, use_graph=True)
    x = dev(torch, inputs.densities(16, nrhs, p.shape[0]), prec)
    out = torch.empty_like(x)
    for it in range(4):
        if it == 2:
            graph.autotune(nrhs)
            eager.autotune(nrhs)
        x.copy_(dev(torch, inputs.densities(100 + it, nrhs, p.shape[0]), prec))
        for adj in (False, True):
            y = graph.apply(x, adjoint=adj, out=out).clone()
            torch.cuda.synchronize()
            z = eager.apply(x, adjoint=adj)
            scratch = (x.abs() ** 2).sum()          # eager work between replays
            torch.cuda.synchronize()
            assert float(scratch) > 0
            if it < 2:
                assert torch.equal(y, z)            # same kernels, same order
            else:                                   # the two plans may tune differently
                assert par(y.cpu().numpy(), z.cpu().numpy()) < 1e-6
    assert graph.misses() == 0


@pytest.mark.parametrize("nrhs", [4, 16])
def test_cousin_eval_mfma_on_off(torch, monkeypatch, nrhs):
    """Cousin-target interpolation for batched right-hand sides on the
    matrix cores (IFGF_COUSIN_MFMA=1) and on the vector units (default):
    both match the oracle, forward and adjoint, on a sphere and on a ragged
    cloud with more than 16 points in some boxes."""
    pts_cases = ((inputs.cube_sphere(20), 5.0 * math.pi),
                 (np.concatenate([inputs.random_box_points(3000, 8), 0.05 * inputs.random_box_points(300, 9)]), 7.0))
    for pts, k in pts_cases:
        a = as_c64(inputs.densities(18, nrhs, pts.shape[0]))
        ref = oracle.ifgf(pts, a, k)["out"]
        ref_adj = np.conj(oracle.ifgf(pts, np.conj(a), k)["out"])
        outs = {}
        for flag in ("1", "0"):
            monkeypatch.setenv("IFGF_COUSIN_MFMA", flag)
            plan = make_plan(pts, k, "mixed", max_nrhs=16)
            outs[flag] = plan.apply(dev(torch, a, "mixed")).cpu().numpy()
            adj = plan.adjoint(dev(torch, a, "mixed")).cpu().numpy()
            assert par(outs[flag], ref) < MIXED_TOL
            assert par(adj, ref_adj) < MIXED_TOL
            assert plan.misses() == 0
        assert par(outs["1"], outs["0"]) < 1e-6
    monkeypatch.delenv("IFGF_COUSIN_MFMA")


@pytest.mark.parametrize("prec,nrhs", [("mixed", 1), ("fp64", 1), ("mixed", 4), ("mixed", 16), ("fp64", 4)])
def test_cousin_two_phase_on_off(torch, monkeypatch, prec, nrhs):
    """Cousin-target interpolation in two phases (pairs in cone order --
    on the matrix cores for batched FP32 -- then per-target sums; default)
    and in one (IFGF_COUSIN_TWO_PHASE=0) both match the oracle, forward and
    adjoint, including boxes with more than 16 points."""
    pts_cases = ((inputs.cube_sphere(20), 5.0 * math.pi),
                 (np.concatenate([inputs.random_box_points(3000, 8), 0.05 * inputs.random_box_points(300, 9)]), 7.0))
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    for pts, k in pts_cases:
        a = inputs.densities(19, nrhs, pts.shape[0])
        ac = a if prec == "fp64" else as_c64(a)
        ref = oracle.ifgf(pts, ac, k)["out"]
        ref_adj = np.conj(oracle.ifgf(pts, np.conj(ac), k)["out"])
        outs = {}
        for flag in ("1", "0"):
            monkeypatch.setenv("IFGF_COUSIN_TWO_PHASE", flag)
            plan = make_plan(pts, k, prec, max_nrhs=16)
            assert sum(plan.stats()["pairs_tabulated"]) > 0
            outs[flag] = plan.apply(dev(torch, a, prec)).cpu().numpy()
            adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
            assert par(outs[flag], ref) < tol
            assert par(adj, ref_adj) < tol
            assert plan.misses() == 0
        assert par(outs["1"], outs["0"]) < (1e-13 if prec == "fp64" else 1e-6)
    monkeypatch.delenv("IFGF_COUSIN_TWO_PHASE")


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("mixed", 1), ("mixed", 4), ("fp64", 16)])
def test_distinct_targets(torch, prec, nrhs):
    """Sources on a sphere, targets off it (outside, inside and a ragged
    cluster): the forward map, its adjoint and the target gradient equal the
    oracle on the same combined point set with zero density at the targets,
    and the forward map is within the IFGF accuracy of the direct sum."""
    src = inputs.cube_sphere(16)
    tgt = np.concatenate([1.3 * inputs.cube_sphere(8), 0.5 * inputs.random_box_points(300, 21),
                          np.array([0.2, -0.1, 0.3]) + 0.02 * inputs.random_box_points(40, 22)])
    n, m = src.shape[0], tgt.shape[0]
    k = 4.0 * math.pi
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    union = np.concatenate([src, tgt])
    a = inputs.densities(23, nrhs, n)
    v = inputs.densities(24, nrhs, m)
    ac, vc = (a, v) if prec == "fp64" else (as_c64(a), as_c64(v))
    pad_a = np.concatenate([ac, np.zeros((nrhs, m), ac.dtype)], axis=1)
    pad_v = np.concatenate([np.zeros((nrhs, n), vc.dtype), vc], axis=1)
    plan = make_plan(src, k, prec, max_nrhs=16, targets=tgt, store_levels=0)
    st = plan.stats()
    assert st["n_sources"] == n and st["n_targets"] == m
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    assert out.shape == (nrhs, m)
    r = oracle.ifgf(union, pad_a, k, grad=True)
    assert par(out, r["out"][:, n:]) < tol
    # the method's own error on this cloud (the GPU equals the oracle above) is
    # about 1.1e-3: the box spanning the targets out to r = 1.3 is larger
    assert rel(out, oracle.direct(src, ac, k, targets=tgt)) < 2e-3
    adj = plan.adjoint(dev(torch, v, prec)).cpu().numpy()
    assert adj.shape == (nrhs, n)
    assert par(adj, np.conj(oracle.ifgf(union, np.conj(pad_v), k)["out"])[:, :n]) < tol
    g = inputs.densities(25, nrhs, m)
    gc = g if prec == "fp64" else as_c64(g)
    got = plan.grad_targets(dev(torch, a, prec), dev(torch, g, prec)).cpu().numpy()
    assert got.shape == (m, 3)
    want = np.einsum("rn,rnc->nc", np.conj(gc), r["grad"][:, n:]).real
    assert par(got, want) < (1e-10 if prec == "fp64" else 1e-4)
    assert plan.misses() == 0


@pytest.mark.parametrize("geom", ["prolate", "oblate", "rough"])
def test_paper_geometries(torch, geom):
    """The other surfaces of Sec. 4 (eqs. defspheroid, defbumpysphere): the
    prolate (0.1, 0.1, 1) and oblate (1, 1, 0.1) spheroids and the rough
    sphere, N = 6144, diameter 4 wavelengths: FP64 equals the oracle, mixed
    within its bar, both within the method's accuracy of the direct sum."""
    pts = {"prolate": lambda: inputs.spheroid(32, (0.1, 0.1, 1.0)),
           "oblate": lambda: inputs.spheroid(32, (1.0, 1.0, 0.1)),
           "rough": lambda: inputs.rough_sphere(32)}[geom]()
    k = 4.0 * math.pi
    a = inputs.densities(26, 1, pts.shape[0])
    ref = oracle.ifgf(pts, a, k)["out"]
    direct = oracle.direct(pts, a, k)
    eps = rel(ref, direct)
    print(f"{geom}: eps_M of the method = {eps:.2e}", flush=True)
    assert eps < 1e-3
    out = make_plan(pts, k, "fp64").apply(dev(torch, a, "fp64")).cpu().numpy()
    assert par(out, ref) < FP64_TOL
    ac = as_c64(a)
    ref32 = oracle.ifgf(pts, ac, k)["out"]
    plan = make_plan(pts, k, "mixed")
    out32 = plan.apply(dev(torch, a, "mixed")).cpu().numpy()
    assert par(out32, ref32) < MIXED_TOL
    assert plan.misses() == 0


def test_argument_errors(torch):
    from paper_2010_02857_amd import ifgf
    p = inputs.cube_sphere(8)
    plan = make_plan(p, 3.0, "fp64", max_nrhs=2)
    x = dev(torch, inputs.densities(1, 3, p.shape[0]), "fp64")
    with pytest.raises(ifgf.IFGFError) as e:
        plan.apply(x)
    assert e.value.status == 1
    with pytest.raises(TypeError):
        plan.apply(x[:1].to(torch.complex64))


# ------------------------------------------------- workload 2, full size

@pytest.fixture(scope="module")
def w2():
    w = inputs.WORKLOADS[2]
    p, a = w.points(), w.densities()
    idx = inputs.error_subset(2, p.shape[0], 1000)
    d = oracle.direct(p, a, w.kappa, targets=p[idx], skip=idx)
    return w, p, a, idx, d


def test_cfg2_full_size_accuracy(torch, w2):
    """N = 393216, kappa a = 32 pi: both paths within 1e-3 of the direct sum
    on 1000 random targets (the paper prints 1.13e-3 for this case, Table
    timings2), and mixed within 1e-5 of FP64 over all N targets."""
    w, p, a, idx, d = w2
    outs = {}
    for prec in ("fp64", "mixed"):
        plan = make_plan(p, w.kappa, prec)
        outs[prec] = plan.apply(dev(torch, a, prec)).cpu().numpy()
        assert plan.misses() == 0
        e = rel(outs[prec][:, idx], d)
        print(f"cfg2 {prec}: eps_M = {e:.3e}", flush=True)
        assert e < 1e-3
        del plan
    assert par(outs["mixed"], outs["fp64"]) < MIXED_TOL


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cfg2_matches_oracle(torch, w2, prec):
    """Full-size parity with the oracle IFGF (about half a minute of CPU per
    precision): FP64 on the complex128 densities, mixed on the same densities
    rounded to complex64 (the oracle upcasts them), in both norms."""
    w, p, a, _, _ = w2
    plan = make_plan(p, w.kappa, prec)
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    del plan
    ref = oracle.ifgf(p, a if prec == "fp64" else as_c64(a), w.kappa)["out"]
    e, ei = rel(out, ref), rel_inf(out, ref)
    print(f"cfg2 {prec} vs oracle: l2 {e:.3e} inf {ei:.3e}", flush=True)
    assert max(e, ei) < (FP64_TOL if prec == "fp64" else MIXED_TOL)


# ------------------------------------------------ plan construction on the GPU

@pytest.mark.parametrize("case", ["cfg1", "cloud", "laplace", "leaf23", "deg46", "lattice"])
def test_gpu_plan_counts_match_oracle(torch, case):
    """The relevant cones marked and numbered on the GPU (rules (i) and (ii)
    of Sec. 3.3.2) give per-level counts equal to the oracle's, as the host
    builder does."""
    kw = {}
    if case == "cfg1":
        w = inputs.WORKLOADS[1]
        p, k = w.points(), w.kappa
    elif case == "cloud":
        p, k, kw = inputs.random_box_points(3000, 5), 25.0, {"levels": 5}
    elif case == "laplace":
        p, k = inputs.cube_sphere(20), 0.0
    elif case == "lattice":
        p, k, kw = inputs.lattice(17), 8.0, {"levels": 4}
    elif case == "leaf23":
        p, k, kw = inputs.cube_sphere(20, 0.25), 15.0, {"leaf": (2, 3)}
    else:
        p, k, kw = inputs.cube_sphere(20), 10.0, {"degrees": (4, 6)}
    st = make_plan(p, k, "fp64", dilate=False, **kw).stats()
    so = oracle.ifgf(p, inputs.densities(1, 1, p.shape[0]), k, **kw)["stats"]
    assert st["D"] == so["D"]
    for key in ("n_boxes", "n_cones", "n_cousin_evals", "n_parent_evals"):
        assert st[key] == so[key], key


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("mixed", 1), ("mixed", 4)])
def test_gpu_plan_equals_host_plan(torch, monkeypatch, prec, nrhs):
    """The plan built on the GPU (relevant cones, slot tables, cousin-pair
    tables in target and cone order) and the one built on the host
    (IFGF_HOST_PLAN=1) have the same counts and the same results, forward
    and adjoint, on a sphere and on a ragged cloud: equal up to the last bits
    of the centred factors G(x_t, x_c) in the pair tables (the device's FP64
    sine and cosine against the host library's)."""
    for pts, k in ((inputs.cube_sphere(24), 6.0 * math.pi), (inputs.random_box_points(5000, 8), 12.0)):
        a = dev(torch, inputs.densities(42, nrhs, pts.shape[0]), prec)
        res = {}
        for flag in ("0", "1"):
            monkeypatch.setenv("IFGF_HOST_PLAN", flag)
            plan = make_plan(pts, k, prec, max_nrhs=16)
            st = plan.stats()
            res[flag] = (st, plan.apply(a).cpu().numpy(), plan.adjoint(a).cpu().numpy())
            assert plan.misses() == 0
            del plan
        (s0, o0, j0), (s1, o1, j1) = res["0"], res["1"]
        for key in ("n_cones", "n_dilated", "pairs_tabulated", "n_frames"):
            assert s0[key] == s1[key], key
        assert sum(s0["pairs_tabulated"]) > 0
        tol = 1e-14 if prec == "fp64" else 1e-6
        assert par(o0, o1) < tol and par(j0, j1) < tol
    monkeypatch.delenv("IFGF_HOST_PLAN")


@pytest.mark.parametrize("tables", [False, True])
@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp64", 4), ("mixed", 1), ("mixed", 4), ("mixed", 16)])
def test_cousin_geo_pairs_on_off(torch, monkeypatch, prec, nrhs, tables):
    """The two-phase cousin evaluation with one thread per pair and the
    one-kernel evaluation (IFGF_COUSIN_GEO_PAIRS=0) both match the oracle,
    forward and adjoint, and each other: on levels without cousin-pair
    tables (IFGF_PAIR_BUDGET_MB=0, geometry per pair) and through the tables
    (two-phase cone-ordered form off, so the per-pair form reads the tables
    in target order)."""
    if tables:
        monkeypatch.setenv("IFGF_COUSIN_TWO_PHASE", "0")
    else:
        monkeypatch.setenv("IFGF_PAIR_BUDGET_MB", "0")
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(43, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    ref = oracle.ifgf(p, ac, k)["out"]
    ref_adj = np.conj(oracle.ifgf(p, np.conj(ac), k)["out"])
    outs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("IFGF_COUSIN_GEO_PAIRS", flag)
        plan = make_plan(p, k, prec, max_nrhs=16)
        assert (sum(plan.stats()["pairs_tabulated"]) > 0) == tables
        outs[flag] = plan.apply(dev(torch, a, prec)).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
        assert par(outs[flag], ref) < tol
        assert par(adj, ref_adj) < tol
        assert plan.misses() == 0
    assert par(outs["1"], outs["0"]) < (1e-13 if prec == "fp64" else 1e-6)
    monkeypatch.delenv("IFGF_COUSIN_GEO_PAIRS")


@pytest.mark.parametrize("prec,nrhs", [("fp64", 4), ("fp64", 16), ("mixed", 4), ("mixed", 16)])
def test_cousin_geo_order(torch, monkeypatch, prec, nrhs):
    """On levels without cousin-pair tables the pairs kept in cone order (a
    4-byte entry per pair) run on the matrix cores; with the order off
    (IFGF_COUSIN_GEO_ORDER=0) one thread per pair.  Both match the oracle,
    forward and adjoint, and the order takes device memory only when built
    (IFGF_GEO_ORDER_BUDGET_MB=0: not built)."""
    monkeypatch.setenv("IFGF_PAIR_BUDGET_MB", "0")
    p = inputs.cube_sphere(20)
    k = 5.0 * math.pi
    a = inputs.densities(44, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    ref = oracle.ifgf(p, ac, k)["out"]
    ref_adj = np.conj(oracle.ifgf(p, np.conj(ac), k)["out"])
    outs, nbytes = {}, {}
    for flag, budget in (("1", None), ("0", None), ("1", "0")):
        monkeypatch.setenv("IFGF_COUSIN_GEO_ORDER", flag)
        if budget is None:
            monkeypatch.delenv("IFGF_GEO_ORDER_BUDGET_MB", raising=False)
        else:
            monkeypatch.setenv("IFGF_GEO_ORDER_BUDGET_MB", budget)
        print(f"geo order {flag} budget {budget}", flush=True)
        plan = make_plan(p, k, prec, max_nrhs=16)
        assert sum(plan.stats()["pairs_tabulated"]) == 0
        nbytes[(flag, budget)] = plan.stats()["device_bytes"]
        out = plan.apply(dev(torch, a, prec)).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
        assert par(out, ref) < tol
        assert par(adj, ref_adj) < tol
        assert plan.misses() == 0
        outs[(flag, budget)] = out
    assert nbytes[("1", None)] > nbytes[("1", "0")]
    assert par(outs[("1", None)], outs[("0", None)]) < (1e-13 if prec == "fp64" else 1e-6)
    # the ordered pairs inside a captured apply: every replay equals the eager
    # result, with eager work in between
    monkeypatch.setenv("IFGF_COUSIN_GEO_ORDER", "1")
    monkeypatch.delenv("IFGF_GEO_ORDER_BUDGET_MB", raising=False)
    gplan = make_plan(p, k, prec, max_nrhs=16, use_graph=True)
    eager = make_plan(p, k, prec, max_nrhs=16)
    x = dev(torch, a, prec)
    y = torch.empty_like(x)
    for it in range(3):
        x.copy_(dev(torch, inputs.densities(90 + it, nrhs, p.shape[0]), prec))
        g = gplan.apply(x, out=y).clone()
        torch.cuda.synchronize()
        e = eager.apply(x)
        scratch = (x.abs() ** 2).sum()
        torch.cuda.synchronize()
        assert float(scratch) > 0
        assert torch.equal(g, e)
    assert gplan.misses() == 0
    monkeypatch.delenv("IFGF_COUSIN_GEO_ORDER")


def test_streams_and_workspace_reallocation(torch):
    """Calls on different streams, the second one growing the workspaces:
    the reallocation waits for the plan's work on the first stream (not for
    the whole device), and every result equals a fresh plan's."""
    p = inputs.cube_sphere(16)
    k = 4.0 * math.pi
    a1 = inputs.densities(71, 1, p.shape[0])
    a16 = inputs.densities(72, 16, p.shape[0])
    ref1 = make_plan(p, k, "fp64", max_nrhs=16).apply(dev(torch, a1, "fp64")).cpu().numpy()
    ref16 = make_plan(p, k, "fp64", max_nrhs=16).apply(dev(torch, a16, "fp64")).cpu().numpy()
    plan = make_plan(p, k, "fp64", max_nrhs=16, store_levels=0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    x1, x16 = dev(torch, a1, "fp64"), dev(torch, a16, "fp64")
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        y1 = plan.apply(x1)
    with torch.cuda.stream(s2):
        s2.wait_stream(s1)      # the caller orders its own buffers; the plan orders its workspaces
        y16 = plan.apply(x16)
    torch.cuda.synchronize()
    assert np.array_equal(y1.cpu().numpy(), ref1)
    assert np.array_equal(y16.cpu().numpy(), ref16)
    with torch.cuda.stream(s1):
        y1b = plan.apply(x1)
    del plan                     # release waits for the plan's streams
    torch.cuda.synchronize()
    assert np.array_equal(y1b.cpu().numpy(), ref1)
