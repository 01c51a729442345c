"""The adaptive octree on the GPU against the oracle, element by element.

A box of level >= 2 with at most leaf_max points is a leaf (the oracle's
reading of the adaptive tree that Sec. 4 and Sec. 5 name): the library
computes its cone values directly on its own level (over the zeros the
child-to-parent step leaves in its slots) and sums its sources directly at
the targets of its neighbour boxes.  Inputs: the graded sphere, whose box
point counts vary by about 1/c^4 = 256 over the surface, so that leaves sit
on several levels.  Bars as in the other parity tests: 1e-12 (FP64) and 1e-5
(mixed, oracle on complex64-rounded inputs), each in the relative l2 and the
relative infinity norm.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2010_02857_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5
K = 10.0
LEVELS = 6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_02857_amd import ifgf
    ifgf.lib()        # the HIP library must be there: no fallback
    return t


def rel(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(np.asarray(y)))


def par(x, y):
    x, y = np.asarray(x), np.asarray(y)
    return max(rel(x, y), float(np.max(np.abs(x - y)) / np.max(np.abs(y))))


def dev(torch, a, prec):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def as_c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def make_plan(p, prec, leaf_max, **kw):
    from paper_2010_02857_amd import ifgf
    kw.setdefault("levels", LEVELS)
    print(f"adaptive plan N={p.shape[0]} prec={prec} leaf_max={leaf_max} {kw}", flush=True)
    return ifgf.Plan(p, K, precision=prec, max_nrhs=16, leaf_max=leaf_max, **kw)


@pytest.fixture(scope="module")
def graded():
    return inputs.graded_sphere(20)


def refs(p, a, leaf_max, **kw):
    kw.setdefault("levels", LEVELS)
    out = oracle.ifgf(p, a, K, leaf_max=leaf_max, **kw)
    adj = np.conj(oracle.ifgf(p, np.conj(a), K, leaf_max=leaf_max, **kw)["out"])
    return out, adj


@pytest.mark.parametrize("leaf_max", [6, 40])
@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp64", 4), ("fp64", 16), ("mixed", 1), ("mixed", 4),
                                       ("mixed", 16)])
def test_adaptive_matches_oracle(torch, graded, prec, nrhs, leaf_max):
    """Forward and adjoint against the oracle's adaptive IFGF; the tree has
    leaves on at least two levels above D; the forward map is within the
    method's accuracy of the direct sum."""
    p = graded
    a = inputs.densities(51, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    r, ref_adj = refs(p, ac, leaf_max)
    plan = make_plan(p, prec, leaf_max)
    st = plan.stats()
    assert st["n_leaf_boxes"] == r["stats"]["n_leaf_boxes"]
    assert sum(1 for x in st["n_leaf_boxes"][:LEVELS] if x > 0) >= 2
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
    assert par(out, r["out"]) < tol
    assert par(adj, ref_adj) < tol
    assert rel(out, oracle.direct(p, ac, K)) < 2e-3
    assert plan.misses() == 0


@pytest.mark.parametrize("prec,nrhs", [("mixed", 1), ("mixed", 16), ("fp64", 1), ("fp64", 4)])
def test_adaptive_every_child_to_parent_variant(torch, graded, prec, nrhs):
    """Every child-to-parent kernel, forced at every level where it applies,
    leaves the leaf boxes' slots to the leaf kernel: forward and adjoint
    match the oracle with each."""
    from paper_2010_02857_amd import ifgf
    p = graded
    a = inputs.densities(52, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    r, ref_adj = refs(p, ac, 8)
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    plan = make_plan(p, prec, 8)
    cand = plan.kernel_candidates(nrhs)
    tested = set()
    for name in ifgf.Plan.C2P_VARIANTS:
        levels = {d: name for d, names in cand.items() if name in names}
        if not levels:
            continue
        print(f"variant {name} at levels {sorted(levels)}", flush=True)
        plan.set_kernel_choice(nrhs, {d: None for d in cand})
        plan.set_kernel_choice(nrhs, levels)
        out = plan.apply(dev(torch, a, prec)).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
        assert par(out, r["out"]) < tol, name
        assert par(adj, ref_adj) < tol, name
        tested.add(name)
    assert plan.misses() == 0
    assert {"geometry", "frames"} <= tested


@pytest.mark.parametrize("prec,store", [("fp64", 1), ("fp64", 0), ("mixed", 1), ("mixed", 0)])
def test_adaptive_grad_targets(torch, graded, prec, store):
    """The target gradient (near field over the leaves' ranges, cousin terms
    of the source boxes) against the oracle's, stored and recomputed."""
    p = graded
    nrhs = 2
    a = inputs.densities(53, nrhs, p.shape[0])
    g = inputs.densities(54, nrhs, p.shape[0])
    ac, gc = (a, g) if prec == "fp64" else (as_c64(a), as_c64(g))
    r = oracle.ifgf(p, ac, K, levels=LEVELS, leaf_max=8, grad=True)
    want = np.einsum("rn,rnc->nc", np.conj(gc), r["grad"]).real
    plan = make_plan(p, prec, 8, store_levels=store)
    x = dev(torch, a, prec)
    plan.apply(x)
    got = plan.grad_targets(x, dev(torch, g, prec)).cpu().numpy()
    assert par(got, want) < (1e-10 if prec == "fp64" else 1e-4)
    assert plan.misses() == 0


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("mixed", 4), ("mixed", 16)])
def test_adaptive_cousin_paths(torch, graded, monkeypatch, prec, nrhs):
    """The cousin stage reads only the cousins that are source boxes, on
    every path: pair tables with the two-phase form (default), one kernel
    per target (IFGF_COUSIN_TWO_PHASE=0), geometry per pair without tables
    (IFGF_PAIR_BUDGET_MB=0), and the one-kernel form without tables
    (IFGF_COUSIN_GEO_PAIRS=0)."""
    p = graded
    a = inputs.densities(55, nrhs, p.shape[0])
    ac = a if prec == "fp64" else as_c64(a)
    r, ref_adj = refs(p, ac, 12)
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    configs = ({}, {"IFGF_COUSIN_TWO_PHASE": "0"}, {"IFGF_PAIR_BUDGET_MB": "0"},
               {"IFGF_PAIR_BUDGET_MB": "0", "IFGF_COUSIN_GEO_PAIRS": "0"})
    for env in configs:
        for key in ("IFGF_COUSIN_TWO_PHASE", "IFGF_PAIR_BUDGET_MB", "IFGF_COUSIN_GEO_PAIRS"):
            monkeypatch.delenv(key, raising=False)
        for key, val in env.items():
            monkeypatch.setenv(key, val)
        print(f"cousin path {env}", flush=True)
        plan = make_plan(p, prec, 12)
        out = plan.apply(dev(torch, a, prec)).cpu().numpy()
        adj = plan.adjoint(dev(torch, a, prec)).cpu().numpy()
        assert par(out, r["out"]) < tol, env
        assert par(adj, ref_adj) < tol, env
        assert plan.misses() == 0


def test_adaptive_gpu_plan_equals_host_plan(torch, graded, monkeypatch):
    """Relevant cones marked on the GPU (source boxes only, rule (i) over all
    cousins of a source box) equal the host builder's and the oracle's
    counts, and give the same result."""
    p = graded
    a = inputs.densities(56, 1, p.shape[0])
    so = oracle.ifgf(p, a, K, levels=LEVELS, leaf_max=8)["stats"]
    outs = []
    for host in ("0", "1"):
        monkeypatch.setenv("IFGF_HOST_PLAN", host)
        plan = make_plan(p, "fp64", 8, dilate=False)
        st = plan.stats()
        for key in ("n_boxes", "n_cones", "n_cousin_evals", "n_parent_evals", "n_src_boxes", "n_leaf_boxes"):
            assert st[key] == so[key], (host, key)
        assert st["n_near_pairs"] == so["n_near_pairs"]
        outs.append(plan.apply(dev(torch, a, "fp64")).cpu().numpy())
    monkeypatch.delenv("IFGF_HOST_PLAN")
    assert par(outs[0], outs[1]) < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adaptive_distinct_targets_and_laplace(torch, graded, prec):
    """Distinct targets (the union plan: zero density at the targets, the
    splitting rule counting both) and kappa = 0, against the oracle on the
    same point sets."""
    from paper_2010_02857_amd import ifgf
    src = graded
    tgt = np.concatenate([inputs.random_box_points(300, 57, 1.8), 1.2 * inputs.cube_sphere(6)])
    n, m = src.shape[0], tgt.shape[0]
    union = np.concatenate([src, tgt])
    a = inputs.densities(58, 4, n)
    ac = a if prec == "fp64" else as_c64(a)
    pad = np.concatenate([ac, np.zeros((4, m), ac.dtype)], axis=1)
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    plan = ifgf.Plan(src, K, precision=prec, max_nrhs=16, levels=LEVELS, targets=tgt, leaf_max=10)
    out = plan.apply(dev(torch, a, prec)).cpu().numpy()
    ref = oracle.ifgf(union, pad, K, levels=LEVELS, leaf_max=10)["out"][:, n:]
    assert par(out, ref) < tol
    assert plan.misses() == 0
    lap = ifgf.Plan(src, 0.0, precision=prec, max_nrhs=16, levels=LEVELS, leaf_max=10)
    out0 = lap.apply(dev(torch, a, prec)).cpu().numpy()
    assert par(out0, oracle.ifgf(src, ac, 0.0, levels=LEVELS, leaf_max=10)["out"]) < tol
    assert lap.misses() == 0


@pytest.mark.parametrize("prec,nrhs", [("mixed", 1), ("fp64", 4)])
def test_adaptive_graph_replay(torch, graded, prec, nrhs):
    """A captured apply of an adaptive plan (the leaf kernels of every level
    inside the graph) replays to the eager result, several times with eager
    work in between."""
    p = graded
    eager = make_plan(p, prec, 8)
    graph = make_plan(p, prec, 8, use_graph=True)
    x = dev(torch, inputs.densities(59, nrhs, p.shape[0]), prec)
    out = torch.empty_like(x)
    for it in range(3):
        x.copy_(dev(torch, inputs.densities(160 + it, nrhs, p.shape[0]), prec))
        y = graph.apply(x, out=out).clone()
        torch.cuda.synchronize()
        z = eager.apply(x)
        scratch = (x.abs() ** 2).sum()
        torch.cuda.synchronize()
        assert float(scratch) > 0
        assert torch.equal(y, z)
    assert graph.misses() == 0
