"""Python binding of libifgf.so (C ABI in include/ifgf.h).

Argument marshalling only: every step of the operator runs in the HIP
library.  PyTorch supplies device memory and the current stream.  If the
library has not been built, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IFGF_LIB: load another build of the same sources (the sanitizer runs)
LIB_PATH = os.environ.get("IFGF_LIB") or os.path.join(HERE, "libifgf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ifgf.h")
MAX_LEVELS = 24

FP64 = 0
MIXED = 1

_STATUS = {0: "IFGF_OK", 1: "IFGF_E_INVALID_ARG", 2: "IFGF_E_OUT_OF_MEMORY", 3: "IFGF_E_HIP",
           4: "IFGF_E_UNSUPPORTED", 5: "IFGF_E_INTERNAL"}


class IFGFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("leaf_ns", ctypes.c_int32),
        ("leaf_nc", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_nrhs", ctypes.c_int32),
        ("store_levels", ctypes.c_int32),
        ("host_only", ctypes.c_int32),
        ("no_dilate", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("workspace_limit", ctypes.c_size_t),
        ("leaf_max", ctypes.c_int32),
    ]


_L = MAX_LEVELS + 1


class Stats(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("n_points", ctypes.c_int32),
        ("H1", ctypes.c_double),
        ("x1", ctypes.c_double * 3),
        ("kappa", ctypes.c_double),
        ("ps", ctypes.c_int32),
        ("pang", ctypes.c_int32),
        ("ns", ctypes.c_int32 * _L),
        ("nc", ctypes.c_int32 * _L),
        ("n_boxes", ctypes.c_int64 * _L),
        ("n_cones", ctypes.c_int64 * _L),
        ("n_cousin_boxes", ctypes.c_int64 * _L),
        ("max_cousin_boxes", ctypes.c_int64 * _L),
        ("n_cousin_evals", ctypes.c_int64 * _L),
        ("n_parent_evals", ctypes.c_int64 * _L),
        ("n_leaf_pairs", ctypes.c_int64),
        ("n_near_pairs", ctypes.c_int64),
        ("n_dilated", ctypes.c_int64),
        ("n_frames", ctypes.c_int64 * _L),
        ("pairs_tabulated", ctypes.c_int32 * _L),
        ("device_bytes", ctypes.c_int64),
        ("t_plan_s", ctypes.c_double),
        ("n_sources", ctypes.c_int64),
        ("n_targets", ctypes.c_int64),
        ("n_src_boxes", ctypes.c_int64 * _L),
        ("n_leaf_boxes", ctypes.c_int64 * _L),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2010_02857_amd._build.build() "
                               "(or __graft_entry__.build()) before using the IFGF operator")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.ifgf_plan_create.argtypes = [P, I64, ctypes.c_double, I32, P, ctypes.POINTER(Options), ctypes.POINTER(P)]
        L.ifgf_plan_create_targets.argtypes = [P, I64, P, I64, ctypes.c_double, I32, P, ctypes.POINTER(Options),
                                               ctypes.POINTER(P)]
        L.ifgf_apply.argtypes = [P, P, I32, P, P]
        L.ifgf_apply_adjoint.argtypes = [P, P, I32, P, P]
        L.ifgf_apply_noalloc.argtypes = [P, P, I32, P, P]
        L.ifgf_grad_targets.argtypes = [P, P, P, I32, P, P]
        L.ifgf_grad_targets_stored.argtypes = [P, P, P, I32, P, P]
        L.ifgf_plan_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.ifgf_plan_check.argtypes = [P, ctypes.POINTER(I64)]
        L.ifgf_plan_destroy.argtypes = [P]
        L.ifgf_plan_profile.argtypes = [P, I32]
        L.ifgf_plan_stage_times.argtypes = [P, P, P]
        L.ifgf_plan_level_times.argtypes = [P, I32, P, P]
        L.ifgf_plan_autotune.argtypes = [P, I32, P]
        L.ifgf_plan_kernel_choice.argtypes = [P, I32, P]
        L.ifgf_plan_set_kernel_choice.argtypes = [P, I32, P]
        L.ifgf_plan_kernel_candidates.argtypes = [P, I32, P]
        L.ifgf_status_string.argtypes = [ctypes.c_int]
        L.ifgf_status_string.restype = ctypes.c_char_p
        L.ifgf_last_error.argtypes = []
        L.ifgf_last_error.restype = ctypes.c_char_p
        for f in (L.ifgf_plan_create, L.ifgf_plan_create_targets, L.ifgf_apply, L.ifgf_apply_adjoint, L.ifgf_grad_targets,
                  L.ifgf_grad_targets_stored, L.ifgf_apply_noalloc, L.ifgf_plan_level_times,
                  L.ifgf_plan_stats, L.ifgf_plan_check, L.ifgf_plan_destroy, L.ifgf_plan_profile,
                  L.ifgf_plan_stage_times, L.ifgf_plan_autotune, L.ifgf_plan_kernel_choice,
                  L.ifgf_plan_set_kernel_choice, L.ifgf_plan_kernel_candidates):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of the functions include/ifgf.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|ifgf_status)\s+(ifgf_\w+)\s*\(", text, re.M)))


def _check(rc: int):
    if rc != 0:
        msg = lib().ifgf_last_error().decode(errors="replace")
        raise IFGFError(rc, msg)


class Plan:
    """An IFGF plan over a fixed point set: the points are both sources and
    targets, or with `targets` given, the field of the sources `points` is
    evaluated at the distinct `targets`.

    points     (n, 3) float64 array-like (host); copied.
    targets    None, or (m, 3) float64 array-like (host); copied.
    k          wavenumber >= 0.
    levels     D, or 0 for H_D about a quarter wavelength.
    degrees    (P_s, P_ang) Chebyshev nodes per cone direction.
    precision  "fp64" (complex128 I/O) or "mixed" (complex64 I/O).
    use_graph  capture apply calls into HIP graphs and replay them.
    leaf_max   adaptive octree: boxes holding at most leaf_max points are not
               split (0: every leaf on level D).
    """

    def __init__(self, points, k: float, levels: int = 0, degrees=(3, 5), precision: str = "fp64",
                 leaf=(1, 2), max_nrhs: int = 16, store_levels: int = -1, host_only: bool = False,
                 dilate: bool = True, workspace_limit: int = 0, use_graph: bool = False, targets=None,
                 device=None, leaf_max: int = 0):
        def host(x):
            if hasattr(x, "detach"):
                x = x.detach().cpu().numpy()
            return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))

        pts = host(points)
        tgt = None if targets is None else host(targets)
        self.n = pts.shape[0]                     # sources
        self.m = self.n if tgt is None else tgt.shape[0]   # targets
        self.k = float(k)
        self.precision = precision
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        opt = Options(int(leaf[0]), int(leaf[1]), FP64 if precision == "fp64" else MIXED, int(max_nrhs),
                      int(store_levels), 1 if host_only else 0, 0 if dilate else 1, 1 if use_graph else 0,
                      int(workspace_limit), int(leaf_max))
        deg = (ctypes.c_int32 * 2)(int(degrees[0]), int(degrees[1]))
        h = ctypes.c_void_p()
        self._h = None
        self.host_only = host_only
        self.device = None

        def create():
            if tgt is None:
                _check(lib().ifgf_plan_create(pts.ctypes.data_as(ctypes.c_void_p), self.n, self.k, int(levels),
                                              ctypes.cast(deg, ctypes.c_void_p), ctypes.byref(opt), ctypes.byref(h)))
            else:
                _check(lib().ifgf_plan_create_targets(pts.ctypes.data_as(ctypes.c_void_p), self.n,
                                                      tgt.ctypes.data_as(ctypes.c_void_p), self.m, self.k,
                                                      int(levels), ctypes.cast(deg, ctypes.c_void_p),
                                                      ctypes.byref(opt), ctypes.byref(h)))

        if not host_only:
            import torch
            self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                       else torch.device(device).index or 0)
            with torch.cuda.device(self.device):
                create()
        else:
            create()
        self._h = h

    # -- housekeeping
    def close(self):
        if self._h is not None and self._h.value:
            lib().ifgf_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        st = Stats()
        _check(lib().ifgf_plan_stats(self._h, ctypes.byref(st)))
        D = st.D
        out = {"D": D, "n_points": st.n_points, "H1": st.H1, "x1": list(st.x1), "kappa": st.kappa,
               "ps": st.ps, "pang": st.pang, "n_leaf_pairs": st.n_leaf_pairs, "n_near_pairs": st.n_near_pairs,
               "n_dilated": st.n_dilated, "device_bytes": st.device_bytes, "t_plan_s": st.t_plan_s,
               "n_sources": st.n_sources, "n_targets": st.n_targets}
        for key in ("ns", "nc", "n_boxes", "n_cones", "n_cousin_boxes", "max_cousin_boxes", "n_cousin_evals",
                    "n_parent_evals", "n_frames", "pairs_tabulated", "n_src_boxes", "n_leaf_boxes"):
            arr = getattr(st, key)
            out[key] = [int(arr[d]) for d in range(D + 1)]
        return out

    def misses(self) -> int:
        m = ctypes.c_int64()
        _check(lib().ifgf_plan_check(self._h, ctypes.byref(m)))
        return int(m.value)

    STAGES = ("permute_in", "nearfield", "leaf_nodes", "cousin_eval", "child_to_parent", "permute_out",
              "near_grad", "cousin_grad", "permute_grad")

    def profile(self, enable: bool = True):
        """Start (clearing totals) or stop per-stage HIP-event timing."""
        _check(lib().ifgf_plan_profile(self._h, 1 if enable else 0))

    def stage_times(self) -> dict:
        """{stage: (milliseconds, launches)} recorded since profile(True)."""
        ms = np.zeros(len(self.STAGES), np.float64)
        cnt = np.zeros(len(self.STAGES), np.int64)
        _check(lib().ifgf_plan_stage_times(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                           cnt.ctypes.data_as(ctypes.c_void_p)))
        return {s: (float(ms[i]), int(cnt[i])) for i, s in enumerate(self.STAGES)}

    def level_times(self, stage: str) -> dict:
        """{level d: (milliseconds, launches)} of one stage since
        profile(True) (levels with launches only)."""
        ms = np.zeros(MAX_LEVELS + 1, np.float64)
        cnt = np.zeros(MAX_LEVELS + 1, np.int64)
        _check(lib().ifgf_plan_level_times(self._h, self.STAGES.index(stage), ms.ctypes.data_as(ctypes.c_void_p),
                                           cnt.ctypes.data_as(ctypes.c_void_p)))
        return {d: (float(ms[d]), int(cnt[d])) for d in range(MAX_LEVELS + 1) if cnt[d]}

    C2P_VARIANTS = ("geometry", "frames", "lds", "mfma", "mfma_geometry", "boxes", "quads", "lds_tiled", "box_acc",
                    "box_acc_half")

    def autotune(self, nrhs: int = 1):
        """Time the child-to-parent kernel variants of every level for nrhs
        right-hand sides on the current stream and keep the fastest."""
        import torch
        with torch.cuda.device(self.device):
            _check(lib().ifgf_plan_autotune(self._h, int(nrhs),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def kernel_choice(self, nrhs: int = 1) -> dict:
        """{level d: variant name} of the child-to-parent step from d to d - 1."""
        v = (ctypes.c_int32 * (MAX_LEVELS + 1))()
        _check(lib().ifgf_plan_kernel_choice(self._h, int(nrhs), ctypes.cast(v, ctypes.c_void_p)))
        return {d: self.C2P_VARIANTS[v[d]] for d in range(MAX_LEVELS + 1) if v[d] >= 0}

    def set_kernel_choice(self, nrhs: int, choice: dict):
        """Force {level d: variant name or None (default rule)} for nrhs
        right-hand sides; levels not named keep their current setting."""
        cur = self.kernel_choice(nrhs)
        v = (ctypes.c_int32 * (MAX_LEVELS + 1))(*([-1] * (MAX_LEVELS + 1)))
        tuned = {d: self.C2P_VARIANTS.index(x) for d, x in cur.items()}
        for d, x in choice.items():
            tuned[d] = -1 if x is None else self.C2P_VARIANTS.index(x)
        for d, x in tuned.items():
            v[d] = x
        _check(lib().ifgf_plan_set_kernel_choice(self._h, int(nrhs), ctypes.cast(v, ctypes.c_void_p)))

    def kernel_candidates(self, nrhs: int = 1) -> dict:
        """{level d: [names of the variants that apply there]}."""
        m = (ctypes.c_int32 * (MAX_LEVELS + 1))()
        _check(lib().ifgf_plan_kernel_candidates(self._h, int(nrhs), ctypes.cast(m, ctypes.c_void_p)))
        return {d: [x for i, x in enumerate(self.C2P_VARIANTS) if (m[d] >> i) & 1]
                for d in range(MAX_LEVELS + 1) if m[d]}

    # -- operator
    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def _prep(self, a, npts=None):
        import torch
        npts = self.n if npts is None else npts
        if not isinstance(a, torch.Tensor) or not a.is_cuda:
            raise TypeError("expected a CUDA (HIP) tensor")
        if a.dtype != self.dtype:
            raise TypeError(f"expected {self.dtype}, got {a.dtype}")
        squeeze = a.dim() == 1
        a2 = a.reshape(1, -1) if squeeze else a
        if a2.dim() != 2 or a2.shape[1] != npts:
            raise ValueError(f"expected shape (nrhs, {npts}) or ({npts},)")
        return a2.contiguous(), squeeze

    def _stream(self, t):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)

    def apply(self, a, adjoint: bool = False, out=None):
        """I = IFGF(a) (or the adjoint operator applied to a).  `out`, if
        given, is a contiguous tensor of a's shape and dtype that receives the
        result (with use_graph, reusing the same a and out replays the
        captured graph)."""
        import torch
        nin, nout = (self.m, self.n) if adjoint else (self.n, self.m)
        a2, squeeze = self._prep(a, nin)
        shape = (a2.shape[0], nout)
        if out is None:
            out = torch.empty(shape, dtype=a2.dtype, device=a2.device)
        else:
            if out.dtype != a2.dtype or out.device != a2.device or out.numel() != shape[0] * shape[1] \
                    or not out.is_contiguous():
                raise ValueError("out must be a contiguous tensor of the output's shape and dtype")
            if out.data_ptr() == a2.data_ptr():
                raise ValueError("out must not alias the densities")
        f = lib().ifgf_apply_adjoint if adjoint else lib().ifgf_apply
        _check(f(self._h, ctypes.c_void_p(a2.data_ptr()), a2.shape[0], ctypes.c_void_p(out.data_ptr()),
                 self._stream(a2)))
        return out.reshape(-1) if squeeze else out.reshape(shape)

    def adjoint(self, v):
        return self.apply(v, adjoint=True)

    def apply_noalloc(self, a, out):
        """IFGF(a) into the preallocated contiguous `out` with no device
        allocation by the library (ifgf_apply_noalloc: workspaces in its
        static per-GPU scratch array)."""
        a2, _ = self._prep(a, self.n)
        if out.dtype != a2.dtype or out.device != a2.device or out.numel() != a2.shape[0] * self.m \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the output's shape and dtype")
        _check(lib().ifgf_apply_noalloc(self._h, ctypes.c_void_p(a2.data_ptr()), a2.shape[0],
                                        ctypes.c_void_p(out.data_ptr()), self._stream(a2)))
        return out

    def grad_targets(self, a, g, stored: bool = False):
        """sum_r Re(conj(g_r) dI_r/dx) for every target, (m, 3) float64.
        stored=True reuses the cone values of the last apply when it took the
        same tensor `a`; the caller guarantees that a has not been modified
        since (ifgf_grad_targets_stored)."""
        import torch
        a2, _ = self._prep(a, self.n)
        g2, _ = self._prep(g, self.m)
        if g2.shape[0] != a2.shape[0]:
            raise ValueError("grad_out must have as many right-hand sides as the densities")
        out = torch.empty((self.m, 3), dtype=torch.float64, device=a2.device)
        f = lib().ifgf_grad_targets_stored if stored else lib().ifgf_grad_targets
        _check(f(self._h, ctypes.c_void_p(a2.data_ptr()), ctypes.c_void_p(g2.data_ptr()),
                 a2.shape[0], ctypes.c_void_p(out.data_ptr()), self._stream(a2)))
        return out


def _function():
    import torch

    class IFGFFunction(torch.autograd.Function):
        """I = IFGF(a) at the plan's points; backward gives the density
        gradient through the adjoint operator and the target-coordinate
        gradient through the differentiated interpolants."""

        @staticmethod
        def forward(ctx, plan, a, targets):
            out = plan.apply(a)
            ctx.plan = plan
            ctx.save_for_backward(a)
            return out

        @staticmethod
        def backward(ctx, g):
            (a,) = ctx.saved_tensors
            plan = ctx.plan
            g = g.contiguous()
            ga = plan.adjoint(g) if ctx.needs_input_grad[1] else None
            gx = None
            if ctx.needs_input_grad[2]:
                # a is a saved tensor: autograd has checked that it was not
                # modified in place since the forward, so the cone values that
                # apply stored for it may be reused
                gx = plan.grad_targets(a, g, stored=True)
            return None, ga, gx

    return IFGFFunction


_FN = None


def apply(plan: Plan, a, targets=None):
    """Differentiable IFGF matvec.  `targets` is the plan's (m, 3) target
    point tensor (the points themselves when sources = targets), passed so
    that a gradient with respect to it can flow."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(plan, a, targets)
