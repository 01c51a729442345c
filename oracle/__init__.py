"""Python access to the plain FP64 CPU oracle (``ifgf_oracle.c``).

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  The GPU library does not
import it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ifgf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# IFGF_ORACLE_LIB: load another build of the same source (the sanitizer runs)
_LOAD = os.environ.get("IFGF_ORACLE_LIB") or _LIB
MAX_LEVELS = 24


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("H1", ctypes.c_double),
        ("x1", ctypes.c_double * 3),
        ("ns", ctypes.c_int32 * (MAX_LEVELS + 1)),
        ("nc", ctypes.c_int32 * (MAX_LEVELS + 1)),
        ("n_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_cones", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_cousin_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("max_cousin_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_cousin_evals", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_parent_evals", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_far_pairs", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_near_pairs", ctypes.c_int64),
        ("n_src_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("n_leaf_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("t_pre", ctypes.c_double),
        ("t_acc", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LOAD == _LIB and not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LOAD)
        P = ctypes.c_void_p
        L.oracle_direct.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_double, P, P,
                                    ctypes.c_int64, P]
        L.oracle_direct_grad.argtypes = L.oracle_direct.argtypes
        L.oracle_ifgf.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P,
                                  ctypes.c_int64, P, P, P, ctypes.POINTER(_Stats)]
        L.oracle_ifgf_ex.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, P, P, ctypes.c_int64, P, P, P, ctypes.POINTER(_Stats)]
        L.oracle_green.argtypes = [ctypes.c_double, P, P, P]
        L.oracle_analytic_factor.argtypes = [ctypes.c_double, P, P, P, P]
        L.oracle_cheb_nodes.argtypes = [ctypes.c_int32, P]
        L.oracle_cheb_interp3.argtypes = [ctypes.c_int32, ctypes.c_int32, P, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, P]
        L.oracle_cone_coords.argtypes = [P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        L.oracle_cone_point.argtypes = [P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P, P, P]
        for f in (L.oracle_direct, L.oracle_direct_grad, L.oracle_ifgf, L.oracle_ifgf_ex):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _dens(dens, n):
    d = np.asarray(dens)
    if d.ndim == 1:
        d = d[None, :]
    if d.shape[1] != n:
        raise ValueError("densities must be (nrhs, n)")
    return np.ascontiguousarray(d.astype(np.complex128))


def _targets(pts, targets, skip):
    if targets is None:
        t = pts
        s = np.arange(pts.shape[0], dtype=np.int64) if skip is None else np.asarray(skip, np.int64)
    else:
        t = _f64(targets).reshape(-1, 3)
        s = (np.full(t.shape[0], -1, np.int64) if skip is None else np.ascontiguousarray(skip, np.int64))
    return np.ascontiguousarray(t), np.ascontiguousarray(s)


def direct(pts, dens, kappa, targets=None, skip=None):
    """Direct sum at targets (default: the source points, self term skipped).
    Returns complex128 (nrhs, m)."""
    pts = _f64(pts).reshape(-1, 3)
    a = _dens(dens, pts.shape[0])
    t, s = _targets(pts, targets, skip)
    out = np.zeros((a.shape[0], t.shape[0]), np.complex128)
    rc = lib().oracle_direct(_p(pts), pts.shape[0], _p(a), a.shape[0], float(kappa), _p(t), _p(s),
                             t.shape[0], _p(out))
    if rc != 0:
        raise ValueError(f"oracle_direct failed ({rc})")
    return out


def direct_grad(pts, dens, kappa, targets=None, skip=None):
    """Gradient of the direct sum w.r.t. target position: complex (nrhs, m, 3)."""
    pts = _f64(pts).reshape(-1, 3)
    a = _dens(dens, pts.shape[0])
    t, s = _targets(pts, targets, skip)
    out = np.zeros((a.shape[0], t.shape[0], 3), np.complex128)
    rc = lib().oracle_direct_grad(_p(pts), pts.shape[0], _p(a), a.shape[0], float(kappa), _p(t), _p(s),
                                  t.shape[0], _p(out))
    if rc != 0:
        raise ValueError(f"oracle_direct_grad failed ({rc})")
    return out


def ifgf(pts, dens, kappa, levels=0, degrees=(3, 5), leaf=(1, 2), targets=None, skip=None,
         grad=False, sig=False, leaf_max=0):
    """Plain FP64 IFGF.  Returns a dict with 'out' (nrhs, m), optional 'grad'
    (nrhs, m, 3), 'sig' (m,) and 'stats' (per-level counts).  leaf_max > 0:
    adaptive octree (boxes holding at most leaf_max points are not split)."""
    pts = _f64(pts).reshape(-1, 3)
    a = _dens(dens, pts.shape[0])
    if targets is None:
        t, s, m = None, None, pts.shape[0]
    else:
        t, s = _targets(pts, targets, skip)
        m = t.shape[0]
    out = np.zeros((a.shape[0], m), np.complex128)
    g = np.zeros((a.shape[0], m, 3), np.complex128) if grad else None
    sg = np.zeros(m, np.uint64) if sig else None
    st = _Stats()
    rc = lib().oracle_ifgf_ex(_p(pts), pts.shape[0], _p(a), a.shape[0], float(kappa), int(levels),
                              int(degrees[0]), int(degrees[1]), int(leaf[0]), int(leaf[1]), int(leaf_max),
                              _p(t), _p(s), m, _p(out), _p(g), _p(sg), ctypes.byref(st))
    if rc != 0:
        raise ValueError(f"oracle_ifgf failed ({rc})")
    D = st.D
    stats = {
        "D": D, "H1": st.H1, "x1": list(st.x1), "n_near_pairs": st.n_near_pairs,
        "t_pre": st.t_pre, "t_acc": st.t_acc,
    }
    for key in ("ns", "nc", "n_boxes", "n_cones", "n_cousin_boxes", "max_cousin_boxes",
                "n_cousin_evals", "n_parent_evals", "n_far_pairs", "n_src_boxes", "n_leaf_boxes"):
        arr = getattr(st, key)
        stats[key] = [int(arr[d]) for d in range(D + 1)]
    res = {"out": out, "stats": stats}
    if grad:
        res["grad"] = g
    if sig:
        res["sig"] = sg
    return res


def green(kappa, x, y):
    out = np.zeros(2)
    lib().oracle_green(float(kappa), _p(_f64(x)), _p(_f64(y)), _p(out))
    return complex(out[0], out[1])


def analytic_factor(kappa, c, x, y):
    out = np.zeros(2)
    lib().oracle_analytic_factor(float(kappa), _p(_f64(c)), _p(_f64(x)), _p(_f64(y)), _p(out))
    return complex(out[0], out[1])


def cheb_nodes(n):
    t = np.zeros(n)
    lib().oracle_cheb_nodes(int(n), _p(t))
    return t


def cheb_interp3(ps, pang, u, loc):
    u = np.ascontiguousarray(np.asarray(u, np.complex128).reshape(ps, pang, pang))
    out = np.zeros(2)
    lib().oracle_cheb_interp3(int(ps), int(pang), _p(u), float(loc[0]), float(loc[1]), float(loc[2]),
                              _p(out))
    return complex(out[0], out[1])


def cone_coords(c, H, ns, nc, x):
    idx = np.zeros(3, np.int32)
    loc = np.zeros(3)
    sth = np.zeros(3)
    lib().oracle_cone_coords(_p(_f64(c)), float(H), int(ns), int(nc), _p(_f64(x)), _p(idx), _p(loc),
                             _p(sth))
    return idx, loc, sth


def cone_point(c, H, ns, nc, idx, loc):
    x = np.zeros(3)
    lib().oracle_cone_point(_p(_f64(c)), float(H), int(ns), int(nc),
                            _p(np.ascontiguousarray(idx, np.int32)), _p(_f64(loc)), _p(x))
    return x
