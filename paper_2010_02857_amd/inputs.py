"""Seeded synthetic inputs for the IFGF workloads.

This module generates points and densities only; it holds none of the
method's arithmetic, so both the GPU library's tests and the CPU oracle's
tests draw their inputs from it.

The paper evaluates the operator on discretisations of a sphere and of
spheroids (Sec. 4, eqs. defspheroid, defbumpysphere) without specifying the
point sets; an equiangular cube-sphere of N = 6 n^2 points stands in for them
here:

* face grid u_i = tan(pi/4 * (2 (i + 0.5) / n - 1)), i = 0..n-1;
* faces in the order +x, -x, +y, -y, +z, -z, the points (+-1, u_i, u_j),
  (u_i, +-1, u_j), (u_i, u_j, +-1) with i outer and j inner;
* every point is projected onto the unit sphere; an oblate spheroid with
  semi-axes (1, 1, c) scales z by c afterwards, a general spheroid scales
  every axis, and the rough sphere moves each point to the radius of eq.
  defbumpysphere along its direction.

Densities are complex Gaussians a = (N(0,1) + i N(0,1)) / sqrt(2) drawn from
``numpy.random.default_rng(1000 + cfg)`` as ``standard_normal((R, N, 2))``;
error-check targets from ``default_rng(2000 + cfg)``; finite-difference
entries from ``default_rng(3000 + cfg)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def cube_sphere(n: int, zscale: float = 1.0) -> np.ndarray:
    """Equiangular cube-sphere with 6 n^2 points, shape (6 n^2, 3), float64."""
    if n < 1:
        raise ValueError("n must be positive")
    i = np.arange(n, dtype=np.float64)
    u = np.tan(math.pi / 4.0 * (2.0 * (i + 0.5) / n - 1.0))
    ui, uj = np.meshgrid(u, u, indexing="ij")          # i outer, j inner
    ui = ui.reshape(-1)
    uj = uj.reshape(-1)
    one = np.ones_like(ui)
    faces = [
        np.stack([one, ui, uj], axis=1),
        np.stack([-one, ui, uj], axis=1),
        np.stack([ui, one, uj], axis=1),
        np.stack([ui, -one, uj], axis=1),
        np.stack([ui, uj, one], axis=1),
        np.stack([ui, uj, -one], axis=1),
    ]
    p = np.concatenate(faces, axis=0)
    p /= np.sqrt((p * p).sum(axis=1, keepdims=True))
    if zscale != 1.0:
        p[:, 2] *= zscale
    return np.ascontiguousarray(p)


def spheroid(n: int, axes=(1.0, 1.0, 0.1)) -> np.ndarray:
    """The spheroid x^2/alpha^2 + y^2/beta^2 + z^2/gamma^2 = 1 of eq.
    defspheroid, as the cube-sphere scaled by (alpha, beta, gamma): oblate
    (1, 1, 0.1) and prolate (0.1, 0.1, 1) in Sec. 4."""
    p = cube_sphere(n)
    p *= np.asarray(axes, dtype=np.float64)[None, :]
    return np.ascontiguousarray(p)


def rough_sphere(n: int, amplitude: float = 0.05, frequency: float = 40.0) -> np.ndarray:
    """The rough sphere of eq. defbumpysphere: the cube-sphere directions at
    radius 1 + amplitude sin(frequency theta) sin(frequency phi), with theta
    the polar angle in [0, pi] and phi the azimuth in [0, 2 pi)."""
    d = cube_sphere(n)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2.0 * math.pi)
    r = 1.0 + amplitude * np.sin(frequency * theta) * np.sin(frequency * phi)
    return np.ascontiguousarray(d * r[:, None])


def graded_sphere(n: int, c: float = 0.25) -> np.ndarray:
    """A locally refined sphere: the cube-sphere mapped by the conformal map
    that scales the stereographic plane (projected from the south pole) by c.
    For c < 1 the points crowd towards the north pole (0, 0, 1): the point
    density there is 1/c^2 times the cube-sphere's, and c^2 times it at the
    south pole, so box point counts vary by a factor of about 1/c^4 over the
    surface (the uneven counts that an adaptive octree targets, Sec. 4)."""
    d = cube_sphere(n)
    den = 1.0 + d[:, 2]
    south = den < 1e-12
    w = np.zeros((d.shape[0], 2))
    w[~south] = c * d[~south, :2] / den[~south, None]
    q = (w * w).sum(axis=1)
    out = np.empty_like(d)
    out[:, 0] = 2.0 * w[:, 0] / (1.0 + q)
    out[:, 1] = 2.0 * w[:, 1] / (1.0 + q)
    out[:, 2] = (1.0 - q) / (1.0 + q)
    out[south] = d[south]
    return np.ascontiguousarray(out)


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: geometry, wavenumber, batch and precision."""
    cfg: int                 # 1-based workload number (seeds derive from it)
    name: str
    n_face: int              # N = 6 n_face^2
    kappa: float
    nrhs: int
    precision: str           # "fp64" or "mixed"
    zscale: float = 1.0      # 1: unit sphere; c < 1: oblate (1, 1, c)

    @property
    def n(self) -> int:
        return 6 * self.n_face * self.n_face

    def points(self) -> np.ndarray:
        return cube_sphere(self.n_face, self.zscale)

    def densities(self, nrhs: int | None = None, n: int | None = None) -> np.ndarray:
        return densities(self.cfg, self.nrhs if nrhs is None else nrhs, self.n if n is None else n)


WORKLOADS = {
    1: Workload(1, "sphere-6144-k4pi", 32, 4.0 * math.pi, 1, "fp64"),
    2: Workload(2, "sphere-393216-k32pi", 256, 32.0 * math.pi, 1, "mixed"),
    3: Workload(3, "oblate-0.25-1572864-k64pi-r16", 512, 64.0 * math.pi, 16, "mixed", 0.25),
    4: Workload(4, "sphere-393216-k32pi-grad", 256, 32.0 * math.pi, 1, "mixed"),
    5: Workload(5, "sphere-6291456-k128pi-r4", 1024, 128.0 * math.pi, 4, "mixed"),
}


def densities(cfg: int, nrhs: int, n: int) -> np.ndarray:
    """Complex128 densities of shape (nrhs, n), seeded by the workload number."""
    rng = np.random.default_rng(1000 + cfg)
    g = rng.standard_normal((nrhs, n, 2))
    return (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)


def error_subset(cfg: int, n: int, m: int) -> np.ndarray:
    """Indices of m distinct random targets for the relative error estimate."""
    rng = np.random.default_rng(2000 + cfg)
    return np.sort(rng.choice(n, size=min(m, n), replace=False)).astype(np.int64)


def fd_entries(cfg: int, n: int, m: int) -> tuple[np.ndarray, np.ndarray]:
    """m random (point index, coordinate) pairs for finite-difference checks."""
    rng = np.random.default_rng(3000 + cfg)
    idx = rng.choice(n, size=min(m, n), replace=False).astype(np.int64)
    comp = rng.integers(0, 3, size=idx.shape[0]).astype(np.int64)
    return idx, comp


def lattice(n: int) -> np.ndarray:
    """n^3 points of a regular grid filling [-1/2, 1/2]^3 (spacing 1/(n-1)).
    With n = 2^j + 1 the points lie on box faces and on the polar axes of box
    centres at every level: a case of ties for the box and cone maps."""
    g = np.arange(n) / (n - 1) - 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1))


def random_box_points(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """n points uniform in [-scale/2, scale/2)^3 (tests of small cases)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray((rng.random((n, 3)) - 0.5) * scale)
