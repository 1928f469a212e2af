"""Seeded synthetic inputs: node sets, evaluation points and manufactured data.

This module is shared by the HIP path's tests/benchmarks and by the CPU oracle.
It holds none of the solver's arithmetic (no kernel entries, no Krylov
steps, no regularisation); it only produces the problem data that the paper's
statement of the problem takes as input (Section 2.1: interior nodes, boundary
nodes, wavenumber, shape parameter, source f and Dirichlet data g).

The paper's own node sets are Gmsh mesh nodes (Section 5) that are not
available; the generators below stand in for them with the same kinds of
distributions the paper names (Halton, uniform random) on the same domains
(unit cube, unit sphere), at the sizes of the workloads this library is
measured on.

Conventions
-----------
* Nodes are float64 arrays of shape (n, 3), xyz interleaved (row-major).
* The node order of a problem is [interior; boundary]; centres = nodes.
* Random draws use numpy's PCG64 (``np.random.default_rng(seed)``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Point generators
# --------------------------------------------------------------------------


def _radical_inverse(idx: np.ndarray, base: int) -> np.ndarray:
    """Van der Corput radical inverse of integer indices in the given base."""
    idx = np.asarray(idx, dtype=np.int64).copy()
    out = np.zeros(idx.shape, dtype=np.float64)
    f = 1.0 / base
    while np.any(idx > 0):
        out += f * (idx % base)
        idx //= base
        f /= base
    return out


def halton_cube(n: int, start: int = 1) -> np.ndarray:
    """First n points of the 3-D Halton sequence (bases 2, 3, 5).

    Indices start at 1 (index 0 is the corner (0,0,0), which lies on the
    boundary and so cannot be an interior node)."""
    idx = np.arange(start, start + n, dtype=np.int64)
    return np.stack([_radical_inverse(idx, b) for b in (2, 3, 5)], axis=1)


def cube_faces_uniform(counts_per_face, seed: int) -> np.ndarray:
    """Uniform random points on the six faces of [0,1]^3.

    Face order: x=0, x=1, y=0, y=1, z=0, z=1; ``counts_per_face`` gives the
    number of points on each."""
    rng = np.random.default_rng(seed)
    pts = []
    for face, cnt in enumerate(counts_per_face):
        axis, side = divmod(face, 2)
        p = rng.random((cnt, 3))
        p[:, axis] = float(side)
        pts.append(p)
    return np.concatenate(pts, axis=0)


def cube_interior_uniform(n: int, seed: int) -> np.ndarray:
    """Uniform random points strictly inside (0,1)^3."""
    rng = np.random.default_rng(seed)
    p = rng.random((n, 3))
    # rng.random draws from [0, 1); exclude the (measure-zero) face x=0.
    p[p == 0.0] = 0.5
    return p


def ball_interior_uniform(n: int, seed: int, radius: float = 1.0) -> np.ndarray:
    """Uniform points in the open ball ||x|| < radius, by rejection from the cube."""
    rng = np.random.default_rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        cand = rng.uniform(-radius, radius, size=(2 * (n - out.shape[0]) + 64, 3))
        keep = cand[np.einsum("ij,ij->i", cand, cand) < radius * radius]
        out = np.concatenate([out, keep], axis=0)
    return np.ascontiguousarray(out[:n])


def sphere_fibonacci(n: int, radius: float = 1.0) -> np.ndarray:
    """Fibonacci lattice on the sphere: z_i = 1-(2i+1)/n, theta_i = i*pi*(3-sqrt5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)


def split_counts(total: int, parts: int):
    """Split ``total`` into ``parts`` near-equal counts, larger ones first."""
    base, rem = divmod(total, parts)
    return [base + (1 if k < rem else 0) for k in range(parts)]


# --------------------------------------------------------------------------
# Manufactured solutions.  Each returns (u, lap_u) as callables of an (n,3)
# array; f = lap_u + kappa^2 u on interior nodes and g = u on boundary nodes.
# --------------------------------------------------------------------------


def u_cube_sines(x: np.ndarray) -> np.ndarray:
    """u = sin(3x) sin(2y) sin(sqrt(12) z); its Laplacian is -25 u."""
    return np.sin(3.0 * x[:, 0]) * np.sin(2.0 * x[:, 1]) * np.sin(math.sqrt(12.0) * x[:, 2])


def u_plane_wave(kappa: float) -> Callable[[np.ndarray], np.ndarray]:
    """u = sin(kappa (x+y+z)/sqrt3); its Laplacian is -kappa^2 u."""

    def u(x: np.ndarray) -> np.ndarray:
        return np.sin(kappa * (x[:, 0] + x[:, 1] + x[:, 2]) / math.sqrt(3.0))

    return u


@dataclasses.dataclass(frozen=True)
class Manufactured:
    """A manufactured solution u with Laplacian -k2 u (k2 = squared wave-vector norm)."""

    name: str
    u: Callable[[np.ndarray], np.ndarray]
    k2: float  # Laplacian(u) = -k2 * u exactly

    def rhs_interior(self, x: np.ndarray, kappa: float) -> np.ndarray:
        """f = Laplacian(u) + kappa^2 u = (kappa^2 - k2) u (zero when kappa^2 == k2)."""
        c = kappa * kappa - self.k2
        if c == 0.0:
            return np.zeros(x.shape[0])
        return c * self.u(x)

    def dirichlet(self, x: np.ndarray) -> np.ndarray:
        return self.u(x)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Problem:
    """One synthetic problem instance."""

    name: str
    x_int: np.ndarray
    x_bnd: np.ndarray
    kappa: float
    eps: float
    f_int: np.ndarray
    g_bnd: np.ndarray
    x_eval: np.ndarray
    u_eval: np.ndarray  # exact solution at x_eval
    ell: int

    @property
    def n_int(self) -> int:
        return self.x_int.shape[0]

    @property
    def n_bnd(self) -> int:
        return self.x_bnd.shape[0]

    @property
    def n(self) -> int:
        return self.n_int + self.n_bnd

    @property
    def nodes(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([self.x_int, self.x_bnd], axis=0))

    @property
    def rhs(self) -> np.ndarray:
        return np.concatenate([self.f_int, self.g_bnd])


def _cube_problem(name, n_int, n_bnd, kappa, eps, ell, seed_bnd, seed_eval, n_eval=2000):
    man = Manufactured("cube_sines", u_cube_sines, 25.0)
    x_int = halton_cube(n_int)
    x_bnd = cube_faces_uniform(split_counts(n_bnd, 6), seed_bnd)
    x_eval = cube_interior_uniform(n_eval, seed_eval)
    return Problem(name, x_int, x_bnd, kappa, eps, man.rhs_interior(x_int, kappa),
                   man.dirichlet(x_bnd), x_eval, man.u(x_eval), ell)


def _sphere_problem(name, n_int, n_bnd, kappa, eps, ell, seed_int, seed_eval, n_eval=2000):
    man = Manufactured("plane_wave", u_plane_wave(kappa), kappa * kappa)
    x_int = ball_interior_uniform(n_int, seed_int)
    x_bnd = sphere_fibonacci(n_bnd)
    x_eval = ball_interior_uniform(n_eval, seed_eval)
    return Problem(name, x_int, x_bnd, kappa, eps, man.rhs_interior(x_int, kappa),
                   man.dirichlet(x_bnd), x_eval, man.u(x_eval), ell)


def cube_small() -> Problem:
    """Unit cube, N=1800 (1200 Halton interior, 600 uniform face nodes), kappa=5, eps=2, ell=60."""
    return _cube_problem("cube_n1800", 1200, 600, 5.0, 2.0, 60, seed_bnd=1, seed_eval=2)


def cube_medium() -> Problem:
    """Unit cube, N=20000 (16000 Halton interior, 4000 face nodes), kappa=20, eps=4, ell=200."""
    return _cube_problem("cube_n20000", 16000, 4000, 20.0, 4.0, 200, seed_bnd=7, seed_eval=8)


def sphere_large() -> Problem:
    """Unit ball, N=100000 (80000 uniform interior, 20000 Fibonacci boundary), kappa=30, eps=6, ell=300."""
    return _sphere_problem("sphere_n100000", 80000, 20000, 30.0, 6.0, 300, seed_int=11, seed_eval=12)


def cube_scaled(n_int: int, n_bnd: int, kappa: float, eps: float, ell: int, seed: int = 21) -> Problem:
    """Cube problem of arbitrary size (Halton interior, uniform faces) for tests."""
    return _cube_problem(f"cube_n{n_int + n_bnd}", n_int, n_bnd, kappa, eps, ell,
                         seed_bnd=seed, seed_eval=seed + 1)


def sphere_scaled(n_int: int, n_bnd: int, kappa: float, eps: float, ell: int, seed: int = 31) -> Problem:
    """Ball problem of arbitrary size (uniform interior, Fibonacci boundary) for tests."""
    return _sphere_problem(f"sphere_n{n_int + n_bnd}", n_int, n_bnd, kappa, eps, ell,
                           seed_int=seed, seed_eval=seed + 1)


WORKLOADS: Dict[str, Callable[[], Problem]] = {
    "cube_n1800": cube_small,
    "cube_n20000": cube_medium,
    "sphere_n100000": sphere_large,
}


# --------------------------------------------------------------------------
# Several right-hand sides per problem: a frequency sweep over cubes with
# Gaussian-blob sources (no manufactured solution; results are compared with
# the FP64 oracle)
# --------------------------------------------------------------------------


def blob_sources(x: np.ndarray, centres: np.ndarray, width: float = 0.1) -> np.ndarray:
    """Rows exp(-|x - c_k|^2 / (2 width^2)) for each centre c_k: (len(centres), len(x))."""
    d2 = ((x[None, :, :] - centres[:, None, :]) ** 2).sum(axis=2)
    return np.exp(-d2 / (2.0 * width * width))


@dataclasses.dataclass
class MultiProblem:
    """One problem with several right-hand sides F (rows [f_int; g_bnd])."""

    name: str
    x_int: np.ndarray
    x_bnd: np.ndarray
    kappa: float
    eps: float
    F: np.ndarray  # nrhs x n
    ell: int

    @property
    def n_int(self) -> int:
        return self.x_int.shape[0]

    @property
    def n_bnd(self) -> int:
        return self.x_bnd.shape[0]

    @property
    def n(self) -> int:
        return self.n_int + self.n_bnd

    @property
    def nrhs(self) -> int:
        return self.F.shape[0]

    @property
    def nodes(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([self.x_int, self.x_bnd], axis=0))


SWEEP_COUNT = 64
SWEEP_NRHS = 16
SWEEP_ELL = 100
SWEEP_SEED = 41


def multi_cube(n_int: int, n_bnd: int, kappa: float, eps: float, nrhs: int, ell: int, seed: int,
               width: float = 0.1) -> MultiProblem:
    """Unit cube (Halton interior, uniform faces) with nrhs blob sources at uniform random
    centres in the cube, g = 0 on the boundary."""
    x_int = halton_cube(n_int)
    x_bnd = cube_faces_uniform(split_counts(n_bnd, 6), seed)
    centres = np.random.default_rng(seed + 1).random((nrhs, 3))
    F = np.zeros((nrhs, n_int + n_bnd))
    F[:, :n_int] = blob_sources(x_int, centres, width)
    return MultiProblem(f"cube_n{n_int + n_bnd}_s{nrhs}", x_int, x_bnd, kappa, eps, F, ell)


def sweep_sizes(count: int = SWEEP_COUNT, seed: int = SWEEP_SEED) -> np.ndarray:
    """Problem sizes of the sweep: N uniform on [2000, 30000]."""
    return np.random.default_rng(seed).integers(2000, 30001, size=count)


def sweep_kappa(k: int, count: int = SWEEP_COUNT) -> float:
    """kappa evenly spaced on [2, 40]."""
    return 2.0 + 38.0 * k / (count - 1)


def sweep_member(k: int, count: int = SWEEP_COUNT, nrhs: int = SWEEP_NRHS, ell: int = SWEEP_ELL,
                 seed: int = SWEEP_SEED) -> MultiProblem:
    """Member k of the frequency sweep: N from sweep_sizes (80 % interior Halton nodes,
    20 % uniform face nodes), kappa from sweep_kappa, eps = 0.2 kappa + 1, nrhs blob sources."""
    n = int(sweep_sizes(count, seed)[k])
    n_int = int(round(0.8 * n))
    kappa = sweep_kappa(k, count)
    return multi_cube(n_int, n - n_int, kappa, 0.2 * kappa + 1.0, nrhs, ell, seed + 1000 + 2 * k)


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal float64 vector (test operands)."""
    return np.random.default_rng(seed).standard_normal(n)


def random_nodes_cube(n: int, seed: int) -> np.ndarray:
    """Seeded uniform nodes in [0,1]^3 (tiny test problems)."""
    return np.random.default_rng(seed).random((n, 3))
