"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers; it contains none of the summation
method's arithmetic.  Every generator uses numpy's PCG64 with a fixed seed so
that the GPU path and the CPU oracle see bit-identical inputs.

Workloads (all 3D, forces i.i.d. N(0,1) per component):

* ``uniform``    -- N points uniform in the unit cube [0,1)^3.
* ``clusters``   -- N points from 8 Gaussian clusters (centres uniform in the
  unit cube, equal weights, isotropic standard deviation ``sigma``); points that
  fall outside [0,1)^3 are redrawn from the same cluster.
* ``periodic``   -- uniform points, forces with the per-component mean removed
  (zero net force).
* ``sphere``     -- points on a perturbed sphere (radius 0.3, relative
  perturbation 0.15 sin(3 theta) cos(4 phi)), sources and a separate target set.
* ``batch``      -- many independent problems with N log-uniform in [1e3, 1e5],
  each uniform or a single Gaussian blob (sigma 0.1, centre in [0.25,0.75]^3)
  chosen by a seeded coin.

The point distributions stand in for the adaptive, clustered inputs the method
is designed for (Sec. "Numerical results": perturbed surfaces and random
points); no external dataset is involved.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.random((n, 3))


def cluster_points(rng: np.random.Generator, n: int, n_clusters: int = 8,
                   sigma: float = 0.02) -> np.ndarray:
    centres = rng.random((n_clusters, 3))
    counts = np.full(n_clusters, n // n_clusters, dtype=np.int64)
    counts[: n - counts.sum()] += 1
    out = []
    for k in range(n_clusters):
        need = int(counts[k])
        got = []
        while need > 0:
            cand = centres[k] + sigma * rng.standard_normal((need + need // 8 + 16, 3))
            ok = np.all((cand >= 0.0) & (cand < 1.0), axis=1)
            cand = cand[ok][:need]
            got.append(cand)
            need -= cand.shape[0]
        out.append(np.concatenate(got, axis=0))
    return np.ascontiguousarray(np.concatenate(out, axis=0))


def blob_points(rng: np.random.Generator, n: int, sigma: float = 0.1) -> np.ndarray:
    centre = 0.25 + 0.5 * rng.random(3)
    pts = []
    need = n
    while need > 0:
        cand = centre + sigma * rng.standard_normal((need + need // 4 + 16, 3))
        ok = np.all((cand >= 0.0) & (cand < 1.0), axis=1)
        cand = cand[ok][:need]
        pts.append(cand)
        need -= cand.shape[0]
    return np.ascontiguousarray(np.concatenate(pts, axis=0))


def sphere_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """Points on a perturbed sphere: r(theta, phi) = 0.3 (1 + 0.15 sin(3 theta)
    cos(4 phi)) around (0.5, 0.5, 0.5), (cos theta, phi) uniform.  A surface
    distribution gives the deep, strongly adaptive trees of the paper's timing
    setup; the perturbation law is this generator's own choice."""
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    th = np.arccos(ct)
    r = 0.3 * (1.0 + 0.15 * np.sin(3.0 * th) * np.cos(4.0 * ph))
    st = np.sqrt(1.0 - ct * ct)
    return np.ascontiguousarray(0.5 + np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1))


def forces(rng: np.random.Generator, n: int, n_rhs: int = 1, zero_mean: bool = False) -> np.ndarray:
    f = rng.standard_normal((n_rhs, n, 3))
    if zero_mean:
        f -= f.mean(axis=1, keepdims=True)
    return f[0] if n_rhs == 1 else f


def make(kind: str, n: int, seed: int, sigma: float = 0.02, n_rhs: int = 1):
    """Return (points (n,3), forces (n,3) or (n_rhs,n,3)) for one workload."""
    rng = _rng(seed)
    if kind == "uniform":
        x = uniform_points(rng, n)
        f = forces(rng, n, n_rhs)
    elif kind == "clusters":
        x = cluster_points(rng, n, 8, sigma)
        f = forces(rng, n, n_rhs)
    elif kind == "periodic":
        x = uniform_points(rng, n)
        f = forces(rng, n, n_rhs, zero_mean=True)
    elif kind == "blob":
        x = blob_points(rng, n, sigma)
        f = forces(rng, n, n_rhs)
    elif kind == "sphere":
        x = sphere_points(rng, n)
        f = forces(rng, n, n_rhs)
    else:
        raise ValueError(f"unknown workload kind {kind!r}")
    return np.ascontiguousarray(x), np.ascontiguousarray(f)


def sphere_targets(m: int, seed: int) -> np.ndarray:
    """A separate target set on the same perturbed sphere (seed + 200)."""
    return sphere_points(_rng(seed + 200), m)


def normals(x: np.ndarray, seed: int, kind: str = "random") -> np.ndarray:
    """Unit vectors n_a for stresslet (double-layer) sources: the radial
    direction from the cube centre for surface points (kind "sphere"), else
    isotropic random directions (seeded with seed + 300)."""
    if kind == "sphere":
        v = np.asarray(x, dtype=np.float64) - 0.5
    else:
        v = _rng(seed + 300).standard_normal((np.asarray(x).shape[0], 3))
    return np.ascontiguousarray(v / np.linalg.norm(v, axis=1, keepdims=True))


def sample_targets(n: int, m: int, seed: int) -> np.ndarray:
    """Sorted distinct target indices (seeded with seed + 100)."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    idx = _rng(seed + 100).choice(n, size=m, replace=False)
    return np.sort(idx).astype(np.int64)


def batch_problems(n_problems: int = 256, base_seed: int = 5000):
    """List of (points, forces) for independent problems, N log-uniform in [1e3,1e5]."""
    meta = _rng(5)
    sizes = np.rint(10.0 ** meta.uniform(3.0, 5.0, size=n_problems)).astype(np.int64)
    kinds = meta.random(n_problems) < 0.5
    out = []
    for i in range(n_problems):
        kind = "uniform" if kinds[i] else "blob"
        out.append(make(kind, int(sizes[i]), base_seed + i, sigma=0.1))
    return out


# Named configurations: (kind, N, seed, sigma, periodic, tol)
CONFIGS = {
    "uniform_1e4": dict(kind="uniform", n=10_000, seed=1, sigma=0.0, periodic=False, tol=1e-6),
    "clusters_1e6": dict(kind="clusters", n=1_000_000, seed=2, sigma=0.02, periodic=False, tol=1e-6),
    "periodic_2e6": dict(kind="periodic", n=2_000_000, seed=3, sigma=0.0, periodic=True, tol=1e-9),
    "clusters_4e6": dict(kind="clusters", n=4_000_000, seed=4, sigma=0.01, periodic=False, tol=1e-6),
    # sources and separate targets on a perturbed sphere
    "sphere_1e6": dict(kind="sphere", n=1_000_000, seed=6, sigma=0.0, periodic=False, tol=1e-6, n_targets=1_000_000),
    # one plan, 32 force vectors (forces shaped (32, N, 3))
    "uniform_2e6_rhs32": dict(kind="uniform", n=2_000_000, seed=5, sigma=0.0, periodic=False, tol=1e-6, n_rhs=32),
}


def config(name: str):
    c = CONFIGS[name]
    x, f = make(c["kind"], c["n"], c["seed"], c["sigma"], c.get("n_rhs", 1))
    return x, f
