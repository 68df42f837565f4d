"""Seeded synthetic TSP instances shaped like the paper's workloads.

The paper measures on TSPLIB instances (hundreds to ~18k cities) and on the
TSP Art instances (100k-200k stipple drawings, Sec. 5.6).  None of those
datasets is used here; these generators stand in for them:

* ``uniform``        -- integer points uniform in [0, 1e6)^2;
* ``gaussian_mixture`` -- isotropic Gaussian clusters (TSPLIB-like structure);
* ``stipple``        -- rejection sampling of a 2-D density made of Gaussian
  blobs plus sinusoidal ridge bands on a 4096^2 pixel grid, scaled to
  [0, 1e6)^2 (a stand-in for stipple-art instances).

This module holds only input generation; it computes nothing of the method.
Every generator returns a C-contiguous ``int32`` array of shape (n, 2) with
unique points.
"""
from dataclasses import dataclass, field
import math

import numpy as np

COORD_MAX = 1_000_000


def _unique_fill(rng, n, propose):
    """Draw points from ``propose(rng, m)`` until n unique in-range points."""
    pts = np.zeros((0, 2), dtype=np.int64)
    seen = set()
    out = []
    while len(out) < n:
        need = n - len(out)
        cand = propose(rng, max(2 * need, 64))
        ok = (cand[:, 0] >= 0) & (cand[:, 0] < COORD_MAX) & \
             (cand[:, 1] >= 0) & (cand[:, 1] < COORD_MAX)
        cand = cand[ok]
        for x, y in cand:
            key = (int(x) << 21) | int(y)
            if key in seen:
                continue
            seen.add(key)
            out.append((int(x), int(y)))
            if len(out) == n:
                break
    del pts
    return np.ascontiguousarray(np.array(out, dtype=np.int32))


def uniform(n, seed):
    rng = np.random.default_rng(seed)
    return _unique_fill(rng, n, lambda r, m: r.integers(0, COORD_MAX, size=(m, 2)))


def gaussian_mixture(n, seed, components=64, sigma_lo=5e3, sigma_hi=4e4):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, COORD_MAX, size=(components, 2))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=components)

    def propose(r, m):
        c = r.integers(0, components, size=m)
        p = centres[c] + r.standard_normal((m, 2)) * sigmas[c, None]
        return np.rint(p).astype(np.int64)

    return _unique_fill(rng, n, propose)


def stipple_density(rng, grid=4096, blobs=200, bands=8):
    """Density on a grid x grid lattice: Gaussian blobs + ridge bands.
    Both terms are separable in x and y, so each is built from outer
    products of 1-D profiles (cos(a + b) = cos a cos b - sin a sin b)."""
    dens = np.zeros((grid, grid), dtype=np.float32)
    ax = np.arange(grid, dtype=np.float32)
    for _ in range(blobs):
        cx, cy = rng.uniform(0, grid, size=2)
        sig = rng.uniform(20, 300)
        amp = rng.uniform(0.2, 1.0)
        r = int(math.ceil(4 * sig))
        x0, x1 = max(0, int(cx) - r), min(grid, int(cx) + r + 1)
        y0, y1 = max(0, int(cy) - r), min(grid, int(cy) + r + 1)
        gx = np.exp(-((ax[x0:x1] - cx) ** 2) / (2 * sig * sig)).astype(np.float32)
        gy = (amp * np.exp(-((ax[y0:y1] - cy) ** 2) / (2 * sig * sig))).astype(np.float32)
        dens[y0:y1, x0:x1] += np.outer(gy, gx)
    band = np.empty((grid, grid), dtype=np.float32)
    tmp = np.empty((grid, grid), dtype=np.float32)
    axd = np.arange(grid, dtype=np.float64)
    for _ in range(bands):
        lam = rng.uniform(256, 2048)
        th = rng.uniform(0, math.pi)
        amp = rng.uniform(0.2, 0.6)
        ph = rng.uniform(0, 2 * math.pi)
        a = (2 * math.pi / lam) * axd * math.cos(th) + ph      # x part
        b = (2 * math.pi / lam) * axd * math.sin(th)           # y part
        np.multiply.outer(np.cos(b).astype(np.float32), np.cos(a).astype(np.float32), out=band)
        np.multiply.outer(np.sin(b).astype(np.float32), np.sin(a).astype(np.float32), out=tmp)
        band -= tmp
        np.maximum(band, 0.0, out=band)
        band *= band
        band *= band
        band *= band
        band *= np.float32(amp)
        dens += band
    return dens


def stipple(n, seed, grid=4096):
    rng = np.random.default_rng(seed)
    dens = stipple_density(rng, grid=grid)
    dmax = float(dens.max())
    scale = COORD_MAX / grid

    def propose(r, m):
        m = max(m, 4096)
        px = r.integers(0, grid, size=m)
        py = r.integers(0, grid, size=m)
        acc = r.uniform(0, dmax, size=m) < dens[py, px]
        px, py = px[acc], py[acc]
        jx = r.uniform(0, 1, size=px.shape[0])
        jy = r.uniform(0, 1, size=py.shape[0])
        x = np.floor((px + jx) * scale).astype(np.int64)
        y = np.floor((py + jy) * scale).astype(np.int64)
        return np.stack([x, y], axis=1)

    return _unique_fill(rng, n, propose)


# --------------------------------------------------------------------------
# Workload definitions (method parameters per workload; names say what they
# are, sizes included).

@dataclass
class Workload:
    name: str
    n: int
    kind: str
    instance_seed: int
    cl_size: int = 16
    bl_size: int = 64
    n_ants: int = 16
    min_new_edges: int = 8
    rho: float = 0.5
    iterations: int = 200
    philox_seed: int = 1
    extra: dict = field(default_factory=dict)

    def points(self):
        return make_points(self.kind, self.n, self.instance_seed)

    def params(self):
        return dict(cl_size=self.cl_size, bl_size=self.bl_size,
                    n_ants=self.n_ants, min_new_edges=self.min_new_edges,
                    rho=self.rho, seed=self.philox_seed)


def make_points(kind, n, seed):
    if kind == "uniform":
        return uniform(n, seed)
    if kind == "gaussian_mixture":
        return gaussian_mixture(n, seed)
    if kind == "cluster16":
        s = math.sqrt(n / 20000.0)
        return gaussian_mixture(n, seed, components=16, sigma_lo=5e3 * s,
                                sigma_hi=4e4 * s)
    if kind == "stipple":
        return stipple(n, seed)
    raise ValueError(kind)


WORKLOADS = {
    # TSPLIB-sized uniform instance, 1000 cities, 16 ants, 8 new edges,
    # retention 0.02, 200 iterations
    "uniform1k": Workload("uniform1k", 1000, "uniform", 1001, n_ants=16,
                          min_new_edges=8, rho=0.02, iterations=200),
    # 20 000 clustered cities (64 Gaussian components), 32 ants, 16 new edges
    "gmm20k": Workload("gmm20k", 20000, "gaussian_mixture", 1002, n_ants=32,
                       min_new_edges=16, rho=0.5, iterations=500),
    # 100 000 stipple-like cities, 64 ants, 32 new edges (stipple-art scale)
    "stipple100k": Workload("stipple100k", 100000, "stipple", 1003, n_ants=64,
                            min_new_edges=32, rho=0.5, iterations=1000),
}


def batch_instances(count=256, seed0=4000, n_lo=200, n_hi=5000):
    """Uneven batch: n log-uniform in [n_lo, n_hi]; even index uniform, odd
    index 16-cluster Gaussian mixture."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        kind = "uniform" if i % 2 == 0 else "cluster16"
        out.append(Workload(f"batch{i}", n, kind, seed0 + i, cl_size=12,
                            n_ants=16, min_new_edges=8, rho=0.5,
                            iterations=300, philox_seed=1))
    return out


def served_requests(count=256, rate=4.0, seed0=5000, n_lo=1000, n_hi=200000,
                    arrival_seed=77):
    """Poisson arrivals of stipple solve requests; returns (arrival_s, Workload)."""
    rng = np.random.default_rng(arrival_seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        rr = np.random.default_rng(seed0 + r)
        n = int(round(math.exp(rr.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append((float(arrivals[r]),
                    Workload(f"req{r}", n, "stipple", seed0 + r, cl_size=16,
                             n_ants=32, min_new_edges=16, rho=0.5,
                             iterations=200, philox_seed=r)))
    return out
