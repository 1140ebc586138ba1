"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle tests.

This module holds no arithmetic of the method itself: it only shapes initial
density fields and draws random numbers.  Coexistence densities, temperatures
and every other physical quantity are passed in by the caller.

* Noise: a splitmix64 stream seeded with ``220509186 + instance_id``; the k-th
  draw (k = 1, 2, ...) is ``u = (x >> 11) * 2**-53`` and the noise is
  ``(2u - 1) * amplitude``, assigned in node order, x fastest; added to the
  density, or (``relative``) applied as a factor ``1 + noise``.
* Droplet: the tanh profile of Eq 26 between given liquid and gas densities,
  centred at node (nx/2, ny/2[, nz/2]), r the Euclidean node distance (no
  periodic image).
* Slab: the same tanh shape across a flat liquid layer occupying the central
  half of one axis (Sec 3.4, flat interface test).

Arrays are indexed [y][x] (2D) or [z][y][x] (3D), x fastest in memory.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 220509186
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(n: int, instance_id: int = 0, start: int = 0) -> np.ndarray:
    """Draws start+1 .. start+n of the splitmix64 stream as doubles in [0, 1)."""
    seed = np.uint64((SEED_BASE + int(instance_id)) % (1 << 64))
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = seed + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def noise(shape, amplitude: float = 1e-6, instance_id: int = 0) -> np.ndarray:
    """Uniform noise in (-amplitude, amplitude) in node order, x fastest."""
    n = int(np.prod(shape))
    out = np.empty(n, np.float64)
    chunk = 1 << 22
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        out[s:s + m] = (2.0 * splitmix64_uniform(m, instance_id, s) - 1.0) * amplitude
    return out.reshape(shape)


def _tanh_shape(dist: np.ndarray, r0: float, W: float, rho_g: float, rho_l: float) -> np.ndarray:
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (dist - r0) / W)


def droplet(shape, radius: float, width: float, rho_g: float, rho_l: float,
            amplitude: float = 1e-6, instance_id: int = 0, center=None, relative: bool = False) -> np.ndarray:
    """Circular (2D, shape (ny, nx)) or spherical (3D, shape (nz, ny, nx)) droplet.

    relative=True applies the noise as rho (1 + n), which keeps the density
    positive when the gas density is below the noise amplitude (low Tr)."""
    shape = tuple(int(s) for s in shape)
    if center is None:
        center = tuple(s // 2 for s in shape)   # node (n/2) on each axis
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    r2 = np.zeros(shape)
    for g, c in zip(grids, center):
        r2 += (g - c) ** 2
    rho = _tanh_shape(np.sqrt(r2), radius, width, rho_g, rho_l)
    if amplitude:
        nz = noise(shape, amplitude, instance_id)
        rho = rho * (1.0 + nz) if relative else rho + nz
    return np.ascontiguousarray(rho)


def slab(shape, axis: int, width: float, rho_g: float, rho_l: float,
         amplitude: float = 1e-6, instance_id: int = 0, relative: bool = False) -> np.ndarray:
    """Flat liquid layer filling the central half of array axis ``axis``."""
    shape = tuple(int(s) for s in shape)
    H = shape[axis]
    c = np.arange(H, dtype=np.float64) - H / 2.0
    dist = np.abs(c)
    prof = _tanh_shape(dist, H / 4.0, width, rho_g, rho_l)
    bshape = [1] * len(shape)
    bshape[axis] = H
    rho = np.broadcast_to(prof.reshape(bshape), shape).copy()
    if amplitude:
        nz = noise(shape, amplitude, instance_id)
        rho = rho * (1.0 + nz) if relative else rho + nz
    return np.ascontiguousarray(rho)


def sweep_instances(n_slabs: int = 48, n_drops: int = 48, seed: int = 0, n_schemes: int = 6,
                    tr_range=(0.2, 0.95), k_range=(0.1, 0.25)):
    """Descriptors of an uneven droplet/slab sweep.

    Slabs are 8 x H with H uniform over multiples of 8 in [128, 1024]; droplets
    have R uniform in [10, 60] and side L uniform over multiples of 8 in
    [max(64, 2R + 64), 256].  Tr, k uniform in the given ranges; scheme id
    uniform over ``n_schemes``.  Returns a list of dicts."""
    rng = np.random.default_rng(SEED_BASE + seed)
    out = []
    for i in range(n_slabs):
        H = int(rng.integers(128 // 8, 1024 // 8 + 1)) * 8
        out.append(dict(kind="slab", nx=8, ny=H, Tr=float(rng.uniform(*tr_range)),
                        k=float(rng.uniform(*k_range)), scheme=int(rng.integers(0, n_schemes)),
                        radius=0.0, instance_id=i))
    for i in range(n_drops):
        R = float(rng.uniform(10.0, 60.0))
        lo = max(64, int(np.ceil((2 * R + 64) / 8.0)) * 8)
        L = int(rng.integers(lo // 8, 256 // 8 + 1)) * 8
        out.append(dict(kind="droplet", nx=L, ny=L, Tr=float(rng.uniform(*tr_range)),
                        k=float(rng.uniform(*k_range)), scheme=int(rng.integers(0, n_schemes)),
                        radius=R, instance_id=n_slabs + i))
    return out
