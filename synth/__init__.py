"""Seeded synthetic inputs for inverse ray-shooting (shared by the HIP path and the oracle).

This module only *draws* inputs: counter-based random numbers, lens fields,
macro-model parameters and the rectangular regions of the ray grid and of
the source map.  It holds none of the method's arithmetic (no deflection,
no lens equation, no binning), so both the GPU path and the CPU oracle may
import it.

Conventions (Thompson et al. 2009, section 1, eqs. 1-2 and section 3.2, eq. 6):
  * lengths are in Einstein radii of a unit-mass lens;
  * a lens record is four float32 values (x1, x2, m, 0);
  * the macro model is (kappa_c, gamma): smooth convergence and external shear.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used
as a counter-based hash: draw i of stream s under seed k is
``mix(key(k, s) + (i + 1) * GOLDEN)`` where ``mix`` is SplitMix64's output
function and ``key(k, s) = mix(k * GOLDEN ^ (s << 32))``.  A uniform double
in [0, 1) is ``(h >> 11) * 2**-53``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream identifiers, one per purpose
STREAM_MASS = 1
STREAM_POS = 2
STREAM_JOBS = 3
STREAM_SAMPLES = 4
STREAM_INIT = 5
STREAM_TILES = 6
STREAM_PROBE = 7


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GOLDEN ^ (np.uint64(stream) << np.uint64(32))
    return mix64(np.array([k], dtype=np.uint64))[0]


def hash_u64(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Counter-based draws h(seed, stream, idx) as uint64."""
    key = stream_key(seed, stream)
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + (idx + np.uint64(1)) * GOLDEN)


def uniform(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) for draws start .. start+count-1."""
    h = hash_u64(seed, stream, np.arange(start, start + count, dtype=np.uint64))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# lens fields
# --------------------------------------------------------------------------

def powerlaw_masses(seed: int, n: int, slope: float = 2.35, m_lo: float = 0.1, m_hi: float = 1.0,
                    stream: int = STREAM_MASS) -> np.ndarray:
    """Masses with dN/dm proportional to m**-slope on [m_lo, m_hi] by inverse CDF (float32).

    Variable lens masses are the paper's section 3.2 extension; the
    Salpeter slope 2.35 on [0.1, 1] is the workload's choice.
    """
    u = uniform(seed, stream, 0, n)
    p = 1.0 - slope
    a, b = m_lo ** p, m_hi ** p
    return np.power(a + u * (b - a), 1.0 / p).astype(np.float32)


def disc_positions(seed: int, n: int, radius: float, stream: int = STREAM_POS) -> np.ndarray:
    """n points uniform in the disc |x| < radius, by rejection from the square (float64, n x 2).

    Candidate j uses draws 2j and 2j+1 of the stream; candidates are taken in
    order and the first n accepted ones are kept.
    """
    out = np.empty((n, 2), dtype=np.float64)
    got, start = 0, 0
    while got < n:
        need = n - got
        batch = int(need * 1.35) + 64
        u = uniform(seed, stream, 2 * start, 2 * batch).reshape(batch, 2)
        xy = (2.0 * u - 1.0) * radius
        ok = (xy[:, 0] * xy[:, 0] + xy[:, 1] * xy[:, 1]) < radius * radius
        acc = xy[ok][:need]
        out[got:got + len(acc)] = acc
        got += len(acc)
        start += batch
    return out


def lens_records(pos: np.ndarray, mass: np.ndarray) -> np.ndarray:
    """Pack (x1, x2, m, 0) float32 records, n x 4."""
    n = len(mass)
    rec = np.zeros((n, 4), dtype=np.float32)
    rec[:, 0] = pos[:, 0].astype(np.float32)
    rec[:, 1] = pos[:, 1].astype(np.float32)
    rec[:, 2] = mass.astype(np.float32)
    return rec


def lens_field(seed: int, n: int, kappa_star: float | None = None, radius: float | None = None,
               equal_mass: bool = False) -> tuple[np.ndarray, float]:
    """A seeded field of n point lenses uniform in a disc centred on the origin.

    Either the disc radius is given, or it follows from the stellar
    convergence kappa_star = sum(m) / R**2 of the realised masses.
    Returns (records n x 4 float32, radius).
    """
    if equal_mass:
        m = np.ones(n, dtype=np.float32)
    else:
        m = powerlaw_masses(seed, n)
    if radius is None:
        if kappa_star is None or kappa_star <= 0:
            raise ValueError("need radius or kappa_star > 0")
        radius = math.sqrt(float(np.sum(m.astype(np.float64))) / kappa_star)
    pos = disc_positions(seed, n, radius)
    return lens_records(pos, m), radius


# --------------------------------------------------------------------------
# regions
# --------------------------------------------------------------------------

def ulp32(x: float) -> float:
    """Spacing of float32 values at magnitude x (x > 0, normal range)."""
    return float(np.spacing(np.float32(x)))


def shooting_region(map_half: tuple[float, float], kappa: float, gamma: float, n: tuple[int, int],
                    lens_radius: float, margin: float = 1.2, floor: float = 0.05):
    """Centred ray-grid rectangle covering the source map's mean preimage.

    The half-width along axis k is margin * map_half_k / max(|lambda_k|, floor)
    with lambda = (1 - kappa - gamma, 1 - kappa + gamma) the mean Jacobian of
    the lens mapping (total convergence kappa).  The cell size is then rounded
    up to a multiple of 2 ulp32(half-width + lens_radius), so every ray
    coordinate lies on a coarse binary lattice.  Returns (lo, hi, n).
    """
    lam = (1.0 - kappa - gamma, 1.0 - kappa + gamma)
    lo, hi = [0.0, 0.0], [0.0, 0.0]
    for k in range(2):
        half = margin * map_half[k] / max(abs(lam[k]), floor)
        q = 2.0 * ulp32(half + lens_radius)
        step = math.ceil((2.0 * half / n[k]) / q) * q
        lo[k] = -0.5 * n[k] * step
        hi[k] = 0.5 * n[k] * step
    return tuple(lo), tuple(hi), tuple(int(v) for v in n)


def smooth_kappa(kappa_star: float, smooth_fraction: float) -> float:
    """kappa_c for a smooth fraction s = kappa_c / (kappa_star + kappa_c)."""
    return kappa_star * smooth_fraction / (1.0 - smooth_fraction)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """One map: lenses, macro model, ray grid and source map."""
    name: str
    lenses: np.ndarray               # n x 4 float32 (x1, x2, m, 0)
    kappa_c: float
    gamma: float
    grid_lo: tuple
    grid_hi: tuple
    grid_n: tuple
    map_lo: tuple
    map_hi: tuple
    map_n: tuple
    kappa_star: float = 0.0
    lens_radius: float = 0.0
    extra: dict = field(default_factory=dict)
    jitter_seed: int | None = None    # None: rays at cell centres; else one seeded random ray per cell

    @property
    def n_rays(self) -> int:
        return int(self.grid_n[0]) * int(self.grid_n[1])

    @property
    def n_lens(self) -> int:
        return int(self.lenses.shape[0])

    def n_av(self) -> float:
        """Rays per source pixel without lensing (pixel area / ray-cell area)."""
        dx = [(self.grid_hi[k] - self.grid_lo[k]) / self.grid_n[k] for k in range(2)]
        dy = [(self.map_hi[k] - self.map_lo[k]) / self.map_n[k] for k in range(2)]
        return dy[0] * dy[1] / (dx[0] * dx[1])


def workload_small(seed: int = 1) -> Workload:
    """100 unit-mass lenses in a disc of radius 12, no macro term, 1000^2 rays on [-10,10]^2,
    100^2 map on [-5,5]^2."""
    lenses, r = lens_field(seed, 100, radius=12.0, equal_mass=True)
    return Workload("small-100lens-1000sq", lenses, 0.0, 0.0, (-10.0, -10.0), (10.0, 10.0), (1000, 1000),
                    (-5.0, -5.0), (5.0, 5.0), (100, 100), kappa_star=100.0 / 144.0, lens_radius=r)


def workload_paper(seed: int = 2, n_lens: int = 100_000, grid: int = 4096, mapn: int = 1024) -> Workload:
    """1e5 power-law lenses, kappa_*=0.45, gamma=0.45, no smooth matter, 4096^2 rays covering the
    shooting region, 1024^2 map over 20x20."""
    ks, g = 0.45, 0.45
    lenses, r = lens_field(seed, n_lens, kappa_star=ks)
    lo, hi, n = shooting_region((10.0, 10.0), ks, g, (grid, grid), r)
    return Workload(f"paper-{n_lens}lens-{grid}sq", lenses, 0.0, g, lo, hi, n, (-10.0, -10.0),
                    (10.0, 10.0), (mapn, mapn), kappa_star=ks, lens_radius=r)


def workload_farfield(seed: int = 4, n_lens: int = 1_000_000, grid: int = 8192, mapn: int = 1024) -> Workload:
    """1e6 power-law lenses, kappa_*=0.6, gamma=0.3, 8192^2 rays, 1024^2 map over 20x20."""
    ks, g = 0.6, 0.3
    lenses, r = lens_field(seed, n_lens, kappa_star=ks)
    lo, hi, n = shooting_region((10.0, 10.0), ks, g, (grid, grid), r)
    return Workload(f"farfield-{n_lens}lens-{grid}sq", lenses, 0.0, g, lo, hi, n, (-10.0, -10.0),
                    (10.0, 10.0), (mapn, mapn), kappa_star=ks, lens_radius=r)


def workload_large(seed: int = 5, n_lens: int = 10_000_000, grid: int = 32768, mapn: int = 2048) -> Workload:
    """1e7 power-law lenses, kappa_*=0.5, gamma=0.5, smooth fraction 0.3, 32768^2 rays, 2048^2 map."""
    ks, g, s = 0.5, 0.5, 0.3
    kc = smooth_kappa(ks, s)
    lenses, r = lens_field(seed, n_lens, kappa_star=ks)
    lo, hi, n = shooting_region((10.0, 10.0), ks + kc, g, (grid, grid), r)
    return Workload(f"large-{n_lens}lens-{grid}sq", lenses, kc, g, lo, hi, n, (-10.0, -10.0),
                    (10.0, 10.0), (mapn, mapn), kappa_star=ks, lens_radius=r)


def batched_jobs(seed: int = 3, n_jobs: int = 64, scale: int = 1) -> list[Workload]:
    """64 maps with N_* log-uniform in [1e3, 1e5], kappa_* ~ U[0.1, 0.8], gamma ~ U[0, 0.6],
    smooth fraction in {0, 0.5}, ray grids in {1024, 2048, 4096}^2, maps in {256, 512, 1024}^2
    over 20x20.  ``scale`` divides grid sides and lens counts (for small test batches)."""
    jobs = []
    u = uniform(seed, STREAM_JOBS, 0, 8 * n_jobs).reshape(n_jobs, 8)
    for j in range(n_jobs):
        n_lens = max(1, int(round(10.0 ** (3.0 + 2.0 * u[j, 0]))) // scale)
        ks = 0.1 + 0.7 * u[j, 1]
        g = 0.6 * u[j, 2]
        s = 0.5 if u[j, 3] >= 0.5 else 0.0
        side = (1024, 2048, 4096)[min(2, int(u[j, 4] * 3))] // scale
        mside = (256, 512, 1024)[min(2, int(u[j, 5] * 3))] // scale
        kc = smooth_kappa(ks, s)
        lenses, r = lens_field(seed * 1000 + j + 1, n_lens, kappa_star=ks)
        lo, hi, n = shooting_region((10.0, 10.0), ks + kc, g, (side, side), r)
        jobs.append(Workload(f"job{j}", lenses, kc, g, lo, hi, n, (-10.0, -10.0), (10.0, 10.0),
                             (mside, mside), kappa_star=ks, lens_radius=r))
    return jobs


def sample_indices(seed: int, total: int, count: int, stream: int = STREAM_PROBE) -> np.ndarray:
    """count distinct sorted indices in [0, total) drawn with the counter hash."""
    count = min(count, total)
    got = np.zeros(0, dtype=np.int64)
    start = 0
    while len(got) < count:
        h = hash_u64(seed, stream, np.arange(start, start + 2 * count, dtype=np.uint64))
        cand = (h % np.uint64(total)).astype(np.int64)
        got = np.unique(np.concatenate([got, cand]))
        start += 2 * count
    sel = hash_u64(seed + 1, stream, np.arange(len(got), dtype=np.uint64))
    order = np.argsort(sel, kind="stable")[:count]
    return np.sort(got[order])


# --------------------------------------------------------------------------
# inputs of the learned far-field fit
# --------------------------------------------------------------------------

def fit_samples(seed: int, n: int = 4096) -> np.ndarray:
    """n tile-local sample points uniform in [-1, 1]^2 (float32, n x 2)."""
    return (uniform(seed, STREAM_SAMPLES, 0, 2 * n).reshape(n, 2) * 2.0 - 1.0).astype(np.float32)


def fit_samples_quads(seed: int, n: int = 4096) -> np.ndarray:
    """n tile-local sample points in [-1, 1]^2 (n a multiple of 256), each coordinate a seeded
    uniform draw, except that samples 64 (4 g + k) + i, k = 0..3, share their first coordinate
    (one draw per quad): n / 4 distinct first and n distinct second coordinates."""
    d = uniform(seed, STREAM_SAMPLES, 0, n // 4 + n) * 2.0 - 1.0
    x = d[: n // 4].reshape(n // 256, 1, 64)
    pts = np.empty((n // 256, 4, 64, 2))
    pts[..., 0] = x
    pts[..., 1] = d[n // 4:].reshape(n // 256, 4, 64)
    return np.ascontiguousarray(pts.reshape(n, 2).astype(np.float32))


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform initial parameters of the 16 -> 64 -> 64 -> 2 network, zero biases
    (float32, 5378 values in the order W1 [64][16], b1, W2 [64][64], b2, W3 [2][64], b3)."""
    p = np.zeros(5378, dtype=np.float64)
    u = uniform(seed, STREAM_INIT, 0, 5378)
    for off, fan_in, fan_out in ((0, 16, 64), (1088, 64, 64), (5248, 64, 2)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        n = fan_in * fan_out
        p[off:off + n] = (2.0 * u[off:off + n] - 1.0) * a
    return p.astype(np.float32)


STREAM_MAP = 10
STREAM_TRACKS = 11


def count_map(seed: int, n: tuple[int, int], mean: float) -> np.ndarray:
    """A seeded uint32 count map of n[1] rows x n[0] columns with the given mean and a heavy
    upper tail (N = floor(4 mean u^3), u uniform), standing in for a magnification map's counts."""
    u = uniform(seed, STREAM_MAP, 0, int(n[0]) * int(n[1])).reshape(int(n[1]), int(n[0]))
    return np.floor(4.0 * mean * u ** 3).astype(np.uint32)


def light_tracks(seed: int, n_tracks: int, lo: tuple[float, float], hi: tuple[float, float],
                 length: float) -> np.ndarray:
    """n_tracks straight tracks (start1, start2, end1, end2): start uniform over [lo, hi), direction
    uniform in angle, the given length (ends may leave the region)."""
    u = uniform(seed, STREAM_TRACKS, 0, 3 * n_tracks).reshape(n_tracks, 3)
    s1 = lo[0] + u[:, 0] * (hi[0] - lo[0])
    s2 = lo[1] + u[:, 1] * (hi[1] - lo[1])
    th = 2.0 * np.pi * u[:, 2]
    return np.stack([s1, s2, s1 + length * np.cos(th), s2 + length * np.sin(th)], 1)


STREAM_VEL = 12


def lens_velocities(seed: int, n: int, sigma: float) -> np.ndarray:
    """n x 2 float32 lens velocities, each component normal with standard deviation sigma
    (Box-Muller on the seeded uniforms)."""
    u = uniform(seed, STREAM_VEL, 0, 2 * n).reshape(n, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
    th = 2.0 * np.pi * u[:, 1]
    return (sigma * np.stack([r * np.cos(th), r * np.sin(th)], 1)).astype(np.float32)
