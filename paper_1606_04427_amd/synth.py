"""Seeded synthetic particle sets, palettes and camera poses.

Stand-ins for the paper's Gadget N-body/SPH snapshot (Sect. 4.1: 50M gas +
5M star particles for single-node tests, 200M + 20M for the GPU comparison),
which is not available.  Every generator here only draws inputs: positions,
smoothing lengths, intensities, colour scalars, species, absorption,
palettes and camera poses.  None of the render arithmetic lives here; the
HIP path and the FP64 oracle both consume these arrays unchanged.

All generators use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ParticleSet:
    x: np.ndarray  # float32 world positions
    y: np.ndarray
    z: np.ndarray
    h: np.ndarray  # float32 smoothing length, world units
    intensity: np.ndarray  # float32
    scalar: np.ndarray  # float32 colour scalar
    species: np.ndarray  # uint8
    absorption: np.ndarray | None = None  # float32, sorted mode
    meta: dict = field(default_factory=dict)
    rgb: np.ndarray | None = None  # float32 (n, 3) colour vector field

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "ParticleSet":
        a = None if self.absorption is None else self.absorption[idx]
        c = None if self.rgb is None else self.rgb[idx]
        return ParticleSet(self.x[idx], self.y[idx], self.z[idx], self.h[idx],
                           self.intensity[idx], self.scalar[idx], self.species[idx],
                           a, dict(self.meta), c)


@dataclass
class Pose:
    eye: tuple
    lookat: tuple
    up: tuple
    fov_y_deg: float
    z_near: float
    width: int
    height: int


def palette(kind: int, n_entries: int = 256) -> np.ndarray:
    """Smooth monotone RGB ramps built from power laws over a dim floor, shape
    (n_entries, 3).

    kind selects the exponents; 0 is a warm ramp (gas), 1 a cold ramp (stars),
    2..7 mixed ramps for a bank of looks."""
    t = np.linspace(0.0, 1.0, n_entries)
    exps = [
        (0.5, 1.5, 4.0),
        (3.0, 1.2, 0.4),
        (1.0, 1.0, 1.0),
        (0.7, 2.5, 1.8),
        (2.0, 0.6, 2.2),
        (1.4, 0.9, 0.5),
        (0.4, 0.8, 3.0),
        (2.6, 2.0, 0.8),
    ]
    er, eg, eb = exps[kind % len(exps)]
    # dim, non-black floor so the lowest scalar still emits
    rgb = 0.04 + 0.96 * np.stack([t ** er, t ** eg, t ** eb], axis=1)
    return np.ascontiguousarray(rgb, dtype=np.float32)


def blobs(n: int, seed: int = 1000, n_blobs: int = 64) -> ParticleSet:
    """Isotropic Gaussian blobs in the unit cube (the 100k-particle workload).

    64 centres uniform in [0.1, 0.9]^3, per-blob width uniform in
    [0.02, 0.1]; positions outside the unit cube are redrawn.  The smoothing
    length is log-normal so that, seen from 2 units away with a 40-degree
    256-px view (0.005687 world units per px at that depth), the projected
    size is log-normal about 2 px, clipped to [0.5, 8] px.  Intensity is
    log-normal (median 1) and is also the colour scalar."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.1, 0.9, size=(n_blobs, 3))
    widths = rng.uniform(0.02, 0.1, size=n_blobs)
    which = rng.integers(0, n_blobs, size=n)
    pos = centres[which] + widths[which, None] * rng.standard_normal((n, 3))
    bad = np.any((pos < 0.0) | (pos > 1.0), axis=1)
    while bad.any():
        k = int(bad.sum())
        pos[bad] = centres[which[bad]] + widths[which[bad], None] * rng.standard_normal((k, 3))
        bad = np.any((pos < 0.0) | (pos > 1.0), axis=1)
    px = np.exp(rng.normal(math.log(2.0), 0.69, size=n)).clip(0.5, 8.0)
    world_per_px = 2.0 * math.tan(math.radians(20.0)) / 128.0
    h = px * world_per_px
    inten = np.exp(rng.normal(0.0, 1.0, size=n))
    pos = pos.astype(np.float32)
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(),
                       h.astype(np.float32), inten.astype(np.float32),
                       inten.astype(np.float32), np.zeros(n, np.uint8),
                       meta={"kind": "blobs", "seed": seed})


def blobs_camera(width: int = 256, height: int = 256) -> Pose:
    return Pose((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 40.0, 1e-3, width, height)


def soneira_peebles(n: int, seed: int = 1001, levels: int = 4, branch: int = 8,
                    lam: float = 3.0, field_frac: float = 0.05,
                    star_frac: float = 0.10, eta: float = 1.3,
                    absorption: bool = False, chunk: int = 1 << 22) -> ParticleSet:
    """Hierarchically clustered set (Soneira-Peebles construction).

    The root sphere (centre 0.5, radius 0.5) holds `branch` child centres drawn
    uniformly inside it, each with radius / lam; repeated `levels` times this
    gives branch**levels leaves.  (1 - field_frac) of the particles go to the
    leaves in equal shares (multinomial), Gaussian about the leaf centre with
    width r_leaf / 2; the rest are uniform in the unit cube.  Particles are
    stored leaf by leaf, the field particles last.

    Species: star_frac of the particles are species 1, the rest species 0
    (the paper's data set has one star per ten gas particles).  The local
    number density n_p is that of the particle's generating component (leaf
    Gaussian plus the uniform field) and the smoothing length follows the SPH
    convention h = eta * n_p^(-1/3).  The colour scalar is n_p (rendered on a
    log scale), the intensity is log-normal.  With absorption=True each
    particle also gets an absorption coefficient uniform in [0.01, 0.5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = np.array([[0.5, 0.5, 0.5]])
    radius = 0.5
    for _ in range(levels):
        k = centres.shape[0]
        d = rng.standard_normal((k, branch, 3))
        d /= np.linalg.norm(d, axis=2, keepdims=True)
        rr = radius * rng.uniform(0.0, 1.0, size=(k, branch, 1)) ** (1.0 / 3.0)
        centres = (centres[:, None, :] + d * rr).reshape(-1, 3)
        radius /= lam
    n_leaves = centres.shape[0]
    n_field = int(round(field_frac * n))
    n_clustered = n - n_field
    per_leaf = rng.multinomial(n_clustered, np.full(n_leaves, 1.0 / n_leaves))
    width = radius / 2.0
    field_density = n_field / 1.0
    x = np.empty(n, np.float32)
    y = np.empty(n, np.float32)
    z = np.empty(n, np.float32)
    dens = np.empty(n, np.float64)
    leaf_of = np.repeat(np.arange(n_leaves), per_leaf)
    norm = (2.0 * math.pi * width * width) ** -1.5
    for s in range(0, n_clustered, chunk):
        e = min(n_clustered, s + chunk)
        off = rng.standard_normal((e - s, 3)) * width
        p = centres[leaf_of[s:e]] + off
        r2 = np.einsum("ij,ij->i", off, off)
        dens[s:e] = per_leaf[leaf_of[s:e]] * norm * np.exp(-0.5 * r2 / (width * width)) + field_density
        x[s:e] = p[:, 0]
        y[s:e] = p[:, 1]
        z[s:e] = p[:, 2]
    if n_field:
        p = rng.uniform(0.0, 1.0, size=(n_field, 3))
        x[n_clustered:] = p[:, 0]
        y[n_clustered:] = p[:, 1]
        z[n_clustered:] = p[:, 2]
        dens[n_clustered:] = field_density
    h = (eta * dens ** (-1.0 / 3.0)).astype(np.float32)
    species = (rng.uniform(0.0, 1.0, size=n) < star_frac).astype(np.uint8)
    inten = np.exp(rng.normal(0.0, 0.5, size=n)).astype(np.float32)
    absorb = rng.uniform(0.01, 0.5, size=n).astype(np.float32) if absorption else None
    return ParticleSet(x, y, z, h, inten, dens.astype(np.float32), species, absorb,
                       meta={"kind": "soneira_peebles", "seed": seed, "levels": levels,
                             "branch": branch, "lam": lam, "n_leaves": n_leaves})


def colour_field(ps: ParticleSet, seed: int = 4001, dim: float = 0.04) -> np.ndarray:
    """A colour vector field for the set, shape (n, 3) float32: a smooth
    function of position (each channel a sinusoid of a random direction, as a
    velocity or magnetic-field direction mapped to RGB would be) in
    [dim, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = np.stack([ps.x, ps.y, ps.z], axis=1).astype(np.float64)
    k = rng.normal(0.0, 6.0, size=(3, 3))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
    c = 0.5 + 0.5 * np.sin(pos @ k.T + ph)
    return np.ascontiguousarray(dim + (1.0 - dim) * c, dtype=np.float32)


def random_poses(count: int, seed: int = 2001, width: int = 1024, height: int = 1024,
                 fov_y_deg: float = 50.0, z_near: float = 0.05,
                 dist_range=(0.6, 3.0)) -> list[Pose]:
    """Camera poses around the unit cube: direction uniform on the sphere,
    distance from the cube centre log-uniform in dist_range (the closest sit
    inside the cube), look-at point = centre + N(0, 0.05^2), random up vector
    orthogonal to the view direction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    c = np.array([0.5, 0.5, 0.5])
    for _ in range(count):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        dist = math.exp(rng.uniform(math.log(dist_range[0]), math.log(dist_range[1])))
        eye = c + dist * d
        look = c + rng.normal(0.0, 0.05, size=3)
        fwd = look - eye
        fwd /= np.linalg.norm(fwd)
        u = rng.standard_normal(3)
        u -= fwd * np.dot(u, fwd)
        u /= np.linalg.norm(u)
        out.append(Pose(tuple(map(float, eye)), tuple(map(float, look)), tuple(map(float, u)),
                        fov_y_deg, z_near, width, height))
    return out


def _look_at_centre(eye, width, height, fov_y_deg, z_near, up_hint=(0.0, 0.0, 1.0)) -> Pose:
    c = np.array([0.5, 0.5, 0.5])
    fwd = c - np.asarray(eye, dtype=np.float64)
    fwd /= np.linalg.norm(fwd)
    u = np.asarray(up_hint, dtype=np.float64)
    u = u - fwd * np.dot(u, fwd)
    if np.linalg.norm(u) < 1e-9:
        u = np.array([0.0, 1.0, 0.0]) - fwd * fwd[1]
    u /= np.linalg.norm(u)
    return Pose(tuple(map(float, eye)), tuple(map(float, c)), tuple(map(float, u)), fov_y_deg,
                z_near, width, height)


def orbit_poses(count: int = 100, radius: float = 1.6, elevation_deg: float = 20.0,
                width: int = 1024, height: int = 1024, fov_y_deg: float = 50.0,
                z_near: float = 0.05) -> list[Pose]:
    """An animation orbit: count frames evenly spaced in azimuth on a circle
    of the given radius around the cube centre, raised by elevation_deg,
    each looking at the centre with z up."""
    c = np.array([0.5, 0.5, 0.5])
    el = math.radians(elevation_deg)
    out = []
    for k in range(count):
        az = 2.0 * math.pi * k / count
        d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        out.append(_look_at_centre(c + radius * d, width, height, fov_y_deg, z_near))
    return out


def sweep_poses(count: int = 6, far: float = 3.0, near: float = 0.6, width: int = 1024,
                height: int = 1024, fov_y_deg: float = 50.0, z_near: float = 0.05,
                direction=(0.6, -0.48, 0.64)) -> list[Pose]:
    """Camera positions from far to near along one direction from the cube
    centre, distances log-spaced, each looking at the centre: projected radii
    grow from pose to pose."""
    c = np.array([0.5, 0.5, 0.5])
    d = np.asarray(direction, dtype=np.float64)
    d /= np.linalg.norm(d)
    out = []
    for k in range(count):
        f = k / max(count - 1, 1)
        dist = math.exp(math.log(far) + f * (math.log(near) - math.log(far)))
        out.append(_look_at_centre(c + dist * d, width, height, fov_y_deg, z_near))
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 3001) -> np.ndarray:
    """Arrival times (s) of a Poisson request stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
