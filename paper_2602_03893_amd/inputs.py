"""Seeded synthetic inputs: acquisition geometries, phantoms and noise.

This module is the one piece shared by the HIP path's tests and the CPU
oracle's tests.  It holds none of the GPAIR method's arithmetic: it only lays
out sensors and kernel centres and draws amplitudes and noise from seeded
generators (``numpy.random.default_rng``).

The paper's own ground truth (a synthetic vascular network volume and its
k-Wave traces) and its in vivo data are not available; seeded vessel trees and
spheres stand in for them, laid out at the paper's shapes (a kernel grid of
256 x 256 x 128 at 0.1 mm and a 1024-element hemispherical array for the in
vivo configuration: Results, "Validation on in vivo experimental results", and
the footnote of its table).

Layouts
 - kernel grid: centres at ((i - (N-1)/2) * spacing, ...), stored [iz][iy][ix]
   (x fastest), float32 metres;
 - sensors: a Fibonacci lattice on the lower hemisphere of radius R centred at
   the grid centre, u_j = (j + 1/2)/N, phi_j = j * pi * (3 - sqrt 5),
   s_j = R (sqrt(1-u^2) cos phi, sqrt(1-u^2) sin phi, -u), float32 metres.
"""
from dataclasses import dataclass, field

import numpy as np

C_SOUND = 1500.0  # m/s
FS = 40e6  # Hz
DT = 1.0 / FS


@dataclass(frozen=True)
class Workload:
    """One acquisition/reconstruction configuration (sizes in kernels, metres)."""
    name: str
    grid: tuple          # (nx, ny, nz)
    spacing: float       # m
    sigma: float         # m, initial / fixed kernel width
    n_sensors: int
    radius: float        # m, hemisphere radius
    n_samples: int
    phantom: str         # "spheres" | "vessels"
    phantom_seed: int
    noise: float         # relative noise level (fraction of trace RMS), 0 = clean
    noise_seed: int
    dt: float = DT
    t0: float = 0.0
    c_sound: float = C_SOUND
    n_sigma: float = 3.0
    sigma_max: float = 0.0   # 0: equal to sigma
    extra: dict = field(default_factory=dict)

    @property
    def n_kernels(self):
        return self.grid[0] * self.grid[1] * self.grid[2]

    @property
    def smax(self):
        return self.sigma_max if self.sigma_max > 0 else self.sigma


# The five configurations of this build (toy, mid-size, paper scale, learned
# warm start training grid, full pipeline).
WORKLOADS = {
    "toy": Workload("toy", (16, 16, 16), 0.2e-3, 0.1e-3, 64, 10e-3, 512,
                    "spheres", 1, 0.0, 0),
    "mid": Workload("mid", (64, 64, 64), 0.1e-3, 0.05e-3, 512, 20e-3, 2048,
                    "vessels", 2, 0.01, 1002),
    "paper": Workload("paper", (256, 256, 128), 0.1e-3, 0.05e-3, 1024, 40e-3, 4096,
                      "vessels", 3, 0.0, 0, sigma_max=0.1e-3),
    "half": Workload("half", (128, 128, 64), 0.2e-3, 0.1e-3, 1024, 40e-3, 4096,
                     "vessels", 0, 0.01, 0),
}
# The simulation study's shapes (its results table): a 512 x 512 x 256 grid
# (0.1 mm, so 51.2 x 51.2 x 25.6 mm) seen by a 102.4 mm square planar array
# (20 mm below the grid centre, 7.2 mm below its lower face) or an R = 60 mm
# hemisphere, each with 64, 256 or 1024 elements.
for _n in (64, 256, 1024):
    WORKLOADS[f"t1_planar_{_n}"] = Workload(
        f"t1_planar_{_n}", (512, 512, 256), 0.1e-3, 0.05e-3, _n, 0.0, 4096, "vessels", 4,
        0.0, 0, sigma_max=0.1e-3, extra={"array": "planar", "width": 102.4e-3,
                                         "plane_z": -20e-3})
    WORKLOADS[f"t1_hemi_{_n}"] = Workload(
        f"t1_hemi_{_n}", (512, 512, 256), 0.1e-3, 0.05e-3, _n, 60e-3, 4096, "vessels", 4,
        0.0, 0, sigma_max=0.1e-3)


def grid_centres(nx, ny, nz, spacing):
    """(nx*ny*nz, 3) float32 centres of a grid centred at the origin, x fastest."""
    xs = (np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0) * spacing
    ys = (np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0) * spacing
    zs = (np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0) * spacing
    out = np.empty((nz, ny, nx, 3), dtype=np.float32)
    out[..., 0] = xs.astype(np.float32)[None, None, :]
    out[..., 1] = ys.astype(np.float32)[None, :, None]
    out[..., 2] = zs.astype(np.float32)[:, None, None]
    return out.reshape(-1, 3)


def planar_array(n, width, z):
    """(n, 3) float32 points of a square array: sqrt(n) x sqrt(n) elements at
    pitch width / sqrt(n), centred on the z axis, in the plane at height z."""
    k = int(round(np.sqrt(n)))
    if k * k != n:
        raise ValueError("planar array: n must be a perfect square")
    a = (np.arange(k, dtype=np.float64) - (k - 1) / 2.0) * (width / k)
    Y, X = np.meshgrid(a, a, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(n, z)], axis=1).astype(np.float32)


def fibonacci_hemisphere(n, radius):
    """(n, 3) float32 points on the lower hemisphere of the given radius."""
    j = np.arange(n, dtype=np.float64)
    u = (j + 0.5) / n
    phi = j * np.pi * (3.0 - np.sqrt(5.0))
    rho = np.sqrt(1.0 - u * u)
    pts = radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), -u], axis=1)
    return pts.astype(np.float32)


def _grid_axes(shape, spacing):
    nx, ny, nz = shape
    return ((np.arange(nx) - (nx - 1) / 2.0) * spacing,
            (np.arange(ny) - (ny - 1) / 2.0) * spacing,
            (np.arange(nz) - (nz - 1) / 2.0) * spacing)


def _paint_ball(vol, axes, centre, radius, value, mode="max"):
    xs, ys, zs = axes
    sl = []
    for ax, c in zip((xs, ys, zs), centre):
        lo = np.searchsorted(ax, c - radius)
        hi = np.searchsorted(ax, c + radius, side="right")
        sl.append((lo, hi))
    (x0, x1), (y0, y1), (z0, z1) = sl
    if x0 >= x1 or y0 >= y1 or z0 >= z1:
        return
    X = xs[x0:x1][None, None, :]
    Y = ys[y0:y1][None, :, None]
    Z = zs[z0:z1][:, None, None]
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2 <= radius * radius
    sub = vol[z0:z1, y0:y1, x0:x1]
    if mode == "set":
        sub[inside] = value
    else:
        np.maximum(sub, np.where(inside, value, 0.0), out=sub)


def spheres_phantom(shape, spacing, n_spheres=3, seed=1, background=0.05,
                    r_range=(0.3e-3, 0.8e-3)):
    """Spheres of value 1 (union) on a zero background, plus U[0, background]
    added to every kernel.  Centres uniform in the inner 60 % of the volume.
    Returns float32 [M] in grid order."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    axes = _grid_axes(shape, spacing)
    ext = np.array([(nx - 1) * spacing, (ny - 1) * spacing, (nz - 1) * spacing])
    for _ in range(n_spheres):
        c = rng.uniform(-0.3, 0.3, 3) * ext
        r = rng.uniform(*r_range)
        _paint_ball(vol, axes, c, r, 1.0, mode="set")
    vol += rng.uniform(0.0, background, vol.shape)
    return vol.reshape(-1).astype(np.float32)


def _segment_paint(vol, axes, p0, p1, radius, value):
    xs, ys, zs = axes
    lo = np.minimum(p0, p1) - radius
    hi = np.maximum(p0, p1) + radius
    x0, x1 = np.searchsorted(xs, lo[0]), np.searchsorted(xs, hi[0], side="right")
    y0, y1 = np.searchsorted(ys, lo[1]), np.searchsorted(ys, hi[1], side="right")
    z0, z1 = np.searchsorted(zs, lo[2]), np.searchsorted(zs, hi[2], side="right")
    if x0 >= x1 or y0 >= y1 or z0 >= z1:
        return
    X = xs[x0:x1][None, None, :]
    Y = ys[y0:y1][None, :, None]
    Z = zs[z0:z1][:, None, None]
    d = p1 - p0
    L2 = float(np.dot(d, d))
    t = ((X - p0[0]) * d[0] + (Y - p0[1]) * d[1] + (Z - p0[2]) * d[2]) / max(L2, 1e-30)
    t = np.clip(t, 0.0, 1.0)
    dist2 = (X - p0[0] - t * d[0]) ** 2 + (Y - p0[1] - t * d[1]) ** 2 + (Z - p0[2] - t * d[2]) ** 2
    sub = vol[z0:z1, y0:y1, x0:x1]
    np.maximum(sub, np.where(dist2 <= radius * radius, value, 0.0), out=sub)


def _rotate_random(rng, direction, max_angle):
    """Perturb a unit vector by an angle uniform in [0, max_angle]."""
    d = direction / np.linalg.norm(direction)
    a = rng.standard_normal(3)
    a -= np.dot(a, d) * d
    a /= np.linalg.norm(a)
    ang = rng.uniform(0.0, max_angle)
    out = np.cos(ang) * d + np.sin(ang) * a
    return out / np.linalg.norm(out)


def vessel_tree_segments(shape, spacing, seed, n_roots=None, depth=6,
                         branch_p=0.3, seg_len=(1e-3, 4e-3),
                         r_range=(0.1e-3, 0.4e-3), max_turn=np.pi / 6):
    """Seeded random branching tree: list of (p0, p1, radius, value)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    half = 0.5 * np.array([(nx - 1) * spacing, (ny - 1) * spacing, (nz - 1) * spacing])
    if n_roots is None:
        n_roots = int(rng.integers(3, 6))
    segs = []
    for _ in range(n_roots):
        value = rng.uniform(0.5, 1.0)
        axis = int(rng.integers(0, 3))
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        start = rng.uniform(-0.8, 0.8, 3) * half
        start[axis] = sign * half[axis]
        heading = np.zeros(3)
        heading[axis] = -sign
        heading = _rotate_random(rng, heading, max_turn)
        radius = rng.uniform(0.25e-3, r_range[1])
        stack = [(start, heading, radius, depth)]
        while stack:
            p, h, rad, left = stack.pop()
            if left <= 0:
                continue
            q = p + h * rng.uniform(*seg_len)
            segs.append((p.copy(), q.copy(), rad, value))
            if np.any(np.abs(q) > half * 1.05):
                continue
            stack.append((q, _rotate_random(rng, h, max_turn), rad, left - 1))
            if rng.uniform() < branch_p:
                child = float(np.clip(rad * rng.uniform(0.7, 0.9), *r_range))
                stack.append((q, _rotate_random(rng, h, np.pi / 3), child, left - 1))
    return segs


def vessel_phantom(shape, spacing, seed, n_spheres_mean=0.0,
                   sphere_r=(0.3e-3, 1.5e-3)):
    """Vessel tree (A_k = max over segments of value * [dist <= radius]) on a
    zero background, optionally with Poisson(n_spheres_mean) spheres of value
    U[0.5, 1].  Returns float32 [M] in grid order."""
    nx, ny, nz = shape
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    axes = _grid_axes(shape, spacing)
    for p0, p1, rad, val in vessel_tree_segments(shape, spacing, seed):
        _segment_paint(vol, axes, p0, p1, rad, val)
    if n_spheres_mean > 0:
        rng = np.random.default_rng(seed + 7919)
        ext = np.array([(nx - 1) * spacing, (ny - 1) * spacing, (nz - 1) * spacing])
        for _ in range(int(rng.poisson(n_spheres_mean))):
            c = rng.uniform(-0.4, 0.4, 3) * ext
            _paint_ball(vol, axes, c, rng.uniform(*sphere_r), rng.uniform(0.5, 1.0))
    return vol.reshape(-1).astype(np.float32)


def phantom(w: Workload):
    if w.phantom == "spheres":
        return spheres_phantom(w.grid, w.spacing, seed=w.phantom_seed)
    return vessel_phantom(w.grid, w.spacing, w.phantom_seed)


def standard_normal(shape, seed, dtype=np.float32):
    """Seeded N(0, 1) draws (noise and random test vectors)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def uniform(shape, seed, lo=0.0, hi=1.0, dtype=np.float32):
    return np.random.default_rng(seed).uniform(lo, hi, shape).astype(dtype)


def sensor_array(w: Workload):
    """(N_d, 3) float32 sensor positions of a workload."""
    if w.extra.get("array") == "planar":
        return planar_array(w.n_sensors, w.extra["width"], w.extra["plane_z"])
    return fibonacci_hemisphere(w.n_sensors, w.radius)


def geometry_arrays(w: Workload):
    """(centres (M,3) float32, sensors (N_d,3) float32) of a workload."""
    return grid_centres(*w.grid, w.spacing), sensor_array(w)


def covariances(m, seed, lo, hi):
    """Seeded anisotropic covariances, (6, m) float32 (rows xx, yy, zz, xy, xz,
    yz, m^2): R diag(s1^2, s2^2, s3^2) R^T with axes s_i ~ U[lo, hi] and R a
    uniformly random rotation (QR of a Gaussian matrix, sign-fixed).  Vectorised
    over kernels; the entries are rounded to float32 once, and the operators
    and the oracle both take those float32 values."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, 3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    s2 = rng.uniform(lo, hi, (m, 3)) ** 2
    c = np.einsum("kij,kj,klj->kil", q, s2, q)
    out = np.stack([c[:, 0, 0], c[:, 1, 1], c[:, 2, 2], c[:, 0, 1], c[:, 0, 2], c[:, 1, 2]])
    return out.astype(np.float32)
