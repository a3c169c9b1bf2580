"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *generates inputs*: acquisition geometries, ellipsoid
phantoms, random rigid poses, per-view motion and smooth detector images.
It contains none of the projector arithmetic (no ray marching, no
interpolation, no gradients of the method), so that the oracle and the HIP
path stay independent while consuming bit-identical inputs.

Conventions (units): millimetres for lengths, radians for the pose angles
(configs quote degrees; the generators convert), mm^-1 for attenuation.
Pose vectors are ordered (tx, ty, tz, gx, gy, gz) as in the paper's notation
table (theta = (t, gamma)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.ndimage import gaussian_filter1d

SEED_BASE = 13304


def rng_for(config_index: int, salt: int = 0) -> np.random.Generator:
    """Generator(PCG64(13304 + config index)); `salt` derives independent sub-streams."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_index, salt]))


@dataclasses.dataclass
class Geom:
    """Cone-beam acquisition + voxel grid description (all lengths in mm).

    Volume memory order is [nz][ny][nx] (x fastest); detector images are
    [nv][nu] (u fastest).  off_u/off_v shift the detector centre in pixels.
    """
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    nu: int
    nv: int
    du: float
    dv: float
    off_u: float = 0.0
    off_v: float = 0.0
    sad: float = 1000.0
    sdd: float = 1500.0
    step: float = 0.5

    def replace(self, **kw) -> "Geom":
        return dataclasses.replace(self, **kw)

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    def proj_shape(self, n_views: int):
        return (n_views, self.nv, self.nu)


# ---------------------------------------------------------------------------
# Workload geometries (sizes of the five benchmark configurations)
# ---------------------------------------------------------------------------

def geom_c1() -> Geom:
    """64^3 at 1 mm; one 128x128 view at 1.5 mm; SAD/SDD 1000/1500; 0.5 mm steps."""
    return Geom(64, 64, 64, 1.0, 1.0, 1.0, 128, 128, 1.5, 1.5)


def geom_c2() -> Geom:
    """256^3 at 0.8 mm; 512x512 view at 0.6 mm; same cone-beam geometry."""
    return Geom(256, 256, 256, 0.8, 0.8, 0.8, 512, 512, 0.6, 0.6)


def geom_c3_recon() -> Geom:
    """512^3 reconstruction grid at 0.375 mm; 512x384 detector at 0.776 mm."""
    return Geom(512, 512, 512, 0.375, 0.375, 0.375, 512, 384, 0.776, 0.776)


def geom_c3_phantom() -> Geom:
    """256^3 phantom at 0.75 mm used to synthesise the c3 projections."""
    return Geom(256, 256, 256, 0.75, 0.75, 0.75, 512, 384, 0.776, 0.776)


# ---------------------------------------------------------------------------
# Phantoms
# ---------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def voxel_centres(n: int, h: float) -> np.ndarray:
    """Voxel-centre coordinates along one axis, origin at the grid centre."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


def _raster_ellipsoid(vol, h, centre, semi, rot, value, mode="add"):
    """Rasterise one ellipsoid at voxel centres into vol[z, y, x] (in place)."""
    nz, ny, nx = vol.shape
    rmax = float(np.max(semi))
    idx = []
    for n, c in zip((nx, ny, nz), centre):
        lo = int(math.floor((c - rmax) / h + (n - 1) / 2.0)) - 1
        hi = int(math.ceil((c + rmax) / h + (n - 1) / 2.0)) + 1
        idx.append((max(lo, 0), min(hi, n - 1)))
    (x0, x1), (y0, y1), (z0, z1) = idx
    if x1 < x0 or y1 < y0 or z1 < z0:
        return
    xs = (np.arange(x0, x1 + 1) - (nx - 1) / 2.0) * h - centre[0]
    ys = (np.arange(y0, y1 + 1) - (ny - 1) / 2.0) * h - centre[1]
    zs = (np.arange(z0, z1 + 1) - (nz - 1) / 2.0) * h - centre[2]
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1) @ rot  # coordinates in the ellipsoid frame
    q = (P[..., 0] / semi[0]) ** 2 + (P[..., 1] / semi[1]) ** 2 + (P[..., 2] / semi[2]) ** 2
    inside = q <= 1.0
    sub = vol[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
    if mode == "add":
        sub[inside] += value
    else:
        sub[inside] = value


def gaussian_smooth(vol: np.ndarray, sigma: float = 1.0) -> np.ndarray:
    """Separable Gaussian (sigma in voxels), truncated at 4 sigma, normalised, zero-padded."""
    out = np.asarray(vol, dtype=np.float64)
    for ax in range(out.ndim):
        out = gaussian_filter1d(out, sigma, axis=ax, mode="constant", cval=0.0, truncate=4.0)
    return out


def ellipsoid_phantom(n: int, h: float, n_ell: int, rng: np.random.Generator,
                      shell: bool = False, sigma: float = 1.0,
                      mu_range=(0.01, 0.05)) -> np.ndarray:
    """Random additive ellipsoid phantom, returned as float32 [n][n][n].

    Centres uniform in a ball of radius 0.35 L, semi-axes uniform in
    [0.05, 0.25] L, uniform random orientation, attenuation uniform in
    mu_range (additive on overlap); an ellipsoid whose bounding sphere reaches
    past 0.5 L - 4 h is redrawn.  Optional high-attenuation shell (0.08/mm,
    4 mm thick, outer semi-axes (0.45, 0.40, 0.42) L) overwrites.  Then a
    sigma = 1 voxel Gaussian smoothing.
    """
    L = n * h
    vol = np.zeros((n, n, n), dtype=np.float64)
    limit = 0.5 * L - 4.0 * h
    if limit <= 0.05 * L:  # no ellipsoid could pass the bounding-sphere rule
        raise ValueError(f"grid of {n} voxels is too small for the ellipsoid recipe")
    placed = 0
    while placed < n_ell:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        centre = d * 0.35 * L * rng.uniform() ** (1.0 / 3.0)
        semi = rng.uniform(0.05, 0.25, size=3) * L
        rot = _random_rotation(rng)
        value = rng.uniform(*mu_range)
        if np.linalg.norm(centre) + semi.max() > limit:
            continue
        _raster_ellipsoid(vol, h, centre, semi, rot, value, "add")
        placed += 1
    if shell:
        outer = np.array([0.45, 0.40, 0.42]) * L
        inner = outer - 4.0
        shell_mask = np.zeros_like(vol)
        _raster_ellipsoid(shell_mask, h, np.zeros(3), outer, np.eye(3), 1.0, "set")
        _raster_ellipsoid(shell_mask, h, np.zeros(3), inner, np.eye(3), 0.0, "set")
        vol[shell_mask > 0.5] = 0.08
    if sigma > 0:
        vol = gaussian_smooth(vol, sigma)
    return vol.astype(np.float32)


# ---------------------------------------------------------------------------
# Poses and motion
# ---------------------------------------------------------------------------

def random_poses(n: int, t_max_mm: float, r_max_deg: float,
                 rng: np.random.Generator) -> np.ndarray:
    """[n][6] float64 poses, translations uniform in +-t_max (mm), rotations uniform in +-r_max (converted to rad)."""
    t = rng.uniform(-t_max_mm, t_max_mm, size=(n, 3))
    r = np.deg2rad(rng.uniform(-r_max_deg, r_max_deg, size=(n, 3)))
    return np.concatenate([t, r], axis=1)


def sinusoidal_motion(n_views: int, amp_t_mm: float, amp_r_deg: float,
                      rng: np.random.Generator) -> np.ndarray:
    """theta_{v,c} = A_c sin(2 pi v / V + phi_c), phi_c uniform in [0, 2 pi)."""
    phase = rng.uniform(0.0, 2.0 * np.pi, size=6)
    amp = np.array([amp_t_mm] * 3 + [np.deg2rad(amp_r_deg)] * 3)
    v = np.arange(n_views)[:, None]
    return amp[None, :] * np.sin(2.0 * np.pi * v / n_views + phase[None, :])


def circular_angles(n_views: int, span_deg: float = 360.0) -> np.ndarray:
    """Gantry angles beta evenly spaced over span (rad, float64)."""
    return np.deg2rad(np.arange(n_views, dtype=np.float64) * span_deg / n_views)


def smooth_images(n_views: int, nv: int, nu: int, rng: np.random.Generator,
                  n_blobs: int = 12, signed: bool = False) -> np.ndarray:
    """[V][nv][nu] float32 smooth random detector images (sums of 2-D Gaussian blobs)."""
    out = np.zeros((n_views, nv, nu), dtype=np.float64)
    uu = np.arange(nu, dtype=np.float64)
    vv = np.arange(nv, dtype=np.float64)
    for v in range(n_views):
        for _ in range(n_blobs):
            cu, cv = rng.uniform(0.1 * nu, 0.9 * nu), rng.uniform(0.1 * nv, 0.9 * nv)
            su, sv = rng.uniform(0.03, 0.2) * nu, rng.uniform(0.03, 0.2) * nv
            amp = rng.uniform(-1.0, 1.0) if signed else rng.uniform(0.2, 1.0)
            out[v] += amp * np.outer(np.exp(-0.5 * ((vv - cv) / sv) ** 2),
                                     np.exp(-0.5 * ((uu - cu) / su) ** 2))
    return out.astype(np.float32)


# ---------------------------------------------------------------------------
# Workload bundles
# ---------------------------------------------------------------------------

def config1_inputs():
    """Config 1: 64^3 phantom (10 ellipsoids), 1 view at beta = 0, pose and target pose (+-5 mm / +-5 deg)."""
    rng = rng_for(0)
    g = geom_c1()
    vol = ellipsoid_phantom(g.nx, g.vx, 10, rng)
    poses = random_poses(1, 5.0, 5.0, rng)
    target_pose = random_poses(1, 5.0, 5.0, rng)
    angles = np.zeros(1)
    return dict(geom=g, vol=vol, angles=angles, poses=poses, target_pose=target_pose)


def config2_inputs(n_poses: int = 64, phantom_n: int | None = None):
    """Config 2: 256^3 phantom (40 ellipsoids + shell), 64 candidate poses (+-10 mm / +-10 deg), beta = 0."""
    rng = rng_for(1)
    g = geom_c2()
    if phantom_n is not None:
        g = g.replace(nx=phantom_n, ny=phantom_n, nz=phantom_n)
    vol = ellipsoid_phantom(g.nx, g.vx, 40, rng, shell=True)
    poses = random_poses(n_poses, 10.0, 10.0, rng)
    target_pose = random_poses(1, 10.0, 10.0, rng)
    angles = np.zeros(n_poses)
    return dict(geom=g, vol=vol, angles=angles, poses=poses, target_pose=target_pose)


def config3_motion(n_views: int = 360):
    """Config 3 acquisition: 360 views over 360 deg, sinusoidal motion 3 mm / 2 deg."""
    rng = rng_for(2)
    angles = circular_angles(n_views)
    motion = sinusoidal_motion(n_views, 3.0, 2.0, rng)
    return dict(angles=angles, poses=motion, rng=rng)


# ---------------------------------------------------------------------------
# Bulk phantoms on the GPU (training-set generation)
# ---------------------------------------------------------------------------

def draw_ellipsoids(n: int, h: float, n_ell: int, rng: np.random.Generator,
                    mu_range=(0.01, 0.05)):
    """The ellipsoid parameters of `ellipsoid_phantom` (same distribution and
    rejection rule): centres [E][3], semi-axes [E][3], rotations [E][3][3],
    attenuations [E]."""
    L = n * h
    limit = 0.5 * L - 4.0 * h
    if limit <= 0.05 * L:  # no ellipsoid could pass the bounding-sphere rule
        raise ValueError(f"grid of {n} voxels is too small for the ellipsoid recipe")
    cs, ss, rs, vs = [], [], [], []
    while len(cs) < n_ell:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        centre = d * 0.35 * L * rng.uniform() ** (1.0 / 3.0)
        semi = rng.uniform(0.05, 0.25, size=3) * L
        rot = _random_rotation(rng)
        value = rng.uniform(*mu_range)
        if np.linalg.norm(centre) + semi.max() > limit:
            continue
        cs.append(centre), ss.append(semi), rs.append(rot), vs.append(value)
    return np.array(cs), np.array(ss), np.array(rs), np.array(vs)


def ellipsoid_phantom_torch(n: int, h: float, n_ell: int, rng: np.random.Generator,
                            device, shell: bool = False, sigma: float = 1.0,
                            mu_range=(0.01, 0.05)):
    """`ellipsoid_phantom`'s recipe rasterised with torch on `device` (FP32
    voxel-centre tests, separable zero-padded Gaussian), for generating many
    phantoms quickly.  Same parameter distribution; voxels on an ellipsoid's
    boundary may differ from the FP64 numpy rasteriser."""
    import torch
    cs, ss, rs, vs = draw_ellipsoids(n, h, n_ell, rng, mu_range)
    ax = (torch.arange(n, device=device, dtype=torch.float32) - (n - 1) / 2.0) * h
    Z, Y, X = torch.meshgrid(ax, ax, ax, indexing="ij")
    P = torch.stack([X, Y, Z], dim=-1)
    vol = torch.zeros((n, n, n), device=device, dtype=torch.float32)
    for c, s, r, v in zip(cs, ss, rs, vs):
        Q = (P - torch.tensor(c, device=device, dtype=torch.float32)) @ \
            torch.tensor(r, device=device, dtype=torch.float32)
        q = ((Q / torch.tensor(s, device=device, dtype=torch.float32)) ** 2).sum(-1)
        vol += float(v) * (q <= 1.0)
    if shell:
        outer = torch.tensor([0.45, 0.40, 0.42], device=device) * n * h
        qo = ((P / outer) ** 2).sum(-1)
        qi = ((P / (outer - 4.0)) ** 2).sum(-1)
        vol = torch.where((qo <= 1.0) & (qi > 1.0), torch.full_like(vol, 0.08), vol)
    if sigma > 0:
        rad = int(math.floor(4.0 * sigma + 0.5))
        k = torch.exp(-0.5 * (torch.arange(-rad, rad + 1, dtype=torch.float64) / sigma) ** 2)
        k = (k / k.sum()).tolist()
        for dim in range(3):
            pad = [0, 0, 0, 0, 0, 0]
            pad[2 * (2 - dim)] = pad[2 * (2 - dim) + 1] = rad
            vp = torch.nn.functional.pad(vol, pad)
            out = torch.zeros_like(vol)
            for j, w in enumerate(k):
                out += w * vp.narrow(dim, j, n)
            vol = out
    return vol.contiguous()


def geom_c5() -> Geom:
    """192^3 at 1 mm; one 256x256 view at 1.2 mm; SAD/SDD 1000/1500; 0.5 mm steps."""
    return Geom(192, 192, 192, 1.0, 1.0, 1.0, 256, 256, 1.2, 1.2)


def config4_problems(device, n_problems: int = 16):
    """The uneven calibration batch: n_problems independent problems, each a
    cubic phantom of N^3 voxels spanning ~200 mm (N from {128, ..., 384},
    20 ellipsoids), 1-8 views at uniform gantry angles on an N_d^2 detector
    (N_d from {256, ..., 768}, pitch 1.5 x 240 mm / N_d) and true poses
    uniform in +-5 mm / +-3 deg.  Returns a list of dicts with geom, vol
    (device FP32), angles and truth (device FP64)."""
    import torch
    rng = rng_for(3, 9)
    out = []
    for _ in range(n_problems):
        n = int(rng.choice([128, 192, 256, 320, 384]))
        h = 200.0 / n
        V = int(rng.integers(1, 9))
        nu = int(rng.choice([256, 384, 512, 640, 768]))
        du = 1.5 * 240.0 / nu
        g = Geom(n, n, n, h, h, h, nu, nu, du, du)
        vol = ellipsoid_phantom_torch(n, h, 20, rng, device)
        angles = torch.tensor(rng.uniform(0, 2 * math.pi, V), dtype=torch.float64, device=device)
        truth = torch.tensor(random_poses(V, 5.0, 3.0, rng), dtype=torch.float64, device=device)
        out.append(dict(geom=g, vol=vol, angles=angles, truth=truth))
    return out


def poisson_log_noise(l, photons: float, generator, scale: float = 1.0):
    """Noisy line integrals of a transmission measurement: per pixel, counts
    N ~ Poisson(photons * exp(-scale * l)) with `photons` unattenuated
    photons, returned as -log(max(N, 1) / photons) / scale (the units of l).
    `scale` maps the line integrals to the attenuation the detector sees
    (1: as given).  l: torch tensor (any shape, any device); `generator` (a
    torch.Generator on l's device) seeds the draws."""
    import torch
    lam = photons * torch.exp(-scale * l.to(torch.float64))
    n = torch.poisson(lam, generator=generator)
    return (-torch.log(n.clamp_min(1.0) / photons) / scale).to(l.dtype)
