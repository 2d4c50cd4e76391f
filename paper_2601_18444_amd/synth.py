"""Seeded synthetic inputs for the NuMagSANS direct-sum path.

This module only makes inputs: point clouds, weights, object offsets, rotation
matrices and detector descriptors, all from ``numpy.random.default_rng(seed)``.
It holds none of the method's arithmetic (no Fourier sums, no cross sections)
and imports nothing else from this repository, so the CPU oracle's tests and
the HIP path can both be fed from it.

The paper's benchmark data (Sec. 4, published separately) is not used; these
generators stand in for it with the shapes and structure of its examples:

* ``sphere_40nm``   -- the runtime-experiment particle of Sec. 4.4 (D = 40 nm on a
  2 nm simple-cubic lattice, 4169 cells) with the uniform magnetization of
  Sec. 4.1, on a 128 x 128 detector, |q_y|, |q_z| <= 1 nm^-1.
* ``vortex_grid``   -- a 64^3 micromagnetic-style grid at 1 nm holding a vortex
  (in-plane curl, Gaussian core of 5 nm, 2 % noise) inside a cylinder, on a
  256 x 256 detector, |q_y|, |q_z| <= 2 nm^-1.
* ``sphere_ensemble``  -- 512 spheres (radii U(5, 15) nm) at random non-overlapping
  centres in a 500 nm cube, 1 nm lattice, tilted uniform moments; stands in for
  the iron-nanoparticle ensemble of Sec. 4.3.  512 x 512 detector, 1.5 nm^-1.
* ``particles_rotations`` -- 64 particles (spheres, cubes, cylinders) with point counts
  log-uniform in [1e3, 2e5] and smooth random unit fields, plus 1000 rotations
  uniform on SO(3); 128 x 128 detector, 1 nm^-1.
* ``vortex_grid_gradient`` -- the vortex grid and a perturbed copy (core shifted 3 nm along x)
  from which the tests make a target cross section.
"""
from __future__ import annotations

import math

import numpy as np

CARTESIAN = 0
POLAR = 1


# ---------------------------------------------------------------------------
# rotations
# ---------------------------------------------------------------------------
def rot_y(alpha_deg: float) -> np.ndarray:
    """Active right-handed rotation about y by alpha (degrees)."""
    a = math.radians(alpha_deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_z(beta_deg: float) -> np.ndarray:
    """Active right-handed rotation about z by beta (degrees)."""
    b = math.radians(beta_deg)
    c, s = math.cos(b), math.sin(b)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def sample_rotation(alpha_deg: float, beta_deg: float) -> np.ndarray:
    """R(alpha, beta) = R_z(beta) R_y(alpha), the sample rotation of Sec. 3.1."""
    return rot_z(beta_deg) @ rot_y(alpha_deg)


def uniform_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """n rotation matrices uniform on SO(3) (K. Shoemake, "Uniform random
    rotations", Graphics Gems III, 1992: a uniform unit quaternion from three
    uniform deviates).  Returns [n, 3, 3]."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    w = a * np.sin(2 * np.pi * u2)
    x = a * np.cos(2 * np.pi * u2)
    y = b * np.sin(2 * np.pi * u3)
    z = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def unit_vectors(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# lattices
# ---------------------------------------------------------------------------
def sphere_lattice(radius: float, a: float, half_offset: bool = False) -> np.ndarray:
    """Points of a simple-cubic lattice a*Z^3 (or a*(Z + 1/2)^3) with |r| <= radius.

    The Sec. 4.4 particle (D = 40 nm, a = 2 nm) has 4169 points on the
    origin-centred lattice."""
    m = int(math.floor(radius / a)) + 1
    g = np.arange(-m, m + 1, dtype=np.float64)
    if half_offset:
        g = g + 0.5
    x, y, z = np.meshgrid(g * a, g * a, g * a, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    r2 = np.sum(pts * pts, axis=1)
    return pts[r2 <= radius * radius * (1 + 1e-12)]


def box_lattice(n, a, corner) -> np.ndarray:
    """n[0] x n[1] x n[2] points corner + (i, j, k) * a (C order: i slowest)."""
    ix, iy, iz = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return np.asarray(corner, dtype=np.float64)[None, :] + idx * np.asarray(a, dtype=np.float64)[None, :]


def detector(kind: int, n0: int, n1: int, qmax: float) -> dict:
    return {"kind": int(kind), "n0": int(n0), "n1": int(n1), "qmax": float(qmax)}


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def sphere_40nm() -> dict:
    """Uniform sphere, R = 20 nm, 2 nm lattice (W = 4169), N = 1, M = e_z."""
    pos = sphere_lattice(20.0, 2.0)
    W = pos.shape[0]
    return {
        "name": "sphere_R20_a2_W4169_det128",
        "pos": pos, "nuc": np.ones(W), "mag": np.tile([0.0, 0.0, 1.0], (W, 1)),
        "obj_offsets": None, "obj_pos": None, "R": np.eye(3),
        "grid": detector(CARTESIAN, 128, 128, 1.0), "n_bins": 64,
    }


def vortex_field(n: int = 64, a: float = 1.0, core: float = 5.0, noise: float = 0.02,
                 radius: float = 32.0, centre_x: float = 0.0, seed: int = 2):
    """64^3 cell centres (i - 31.5) a, cylinder rho <= radius about z: N = 1, vortex
    m_z = exp(-rho^2 / (2 core^2)), in-plane curl, Gaussian noise, unit norm;
    zero outside.  ``centre_x`` shifts the vortex core along x (same noise)."""
    rng = np.random.default_rng(seed)
    c = (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * a
    pos = box_lattice((n, n, n), (a, a, a), (c[0], c[0], c[0]))
    x, y = pos[:, 0], pos[:, 1]
    inside = (x * x + y * y) <= radius * radius
    xs = x - centre_x
    rho = np.sqrt(xs * xs + y * y)
    mz = np.exp(-rho * rho / (2.0 * core * core))
    inpl = np.sqrt(np.clip(1.0 - mz * mz, 0.0, None))
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(rho > 0, -y / rho, 0.0)
        uy = np.where(rho > 0, xs / rho, 0.0)
    m = np.stack([inpl * ux, inpl * uy, mz], axis=1)
    m = m + noise * rng.standard_normal(m.shape)
    m = m / np.linalg.norm(m, axis=1, keepdims=True)
    m[~inside] = 0.0
    nuc = inside.astype(np.float64)
    return pos, nuc, m


def vortex_grid(n: int = 64, det: int = 256, qmax: float = 2.0, seed: int = 2) -> dict:
    pos, nuc, mag = vortex_field(n=n, seed=seed)
    c0 = -(n - 1) / 2.0
    return {
        "name": f"vortex_grid{n}_det{det}",
        "pos": pos, "nuc": nuc, "mag": mag, "obj_offsets": None, "obj_pos": None,
        "R": np.eye(3), "grid": detector(CARTESIAN, det, det, qmax), "n_bins": det // 2,
        "regular": {"n": (n, n, n), "origin": (c0, c0, c0), "step": (1.0, 1.0, 1.0)},
    }


def vortex_grid_gradient(n: int = 64, det: int = 256, qmax: float = 2.0, seed: int = 2, shift: float = 3.0):
    """Configuration for the gradient: the vortex grid and the perturbed target field."""
    base = vortex_grid(n=n, det=det, qmax=qmax, seed=seed)
    tpos, tnuc, tmag = vortex_field(n=n, seed=seed, centre_x=shift)
    base["target_field"] = {"pos": tpos, "nuc": tnuc, "mag": tmag}
    base["name"] = f"vortex_grid{n}_det{det}_grad"
    return base


def vortex_field_sweep(n_snap: int, n: int = 64, seed: int = 2, h_max: float = 1.0):
    """Loop-mode stand-in (a field sweep): the vortex field of ``vortex_field`` with a
    uniform field-like component h_b e_z added and the moments renormalised, for
    h_b evenly spaced in [-h_max, h_max] (b < n_snap).  Returns (nuc [W],
    mag [n_snap, W, 3], regular-grid descriptor, h)."""
    pos, nuc, m = vortex_field(n=n, seed=seed)
    inside = nuc > 0
    h = np.linspace(-h_max, h_max, n_snap) if n_snap > 1 else np.zeros(1)
    mags = np.empty((n_snap,) + m.shape)
    for b in range(n_snap):
        mb = m + h[b] * np.array([0.0, 0.0, 1.0])
        nrm = np.linalg.norm(mb, axis=1, keepdims=True)
        mb = np.where(nrm > 0, mb / np.where(nrm > 0, nrm, 1.0), 0.0)
        mb[~inside] = 0.0
        mags[b] = mb
    c0 = -(n - 1) / 2.0
    regular = {"n": (n, n, n), "origin": (c0, c0, c0), "step": (1.0, 1.0, 1.0)}
    return nuc, mags, regular, h


def tilted_moment(e: np.ndarray, tilt_deg: float) -> np.ndarray:
    """Rotate the unit vector e toward +z by tilt_deg inside span(e, z), stopping at z."""
    z = np.array([0.0, 0.0, 1.0])
    ang = math.acos(max(-1.0, min(1.0, float(e @ z))))
    t = math.radians(tilt_deg)
    if t >= ang or ang < 1e-12:
        return z.copy()
    perp = e - (e @ z) * z
    perp = perp / np.linalg.norm(perp)
    new = ang - t
    return math.cos(new) * z + math.sin(new) * perp


def sphere_ensemble(n_spheres: int = 512, box: float = 500.0, rmin: float = 5.0, rmax: float = 15.0,
               a: float = 1.0, det: int = 512, qmax: float = 1.5, seed: int = 3) -> dict:
    """Ensemble of non-overlapping spheres by random sequential addition."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(rmin, rmax, n_spheres)
    centres = np.zeros((n_spheres, 3))
    half = box / 2.0
    for k in range(n_spheres):
        for _ in range(100000):
            c = rng.uniform(-half + radii[k], half - radii[k], 3)
            if k == 0:
                break
            d = np.linalg.norm(centres[:k] - c[None, :], axis=1)
            if np.all(d > radii[:k] + radii[k] + a):
                break
        else:
            raise RuntimeError("random sequential addition failed")
        centres[k] = c
    axes = unit_vectors(n_spheres, rng)
    tilts = rng.uniform(0.0, 60.0, n_spheres)
    pos_list, mag_list, off = [], [], [0]
    for k in range(n_spheres):
        pts = sphere_lattice(radii[k], a)
        m = tilted_moment(axes[k], tilts[k])
        pos_list.append(pts)
        mag_list.append(np.tile(m, (pts.shape[0], 1)))
        off.append(off[-1] + pts.shape[0])
    pos = np.concatenate(pos_list)
    return {
        "name": f"spheres{n_spheres}_det{det}",
        "pos": pos, "nuc": np.ones(pos.shape[0]), "mag": np.concatenate(mag_list),
        "obj_offsets": np.array(off, dtype=np.int64), "obj_pos": centres, "R": np.eye(3),
        "grid": detector(CARTESIAN, det, det, qmax), "n_bins": det // 2,
    }


def _shape_points(shape: str, n_target: float, a: float = 1.0) -> np.ndarray:
    if shape == "sphere":
        r = (3.0 * n_target / (4.0 * math.pi)) ** (1.0 / 3.0) * a
        return sphere_lattice(r, a)
    if shape == "cube":
        s = max(1, int(round(n_target ** (1.0 / 3.0))))
        c = -(s - 1) / 2.0 * a
        return box_lattice((s, s, s), (a, a, a), (c, c, c))
    # cylinder with h = 2 r: N = pi r^2 * 2r
    r = (n_target / (2.0 * math.pi)) ** (1.0 / 3.0) * a
    m = int(math.floor(r / a)) + 1
    g = np.arange(-m, m + 1, dtype=np.float64) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    keep = (pts[:, 0] ** 2 + pts[:, 1] ** 2 <= r * r) & (np.abs(pts[:, 2]) <= r)
    return pts[keep]


def particles_rotations(n_particles: int = 64, n_rot: int = 1000, nmin: float = 1e3, nmax: float = 2e5,
                 det: int = 128, qmax: float = 1.0, seed: int = 4, scale_counts: float = 1.0) -> dict:
    """Particles of uneven size with smooth random unit magnetization fields and
    shared uniform rotations (dilute sample, orientational average)."""
    rng = np.random.default_rng(seed)
    shapes = rng.choice(["sphere", "cube", "cylinder"], n_particles)
    counts = np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_particles)) * scale_counts
    pos_list, mag_list, off = [], [], [0]
    for k in range(n_particles):
        pts = _shape_points(str(shapes[k]), counts[k])
        u = unit_vectors(1, rng)[0]
        v = unit_vectors(3, rng)
        kdir = unit_vectors(3, rng)
        kmag = rng.uniform(0.05, 0.5, 3)
        phi = rng.uniform(0.0, 2 * math.pi, 3)
        field = np.tile(u, (pts.shape[0], 1))
        for i in range(3):
            field = field + 0.5 * v[i][None, :] * np.cos(pts @ (kmag[i] * kdir[i]) + phi[i])[:, None]
        field = field / np.linalg.norm(field, axis=1, keepdims=True)
        pos_list.append(pts)
        mag_list.append(field)
        off.append(off[-1] + pts.shape[0])
    pos = np.concatenate(pos_list)
    rots = uniform_rotations(n_rot, rng)
    return {
        "name": f"particles{n_particles}_rot{n_rot}_det{det}",
        "pos": pos, "nuc": np.ones(pos.shape[0]), "mag": np.concatenate(mag_list),
        "obj_offsets": np.array(off, dtype=np.int64), "obj_pos": None, "rotations": rots,
        "grid": detector(CARTESIAN, det, det, qmax), "n_bins": det // 2,
        "shapes": [str(s) for s in shapes],
    }


def random_cloud(n: int, extent: float, seed: int, with_nuc: bool = True, with_mag: bool = True) -> dict:
    """Unstructured random points and weights (for parity cases and pins)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-extent, extent, (n, 3))
    nuc = rng.standard_normal(n) if with_nuc else None
    mag = rng.standard_normal((n, 3)) if with_mag else None
    return {"pos": pos, "nuc": nuc, "mag": mag}
