"""The seeded synthetic inputs hold the recipes stated for them: sizes, lattices,
field norms, object placement and rotations (no method arithmetic is involved)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2601_18444_amd import synth  # noqa: E402


def test_sphere_40nm_lattice():
    """D = 40 nm on a 2 nm simple-cubic lattice, |r| <= 20 nm inclusive: 4169 points;
    N = 1, M = e_z; 128 x 128 detector on [-1, 1]^2."""
    c = synth.sphere_40nm()
    pos = c["pos"]
    assert pos.shape == (4169, 3)
    assert np.all(np.linalg.norm(pos, axis=1) <= 20.0 + 1e-12)
    assert np.array_equal(pos, 2.0 * np.round(pos / 2.0))
    assert np.all(c["nuc"] == 1.0) and np.all(c["mag"] == np.array([0.0, 0.0, 1.0]))
    assert c["grid"] == {"kind": 0, "n0": 128, "n1": 128, "qmax": 1.0}


def test_vortex_grid_recipe():
    """64^3 cells at 1 nm, centres (i - 31.5) nm; inside rho <= 32 nm: N = 1 and a unit
    moment, zero outside; the core (m_z near 1) on the axis and the in-plane curl
    along (-y, x); the gradient's target has the core moved 3 nm along x."""
    c = synth.vortex_grid()
    pos, nuc, mag = c["pos"], c["nuc"], c["mag"]
    assert pos.shape == (262144, 3)
    assert np.allclose(np.unique(pos[:, 0]), np.arange(64) - 31.5)
    rho = np.hypot(pos[:, 0], pos[:, 1])
    inside = rho <= 32.0
    assert np.array_equal(nuc, inside.astype(float))
    assert np.allclose(np.linalg.norm(mag[inside], axis=1), 1.0)
    assert np.all(mag[~inside] == 0.0)
    core = inside & (rho < 1.0)
    assert np.mean(mag[core, 2]) > 0.9
    ring = inside & (rho > 20.0)
    curl = (-pos[ring, 1] * mag[ring, 0] + pos[ring, 0] * mag[ring, 1]) / rho[ring]
    assert np.mean(curl) > 0.9 and np.mean(np.abs(mag[ring, 2])) < 0.1
    assert c["grid"] == {"kind": 0, "n0": 256, "n1": 256, "qmax": 2.0}
    tf = synth.vortex_grid_gradient()["target_field"]
    assert np.array_equal(tf["pos"], pos)
    tin = np.hypot(tf["pos"][:, 0], tf["pos"][:, 1]) <= 32.0
    j = np.argmax(np.where(tin, tf["mag"][:, 2], -2.0))
    assert abs(tf["pos"][j, 0] - 3.0) <= 0.5 and abs(tf["pos"][j, 1]) <= 0.5


def test_sphere_ensemble_recipe():
    """512 spheres, radii in [5, 15] nm, 1 nm lattice in local coordinates, centres
    inside the 500 nm cube without overlaps; N = 1 and one unit moment per sphere;
    2625870 points; 512 x 512 detector on [-1.5, 1.5]^2."""
    c = synth.sphere_ensemble()
    off, cen, pos = c["obj_offsets"], c["obj_pos"], c["pos"]
    assert len(off) == 513 and off[-1] == pos.shape[0] == 2625870
    assert np.array_equal(pos, np.round(pos))
    r = np.array([np.linalg.norm(pos[off[k]:off[k + 1]], axis=1).max() for k in range(512)])
    assert r.min() >= 4.0 and r.max() <= 15.0
    assert np.all(np.abs(cen) + r[:, None] <= 250.0)
    d = np.linalg.norm(cen[:, None, :] - cen[None, :, :], axis=2) + np.eye(512) * 1e9
    assert np.all(d >= r[:, None] + r[None, :])
    assert np.all(c["nuc"] == 1.0)
    m = c["mag"]
    assert np.allclose(np.linalg.norm(m, axis=1), 1.0)
    for k in range(512):
        assert np.all(m[off[k]:off[k + 1]] == m[off[k]])
    assert c["grid"] == {"kind": 0, "n0": 512, "n1": 512, "qmax": 1.5}


def test_particles_rotations_recipe():
    """64 particles (spheres, cubes, cylinders) with 1331 ... 173157 points, 2298012 in
    total, unit moments; 1000 rotations in SO(3); 128 x 128 detector on [-1, 1]^2."""
    c = synth.particles_rotations()
    cnt = np.diff(c["obj_offsets"])
    assert cnt.size == 64 and cnt.sum() == 2298012 and cnt.min() == 1331 and cnt.max() == 173157
    assert set(c["shapes"]) <= {"sphere", "cube", "cylinder"}
    assert np.allclose(np.linalg.norm(c["mag"], axis=1), 1.0)
    R = c["rotations"]
    assert R.shape == (1000, 3, 3)
    assert np.max(np.abs(np.einsum("nji,njk->nik", R, R) - np.eye(3))) < 1e-12
    assert np.allclose(np.linalg.det(R), 1.0)
    assert c["grid"] == {"kind": 0, "n0": 128, "n1": 128, "qmax": 1.0}
