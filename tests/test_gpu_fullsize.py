"""Component-wise parity at full configuration sizes.

* Gradient (the 64^3 vortex grid on the 256 x 256 detector; loss on the
  unpolarized cross section, Sec. 2.4): 100 seeded components of dL/dn and
  dL/dm from the HIP adjoint against FP64 central finite differences of the
  loss.  The oracle computes the raw sums S of the sample and of the target
  field; each perturbed loss is a rank-1 update of S (one weight changes by
  +-h, so S_c changes by +-h exp(-i q.X_j) at every pixel) followed by the
  oracle's cross sections.  L is a quartic polynomial in one weight, so the
  central difference carries exactly h^2 L'''/6, which Richardson extrapolation
  over h and h/2 removes: the reference is exact up to rounding.  Tolerance:
  |g - g_FD| <= 1e-4 |g_FD| on components with |g_FD| >= 1e-3 max|g_FD|, else
  <= 1e-7 max|g_FD|.
* The benchmark's launch configuration: the same vortex sums and gradient under the
  shapes the autotuner picks on the machine, against the oracle (sums, sampled) and
  the default shapes (to rounding).
* Orientational averages (64 particles of 1,331-173,157 points, 1,000 rotations,
  128 x 128 detector; Sec. 3.3 dilute limit): every particle's averaged spectral
  matrix against the oracle over all 1,000 rotations on sampled pixels (this
  covers the largest particle, whose work is cut into many rotation ranges), and
  every particle under 4 seeded rotations on more pixels.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402
from tests.helpers import amp_to_complex, gated_rel_err, max_norm_err  # noqa: E402

DEV = "cuda:0"
TOL = 1e-5


def _oracle_sums(orc, field, qy, qz):
    """Oracle sums of the points with a nonzero weight (the others add exact zeros)."""
    nz = (field["nuc"] != 0) | np.any(field["mag"] != 0, axis=1)
    return orc.amplitudes(field["pos"][nz], field["nuc"][nz], field["mag"][nz], qy, qz)


def test_vortex_gradient_components_against_finite_differences(orc):
    cfg = synth.vortex_grid_gradient()
    g = cfg["grid"]
    qy, qz, qhat = orc.pixels(g["kind"], g["n0"], g["n1"], g["qmax"])
    print("C5: oracle sums of the sample and of the target field (2 x 1.4e10 terms)", flush=True)
    S = _oracle_sums(orc, cfg, qy, qz)
    ST = _oracle_sums(orc, cfg["target_field"], qy, qz)
    k = dict(V=1.0, bH=1.0, scale=1.0, P=(0.0, 0.0, 1.0))
    T = orc.cross_sections(ST, qhat, **k)["UNPOL"]
    qn = np.sqrt(qy * qy + qz * qz)
    w = np.where(qn <= g["qmax"], 1.0 / (T + 1e-3 * T.max()) ** 2, 0.0)

    def loss(A):
        I = orc.cross_sections(A, qhat, **k)["UNPOL"]
        return float(np.sum(w * (I - T) ** 2))

    L0 = loss(S)
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    s = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], device=DEV)
    print("C5: HIP loss and gradient", flush=True)
    lt, dn, dm = numag.grad(s, grid, numag.consts(**k), weight=torch.as_tensor(w, device=DEV),
                            target=torch.as_tensor(T, device=DEV))
    torch.cuda.synchronize()
    assert abs(lt.item() - L0) <= 1e-9 * abs(L0)
    gpu = np.concatenate([dn.cpu().numpy()[:, None], dm.cpu().numpy()], axis=1)  # [W, 4]: N, Mx, My, Mz

    W = cfg["pos"].shape[0]
    comp = np.random.default_rng(5).choice(4 * W, 100, replace=False)
    pos = cfg["pos"]
    print("C5: 100 components by Richardson-extrapolated central differences", flush=True)
    fd = np.zeros(comp.size)
    for i, cidx in enumerate(comp):
        j, c = divmod(int(cidx), 4)
        e = np.exp(-1j * (qy * pos[j, 1] + qz * pos[j, 2]))  # exp(-i q.X_j), q = (0, q_y, q_z), R = I

        def L(h):
            A = S.copy()
            A[:, c] += h * e
            return loss(A)

        def D(h):
            return (L(h) - L(-h)) / (2.0 * h)

        h = 1e-3
        fd[i] = (4.0 * D(h / 2) - D(h)) / 3.0
    got = gpu.reshape(-1)[comp]
    big = np.max(np.abs(fd))
    assert big > 0
    for i in range(comp.size):
        err = abs(got[i] - fd[i])
        if abs(fd[i]) >= 1e-3 * big:
            assert err <= 1e-4 * abs(fd[i]), (int(comp[i]), got[i], fd[i])
        else:
            assert err <= 1e-7 * big, (int(comp[i]), got[i], fd[i])


def _check_spec(gpu, ref):
    for v in range(16):
        e = gated_rel_err(gpu[:, v], ref[:, v])
        assert e <= TOL, f"spectral entry {v}: {e:.3e}"


def test_orientational_average_every_particle_full_rotation_set(orc):
    cfg = synth.particles_rotations()
    g = cfg["grid"]
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    s = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], obj_offsets=cfg["obj_offsets"], device=DEV)
    rots = cfg["rotations"]
    off = cfg["obj_offsets"]
    K = off.size - 1
    qy, qz, _ = orc.pixels(0, g["n0"], g["n1"], g["qmax"])
    print("C4: 64 particles x 1000 rotations on the GPU", flush=True)
    _, spec = numag.amplitudes(s, grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
    spec = spec.cpu().numpy()
    # all 1000 rotations, every particle, on 4 pixels
    idx = np.sort(np.random.default_rng(46).choice(qy.size, 4, replace=False))
    print("C4: oracle, 64 particles x 1000 rotations x 4 pixels", flush=True)
    # The oracle parallelises over pixels, so with 4 pixels it uses 4 threads: the
    # rotations run concurrently from a thread pool (the library call releases the
    # interpreter lock) and are accumulated in rotation order.
    def one_rotation(R):
        return orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[idx], qz[idx], R=R, obj_offsets=off,
                              per_object=True)

    acc = np.zeros((K, idx.size, 16))
    with ThreadPoolExecutor(max_workers=4) as pool:
        for F in pool.map(one_rotation, rots):
            for kk in range(K):
                acc[kk] += orc.spectral(F[kk])
    acc /= len(rots)
    for kk in range(K):
        _check_spec(spec[kk][idx], acc[kk])
    # every particle under 4 seeded rotations, 32 pixels
    rots4 = synth.uniform_rotations(4, np.random.default_rng(47))
    print("C4: 64 particles x 4 rotations, GPU and oracle on 32 pixels", flush=True)
    _, spec4 = numag.amplitudes(s, grid, rot=rots4, mode=numag.MODE_DILUTE, spec_per_object=True)
    spec4 = spec4.cpu().numpy()
    idx = np.sort(np.random.default_rng(48).choice(qy.size, 32, replace=False))
    acc = np.zeros((K, idx.size, 16))
    for R in rots4:
        F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[idx], qz[idx], R=R, obj_offsets=off,
                           per_object=True)
        for kk in range(K):
            acc[kk] += orc.spectral(F[kk])
    acc /= len(rots4)
    for kk in range(K):
        _check_spec(spec4[kk][idx], acc[kk])
    # the summed average equals the sum of the per-particle ones
    _, tot = numag.amplitudes(s, grid, rot=rots4, mode=numag.MODE_DILUTE, spec_per_object=False)
    assert max_norm_err(tot[0].cpu().numpy(), spec4.sum(axis=0)) <= 1e-12


def test_benchmark_launch_configuration_full_size(orc):
    """The benchmark step's configuration: the 64^3 vortex on the 256 x 256 detector
    with the launch shapes the autotuner picks on this machine (as bench.py does before
    it times).  Direct sums against the oracle on 128 sampled pixels (and against the
    library-default shapes to rounding); the loss gradient under the tuned adjoint
    shape against the default-shape gradient, which the finite-difference test above
    checks against the oracle."""
    cfg = synth.vortex_grid_gradient()
    g = cfg["grid"]
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    W = cfg["pos"].shape[0]
    s = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], device=DEV)
    k = numag.consts(V=1.0, bH=1.0, scale=1.0, P=(0.0, 0.0, 1.0))
    tf = cfg["target_field"]
    ts = numag.Sample(pos=tf["pos"], nuc=tf["nuc"], mag=tf["mag"], device=DEV)
    numag.tune_clear()
    try:
        tamp, _ = numag.amplitudes(ts, grid)
        T = numag.cross_section(grid, amp=tamp, c=k, obs=("UNPOL",))[0, 0].clone()
        w = (1.0 / (T + 1e-3 * T.max()) ** 2).contiguous()
        a_def, _ = numag.amplitudes(s, grid)
        a_def = a_def.clone()
        g_def = [t.clone() for t in numag.grad(s, grid, k, weight=w, target=T, amp=a_def[0])]
        print("tuned shapes:", numag.autotune(s, grid, numag.TUNE_DIRECT),
              numag.autotune(s, grid, numag.TUNE_ADJOINT), flush=True)
        a_tun, _ = numag.amplitudes(s, grid)
        g_tun = numag.grad(s, grid, k, weight=w, target=T, amp=a_tun[0])
        torch.cuda.synchronize()
    finally:
        numag.tune_clear()
    gpu = amp_to_complex(a_tun[0])
    assert max_norm_err(gpu, amp_to_complex(a_def[0])) <= 1e-12
    qy, qz, _ = orc.pixels(g["kind"], g["n0"], g["n1"], g["qmax"])
    idx = np.sort(np.random.default_rng(96).choice(qy.size, 128, replace=False))
    ref = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[idx], qz[idx])
    for c in range(4):
        assert gated_rel_err(gpu[idx, c], ref[:, c]) <= TOL, c
    assert abs(float(g_tun[0]) - float(g_def[0])) <= 1e-12 * abs(float(g_def[0]))
    for a, b in zip(g_tun[1:], g_def[1:]):
        assert float((a - b).abs().max()) <= 1e-10 * float(b.abs().max())
