"""Randomized parity sweep: 24 seeded random configurations of detector kind and
size (odd and even, 1 to 69 rows and columns), q_max, object counts and sizes
(including empty objects and samples), channel subsets, rotations, object mode
(coherent, dilute with several rotations, split) and path (direct or half
detector), each against the FP64 oracle; coherent cases also check the loss and
gradient.  A second sweep of 16 seeded regular-grid cases runs the separable
matrix-core paths (FP64 and its half-detector variant) in batches of snapshots.
Every case has its own seed, so a failure names a reproducible case."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402
from tests.helpers import amp_to_complex, gated_rel_err, max_norm_err  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("case", range(24))
def test_random_configuration(orc, case):
    rng = np.random.default_rng(1000 + case)
    kind = int(rng.integers(0, 2))
    n0, n1 = int(rng.integers(1, 70)), int(rng.integers(1, 70))
    if kind == 1 and case % 2 == 0:
        n1 += n1 % 2  # an even n_theta admits the half-detector path
    qmax = float(rng.uniform(0.2, 2.5))
    mode = case % 3
    path = numag.PATH_DIRECT_HERMITIAN if (case // 3) % 2 and not (kind == 1 and n1 % 2) else numag.PATH_DIRECT
    K = int(rng.integers(1, 6))
    sizes = rng.integers(0, 3000 // K + 1, K)
    if case == 5:
        sizes[:] = 0  # an empty sample
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    W = int(off[-1])
    ext = float(rng.uniform(1, 15))
    pos = rng.uniform(-ext, ext, (W, 3))
    nuc, mag = rng.standard_normal(W), rng.standard_normal((W, 3))
    chan = case % 4 if case % 4 < 3 else 0  # 0 all channels, 1 nuclear only, 2 magnetic only
    n_rot = int(rng.integers(1, 9)) if mode == 1 else 1
    rots = synth.uniform_rotations(n_rot, rng)
    obj_pos = rng.uniform(-20, 20, (K, 3))
    s = numag.Sample(pos=pos, nuc=nuc if chan != 2 else None, mag=mag if chan != 1 else None,
                     obj_offsets=off if K > 1 else None, obj_pos=obj_pos if mode != 1 else None, device=DEV)
    on = nuc if chan != 2 else np.zeros(W)
    om = mag if chan != 1 else np.zeros((W, 3))
    grid = numag.qgrid(kind, n0, n1, qmax)
    qy, qz, qhat = orc.pixels(kind, n0, n1, qmax)
    offs = off if K > 1 else None
    if mode == 0:
        amp, _ = numag.amplitudes(s, grid, rot=rots[0], path=path)
        A = orc.amplitudes(pos, on, om, qy, qz, R=rots[0], obj_offsets=offs, obj_pos=obj_pos)
        if W == 0:
            assert torch.count_nonzero(amp).item() == 0
            return
        gpu = amp_to_complex(amp[0])
        for c in range(4):
            assert gated_rel_err(gpu[:, c], A[:, c]) <= 1e-9, c
        T = rng.uniform(0, 5, qy.size)
        w = rng.uniform(0.5, 1.5, qy.size)
        L, dn, dm = orc.loss_grad(pos, on, om, qy, qz, qhat, T, w, R=rots[0], obj_offsets=offs, obj_pos=obj_pos)
        loss, gdn, gdm = numag.grad(s, grid, numag.consts(), weight=torch.as_tensor(w, device=DEV),
                                    target=torch.as_tensor(T, device=DEV), rot=rots[0], path=path)
        assert abs(loss.item() - L) <= 1e-9 * abs(L)
        if chan != 2:
            assert max_norm_err(gdn.cpu().numpy(), dn) <= 1e-8
        if chan != 1:
            assert max_norm_err(gdm.cpu().numpy(), dm) <= 1e-8
    elif mode == 1:
        _, spec = numag.amplitudes(s, grid, rot=rots, path=path, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec = spec.cpu().numpy()
        for k in range(K):
            sl = slice(off[k], off[k + 1])
            if off[k + 1] == off[k]:
                assert np.count_nonzero(spec[k]) == 0
                continue
            Fs = [orc.amplitudes(pos[sl], on[sl], om[sl], qy, qz, R=R) for R in rots]
            assert max_norm_err(spec[k], orc.spectral(np.stack(Fs)) / len(rots)) <= 1e-9, k
    else:
        amp, spec = numag.amplitudes(s, grid, rot=rots[0], path=path, mode=numag.MODE_SPLIT)
        if W == 0:
            assert torch.count_nonzero(amp).item() == 0 and torch.count_nonzero(spec).item() == 0
            return
        A = orc.amplitudes(pos, on, om, qy, qz, R=rots[0], obj_offsets=offs, obj_pos=obj_pos)
        F = orc.amplitudes(pos, on, om, qy, qz, R=rots[0], obj_offsets=offs, obj_pos=obj_pos, per_object=True)
        assert max_norm_err(amp_to_complex(amp[0]), A) <= 1e-9
        assert max_norm_err(spec[0].cpu().numpy(), orc.spectral(F)) <= 1e-9


@pytest.mark.parametrize("case", range(16))
def test_random_separable_configuration(orc, case):
    """Seeded random regular grids (1 to 40 cells per axis, random steps and origins),
    Cartesian detectors (1 to 90 rows and columns), q_max, channel subsets and
    snapshot counts (up to 240, so that large batches take the four-channel-set
    tiles) on the FP64 separable path or its Hermitian variant: two snapshots
    against the oracle on sampled pixels, and each equal to its single call."""
    rng = np.random.default_rng(2000 + case)
    n = tuple(int(v) for v in rng.integers(1, 41, 3))
    while n[0] * n[1] * n[2] > 20000:
        n = (max(1, n[0] // 2), n[1], n[2])
    step = tuple(float(v) for v in rng.uniform(0.3, 2.0, 3))
    origin = tuple(float(v) for v in rng.uniform(-30, 5, 3))
    W = n[0] * n[1] * n[2]
    n0, n1 = int(rng.integers(1, 91)), int(rng.integers(1, 91))
    qmax = float(rng.uniform(0.2, 2.5))
    B = int(rng.integers(1, 13)) if case % 4 else int(rng.integers(100, 241))
    chan = case % 3  # 0 all channels, 1 nuclear only, 2 magnetic only
    path = numag.PATH_SEPARABLE_F64_HERMITIAN if case % 2 else numag.PATH_SEPARABLE_F64
    nuc = rng.standard_normal((B, W)) if chan != 2 else None
    mag = rng.standard_normal((B, W, 3)) if chan != 1 else None
    grid = numag.qgrid(0, n0, n1, qmax)
    points = numag.regular_grid(n, origin, step)
    amp = numag.amplitudes_snapshots(points, grid, nuc=nuc, mag=mag, path=path, device=DEV)
    pos = synth.box_lattice(n, step, origin)
    qy, qz, _ = orc.pixels(0, n0, n1, qmax)
    idx = np.sort(rng.choice(qy.size, min(qy.size, 48), replace=False))
    reg = {"n": n, "origin": origin, "step": step}
    for b in sorted({0, B - 1}):
        nb = nuc[b] if nuc is not None else None
        mb = mag[b] if mag is not None else None
        ref = orc.amplitudes(pos, nb if nb is not None else np.zeros(W), mb if mb is not None else np.zeros((W, 3)),
                             qy[idx], qz[idx])
        gpu = amp_to_complex(amp[b])[idx]
        for c in range(4):
            if np.max(np.abs(ref[:, c])) == 0:
                assert np.max(np.abs(gpu[:, c])) == 0, (b, c)
            else:
                assert gated_rel_err(gpu[:, c], ref[:, c]) <= 1e-9, (b, c)
        single = numag.Sample(nuc=nb, mag=mb, regular=reg, n_points=W, device=DEV)
        one, _ = numag.amplitudes(single, grid, path=path)
        assert torch.equal(amp[b], one[0]), f"snapshot {b} differs from its single call"
