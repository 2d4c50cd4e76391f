"""The launch-shape autotuner on the GPU: numag_autotune picks a valid shape for
each kernel, and every candidate shape of each kernel (set explicitly in the
table) gives sums, spectral matrices and gradients within the accuracy gate of
the FP64 oracle (relative error <= 1e-5 at pixels >= 1e-6 of the maximum; Sec. 3.3
DSFT, dilute limit; Sec. 2.4 loss).  Shapes only re-cut the work, so the
sums under different shapes also agree with each other to rounding.
"""
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


@pytest.fixture(autouse=True)
def _clean_table():
    numag.tune_clear()
    yield
    numag.tune_clear()


def _check(gpu, ref):
    for c in range(ref.shape[-1]):
        if np.max(np.abs(ref[..., c])) > 0:
            assert gated_rel_err(gpu[..., c], ref[..., c]) <= TOL, c


def _direct_shapes(grid):
    if grid.kind == numag.GRID_POLAR:
        shapes = [1, 0] if grid.n0 <= 32 else [0, 2, 3, 4]
        return [(s, t) for s in shapes for t in (256, 1024)]
    return [(l, t) for l in (8, 16, 32, 64) for t in (512, 2048, 4096)]


@pytest.mark.parametrize("kind,n0,n1", [(0, 70, 130), (0, 33, 300), (1, 150, 70), (1, 300, 37), (1, 20, 130)])
def test_every_direct_shape_within_gate(orc, kind, n0, n1):
    cl = synth.random_cloud(5000, 10.0, seed=31)
    s = numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV)
    grid = numag.qgrid(kind, n0, n1, 1.2)
    R = synth.sample_rotation(25.0, 40.0)
    qy, qz, _ = orc.pixels(kind, n0, n1, 1.2)
    ref = orc.amplitudes(cl["pos"], cl["nuc"], cl["mag"], qy, qz, R=R)
    first = None
    for shape in _direct_shapes(grid):
        numag.tune_set(numag.TUNE_DIRECT, grid, 5000, shape)
        assert numag.tune_get(numag.TUNE_DIRECT, grid, 5000)[1] == shape
        amp, _ = numag.amplitudes(s, grid, rot=R)
        a = amp_to_complex(amp[0])
        _check(a, ref)
        if first is None:
            first = a
        assert max_norm_err(a, first) <= 1e-12, shape


def test_autotune_direct_and_adjoint_keep_parity(orc):
    cl = synth.random_cloud(20000, 12.0, seed=32)
    s = numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV)
    for kind, n0, n1 in [(0, 96, 96), (1, 130, 64)]:
        grid = numag.qgrid(kind, n0, n1, 1.0)
        chosen = numag.autotune(s, grid, numag.TUNE_DIRECT)
        d, cur, tuned = numag.tune_get(numag.TUNE_DIRECT, grid, 20000)
        assert tuned and cur == chosen
        qy, qz, qhat = orc.pixels(kind, n0, n1, 1.0)
        amp, _ = numag.amplitudes(s, grid)
        _check(amp_to_complex(amp[0]), orc.amplitudes(cl["pos"], cl["nuc"], cl["mag"], qy, qz))
        # the adjoint: tuned, then every candidate against the oracle gradient
        numag.autotune(s, grid, numag.TUNE_ADJOINT)
        assert numag.tune_get(numag.TUNE_ADJOINT, grid, 20000)[2]
        rng = np.random.default_rng(33)
        T = rng.uniform(0.0, 1.0, qy.size)
        w = rng.uniform(0.5, 1.5, qy.size)
        L, dn, dm = orc.loss_grad(cl["pos"], cl["nuc"], cl["mag"], qy, qz, qhat, T, w)
        for target in (0, 2048, 4096, 8192):
            if target:
                numag.tune_set(numag.TUNE_ADJOINT, grid, 20000, (0, target))
            loss, gdn, gdm = numag.grad(s, grid, numag.consts(), weight=torch.as_tensor(w, device=DEV),
                                        target=torch.as_tensor(T, device=DEV))
            assert abs(loss.item() - L) <= 1e-9 * abs(L)
            assert max_norm_err(gdn.cpu().numpy(), dn) <= 1e-9
            assert max_norm_err(gdm.cpu().numpy(), dm) <= 1e-9


@pytest.mark.parametrize("kind,n0,n1", [(0, 48, 80), (1, 140, 40), (1, 24, 64)])
def test_autotune_objects_and_every_object_shape(orc, kind, n0, n1):
    """Dilute per-object orientational averages: the persistent kernel under the
    tuned shape and under every candidate (Cartesian: lanes per row; polar: the
    workgroup shape; x work items)."""
    rng = np.random.default_rng(34)
    sizes = [1500, 40, 3100, 700]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    W = int(off[-1])
    pos = rng.uniform(-7.0, 7.0, (W, 3))
    nuc = rng.standard_normal(W)
    mag = rng.standard_normal((W, 3))
    s = numag.Sample(pos=pos, nuc=nuc, mag=mag, obj_offsets=off, device=DEV)
    grid = numag.qgrid(kind, n0, n1, 1.1)
    rots = synth.uniform_rotations(6, np.random.default_rng(35))
    chosen = numag.autotune(s, grid, numag.TUNE_OBJECTS, rot=rots)
    assert numag.tune_get(numag.TUNE_OBJECTS, grid, W)[1] == chosen
    qy, qz, _ = orc.pixels(kind, n0, n1, 1.1)
    acc = np.zeros((len(sizes), qy.size, 16))
    for R in rots:
        F = orc.amplitudes(pos, nuc, mag, qy, qz, R=R, obj_offsets=off, per_object=True)
        for k in range(len(sizes)):
            acc[k] += orc.spectral(F[k])
    acc /= len(rots)
    if kind == numag.GRID_POLAR:
        shapes = [(sh, t) for sh in ((1, 0) if n0 <= 32 else (0, 2, 3, 4)) for t in (64, 1024)]
    else:
        shapes = [(l, t) for l in (8, 16, 32) for t in (64, 1024, 4096)]
    for shape in [None] + shapes:
        if shape is not None:
            numag.tune_set(numag.TUNE_OBJECTS, grid, W, shape)
        _, spec = numag.amplitudes(s, grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec = spec.cpu().numpy()
        for k in range(len(sizes)):
            for v in range(16):
                assert gated_rel_err(spec[k][:, v], acc[k][:, v]) <= TOL, (shape, k, v)


def test_autotune_cache_file_round_trip(tmp_path):
    """numag_autotune writes the cache file named by NUMAG_AUTOTUNE_CACHE when the
    process starts with it set (checked in a child process)."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = tmp_path / "shapes.txt"
    code = ("import sys; sys.path.insert(0, sys.argv[1]); from paper_2601_18444_amd import numag, synth; "
            "cl = synth.random_cloud(3000, 8.0, seed=36); "
            "s = numag.Sample(pos=cl['pos'], nuc=cl['nuc'], mag=cl['mag'], device='cuda:0'); "
            "g = numag.qgrid(1, 64, 64, 1.0); print(numag.autotune(s, g, numag.TUNE_DIRECT))")
    env = dict(os.environ, NUMAG_AUTOTUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code, root], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [l for l in path.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 1 and lines[0].split()[1] == "direct" and lines[0].split()[3:5] == ["64", "64"]


def test_hermitian_gradient_workspace_follows_the_half_detector_shape():
    """On the half-detector path the adjoint runs on half of the detector with that
    part's launch shape, and its workspace is sized for that shape whatever the
    whole detector's is: a small adjoint target pinned for the whole detector (few
    row splits) and none for the half (the default, many splits).  The gradient
    equals the one computed with an empty table bit for bit."""
    cl = synth.random_cloud(40000, 20.0, seed=95)
    W = cl["pos"].shape[0]
    s = numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV)
    grid = numag.qgrid(0, 96, 80, 1.1)
    c = numag.consts(V=2.0, bH=0.7)
    weight = torch.ones(grid.n_pixels, dtype=torch.float64, device=DEV)
    target = torch.full((grid.n_pixels,), 0.5, dtype=torch.float64, device=DEV)
    H = numag.PATH_DIRECT_HERMITIAN
    ref = [t.clone() for t in numag.grad(s, grid, c, weight, target, path=H)]
    numag.tune_set(numag.TUNE_ADJOINT, grid, W, shape=(0, 64), path=numag.PATH_DIRECT)
    assert numag.tune_get(numag.TUNE_ADJOINT, grid, W, path=H)[2] is False  # the half has no entry
    numag.clear_workspace_cache()  # the binding allocates exactly what the library asks for
    got = numag.grad(s, grid, c, weight, target, path=H)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    # and the whole-detector gradient under the pinned shape agrees with it to rounding
    full = numag.grad(s, grid, c, weight, target)
    torch.cuda.synchronize()
    for a, b in zip(full[1:], ref[1:]):
        assert float((a - b).abs().max()) <= 1e-10 * float(b.abs().max())


def _pin_random_shapes(rng, grid, W, kind, n0):
    """Random valid table entries for every kernel on the whole and the half detector."""
    for path in (numag.PATH_DIRECT, numag.PATH_DIRECT_HERMITIAN):
        if kind == 1 and path == numag.PATH_DIRECT_HERMITIAN and grid.n1 % 2:
            continue
        polar_shapes = [0, 2, 3, 4] + ([1] if n0 <= 32 else [])
        sh = int(rng.choice([8, 16, 32, 64])) if kind == 0 else int(rng.choice(polar_shapes))
        numag.tune_set(numag.TUNE_DIRECT, grid, W, shape=(sh, int(rng.choice([64, 1024, 8192]))), path=path)
        numag.tune_set(numag.TUNE_ADJOINT, grid, W, shape=(0, int(rng.choice([16, 512, 16384]))), path=path)
        sh = int(rng.choice([8, 16, 32, 64])) if kind == 0 else int(rng.choice(polar_shapes))
        numag.tune_set(numag.TUNE_OBJECTS, grid, W, shape=(sh, int(rng.choice([32, 2048, 8192]))), path=path)


@pytest.mark.parametrize("case", range(10))
def test_random_pinned_shapes_size_their_workspaces(orc, case):
    """Every workspace (sums, allocation-free sums, gradient, dilute objects) is sized
    for the launch shape its kernels take, whatever shapes the table holds for the
    whole and the half detector: random entries for every kernel, then every entry
    point against the oracle on both paths."""
    rng = np.random.default_rng(70000 + case)
    kind = int(rng.integers(0, 2))
    n0, n1 = int(rng.integers(1, 90)), int(rng.integers(1, 90))
    if kind == 1:
        n1 += n1 % 2
    qmax = float(rng.uniform(0.2, 2.5))
    K = int(rng.integers(2, 5))
    sizes = rng.integers(1, 4000 // K + 1, K)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    W = int(off[-1])
    pos = rng.uniform(-10, 10, (W, 3))
    nuc, mag = rng.standard_normal(W), rng.standard_normal((W, 3))
    grid = numag.qgrid(kind, n0, n1, qmax)
    _pin_random_shapes(rng, grid, W, kind, n0)
    numag.clear_workspace_cache()
    qy, qz, qhat = orc.pixels(kind, n0, n1, qmax)
    R = synth.uniform_rotations(2, rng)
    s1 = numag.Sample(pos=pos, nuc=nuc, mag=mag, device=DEV)
    sK = numag.Sample(pos=pos, nuc=nuc, mag=mag, obj_offsets=off, device=DEV)
    A = orc.amplitudes(pos, nuc, mag, qy, qz, R=R[0])
    T, w = rng.uniform(0, 5, qy.size), rng.uniform(0.5, 1.5, qy.size)
    L, dn, dm = orc.loss_grad(pos, nuc, mag, qy, qz, qhat, T, w, R=R[0])
    for path in (numag.PATH_DIRECT, numag.PATH_DIRECT_HERMITIAN):
        amp, _ = numag.amplitudes(s1, grid, rot=R[0], path=path)
        for c in range(4):
            assert gated_rel_err(amp_to_complex(amp[0])[:, c], A[:, c]) <= 1e-9, (path, c)
        na = numag.amplitudes_noalloc(s1, grid, rot=R[0], path=path)
        assert max_norm_err(amp_to_complex(na[0]), amp_to_complex(amp[0])) <= 1e-11
        loss, gdn, gdm = numag.grad(s1, grid, numag.consts(), weight=torch.as_tensor(w, device=DEV),
                                    target=torch.as_tensor(T, device=DEV), rot=R[0], path=path)
        assert abs(loss.item() - L) <= 1e-9 * abs(L)
        assert max_norm_err(gdn.cpu().numpy(), dn) <= 1e-8 and max_norm_err(gdm.cpu().numpy(), dm) <= 1e-8
        _, spec = numag.amplitudes(sK, grid, rot=R, path=path, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec = spec.cpu().numpy()
        for k in range(K):
            sl = slice(off[k], off[k + 1])
            Fs = [orc.amplitudes(pos[sl], nuc[sl], mag[sl], qy, qz, R=Rr) for Rr in R]
            assert max_norm_err(spec[k], orc.spectral(np.stack(Fs)) / len(R)) <= 1e-9, (path, k)
