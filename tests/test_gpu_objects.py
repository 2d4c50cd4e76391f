"""Parity of the object and orientation path (dilute / split modes, many
rotations, persistent launch, HIP-graph replay) with the FP64 oracle.

The oracle side forms the dilute cross sections as sum_k obs(F_k) and the
spectral matrix as sum_k F_k F_k^H from its per-object sums; the GPU side
accumulates the spectral matrix in its kernel and evaluates the cross
sections as linear functionals of it.  Tolerance: the accuracy gate
(relative error <= 1e-5 at pixels >= 1e-6 of the maximum)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402
from tests.helpers import amp_to_complex, gated_rel_err, max_norm_err  # noqa: E402

TOL = 1e-5
DEV = "cuda:0"


def _objects(seed, sizes, extent=4.0, spread=30.0):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    W = int(off[-1])
    return {"pos": rng.uniform(-extent, extent, (W, 3)), "nuc": rng.standard_normal(W),
            "mag": rng.standard_normal((W, 3)), "obj_offsets": off,
            "obj_pos": rng.uniform(-spread, spread, (len(sizes), 3))}


def _sample(cfg):
    return numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], obj_offsets=cfg["obj_offsets"],
                        obj_pos=cfg.get("obj_pos"), device=DEV)


def _check_spec(G, Gref):
    # diagonal entries and complex off-diagonal entries, gated per entry; an entry
    # whose reference stays below 1e-12 of the matrix's largest entry is zero in
    # exact arithmetic (e.g. Im G_ab of a one-point object) and is compared in
    # absolute terms against that scale
    scale = np.max(np.abs(Gref))
    for v in range(16):
        if np.max(np.abs(Gref[:, v])) <= 1e-12 * scale:
            assert np.max(np.abs(G[:, v])) <= 1e-12 * scale, v
            continue
        e = gated_rel_err(G[:, v], Gref[:, v])
        assert e <= TOL or max_norm_err(G[:, v], Gref[:, v]) <= 1e-12, (v, e)


def test_split_mode_form_factor_and_interference(orc):
    """Sec. 3.3 summation relation: split mode returns the coherent total and the
    form-factor spectral matrix; every cross section splits into form factor +
    interparticle interference."""
    cfg = _objects(40, [10, 400, 37, 250, 123])
    R = synth.sample_rotation(25.0, 65.0)
    n0, n1, qmax = 48, 72, 1.1
    grid = numag.qgrid(0, n0, n1, qmax)
    amp, spec = numag.amplitudes(_sample(cfg), grid, rot=R, mode=numag.MODE_SPLIT)
    qy, qz, qhat = orc.pixels(0, n0, n1, qmax)
    A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, R=R, obj_offsets=cfg["obj_offsets"],
                       obj_pos=cfg["obj_pos"])
    F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, R=R, obj_offsets=cfg["obj_offsets"],
                       obj_pos=cfg["obj_pos"], per_object=True)
    a = amp_to_complex(amp[0])
    for c in range(4):
        assert gated_rel_err(a[:, c], A[:, c]) <= TOL
    _check_spec(spec[0].cpu().numpy(), orc.spectral(F))
    k = dict(V=2.0, bH=0.7, scale=1.0, P=(0.0, 0.6, 0.8))
    ff = numag.cross_section(grid, spec=spec, c=numag.consts(**k), obs=numag.OBSERVABLES)[0].cpu().numpy()
    tot = numag.cross_section(grid, amp=amp, c=numag.consts(**k), obs=numag.OBSERVABLES)[0].cpu().numpy()
    ff_ref = orc.cross_sections(F, qhat, **k)       # sum_k obs(F_k)
    tot_ref = orc.cross_sections(A, qhat, **k)
    for i, name in enumerate(numag.OBSERVABLES):
        assert gated_rel_err(ff[i], ff_ref[name]) <= TOL, name
        assert gated_rel_err(tot[i], tot_ref[name]) <= TOL, name
        # interference = total - form factor, both sides
        assert max_norm_err(tot[i] - ff[i], tot_ref[name] - ff_ref[name]) <= 1e-9, name


def test_dilute_per_object_rotation_average(orc):
    """Dilute sample, many rotations, one spectral matrix per object averaged
    over the rotations (the orientational average of the batched path)."""
    cfg = _objects(41, [60, 5, 140], spread=0.0)
    rots = synth.uniform_rotations(7, np.random.default_rng(42))
    n0, n1, qmax = 32, 40, 1.3
    grid = numag.qgrid(0, n0, n1, qmax)
    _, spec = numag.amplitudes(_sample(cfg), grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
    spec = spec.cpu().numpy()
    qy, qz, qhat = orc.pixels(0, n0, n1, qmax)
    off = cfg["obj_offsets"]
    for k in range(3):
        sl = slice(off[k], off[k + 1])
        Fs = [orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R) for R in rots]
        Gref = orc.spectral(np.stack(Fs)) / len(rots)
        _check_spec(spec[k], Gref)
    # summed over objects
    _, tot = numag.amplitudes(_sample(cfg), grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=False)
    assert max_norm_err(tot[0].cpu().numpy(), spec.sum(axis=0)) <= 1e-12


def test_dilute_single_object_equals_coherent(orc):
    """A single object has no interparticle interference: the dilute cross
    sections equal the coherent ones."""
    cl = synth.random_cloud(900, 6.0, seed=43)
    grid = numag.qgrid(0, 30, 50, 1.0)
    s = numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV)
    amp, _ = numag.amplitudes(s, grid)
    _, spec = numag.amplitudes(s, grid, mode=numag.MODE_DILUTE)
    x1 = numag.cross_section(grid, amp=amp, obs=numag.OBSERVABLES)[0].cpu().numpy()
    x2 = numag.cross_section(grid, spec=spec, obs=numag.OBSERVABLES)[0].cpu().numpy()
    assert max_norm_err(x2, x1) <= 1e-12


def test_batched_orientations_graph_replay_c4_subsample(orc):
    """64 particles of uneven size (1e3-2e5 points) under 1000 uniform rotations on
    a 128 x 128 detector: one persistent launch recorded into a HIP graph.  The
    replays (with eager work in between) equal the eager result bit for bit,
    and the two smallest particles are checked against the oracle over all
    1000 rotations on 48 sampled pixels."""
    cfg = synth.particles_rotations()
    g = cfg["grid"]
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    s = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], obj_offsets=cfg["obj_offsets"], device=DEV)
    rots = cfg["rotations"]
    b = numag.BatchedOrientations(s, grid, rots, spec_per_object=True)
    ref = b.eager().clone()
    torch.cuda.synchronize()
    for _ in range(2):
        out = b.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        _ = torch.ones(1000, device=DEV).sum().item()  # eager work between replays
    spec = ref.cpu().numpy()
    off = cfg["obj_offsets"]
    sizes = np.diff(off)
    small = np.argsort(sizes)[:2]
    qy, qz, qhat = orc.pixels(0, g["n0"], g["n1"], g["qmax"])
    rng = np.random.default_rng(44)
    idx = np.sort(rng.choice(qy.size, 48, replace=False))
    for k in small:
        sl = slice(off[k], off[k + 1])
        acc = np.zeros((idx.size, 16))
        for R in rots:
            acc += orc.spectral(orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy[idx], qz[idx], R=R))
        _check_spec(spec[k][idx], acc / len(rots))
    # orientation-averaged unpolarized pattern of every particle is finite and >= 0
    un = numag.cross_section(grid, spec=ref, obs=("UNPOL",))[:, 0].cpu().numpy()
    assert np.all(np.isfinite(un)) and un.min() >= -1e-9 * un.max()


def test_sphere_ensemble_split_full_size_sampled(orc):
    """512 spheres (2.6e6 points, random non-overlapping centres in a 500 nm cube)
    on a 512 x 512 detector in split mode: form factor, interparticle
    interference and the spin-flip cross section, on 40 sampled pixels."""
    cfg = synth.sphere_ensemble()
    g = cfg["grid"]
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    amp, spec = numag.amplitudes(_sample(cfg), grid, mode=numag.MODE_SPLIT)
    k = dict(V=1.0, bH=1.0, scale=1.0, P=(0.0, 0.0, 1.0))
    obs = ("N", "M", "SF", "UNPOL")
    ff = numag.cross_section(grid, spec=spec, c=numag.consts(**k), obs=obs)[0].cpu().numpy()
    tot = numag.cross_section(grid, amp=amp, c=numag.consts(**k), obs=obs)[0].cpu().numpy()
    qy, qz, qhat = orc.pixels(0, g["n0"], g["n1"], g["qmax"])
    rng = np.random.default_rng(45)
    idx = np.sort(rng.choice(qy.size, 40, replace=False))
    F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[idx], qz[idx], obj_offsets=cfg["obj_offsets"],
                       obj_pos=cfg["obj_pos"], per_object=True)
    A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[idx], qz[idx], obj_offsets=cfg["obj_offsets"],
                       obj_pos=cfg["obj_pos"])
    ff_ref = orc.cross_sections(F, qhat[idx], **k)
    tot_ref = orc.cross_sections(A, qhat[idx], **k)
    for i, name in enumerate(obs):
        assert gated_rel_err(ff[i][idx], ff_ref[name]) <= TOL, name
        assert gated_rel_err(tot[i][idx], tot_ref[name]) <= TOL, name
        interf = tot_ref[name] - ff_ref[name]
        scale = np.max(np.abs(tot_ref[name]))
        assert np.max(np.abs((tot[i][idx] - ff[i][idx]) - interf)) <= 1e-8 * scale, name


@pytest.mark.parametrize("mode", ["dilute", "split"])
def test_empty_and_single_point_objects(orc, mode):
    """Objects with zero points (their spectral matrix is zero) and with one point
    (|F|^2 = w^2 at every pixel), next to ordinary ones, on a detector wide enough
    for the widest lane layout (two column blocks)."""
    cfg = _objects(47, [0, 1, 37, 0, 129, 1], spread=12.0)
    n0, n1, qmax = 9, 530, 1.1
    grid = numag.qgrid(0, n0, n1, qmax)
    qy, qz, qhat = orc.pixels(0, n0, n1, qmax)
    off = cfg["obj_offsets"]
    if mode == "dilute":
        R = synth.sample_rotation(70, 15)
        _, spec = numag.amplitudes(_sample(cfg), grid, rot=R, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec = spec.cpu().numpy()
        for k in range(6):
            sl = slice(off[k], off[k + 1])
            if off[k + 1] == off[k]:
                assert np.count_nonzero(spec[k]) == 0, k
                continue
            F = orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R)
            _check_spec(spec[k], orc.spectral(F))
            if off[k + 1] - off[k] == 1:
                j = off[k]
                w = np.concatenate([[cfg["nuc"][j]], R @ cfg["mag"][j]])
                assert np.allclose(spec[k][:, :4], (w ** 2)[None, :], rtol=1e-12, atol=0)
    else:
        amp, spec = numag.amplitudes(_sample(cfg), grid, mode=numag.MODE_SPLIT)
        A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, obj_offsets=off, obj_pos=cfg["obj_pos"])
        F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, obj_offsets=off, obj_pos=cfg["obj_pos"],
                           per_object=True)
        gpu = amp_to_complex(amp[0])
        for c in range(4):
            assert gated_rel_err(gpu[:, c], A[:, c]) <= TOL, c
        _check_spec(spec[0].cpu().numpy(), orc.spectral(F))


@pytest.mark.parametrize("mode", ["dilute", "split"])
def test_object_modes_on_polar_detector(orc, mode):
    """Dilute (several rotations, one spectral matrix per object) and split modes on
    the paper's polar (q, theta) detector, with an empty object."""
    cfg = _objects(48, [90, 0, 33, 150], spread=14.0)
    nq, nt, qmax = 21, 36, 1.2
    grid = numag.qgrid(1, nq, nt, qmax)
    qy, qz, qhat = orc.pixels(1, nq, nt, qmax)
    off = cfg["obj_offsets"]
    if mode == "dilute":
        rots = synth.uniform_rotations(3, np.random.default_rng(49))
        _, spec = numag.amplitudes(_sample(cfg), grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec = spec.cpu().numpy()
        for k in range(4):
            sl = slice(off[k], off[k + 1])
            if off[k + 1] == off[k]:
                assert np.count_nonzero(spec[k]) == 0
                continue
            Fs = [orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R) for R in rots]
            _check_spec(spec[k], orc.spectral(np.stack(Fs)) / len(rots))
    else:
        amp, spec = numag.amplitudes(_sample(cfg), grid, mode=numag.MODE_SPLIT)
        A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, obj_offsets=off, obj_pos=cfg["obj_pos"])
        F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, obj_offsets=off, obj_pos=cfg["obj_pos"],
                           per_object=True)
        gpu = amp_to_complex(amp[0])
        for c in range(4):
            assert gated_rel_err(gpu[:, c], A[:, c]) <= TOL, c
        _check_spec(spec[0].cpu().numpy(), orc.spectral(F))


@pytest.mark.parametrize("kind,n0,n1,mode", [(0, 33, 40, "dilute"), (0, 32, 41, "split"), (1, 17, 36, "dilute"),
                                             (1, 16, 24, "split")])
def test_hermitian_object_modes(orc, kind, n0, n1, mode):
    """The half-detector path in the object modes: rows [0, ceil(n0/2)) of a
    Cartesian detector (theta in [0, pi) of a polar one) are summed and the rest
    follows from G(-q) = conj G(q) and, in split mode, A(-q) = conj A(q) (real
    weights, also after rotation).  Checked against the oracle at every pixel and
    against the full path, which it must equal up to rounding (a mirrored pixel
    takes its partner's conjugate, at -q within an ulp).  With an empty object
    and, for the dilute Cartesian case, the batched graph replay."""
    cfg = _objects(50, [70, 0, 25, 120], spread=12.0)
    qmax = 1.1
    grid = numag.qgrid(kind, n0, n1, qmax)
    qy, qz, qhat = orc.pixels(kind, n0, n1, qmax)
    off = cfg["obj_offsets"]
    H = numag.PATH_DIRECT_HERMITIAN
    if mode == "dilute":
        rots = synth.uniform_rotations(3, np.random.default_rng(51))
        _, spec = numag.amplitudes(_sample(cfg), grid, rot=rots, path=H, mode=numag.MODE_DILUTE,
                                   spec_per_object=True)
        _, full = numag.amplitudes(_sample(cfg), grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
        spec, full = spec.cpu().numpy(), full.cpu().numpy()
        for k in range(4):
            sl = slice(off[k], off[k + 1])
            if off[k + 1] == off[k]:
                assert np.count_nonzero(spec[k]) == 0
                continue
            Fs = [orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R) for R in rots]
            _check_spec(spec[k], orc.spectral(np.stack(Fs)) / len(rots))
            assert max_norm_err(spec[k], full[k]) <= 1e-11, k
        if kind == 0:
            b = numag.BatchedOrientations(_sample(cfg), grid, rots, spec_per_object=True, path=H)
            ref = b.eager().clone()
            torch.cuda.synchronize()
            assert max_norm_err(ref.cpu().numpy(), spec) <= 1e-14
            for _ in range(2):
                out = b.replay()
                torch.cuda.synchronize()
                assert torch.equal(out, ref)
                _ = torch.ones(1000, device=DEV).sum().item()  # eager work between replays
    else:
        R = synth.sample_rotation(20.0, 50.0)
        amp, spec = numag.amplitudes(_sample(cfg), grid, rot=R, path=H, mode=numag.MODE_SPLIT)
        ampf, specf = numag.amplitudes(_sample(cfg), grid, rot=R, mode=numag.MODE_SPLIT)
        A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, R=R, obj_offsets=off, obj_pos=cfg["obj_pos"])
        F = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz, R=R, obj_offsets=off, obj_pos=cfg["obj_pos"],
                           per_object=True)
        gpu = amp_to_complex(amp[0])
        for c in range(4):
            assert gated_rel_err(gpu[:, c], A[:, c]) <= TOL, c
        _check_spec(spec[0].cpu().numpy(), orc.spectral(F))
        assert max_norm_err(amp.cpu().numpy(), ampf.cpu().numpy()) <= 1e-11
        assert max_norm_err(spec.cpu().numpy(), specf.cpu().numpy()) <= 1e-11


def test_workspace_reuse_never_reads_stale_tables():
    """Object modes take their tables from the start of the workspace.  A plain
    call uploads them on every call, so a workspace freed and allocated again at
    the same address with foreign bytes in it gives the right result for another
    sample.  A plan's calls read the tables its upload left there, guarded by the
    plan's tag: a workspace whose tables were overwritten, or that holds another
    plan's upload, gives NaN; uploading again restores the result bit for bit."""
    cfg = _objects(52, [40, 90, 15], spread=0.0)
    rots = synth.uniform_rotations(4, np.random.default_rng(53))
    grid = numag.qgrid(0, 20, 28, 1.0)
    s = _sample(cfg)
    nws = numag.workspace_size(s, grid, len(rots), numag.PATH_DIRECT, numag.MODE_DILUTE)
    ws = torch.empty(nws, dtype=torch.uint8, device=DEV)
    _, ref = numag.amplitudes(s, grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True, ws=ws)
    ref = ref.clone()
    torch.cuda.synchronize()
    addr = ws.data_ptr()
    del ws
    # another sample (other offsets) on a buffer allocated after the free, full of foreign bytes
    cfg2 = _objects(54, [70, 5, 60], spread=0.0)
    s2 = _sample(cfg2)
    ws2 = torch.full((nws,), 0xFF, dtype=torch.uint8, device=DEV)
    print("workspace reallocated at the same address:", ws2.data_ptr() == addr, flush=True)
    _, got2 = numag.amplitudes(s2, grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True, ws=ws2)
    _, want2 = numag.amplitudes(s2, grid, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True,
                                ws=torch.empty(nws, dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(got2, want2)
    # plans: one upload, many calls; overwritten or foreign tables give NaN
    for kind in (0, 1):
        g = numag.qgrid(kind, 20, 28, 1.0)
        pa = numag.Plan(s, g, rots, mode=numag.MODE_DILUTE, spec_per_object=True)
        pb = numag.Plan(s, g, rots[::-1].copy(), mode=numag.MODE_DILUTE, spec_per_object=True)
        pa.upload()
        _, a1 = pa()
        _, a2 = pa()
        a1 = a1.clone()
        torch.cuda.synchronize()
        assert torch.equal(a1, a2) and float(a1.abs().max()) > 0.0
        _, direct = numag.amplitudes(s, g, rot=rots, mode=numag.MODE_DILUTE, spec_per_object=True)
        assert max_norm_err(a1.cpu().numpy(), direct.cpu().numpy()) <= 1e-12
        pa.ws.zero_()
        _, z = pa()
        torch.cuda.synchronize()
        assert torch.isnan(z).all(), kind
        pa.upload()
        _, a3 = pa()
        torch.cuda.synchronize()
        assert torch.equal(a3, a1)
        _, f = pb(ws=pa.ws)  # pa's tables, pb's tag
        torch.cuda.synchronize()
        assert torch.isnan(f).all(), kind


@pytest.mark.parametrize("nq,nt,path", [(24, 30, 0), (40, 36, 0), (40, 36, 3), (130, 20, 0), (130, 20, 3)])
def test_dilute_polar_rotation_groups(orc, nq, nt, path):
    """Dilute mode on a polar detector runs each object over groups of rotations
    (one launch sequence per group, as many rotations as the sample's buffers
    and the chip take): objects from 1 to 3000 points and an empty one give
    groups of one rotation up to all 37, on 4-wave (24 q rows) and 8-wave (40 q
    rows; 130 q rows: three row blocks, whose starts are powers of the q step)
    kernels and on the half-detector path; every object's orientational average
    against the oracle."""
    cfg = _objects(64, [5, 200, 3000, 0, 40, 1, 800], spread=0.0)
    rots = synth.uniform_rotations(37, np.random.default_rng(65))
    qmax = 1.1
    grid = numag.qgrid(1, nq, nt, qmax)
    qy, qz, _ = orc.pixels(1, nq, nt, qmax)
    _, spec = numag.amplitudes(_sample(cfg), grid, rot=rots, path=path, mode=numag.MODE_DILUTE,
                               spec_per_object=True)
    spec = spec.cpu().numpy()
    off = cfg["obj_offsets"]
    for k in range(len(off) - 1):
        sl = slice(off[k], off[k + 1])
        if off[k + 1] == off[k]:
            assert np.count_nonzero(spec[k]) == 0
            continue
        Fs = [orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R) for R in rots]
        _check_spec(spec[k], orc.spectral(np.stack(Fs)) / len(rots))
    # summed over objects
    _, tot = numag.amplitudes(_sample(cfg), grid, rot=rots, path=path, mode=numag.MODE_DILUTE)
    assert max_norm_err(tot[0].cpu().numpy(), spec.sum(axis=0)) <= 1e-12


@pytest.mark.parametrize("path", [0, 3])
def test_batched_orientations_graph_replay_polar(orc, path):
    """The orientation batch on a polar detector: the plan's kernels (rotation
    groups on the polar direct kernel) recorded into a HIP graph; every replay,
    with eager work in between, equals the eager result bit for bit, and one
    object's average equals the oracle's."""
    cfg = _objects(66, [5, 200, 3000, 0, 40], spread=0.0)
    rots = synth.uniform_rotations(12, np.random.default_rng(67))
    qmax = 1.1
    grid = numag.qgrid(1, 40, 36, qmax)
    b = numag.BatchedOrientations(_sample(cfg), grid, rots, spec_per_object=True, path=path)
    ref = b.eager().clone()
    torch.cuda.synchronize()
    for _ in range(3):
        out = b.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        _ = torch.ones(1000, device=DEV).sum().item()  # eager work between replays
    off = cfg["obj_offsets"]
    k = 2
    sl = slice(off[k], off[k + 1])
    qy, qz, _ = orc.pixels(1, 40, 36, qmax)
    Fs = [orc.amplitudes(cfg["pos"][sl], cfg["nuc"][sl], cfg["mag"][sl], qy, qz, R=R) for R in rots]
    _check_spec(ref[k].cpu().numpy(), orc.spectral(np.stack(Fs)) / len(rots))
