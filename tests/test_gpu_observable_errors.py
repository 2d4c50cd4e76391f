"""Gated relative error of every observable (Sec. 2.1-2.4 cross sections) against
the FP64 oracle, per FP64 path: the direct sums, their half-detector (Hermitian)
variant, the separable matrix-core sums and their Hermitian variant.  C1 (the
uniform 20 nm sphere on a 128 x 128 detector) over every pixel; C2 (the 64^3 vortex
on 256 x 256) on 256 sampled pixels.  The separable paths take C1 as its 21^3
lattice box with zero weights outside the sphere.  Each value is printed (the
figures quoted with the paths' documentation) and checked against the 1e-5 gate;
q = 0 is excluded, as in the other parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402
from tests.helpers import gated_rel_err, zero_q_mask  # noqa: E402

DEV = "cuda:0"
PATHS = (("direct", numag.PATH_DIRECT), ("direct_hermitian", numag.PATH_DIRECT_HERMITIAN),
         ("separable_f64", numag.PATH_SEPARABLE_F64), ("separable_f64_hermitian", numag.PATH_SEPARABLE_F64_HERMITIAN))


def _c1_box():
    """The C1 sphere as a regular 21^3 box of 2 nm cells, weights zero outside."""
    n, a, corner = (21, 21, 21), (2.0, 2.0, 2.0), (-20.0, -20.0, -20.0)
    box = synth.box_lattice(n, a, corner)
    inside = np.linalg.norm(box, axis=1) <= 20.0 + 1e-9
    nuc = inside.astype(np.float64)
    mag = np.zeros((box.shape[0], 3))
    mag[inside, 2] = 1.0
    return {"n": n, "origin": corner, "step": a}, box.shape[0], nuc, mag, int(inside.sum())


@pytest.mark.parametrize("case", ["C1_sphere_all_pixels", "C2_vortex_sampled"])
def test_observable_errors_per_path(orc, case):
    if case.startswith("C1"):
        cfg = synth.sphere_40nm()
        reg, Wbox, nbox, mbox, n_in = _c1_box()
        assert n_in == cfg["pos"].shape[0]
        idx = None
    else:
        cfg = synth.vortex_grid()
        reg, Wbox, nbox, mbox = cfg["regular"], cfg["pos"].shape[0], cfg["nuc"], cfg["mag"]
        idx = 256
    g = cfg["grid"]
    grid = numag.qgrid(g["kind"], g["n0"], g["n1"], g["qmax"])
    qy, qz, qhat = orc.pixels(g["kind"], g["n0"], g["n1"], g["qmax"])
    sel = np.arange(qy.size) if idx is None else np.sort(np.random.default_rng(90).choice(qy.size, idx, replace=False))
    ref = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy[sel], qz[sel])
    oref = orc.cross_sections(ref, qhat[sel])
    zq = zero_q_mask(qy[sel], qz[sel])
    direct_sample = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], device=DEV)
    box_sample = numag.Sample(nuc=nbox, mag=mbox, regular=reg, n_points=Wbox, device=DEV)
    worst = 0.0
    for name, path in PATHS:
        s = box_sample if name.startswith("separable") else direct_sample
        amp, _ = numag.amplitudes(s, grid, path=path)
        xs = numag.cross_section(grid, amp=amp, obs=numag.OBSERVABLES)[0].cpu().numpy()[:, sel]
        errs = {o: gated_rel_err(xs[i], oref[o], zq) for i, o in enumerate(numag.OBSERVABLES)}
        print(f"{case} {name}: " + ", ".join(f"{o} {e:.1e}" for o, e in errs.items()), flush=True)
        for o, e in errs.items():
            assert e <= 1e-5, f"{case} {name} {o}: {e:.3e}"
        worst = max(worst, max(errs.values()))
    print(f"{case} worst over paths and observables: {worst:.2e}", flush=True)
