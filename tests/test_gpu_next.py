"""Parity of the 2D correlation function (eq. crav2d) and the angular spectrum
(eqs. CosineSinceIntensities, ModalAmplitudes) with the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402
from tests.helpers import max_norm_err  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("kind,n0,n1,rkind,r0,r1", [(1, 37, 64, 1, 10, 16), (0, 40, 53, 0, 21, 17),
                                                     (1, 20, 30, 0, 9, 12), (0, 33, 33, 1, 7, 24),
                                                     (1, 20, 30, 1, 9, 15), (0, 25, 31, 0, 1, 8)])
def test_correlation_2d_vs_oracle(orc, kind, n0, n1, rkind, r0, r1):
    """Six data sets (the four weight channels carry four at a time, plus a partial
    group) on both detector kinds and both real-space grid kinds."""
    rng = np.random.default_rng(50 + n0)
    P = n0 * n1
    f = rng.standard_normal((6, P))
    qmax, rmax = 1.2, 25.0
    grid = numag.qgrid(kind, n0, n1, qmax)
    rgrid = numag.qgrid(rkind, r0, r1, rmax)
    C = numag.correlation_2d(grid, torch.as_tensor(f, device=DEV), rgrid).cpu().numpy()
    C = C[..., 0] + 1j * C[..., 1]
    ref = orc.correlation_2d(kind, n0, n1, qmax, f, rkind, r0, r1, rmax)
    assert max_norm_err(C, ref) <= 1e-10


@pytest.mark.parametrize("n_f", [1, 3, 5, 7])
@pytest.mark.parametrize("kind,n0,n1,rkind,r0,r1", [(1, 24, 40, 1, 9, 16), (0, 27, 31, 0, 13, 11)])
def test_correlation_2d_every_channel_grouping(orc, kind, n0, n1, rkind, r0, r1, n_f):
    """Groups of one data set (one weight channel), of two or three (channels 1-3) and
    of four, alone and after a full group, against the oracle."""
    rng = np.random.default_rng(70 + n_f + n0)
    f = rng.standard_normal((n_f, n0 * n1))
    qmax, rmax = 1.1, 20.0
    grid = numag.qgrid(kind, n0, n1, qmax)
    rgrid = numag.qgrid(rkind, r0, r1, rmax)
    C = numag.correlation_2d(grid, torch.as_tensor(f, device=DEV), rgrid).cpu().numpy()
    ref = orc.correlation_2d(kind, n0, n1, qmax, f, rkind, r0, r1, rmax)
    assert C.shape == (n_f, r0 * r1, 2)
    assert max_norm_err(C[..., 0] + 1j * C[..., 1], ref) <= 1e-10


def test_correlation_2d_of_sphere_cross_section(orc):
    """C of the unpolarized sphere cross section on a polar detector (the use of
    Sec. 4.1, Fig. 6d): the GPU pipeline sums -> cross section -> correlation
    against the oracle's."""
    cfg = synth.sphere_40nm()
    nq, nt, qmax = 48, 72, 1.0
    grid = numag.qgrid(1, nq, nt, qmax)
    s = numag.Sample(pos=cfg["pos"], nuc=cfg["nuc"], mag=cfg["mag"], device=DEV)
    amp, _ = numag.amplitudes(s, grid)
    sf = numag.cross_section(grid, amp=amp, obs=("SF", "UNPOL"))[0]
    rgrid = numag.qgrid(0, 31, 31, 40.0)
    C = numag.correlation_2d(grid, sf, rgrid).cpu().numpy()
    qy, qz, qhat = orc.pixels(1, nq, nt, qmax)
    A = orc.amplitudes(cfg["pos"], cfg["nuc"], cfg["mag"], qy, qz)
    o = orc.cross_sections(A, qhat)
    ref = orc.correlation_2d(1, nq, nt, qmax, np.stack([o["SF"], o["UNPOL"]]), 0, 31, 31, 40.0)
    assert max_norm_err(C[..., 0] + 1j * C[..., 1], ref) <= 1e-9


def test_angular_spectrum_vs_oracle(orc):
    rng = np.random.default_rng(60)
    nq, nt, kmax = 11, 40, 9
    f = rng.standard_normal((3, nq * nt))
    grid = numag.qgrid(1, nq, nt, 1.0)
    Is, Ic, As, Ac = numag.angular_spectrum(grid, torch.as_tensor(f, device=DEV), kmax)
    for s in range(3):
        Isr, Icr = orc.angular_spectrum(f[s], nq, nt, kmax)
        assert max_norm_err(Is[s].cpu().numpy(), Isr) <= 1e-12
        assert max_norm_err(Ic[s].cpu().numpy(), Icr) <= 1e-12
        Asr, Acr = orc.modal_amplitudes(Isr, Icr)
        assert max_norm_err(As[s].cpu().numpy(), Asr) <= 1e-12
        assert max_norm_err(Ac[s].cpu().numpy(), Acr) <= 1e-12


@pytest.mark.parametrize("kind,n0,n1", [(0, 33, 41), (1, 25, 48)])
def test_spectral_matrix_export(orc, kind, n0, n1):
    """Sec. 3.4 export G_ab = A_a conj(A_b) on both detector kinds: against the
    oracle's spectral matrix of the oracle's sums, and the identity with the
    cross sections (computed from G or from the amplitudes, the same numbers)."""
    cl = synth.random_cloud(1800, 9.0, seed=61)
    grid = numag.qgrid(kind, n0, n1, 1.3)
    s = numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV)
    R = synth.sample_rotation(20, 75)
    amp, _ = numag.amplitudes(s, grid, rot=R)
    G = numag.spectral_matrix(grid, amp)
    qy, qz, _ = orc.pixels(kind, n0, n1, 1.3)
    Gref = orc.spectral(orc.amplitudes(cl["pos"], cl["nuc"], cl["mag"], qy, qz, R=R))
    assert max_norm_err(G[0].cpu().numpy(), Gref) <= 1e-9
    xa = numag.cross_section(grid, amp=amp, obs=numag.OBSERVABLES)
    xg = numag.cross_section(grid, spec=G, obs=numag.OBSERVABLES)
    assert max_norm_err(xg.cpu().numpy(), xa.cpu().numpy()) <= 1e-12
