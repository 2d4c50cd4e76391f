"""Zero-size inputs at the boundary give what their definitions fix: a sum over no
points is zero on every detector kind, path and rotation; the loss of a zero cross
section is sum_p w_p T_p^2 (Sec. 2.4) with empty gradients; every observable of zero
sums is zero, and so are their azimuthal average and 2D correlation; an empty
snapshot batch is refused with an error."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402

DEV = "cuda:0"


def _empty_sample():
    return numag.Sample(pos=np.zeros((0, 3)), nuc=np.zeros(0), mag=np.zeros((0, 3)), device=DEV)


GRIDS = [(numag.GRID_CARTESIAN, 16, 18, 1.0), (numag.GRID_POLAR, 12, 16, 1.0)]


@pytest.mark.parametrize("kind,n0,n1,qmax", GRIDS)
@pytest.mark.parametrize("path", [numag.PATH_DIRECT, numag.PATH_DIRECT_HERMITIAN])
def test_no_points_gives_zero_sums(kind, n0, n1, qmax, path):
    grid = numag.qgrid(kind, n0, n1, qmax)
    rots = np.stack([synth.sample_rotation(a, b) for a, b in ((0.0, 0.0), (30.0, 45.0), (90.0, 10.0))])
    amp, _ = numag.amplitudes(_empty_sample(), grid, rot=rots, path=path)
    torch.cuda.synchronize()
    assert amp.shape == (3, grid.n_pixels, 4, 2)
    assert torch.count_nonzero(amp).item() == 0
    xs = numag.cross_section(grid, amp=amp, obs=numag.OBSERVABLES)
    assert torch.count_nonzero(xs).item() == 0


@pytest.mark.parametrize("kind,n0,n1,qmax", GRIDS)
@pytest.mark.parametrize("path", [numag.PATH_DIRECT, numag.PATH_DIRECT_HERMITIAN])
def test_no_points_loss_and_gradient(kind, n0, n1, qmax, path):
    grid = numag.qgrid(kind, n0, n1, qmax)
    rng = np.random.default_rng(91)
    T = rng.uniform(0.0, 2.0, grid.n_pixels)
    w = rng.uniform(0.5, 1.5, grid.n_pixels)
    target = torch.as_tensor(T, device=DEV)
    weight = torch.as_tensor(w, device=DEV)
    loss, dn, dm = numag.grad(_empty_sample(), grid, numag.consts(V=2.0, bH=0.7), weight, target, path=path)
    torch.cuda.synchronize()
    assert dn.shape == (0,) and dm.shape == (0, 3)
    ref = float(np.sum(w * T * T))
    assert abs(loss.item() - ref) <= 1e-13 * ref
    # backward form (upstream gradient in `weight`, no target): nothing to return
    loss2, dn2, dm2 = numag.grad(_empty_sample(), grid, numag.consts(), weight, None, path=path)
    torch.cuda.synchronize()
    assert loss2 is None and dn2.numel() == 0 and dm2.numel() == 0


def test_zero_field_epilogues():
    grid = numag.qgrid(numag.GRID_CARTESIAN, 32, 32, 1.0)
    f = torch.zeros((2, grid.n_pixels), dtype=torch.float64, device=DEV)
    I, cnt = numag.azimuthal_average(grid, f, 8)
    torch.cuda.synchronize()
    filled = cnt.cpu().numpy() > 0
    assert filled.any()
    assert torch.count_nonzero(I[:, torch.as_tensor(filled, device=DEV)]).item() == 0
    C = numag.correlation_2d(grid, f, numag.qgrid(numag.GRID_POLAR, 6, 8, 5.0))
    torch.cuda.synchronize()
    assert torch.count_nonzero(C).item() == 0
    # no data sets: valid, nothing written
    I0, _ = numag.azimuthal_average(grid, f[:0], 8)
    C0 = numag.correlation_2d(grid, f[:0], numag.qgrid(numag.GRID_POLAR, 6, 8, 5.0))
    torch.cuda.synchronize()
    assert I0.shape == (0, 8) and C0.shape[0] == 0


def test_empty_snapshot_batch_is_refused():
    points = numag.regular_grid((4, 4, 4), (-1.5, -1.5, -1.5), (1.0, 1.0, 1.0))
    grid = numag.qgrid(numag.GRID_CARTESIAN, 8, 8, 1.0)
    with pytest.raises(numag.NumagError):
        numag.amplitudes_snapshots(points, grid, nuc=np.zeros((0, 64)), mag=np.zeros((0, 64, 3)), device=DEV)


def test_no_amplitude_sets():
    grid = numag.qgrid(numag.GRID_CARTESIAN, 8, 10, 1.0)
    amp = torch.empty((0, grid.n_pixels, 4, 2), dtype=torch.float64, device=DEV)
    xs = numag.cross_section(grid, amp=amp, obs=numag.OBSERVABLES)
    spec = numag.spectral_matrix(grid, amp)
    xs2 = numag.cross_section(grid, spec=spec, obs=("UNPOL", "SF"))
    torch.cuda.synchronize()
    assert xs.shape == (0, len(numag.OBSERVABLES), grid.n_pixels)
    assert spec.shape == (0, grid.n_pixels, 16) and xs2.shape == (0, 2, grid.n_pixels)
