"""Calls enqueued on different streams may overlap; the binding gives each stream its
own workspace.  Sums and gradients computed on two streams at once equal the same
calls made one after the other on one stream, bit for bit."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_18444_amd import numag, synth  # noqa: E402

DEV = "cuda:0"


def _samples():
    out = []
    for seed in (80, 81):
        cl = synth.random_cloud(30000, 20.0, seed=seed)
        out.append(numag.Sample(pos=cl["pos"], nuc=cl["nuc"], mag=cl["mag"], device=DEV))
    return out


def test_direct_sums_and_gradients_on_two_streams():
    grid = numag.qgrid(0, 96, 112, 1.1)
    c = numag.consts(V=2.0, bH=0.7)
    weight = torch.ones(grid.n_pixels, dtype=torch.float64, device=DEV)
    target = torch.full((grid.n_pixels,), 0.5, dtype=torch.float64, device=DEV)
    samples = _samples()
    # reference: one stream, one call after the other
    ref_amp = [numag.amplitudes(s, grid)[0].clone() for s in samples]
    ref_grad = [[t.clone() for t in numag.grad(s, grid, c, weight, target)] for s in samples]
    torch.cuda.synchronize()
    numag.clear_workspace_cache()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    amps, grads = [None, None], [None, None]
    for rep in range(2):  # the second round reuses each stream's cached workspace
        for i, (st, s) in enumerate(zip(streams, samples)):
            with torch.cuda.stream(st):
                amps[i] = numag.amplitudes(s, grid)[0]
                grads[i] = numag.grad(s, grid, c, weight, target)
        for st in streams:
            torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(amps[i], ref_amp[i]), f"sums of sample {i}, round {rep}"
            for a, b in zip(grads[i], ref_grad[i]):
                assert torch.equal(a, b), f"gradient of sample {i}, round {rep}"
