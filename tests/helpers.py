"""Shared test helpers: the error metric and oracle/HIP glue (no method arithmetic)."""
import numpy as np

GATE = 1e-6  # pixels with |X_ref| >= GATE * max|X_ref| are gated


def gated_rel_err(x, ref, exclude=None):
    """max over gated pixels of |x - ref| / |ref|; gate = |ref| >= 1e-6 max|ref|
    (complex amplitudes use the modulus); `exclude` masks pixels (q = 0)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    mag = np.abs(ref)
    ok = np.ones(ref.shape, dtype=bool)
    if exclude is not None:
        ok &= ~exclude
    if not np.any(mag[ok] > 0):
        return float(np.max(np.abs(x - ref))) if x.size else 0.0
    gate = ok & (mag >= GATE * mag[ok].max())
    return float(np.max(np.abs(x - ref)[gate] / mag[gate]))


def max_norm_err(x, ref):
    ref = np.asarray(ref)
    scale = np.max(np.abs(ref)) if ref.size else 1.0
    if scale == 0:
        scale = 1.0
    return float(np.max(np.abs(np.asarray(x) - ref)) / scale) if ref.size else 0.0


def amp_to_complex(amp_t):
    """[..., P, 4, 2] float64 tensor -> complex numpy [..., P, 4]."""
    a = amp_t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def zero_q_mask(qy, qz):
    return (np.asarray(qy) == 0) & (np.asarray(qz) == 0)
