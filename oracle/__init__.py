"""FP64 CPU oracle for the NuMagSANS direct-Fourier-sum path (arXiv 2601.18444).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2601_18444_amd`` and never imports it.

The arithmetic lives in ``numag_oracle.c`` (plain C, FP64, libm sin/cos, OpenMP
over output elements only).  This module marshals numpy arrays into it and
holds the detector definition (Sec. 2.1 eq. qdef; Sec. 3.1 q_max and the
resolutions; Sec. 3.2 the polar coordinates q_y = q sin(theta),
q_z = q cos(theta)):

* Cartesian detector: q_i = -q_max + i * (2 q_max / (n - 1)), i < n, computed
  in FP64 exactly as written (one product, one sum); pixel p = i_y * n_z + i_z.
* Polar detector: q_i = i * (q_max / (n_q - 1)), theta_m = 2 pi m / n_theta;
  pixel p = i_q * n_theta + m.
* qhat = (0, q_y, q_z) / |q|; on a Cartesian detector the q = 0 pixel (only
  present for odd n) takes qhat = e_z; on a polar detector qhat is
  (0, sin theta_m, cos theta_m) for every pixel of column m, q = 0 included.

Parity status: pinned by tests/test_oracle_pins.py (closed forms, brute force,
identities and the worked examples of Sec. 4.1 and 4.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "numag_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OBSERVABLES = ("N", "M", "NM", "P", "CHI", "SF", "PP", "MM", "PM", "MP", "PLUS", "MINUS", "UNPOL")

CARTESIAN = 0
POLAR = 1


def build(force: bool = True) -> str:
    """Compile numag_oracle.c into liboracle.so with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        lib.orc_amplitudes.argtypes = [i64, P, P, P, i64, P, P, P, i64, P, P, ctypes.c_int, P]
        lib.orc_spectral.argtypes = [i64, i64, P, P]
        lib.orc_cross_sections.argtypes = [i64, i64, P, P, d, d, d, P, P, P]
        lib.orc_azimuthal_average.argtypes = [ctypes.c_int, i64, i64, P, P, i64, P, i64, d, P, P]
        lib.orc_correlation.argtypes = [i64, P, i64, P, i64, P, d, P, P]
        lib.orc_loss_grad.argtypes = [i64, P, P, P, i64, P, P, P, i64, P, P, P, d, d, d, P, P, P, P, P]
        lib.orc_angular_spectrum.argtypes = [i64, i64, P, i64, P, P]
        lib.orc_correlation_2d.argtypes = [i64, P, P, P, i64, P, i64, P, P, P]
        lib.orc_correlation_2d.restype = None
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        for f in (lib.orc_amplitudes, lib.orc_spectral, lib.orc_cross_sections,
                  lib.orc_azimuthal_average, lib.orc_correlation, lib.orc_loss_grad,
                  lib.orc_angular_spectrum):
            f.restype = None
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(_load().orc_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# --------------------------------------------------------------------------
# Detector (Sec. 2.1, Sec. 3.1, Sec. 3.2)
# --------------------------------------------------------------------------
def axis(n: int, qmax: float) -> np.ndarray:
    """Cartesian detector axis q_i = -q_max + i * (2 q_max / (n - 1))."""
    if n == 1:
        return np.zeros(1)
    step = (2.0 * qmax) / (n - 1)
    i = np.arange(n, dtype=np.float64)
    return -qmax + i * step


def pixels(kind: int, n0: int, n1: int, qmax: float):
    """Pixel list (qy, qz, qhat[P,3]) of a detector, in pixel order."""
    if kind == CARTESIAN:
        ay, az = axis(n0, qmax), axis(n1, qmax)
        qy = np.repeat(ay, n1)
        qz = np.tile(az, n0)
        qn = np.sqrt(qy * qy + qz * qz)
        qhat = np.zeros((qy.size, 3))
        nz = qn > 0
        qhat[nz, 1] = qy[nz] / qn[nz]
        qhat[nz, 2] = qz[nz] / qn[nz]
        qhat[~nz, 2] = 1.0
        return qy, qz, qhat
    if kind == POLAR:
        q = np.zeros(n0) if n0 == 1 else np.arange(n0, dtype=np.float64) * (qmax / (n0 - 1))
        th = 2.0 * np.pi * np.arange(n1, dtype=np.float64) / n1
        qq = np.repeat(q, n1)
        tt = np.tile(th, n0)
        qy = qq * np.sin(tt)
        qz = qq * np.cos(tt)
        qhat = np.stack([np.zeros_like(tt), np.sin(tt), np.cos(tt)], axis=1)
        return qy, qz, qhat
    raise ValueError("unknown detector kind")


def qhat_of(qy, qz):
    """qhat for an explicit Cartesian pixel list (q = 0 -> e_z)."""
    qy = np.asarray(qy, dtype=np.float64)
    qz = np.asarray(qz, dtype=np.float64)
    qn = np.sqrt(qy * qy + qz * qz)
    qhat = np.zeros((qy.size, 3))
    nz = qn > 0
    qhat[nz, 1] = qy[nz] / qn[nz]
    qhat[nz, 2] = qz[nz] / qn[nz]
    qhat[~nz, 2] = 1.0
    return qhat


# --------------------------------------------------------------------------
# Sums, spectra, observables
# --------------------------------------------------------------------------
def amplitudes(pos, nuc, mag, qy, qz, R=None, obj_offsets=None, obj_pos=None,
               per_object=False) -> np.ndarray:
    """Raw discrete Fourier sums (Sec. 3.3).  Returns complex [P,4] or [K,P,4]."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    W = pos.shape[0]
    nuc = _f64(nuc)
    mag = _f64(mag, (-1, 3)) if mag is not None else None
    R = np.eye(3) if R is None else _f64(R, (3, 3))
    qy = _f64(qy)
    qz = _f64(qz)
    if obj_offsets is None:
        K, off = 1, None
    else:
        off = np.ascontiguousarray(obj_offsets, dtype=np.int64)
        K = off.size - 1
    op = _f64(obj_pos, (-1, 3)) if obj_pos is not None else None
    n_sets = K if per_object else 1
    out = np.zeros((n_sets, qy.size, 4), dtype=np.complex128)
    lib.orc_amplitudes(W, _ptr(pos), _ptr(nuc), _ptr(mag), K, _ptr(off), _ptr(op), _ptr(R),
                       qy.size, _ptr(qy), _ptr(qz), int(bool(per_object)), _ptr(out))
    return out if per_object else out[0]


def spectral(amp) -> np.ndarray:
    """G = sum over sets of A A^H, packed as 16 reals per pixel."""
    lib = _load()
    a = np.ascontiguousarray(amp, dtype=np.complex128)
    if a.ndim == 2:
        a = a[None]
    G = np.zeros((a.shape[1], 16))
    lib.orc_spectral(a.shape[0], a.shape[1], _ptr(a), _ptr(G))
    return G


def cross_sections(amp, qhat, V=1.0, bH=1.0, scale=1.0, P=(0.0, 0.0, 1.0), return_imag=False):
    """All 13 observables of Sec. 2, summed over amplitude sets.  Returns dict name -> [P]."""
    lib = _load()
    a = np.ascontiguousarray(amp, dtype=np.complex128)
    if a.ndim == 2:
        a = a[None]
    qhat = _f64(qhat, (-1, 3))
    Ph = _f64(P, (3,))
    out = np.zeros((len(OBSERVABLES), a.shape[1]))
    imag = np.zeros(1)
    lib.orc_cross_sections(a.shape[0], a.shape[1], _ptr(a), _ptr(qhat), float(V), float(bH),
                           float(scale), _ptr(Ph), _ptr(out), _ptr(imag))
    res = {name: out[i] for i, name in enumerate(OBSERVABLES)}
    if return_imag:
        return res, float(imag[0])
    return res


def azimuthal_average(kind, n0, n1, qmax, f, n_bins, qmax_avg=None):
    """Azimuthal average (eq. iqazi).  f is [n_f, P]; returns (I[n_f, n_bins], count[n_bins])."""
    lib = _load()
    f = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
    qy, qz, _ = pixels(kind, n0, n1, qmax)
    if qmax_avg is None:
        qmax_avg = qmax
    I = np.zeros((f.shape[0], n_bins))
    cnt = np.zeros(n_bins, dtype=np.int64)
    lib.orc_azimuthal_average(int(kind), n0, n1, _ptr(qy), _ptr(qz), f.shape[0], _ptr(f), n_bins,
                              float(qmax_avg), _ptr(I), _ptr(cnt))
    return I, cnt


def bin_centres(n_bins, qmax_avg):
    """Annulus centres (b + 1/2) dq of the Cartesian azimuthal average."""
    dq = qmax_avg / n_bins
    return (np.arange(n_bins) + 0.5) * dq


def correlation(q, I, r, scale=1.0):
    """c(r), p(r) of eqs. crrad/prrad by the trapezoidal rule.  I is [n_f, n_q]."""
    lib = _load()
    q = _f64(q)
    I = np.ascontiguousarray(np.atleast_2d(I), dtype=np.float64)
    r = _f64(r)
    c = np.zeros((I.shape[0], r.size))
    p = np.zeros_like(c)
    lib.orc_correlation(q.size, _ptr(q), I.shape[0], _ptr(I), r.size, _ptr(r), float(scale),
                        _ptr(c), _ptr(p))
    return c, p


def loss_grad(pos, nuc, mag, qy, qz, qhat, target, weight, V=1.0, bH=1.0, scale=1.0, R=None,
              obj_offsets=None, obj_pos=None):
    """Loss sum_p w_p (I_p - T_p)^2 on the unpolarized cross section and its gradient."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    W = pos.shape[0]
    nuc = _f64(nuc)
    mag = _f64(mag, (-1, 3)) if mag is not None else None
    R = np.eye(3) if R is None else _f64(R, (3, 3))
    qy, qz = _f64(qy), _f64(qz)
    qhat = _f64(qhat, (-1, 3))
    T, w = _f64(target), _f64(weight)
    if obj_offsets is None:
        K, off = 1, None
    else:
        off = np.ascontiguousarray(obj_offsets, dtype=np.int64)
        K = off.size - 1
    op = _f64(obj_pos, (-1, 3)) if obj_pos is not None else None
    loss = np.zeros(1)
    dn = np.zeros(W)
    dm = np.zeros((W, 3))
    lib.orc_loss_grad(W, _ptr(pos), _ptr(nuc), _ptr(mag), K, _ptr(off), _ptr(op), _ptr(R),
                      qy.size, _ptr(qy), _ptr(qz), _ptr(qhat), float(V), float(bH), float(scale),
                      _ptr(T), _ptr(w), _ptr(loss), _ptr(dn), _ptr(dm))
    return float(loss[0]), dn, dm


def quadrature_weights(kind, n0, n1, qmax):
    """Trapezoidal weights of int d^2q over a detector (Sec. 2.5 trapezoidal rule).
    Polar: q dq dtheta with weight h_i q_i dtheta, h_i = dq (1/2 at q = 0 and q_max),
    periodic in theta.  Cartesian: dq_y dq_z with 1/2 on edge rows and columns."""
    if kind == POLAR:
        dq = qmax / (n0 - 1) if n0 > 1 else 0.0
        q = np.arange(n0, dtype=np.float64) * dq
        h = np.full(n0, dq)
        h[0] *= 0.5
        h[-1] *= 0.5
        dth = 2.0 * np.pi / n1
        return np.repeat(h * q * dth, n1)
    cy = np.ones(n0)
    cz = np.ones(n1)
    cy[[0, -1]] = 0.5
    cz[[0, -1]] = 0.5
    dqy = 2.0 * qmax / (n0 - 1) if n0 > 1 else 1.0
    dqz = 2.0 * qmax / (n1 - 1) if n1 > 1 else 1.0
    return (np.outer(cy, cz) * dqy * dqz).reshape(-1)


def real_space_points(kind, n0, n1, rmax):
    """Output points of the 2D correlation: Cartesian r on [-rmax, rmax]^2 like the
    detector axes, or polar rho_a = a rmax/(n0 - 1), alpha_b = 2 pi b / n1 with
    r = rho (sin alpha, cos alpha)."""
    qy, qz, _ = pixels(kind, n0, n1, rmax)
    return qy, qz


def correlation_2d(kind, n0, n1, qmax, f, rkind, r0, r1, rmax):
    """eq. crav2d: C on the real-space grid (rkind, r0, r1, rmax) from data sets f
    [n_f, P] on the detector (kind, n0, n1, qmax).  Returns complex [n_f, R]."""
    lib = _load()
    f = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
    qy, qz, _ = pixels(kind, n0, n1, qmax)
    wq = np.ascontiguousarray(quadrature_weights(kind, n0, n1, qmax))
    ry, rz = real_space_points(rkind, r0, r1, rmax)
    ry, rz = np.ascontiguousarray(ry), np.ascontiguousarray(rz)
    out = np.zeros((f.shape[0], ry.size), dtype=np.complex128)
    lib.orc_correlation_2d(qy.size, _ptr(qy), _ptr(qz), _ptr(wq), f.shape[0], _ptr(f), ry.size, _ptr(ry),
                           _ptr(rz), _ptr(out))
    return out


def modal_amplitudes(Is, Ic):
    """eq. ModalAmplitudes: a_k = sum_i I_k(q_i), A_k = a_k / sum_j sqrt(a_j^s^2 + a_j^c^2)."""
    a_s = np.sum(Is, axis=0)
    a_c = np.sum(Ic, axis=0)
    norm = np.sum(np.sqrt(a_s ** 2 + a_c ** 2))
    return a_s / norm, a_c / norm


def angular_spectrum(f_polar, n_q, n_theta, k_max):
    """Modal intensities (eq. CosineSinceIntensities) on a polar detector: (Is, Ic) [n_q, k_max+1]."""
    lib = _load()
    f = _f64(f_polar, (n_q * n_theta,))
    Is = np.zeros((n_q, k_max + 1))
    Ic = np.zeros_like(Is)
    lib.orc_angular_spectrum(n_q, n_theta, _ptr(f), k_max, _ptr(Is), _ptr(Ic))
    return Is, Ic
