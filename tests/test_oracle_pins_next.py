"""Pins of the oracle's 2D correlation function (eq. crav2d) and modal
amplitudes (eq. ModalAmplitudes) against closed forms."""
import math

import numpy as np


def test_correlation_2d_isotropic_gaussian_polar(orc):
    """On the paper's polar detector, an isotropic Gaussian f = exp(-q^2 a^2) has
    C(rho, alpha) = 2 pi int exp(-q^2 a^2) J0(q rho) q dq = (pi / a^2) exp(-rho^2 / (4 a^2))
    for every alpha (a Hankel-transform pair); the trapezoidal rule in q (step
    3/399) is accurate to ~1e-5 of the peak."""
    a = 2.0
    nq, nt, qmax = 400, 96, 3.0
    qy, qz, _ = orc.pixels(orc.POLAR, nq, nt, qmax)
    f = np.exp(-(qy ** 2 + qz ** 2) * a * a)
    C = orc.correlation_2d(orc.POLAR, nq, nt, qmax, f, orc.POLAR, 12, 7, 10.0)[0]
    ry, rz = orc.real_space_points(orc.POLAR, 12, 7, 10.0)
    rho2 = ry ** 2 + rz ** 2
    expect = math.pi / a ** 2 * np.exp(-rho2 / (4 * a * a))
    assert np.max(np.abs(C - expect)) < 1e-4 * expect.max()


def test_correlation_2d_anisotropic_gaussian_cartesian(orc):
    """On a Cartesian detector, f = exp(-(q_y^2 a^2 + q_z^2 b^2)) has
    C(r) = (pi / (a b)) exp(-r_y^2 / (4 a^2) - r_z^2 / (4 b^2)): the y and z axes are
    not interchangeable, so a swapped axis or a flipped phase sign fails."""
    a, b = 1.5, 2.5
    n, qmax = 161, 4.0
    qy, qz, _ = orc.pixels(orc.CARTESIAN, n, n, qmax)
    f = np.exp(-(qy ** 2 * a * a + qz ** 2 * b * b))
    C = orc.correlation_2d(orc.CARTESIAN, n, n, qmax, f, orc.CARTESIAN, 9, 11, 8.0)[0]
    ry, rz = orc.real_space_points(orc.CARTESIAN, 9, 11, 8.0)
    expect = math.pi / (a * b) * np.exp(-ry ** 2 / (4 * a * a) - rz ** 2 / (4 * b * b))
    assert np.max(np.abs(C - expect)) < 1e-6 * expect.max()
    # an odd pattern gives an imaginary correlation with the sign of exp(+i q.r)
    g = qy * f
    Cg = orc.correlation_2d(orc.CARTESIAN, n, n, qmax, g, orc.CARTESIAN, 9, 11, 8.0)[0]
    # int q_y exp(-q_y^2 a^2) exp(i q_y r_y) dq_y = i r_y sqrt(pi) / (2 a^3) exp(-r_y^2 / 4a^2)
    expect_g = 1j * ry / (2 * a * a) * expect
    assert np.max(np.abs(Cg - expect_g)) < 1e-6 * np.abs(expect_g).max()


def test_modal_amplitudes_normalisation(orc):
    """eq. ModalAmplitudes: sin^2 gives A0c = 1/2, A2c = -1/2 (ratio -1) and the
    normalisation makes sum_k sqrt(As^2 + Ac^2) = 1."""
    nq, nt = 5, 24
    th = 2 * np.pi * np.arange(nt) / nt
    f = np.tile(np.sin(th) ** 2, nq)
    Is, Ic = orc.angular_spectrum(f, nq, nt, 6)
    As, Ac = orc.modal_amplitudes(Is, Ic)
    assert abs(Ac[0] - 0.5) < 1e-12 and abs(Ac[2] + 0.5) < 1e-12
    assert abs(np.sum(np.sqrt(As ** 2 + Ac ** 2)) - 1.0) < 1e-12


def test_modal_amplitudes_sin2cos2(orc):
    """sin^2 cos^2 = (1 - cos 4 theta)/8: I0 = 1/8, I4c = -1/8, every other mode 0, so
    A0c/A4c = -1 (the ratio the paper quotes for this pattern)."""
    nq, nt = 4, 32
    th = 2 * np.pi * np.arange(nt) / nt
    f = np.tile(np.sin(th) ** 2 * np.cos(th) ** 2, nq)
    Is, Ic = orc.angular_spectrum(f, nq, nt, 8)
    assert np.allclose(Ic[:, 0], 0.125, atol=1e-13) and np.allclose(Ic[:, 4], -0.125, atol=1e-13)
    others = [k for k in range(9) if k not in (0, 4)]
    assert np.max(np.abs(Ic[:, others])) < 1e-13 and np.max(np.abs(Is)) < 1e-13
    As, Ac = orc.modal_amplitudes(Is, Ic)
    assert abs(Ac[0] / Ac[4] + 1.0) < 1e-12
