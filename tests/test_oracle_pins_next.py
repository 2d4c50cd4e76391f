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


def test_correlation_2d_abel_relation_to_1d_correlation(orc):
    """Sec. 2.6: for an isotropic cross section the azimuthally constant C(rho) and
    c(r) of eq. crrad are related by an Abel transform.  The detector plane is the
    q_x = 0 slice of the 3D transform, so its 2D inverse transform is the projection
    of c along the beam: C(rho) = 4 pi^2 int c(sqrt(rho^2 + x^2)) dx over the whole
    x axis.  Both sides come from the oracle (eq. crav2d on a polar detector, eq.
    crrad on its q axis) for I(q) = (1 + q^2 a^2) exp(-q^2 b^2), which is not a
    Hankel pair of either closed form; the x integral uses Gauss-Legendre nodes.
    The two trapezoidal rules in q differ by their Euler-Maclaurin end terms at
    q = 0: the 2D integrand q f J0 has slope f(0) there, the 1D one q^2 I j0 slope
    zero, so the 2D sum lies 2 pi h^2 / 12 f(0) below the integral (q step h); that
    term bounds the comparison.  The paper's remark that c is not the azimuthal average of C is
    checked too: C(rho) / C(0) and c(rho) / c(0) differ by far more."""
    a, b = 3.0, 1.5
    nq, nt, qmax = 400, 64, 6.0
    qy, qz, _ = orc.pixels(orc.POLAR, nq, nt, qmax)
    q2 = qy ** 2 + qz ** 2
    f = (1.0 + q2 * a * a) * np.exp(-q2 * b * b)
    nr, na, rmax = 11, 5, 10.0
    C = orc.correlation_2d(orc.POLAR, nq, nt, qmax, f, orc.POLAR, nr, na, rmax)[0].reshape(nr, na)
    # isotropic data: the same value at every alpha, and real
    assert np.max(np.abs(C - C[:, :1])) < 1e-12 * np.abs(C).max()
    assert np.max(np.abs(C.imag)) < 1e-12 * np.abs(C).max()
    rho = np.arange(nr) * rmax / (nr - 1)
    q = np.arange(1, nq) * qmax / (nq - 1)  # the detector's q rows (q = 0 adds nothing)
    Iq = (1.0 + q * q * a * a) * np.exp(-q * q * b * b)
    x, wx = np.polynomial.legendre.leggauss(160)
    X = 24.0  # c(r) < 1e-25 c(0) beyond
    x, wx = (x + 1.0) * X / 2.0, wx * X / 2.0
    r = np.sqrt(rho[:, None] ** 2 + x[None, :] ** 2)
    c, _ = orc.correlation(q, Iq[None, :], r.reshape(-1))
    abel = 8.0 * math.pi ** 2 * (c[0].reshape(r.shape) @ wx)
    h = qmax / (nq - 1)
    assert np.max(np.abs(C[:, 0].real - abel)) < 2.0 * (2.0 * math.pi * h * h / 12.0) * f.max()
    c_rho, _ = orc.correlation(q, Iq[None, :], rho)
    assert np.max(np.abs(C[:, 0].real / C[0, 0].real - c_rho[0] / c_rho[0, 0])) > 0.05


def test_correlation_2d_of_uniform_sphere(orc):
    """For a uniform sphere of radius R, f = |F|^2 with F = V 3 j1(qR) / (qR) is the
    transform of the autocorrelation V gamma0(r), gamma0 = 1 - 3r/(4R) + r^3/(16R^3)
    for r <= 2R (the same closed form as the 1D sphere pin), so eq. crav2d gives
    C(rho) = 8 pi^2 V int_0^sqrt(4R^2 - rho^2) gamma0(sqrt(rho^2 + x^2)) dx.  The
    oracle's trapezoid in q lies 2 pi h^2 / 12 f(0) below the integral (the
    Euler-Maclaurin end term at q = 0, q step h) and misses the tail beyond q_max,
    at most 2 pi int |F|^2 q dq ~ 4.5 pi V^2 / (R^4 q_max^2) (at rho = 0); the
    theta trapezoid is exact once n_theta exceeds q_max rho."""
    R = 5.0
    V = 4.0 / 3.0 * math.pi * R ** 3
    nq, nt, qmax = 2001, 256, 20.0
    qy, qz, _ = orc.pixels(orc.POLAR, nq, nt, qmax)
    x = np.sqrt(qy ** 2 + qz ** 2) * R
    xs = np.where(x > 1e-3, x, 1.0)
    F = V * np.where(x > 1e-3, 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3, 1.0 - x * x / 10.0)
    f = F * F
    nr, na, rmax = 6, 4, 2.0 * R * 5.0 / 6.0
    C = orc.correlation_2d(orc.POLAR, nq, nt, qmax, f, orc.POLAR, nr, na, rmax)[0].reshape(nr, na)
    rho = np.arange(nr) * rmax / (nr - 1)
    g, w = np.polynomial.legendre.leggauss(64)
    expect = np.empty(nr)
    for i, p in enumerate(rho):
        L = math.sqrt(4.0 * R * R - p * p)
        r = np.sqrt(p * p + ((g + 1.0) * L / 2.0) ** 2)
        expect[i] = 8.0 * math.pi ** 2 * V * np.sum((1.0 - 0.75 * r / R + r ** 3 / (16.0 * R ** 3)) * w * L / 2.0)
    h = qmax / (nq - 1)
    end = 2.0 * math.pi * h * h / 12.0 * V * V
    tail = 4.5 * math.pi * V * V / (R ** 4 * qmax ** 2)
    for j in range(na):
        assert np.max(np.abs(C[:, j].real - (expect - end))) < 1.25 * tail
    assert np.max(np.abs(C.imag)) < 1e-9 * expect[0]
    assert tail < 2e-4 * expect[0]
