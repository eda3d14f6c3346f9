"""Velocity autocorrelation functions of a neutrally buoyant no-slip sphere
(Sec. III.A): the reference curves the single-particle runs are compared to.

C_T is the inverse Fourier transform of Eq. (VACF_fourier) with the
frequency-dependent translational friction of Eq. (translational_friction);
C_R is the inverse Laplace transform of Eq. (AVACF_laplace) with its
rotational friction.  Reading of a garbled symbol: the compressibility
parameter is zeta = w R / sqrt(c0^2 - i w (4 eta/3 + eta_b)/rho) with the real
frequency w, so that 1 - i zeta = 1 + s R / c0 for s = -i w.  Taking s = -i w
in place of w makes the transform non-causal (a nonzero C_T at t < 0) and
breaks the Green-Kubo sum rule; this reading satisfies both (see the pins).
The transform is one-sided: at t = 0 the quadrature returns C_T(0+)/2.
Solvent constants as the paper quotes them: c0 = 1, nu0 = 0.792,
eta_b = 1.22, rho0 = 5, eta0 = rho0 nu0.
"""
import math

import numpy as np

RHO0, NU0, C0, ETA_B = 5.0, 0.792, 1.0, 1.22
ETA0 = RHO0 * NU0


def gamma_t(w, R, eta=ETA0, nu=NU0, rho=RHO0, c0=C0, eta_b=ETA_B):
    """Translational friction at angular frequency w (complex; w != 0)."""
    w = np.asarray(w, dtype=np.complex128)
    x = R * np.sqrt(-1j * w / nu)
    zeta = w * R / np.sqrt(c0 * c0 - 1j * w * (4.0 * eta / 3.0 + eta_b) / rho)
    num = (1.0 + x) * (9.0 - 9.0j * zeta - 2.0 * zeta ** 2) + x ** 2 * (1.0 - 1j * zeta)
    den = 2.0 * x ** 2 * (1.0 - 1j * zeta) - (1.0 + x) * zeta ** 2 - x ** 2 * zeta ** 2
    return (4.0 * math.pi / 3.0) * eta * R * x ** 2 * num / den


def ct_theory(t, R, kT=1.0, dw=1e-3, wmax=1e3, M=None, **fluid):
    """C_T(t) = (3 kT / 2 pi) int e^{-i w t} / (gamma_T - i w M_S) dw by the
    trapezoid rule on [-wmax, wmax] with step dw (the paper's quadrature);
    gamma_T(0) = 6 pi eta R (its limit) at w = 0.  M: a particle mass in place
    of the neutrally buoyant M_S (the same friction, another inertia)."""
    rho = fluid.get("rho", RHO0)
    eta = fluid.get("eta", ETA0)
    MS = 4.0 * math.pi * R ** 3 * rho / 3.0 if M is None else float(M)
    n = int(round(wmax / dw))
    w = dw * np.arange(1, n + 1)
    f = 1.0 / (gamma_t(w, R, **fluid) - 1j * w * MS)
    f0 = 1.0 / (6.0 * math.pi * eta * R)
    out = []
    for tt in np.atleast_1d(t):
        # the integrand at -w is the conjugate of that at w: twice the real part
        # of the half-line sum (end point weighted 1/2), plus the w = 0 point
        s = np.sum(np.exp(-1j * w * tt) * f) - 0.5 * np.exp(-1j * w[-1] * tt) * f[-1]
        out.append(3.0 * kT / (2.0 * math.pi) * dw * (f0 + 2.0 * s.real))
    return np.array(out)


def cr_theory(t, R, kT=1.0, eta=ETA0, nu=NU0, rho=RHO0, I=None):
    """C_R(t): inverse Laplace transform of (3 kT / I_S) / (s + gamma_R(s) / I_S)
    with gamma_R = 8 pi eta R^3 [1 + (R^2 s/nu) / (3 (1 + sqrt(R^2 s / nu)))],
    I_S = 2 M_S R^2 / 5 (mpmath's numerical inversion, as in the paper).  I: a
    moment of inertia in place of I_S."""
    import mpmath as mp
    MS = 4.0 * math.pi * R ** 3 * rho / 3.0
    IS = 2.0 * MS * R * R / 5.0 if I is None else float(I)

    def F(s):
        a = R * R * s / nu
        g = 8.0 * mp.pi * eta * R ** 3 * (1 + a / (3 * (1 + mp.sqrt(a))))
        return (3.0 * kT / IS) / (s + g / IS)

    return np.array([float(mp.invertlaplace(F, float(tt), method="talbot")) for tt in np.atleast_1d(t)])
