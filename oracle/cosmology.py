"""Background cosmology for the oracle (flat LambdaCDM, radiation neglected).

Units: time in 1/H0, scale factor a (a=1 today), wavenumbers in h/Mpc where a power
spectrum is involved.

Sec. 2.1 sets the initial conditions from an analytic matter transfer function; the paper
uses Eisenstein & Hu, the workloads here use the BBKS form with P(k) = A k^{n_s} T(q)^2,
q = k / (Omega_m h), normalised to sigma_8 with a top-hat of radius 8 Mpc/h.  The linear
growth factor is the Heath (1977) integral, valid for dust + Lambda.
"""

import math

from scipy import integrate


def hubble_e(a, om):
    """E(a) = H(a)/H0 = sqrt(Om a^-3 + OL) for a flat universe."""
    return math.sqrt(om / a ** 3 + (1.0 - om))


def time_of_a(a, om):
    """Cosmic time t(a) in 1/H0: the closed form of da/dt = a E(a) for flat dust + Lambda."""
    ol = 1.0 - om
    return 2.0 / (3.0 * math.sqrt(ol)) * math.asinh(math.sqrt(ol / om) * a ** 1.5)


def a_of_time(t, om):
    """Inverse of time_of_a: a(t) = (Om/OL)^(1/3) sinh^(2/3)(1.5 sqrt(OL) t)."""
    ol = 1.0 - om
    return (om / ol) ** (1.0 / 3.0) * math.sinh(1.5 * math.sqrt(ol) * t) ** (2.0 / 3.0)


def _heath_integral(a, om):
    f = lambda x: 1.0 / (x * hubble_e(x, om)) ** 3 if x > 0 else 0.0
    val, _ = integrate.quad(f, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def growth_unnormalised(a, om):
    """D_u(a) = (5 Om / 2) E(a) int_0^a da' / (a' E(a'))^3; D_u -> a as a -> 0."""
    return 2.5 * om * hubble_e(a, om) * _heath_integral(a, om)


def growth(a, om):
    """Linear growth factor normalised to D(1) = 1."""
    return growth_unnormalised(a, om) / growth_unnormalised(1.0, om)


def growth_rate(a, om):
    """f = dlnD/dlna = -3 Om/(2 a^3 E^2) + 5 Om / (2 a^2 E^2 D_u)  (derivative of D_u above)."""
    e2 = hubble_e(a, om) ** 2
    return -1.5 * om / (a ** 3 * e2) + 2.5 * om / (a * a * e2 * growth_unnormalised(a, om))


def growth_momentum(a, om):
    """G(a) = a^2 dD/dt for t in 1/H0: with dD/dt = (dD/da) a E(a) and f = dlnD/dlna this is
    a^2 E(a) f(a) D(a).  For the linear growing mode x = q + D Psi_0 the momentum p = a^2 dx/dt
    of the particle step (eq. dm_hamil) is G Psi_0."""
    return a * a * hubble_e(a, om) * growth_rate(a, om) * growth(a, om)


def growth_force(a, om):
    """F(a) = dG/dt = (3 Om / 2a) D(a): the growth equation of linear theory,
    d(a^2 dD/dt)/dt = (3/2) Om D / a (t in 1/H0).  For the growing mode the particle force
    g = -grad phi with lap phi = (3 Om / 2a) delta (Sec. 2.2) is F Psi_0."""
    return 1.5 * om * growth(a, om) / a


def fastpm_factors(a0, a_half, a1, om):
    """Kick and drift factors of one kick-drift-kick step from a0 to a1 through a_half that
    are exact for the linear growing mode (the modified KDK of FastPM, which the paper uses
    for its particle mesh, Sec. 2.2).  With p = G Psi_0, g = F Psi_0 and x - q = D Psi_0 along
    that mode, the opening half kick with g(a0), the drift with p(a_half) and the closing half
    kick with g(a1) reproduce the mode exactly when
        opening kick  K0 = (G(a_half) - G(a0)) / F(a0),
        drift         Dr = (D(a1) - D(a0)) / G(a_half),
        closing kick  K1 = (G(a1) - G(a_half)) / F(a1);
    the plain leapfrog in t uses dt/2, dt / a_half^2 and dt/2 (their limit for small dt).
    Returns (K0, Dr, K1)."""
    g0, gh, g1 = (growth_momentum(a, om) for a in (a0, a_half, a1))
    k0 = (gh - g0) / growth_force(a0, om)
    dr = (growth(a1, om) - growth(a0, om)) / gh
    k1 = (g1 - gh) / growth_force(a1, om)
    return k0, dr, k1


def bbks_transfer(q, log=math.log):
    """BBKS (Bardeen et al. 1986) transfer function of q = k / (Om h) with k in h/Mpc.
    Works on floats, or on tensors with log=torch.log (q > 0)."""
    return (log(1.0 + 2.34 * q) / (2.34 * q)
            * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)


def eh_nowiggle_transfer(k, om, ob, h, tcmb=2.7255, log=math.log, sqrt=math.sqrt):
    """Eisenstein & Hu (1998, Sec. 4.2) fitting formula without the baryon oscillations, the
    transfer function family the paper sets its initial conditions with (Sec. 2.1).  k in
    h/Mpc.  With theta = T_cmb / 2.7 K, w_m = Om h^2, w_b = Ob h^2, f_b = Ob / Om:
        s       = 44.5 ln(9.83 / w_m) / sqrt(1 + 10 w_b^(3/4))  [Mpc]   (sound horizon fit)
        alpha   = 1 - 0.328 ln(431 w_m) f_b + 0.38 ln(22.3 w_m) f_b^2
        Gamma   = Om h (alpha + (1 - alpha) / (1 + (0.43 k h s)^4))
        q       = k theta^2 / Gamma
        T       = L / (L + C q^2),  L = ln(2 e + 1.8 q),  C = 14.2 + 731 / (1 + 62.5 q).
    Works on floats, or on tensors with log=torch.log, sqrt=torch.sqrt (k > 0)."""
    theta2 = (tcmb / 2.7) ** 2
    wm, wb, fb = om * h * h, ob * h * h, ob / om
    s = 44.5 * math.log(9.83 / wm) / math.sqrt(1.0 + 10.0 * wb ** 0.75)
    alpha = 1.0 - 0.328 * math.log(431.0 * wm) * fb + 0.38 * math.log(22.3 * wm) * fb * fb
    gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta2 / gamma
    big_l = log(2.0 * math.e + 1.8 * q)
    big_c = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return big_l / (big_l + big_c * q * q)


TRANSFER_BBKS, TRANSFER_EH = 0, 1


def transfer(k, om, ob, h, kind, log=math.log, sqrt=math.sqrt):
    """The matter transfer function of wavenumber k [h/Mpc]: BBKS of q = k / (Om h), or
    Eisenstein & Hu without wiggles."""
    if kind == TRANSFER_EH:
        return eh_nowiggle_transfer(k, om, ob, h, log=log, sqrt=sqrt)
    return bbks_transfer(k / (om * h), log=log)


def omega_m_of_a(a, om):
    """Omega_m(a) = Om a^-3 / E(a)^2."""
    return om / (a ** 3 * hubble_e(a, om) ** 2)


def lpt2_factors(a, om):
    """Second-order LPT at scale factor a: (D2 / D1^2, f2) with the fits of Bouchet et al.
    (1995), D2 = -(3/7) D1^2 Omega_m(a)^(-1/143) and f2 = dln D2 / dln a = 2 Omega_m(a)^(6/11)."""
    w = omega_m_of_a(a, om)
    return -3.0 / 7.0 * w ** (-1.0 / 143.0), 2.0 * w ** (6.0 / 11.0)


def _tophat(x):
    if x < 1e-4:
        return 1.0 - x * x / 10.0
    return 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3


def sigma_r(pk, radius):
    """sigma(R)^2 = 1/(2 pi^2) int k^2 P(k) W(kR)^2 dk, integrated in ln k."""
    f = lambda lnk: (math.exp(3 * lnk) * pk(math.exp(lnk)) * _tophat(math.exp(lnk) * radius) ** 2)
    pts = [math.log(x) for x in (1e-3, 1e-2, 0.1, 1.0, 10.0)]
    val, _ = integrate.quad(f, math.log(1e-7), math.log(1e4), points=pts, limit=2000,
                            epsabs=0.0, epsrel=1e-11)
    return math.sqrt(val / (2.0 * math.pi ** 2))


def spectrum_amplitude(om, h, n_s, sigma8, kind=TRANSFER_BBKS, ob=0.05):
    """A such that P(k) = A k^n_s T(k)^2 has sigma(8 Mpc/h) = sigma8 today."""
    shape = lambda k: k ** n_s * transfer(k, om, ob, h, kind) ** 2 if k > 0 else 0.0
    s = sigma_r(shape, 8.0)
    return (sigma8 / s) ** 2


def linear_power(k, om, h, n_s, amp):
    """P(k) [(Mpc/h)^3] at a = 1; k in h/Mpc; P(0) = 0."""
    if k <= 0.0:
        return 0.0
    return amp * k ** n_s * bbks_transfer(k / (om * h)) ** 2
