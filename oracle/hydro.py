"""Gas dynamics of the oracle: comoving Euler equations in conservation form, solved with
the relaxing total-variation-diminishing scheme (Jin & Xin relaxation, Trac & Pen 2003) with
a two-stage Runge-Kutta step and Strang dimensional splitting (Sec. 2.3, 2.3.1, 2.3.2).

State vector per cell (eq. conservation):  Q = (rho, a rho U_x, a rho U_y, a rho U_z, a^2 rho E)
with comoving gas density rho, peculiar velocity U and specific total energy E = e + U^2/2.
Fluxes along direction d (eq. cont, eq. momentum, eq. ev with gamma = 5/3):
    F_rho = rho U_d / a
    F_mj  = rho U_d U_j + p delta_jd        (pressure in the momentum flux: conservative form)
    F_E   = a U_d (rho E + p)
The internal-energy source S_e is not applied: the energy variable is the total energy,
whose flux already carries the pdV work (a reading: the paper lists S_e beside a total-
energy equation whose flux has the pressure work).

Dual energy (an option; Sec. 2.3 names the dual-energy formalism as the extension of its
single-energy scheme without fixing one): a sixth conserved component S = (a^2 rho e)
rho^(1-gamma), the entropy variable, is advected with the flux S U_d / a.  With gamma = 5/3,
S / rho = a^2 e rho^(1-gamma) is a function of the proper entropy p_prop / rho_prop^gamma alone,
so it is carried unchanged by the flow wherever the flow is adiabatic.  The equation of state
takes the specific internal energy from the total energy, e_E = E - U^2/2, where
e_E > eta1 E, and from the entropy, e_S = S rho^(gamma-2) / a^2, elsewhere (kinetic energy
dominating: e_E is then a small difference of large numbers); at the end of each step S is
reset from the total energy where e_E >= eta2 E, so shocks, which raise the entropy, feed it.
The selection and synchronisation rule and eta1 = 1e-3, eta2 = 0.1 are those of Bryan et al.
(1995); the entropy in place of an internal-energy equation follows Ryu et al. (1993), and
needs no pdV source term.

Units: length in cells (Delta x = 1), time in 1/H0, velocity in cells*H0.
Arrays are indexed [component, z, y, x] (x fastest); axis d = 0, 1, 2 means x, y, z.
"""

import torch


def shift(f, d, s):
    """Value of f at cell j+s along axis d (periodic); f is [..., z, y, x]."""
    return torch.roll(f, shifts=-s, dims=f.dim() - 1 - d)


DUAL_ETA1 = 1e-3   # below this fraction of E, e comes from the entropy
DUAL_ETA2 = 0.1    # at or above it, the entropy is reset from the total energy


def entropy_energy(q, a, gamma):
    """e_S = S rho^(gamma-2) / a^2: the specific internal energy held by the entropy S."""
    return q[5] * q[0] ** (gamma - 2.0) / (a * a)


def internal_energy(q, a, gamma):
    """(e, U): the specific internal energy before the floor and the peculiar velocity.
    Single energy (five components): e = E - U^2/2.  Dual energy (six): that where it
    exceeds eta1 E, else e_S (module docstring)."""
    rho = q[0]
    u = q[1:4] / (a * rho)
    big_e = q[4] / (a * a * rho)
    e = big_e - 0.5 * (u * u).sum(0)
    if q.shape[0] > 5:
        e = torch.where(e > DUAL_ETA1 * big_e, e, entropy_energy(q, a, gamma))
    return e, u


def entropy_of_total(q, gamma):
    """S = (a^2 rho E - |a rho U|^2 / (2 rho)) rho^(1-gamma): the entropy variable of the
    internal energy that the total energy holds."""
    rho = q[0]
    return (q[4] - 0.5 * (q[1:4] * q[1:4]).sum(0) / rho) * rho ** (1.0 - gamma)


def dual_sync(q, a, gamma):
    """End-of-step synchronisation of the dual-energy state: S from the total energy where
    e_E >= eta2 E, unchanged elsewhere."""
    rho = q[0]
    u = q[1:4] / (a * rho)
    big_e = q[4] / (a * a * rho)
    e = big_e - 0.5 * (u * u).sum(0)
    s = torch.where(e >= DUAL_ETA2 * big_e, entropy_of_total(q, gamma), q[5])
    return torch.cat([q[:5], s[None]])


def primitives(q, a, gamma, e_floor):
    """Velocity, pressure and sound speed from Q at scale factor a.

    The specific internal energy e (internal_energy) is floored at e_floor only inside the
    equation of state (pressure, sound speed); the stored total energy is never changed,
    so the conservation form is untouched.  p = (gamma-1) rho e, c_s = sqrt(gamma p/rho).
    """
    rho = q[0]
    e, u = internal_energy(q, a, gamma)
    e_eff = torch.clamp(e, min=e_floor)
    p = (gamma - 1.0) * rho * e_eff
    cs = torch.sqrt(gamma * p / rho)
    return u, p, cs


def flux_and_speed(q, a, d, gamma, e_floor, sign_ud=None):
    """Cell-centred flux F along d and the freezing speed c = (|U_d| + c_s)/a (Sec. 2.3.1).

    The 1/a in c is the comoving signal speed in cells per unit time: the continuity flux is
    rho U/a, so the characteristic speeds of this system are (U_d +- c_s)/a.
    sign_ud (optional, +-1 per cell) fixes the side of the kink of |U_d| (|U_d| = sign U_d);
    only derivative checks at a kink use it."""
    rho = q[0]
    u, p, cs = primitives(q, a, gamma, e_floor)
    ud = u[d]
    mom = [rho * ud * u[j] + (p if j == d else 0.0) for j in range(3)]
    extra = [q[5] * ud / a] if q.shape[0] > 5 else []
    f = torch.stack([rho * ud / a] + mom + [a * ud * (q[4] / (a * a) + p)] + extra)
    c = ((ud.abs() if sign_ud is None else sign_ud * ud) + cs) / a
    return f, c


LIMITER_EPS = 1e-20


def van_leer(x, y, eps=LIMITER_EPS, take=None):
    """Harmonic-mean (van Leer) flux limiter with a small guard epsilon (Sec. 2.3.2).

    phi(x, y) = (x y + |x y|) / (x + y + eps sgn(x+y)), sgn(0) = +1: equal to
    2xy/(x+y+eps sgn) when x and y share a sign and 0 otherwise, so it is never 0/0
    (a reading: the paper's form 2xy/(x+y+eps) leaves opposite signs and x + y < 0 open).
    take (optional, per element: a boolean or a weight 0, 1/2 or 1) fixes the branch in place
    of the test x y > 0: w 2xy/(x+y+eps sgn) with w = 1 (true) or 0 (false).  w = 1/2 is the
    mean of the two sides, whose derivative is that of the |x y| form itself at x y = 0 exactly
    (where |.| has the derivative sign(0) = 0).  Only derivative checks at the kink x y = 0
    use it."""
    s = x + y
    sg = torch.where(s >= 0, torch.ones_like(s), -torch.ones_like(s))
    xy = x * y
    if take is None:
        return (xy + xy.abs()) / (s + eps * sg)
    w = take.to(xy.dtype)
    return torch.where(w > 0, w * (2.0 * xy / (s + eps * sg)), torch.zeros_like(xy))


def split_fluxes(q, a, d, gamma, e_floor, sign_ud=None):
    """Right- and left-moving fluxes F^R = c Q^R, F^L = c Q^L of the relaxation system with
    Q^R = (Q + F/c)/2 and Q^L = (Q - F/c)/2, so that F = F^R - F^L (Sec. 2.3.1)."""
    f, c = flux_and_speed(q, a, d, gamma, e_floor, sign_ud)
    return 0.5 * (c * q + f), 0.5 * (c * q - f)


def sweep_kinks(q, d, dt, a_stage1, a_stage2, gamma, e_floor):
    """The quantities whose signs decide the non-smooth choices of sweep(): U_d at each
    stage (the kink of |U_d|) and the two slopes of every limited face and component,
    right-moving (x_r, y_r) and left-moving (x_l, y_l).  Returned as a dict of tensors, with
    the scale each is compared against (for telling which lie within rounding of a kink)."""
    with torch.no_grad():
        u1 = primitives(q, a_stage1, gamma, e_floor)[0][d]
        fr, fl = split_fluxes(q, a_stage1, d, gamma, e_floor)
        f1 = fr - shift(fl, d, 1)
        qh = q - 0.5 * dt * (f1 - shift(f1, d, -1))
        u2 = primitives(qh, a_stage2, gamma, e_floor)[0][d]
        fr, fl = split_fluxes(qh, a_stage2, d, gamma, e_floor)
        fr_m1, fr_p1 = shift(fr, d, -1), shift(fr, d, 1)
        fl_p1, fl_p2 = shift(fl, d, 1), shift(fl, d, 2)
        return {"u1": (u1, primitives(q, a_stage1, gamma, e_floor)[0].abs().sum(0)),
                "u2": (u2, primitives(qh, a_stage2, gamma, e_floor)[0].abs().sum(0)),
                "x_r": (fr - fr_m1, fr.abs() + fr_m1.abs()),
                "y_r": (fr_p1 - fr, fr_p1.abs() + fr.abs()),
                "x_l": (fl_p1 - fl, fl_p1.abs() + fl.abs()),
                "y_l": (fl_p2 - fl_p1, fl_p2.abs() + fl_p1.abs())}


def sweep(q, d, dt, a_stage1, a_stage2, gamma, e_floor, eps=LIMITER_EPS, branches=None):
    """One dimensional relaxing-TVD sweep of the whole grid along axis d over a full dt.

    Stage 1 (eq. TVD_halfstep): first-order upwind interface fluxes
        F_{n+1/2} = F^R_n - F^L_{n+1},  Q^{1/2}_n = Q_n - dt/2 (F_{n+1/2} - F_{n-1/2}).
    Stage 2 (eq. TVD_fullstep): second-order fluxes of Q^{1/2} with the limiter applied to
    each wave and component,
        F^R_{n+1/2} = F^R_n + phi((F^R_n - F^R_{n-1})/2, (F^R_{n+1} - F^R_n)/2)
        F^L_{n+1/2} = F^L_{n+1} - phi((F^L_{n+1} - F^L_n)/2, (F^L_{n+2} - F^L_{n+1})/2)
    and Q^{new}_n = Q_n - dt (F_{n+1/2} - F_{n-1/2}).  The freezing speed is recomputed at
    each stage; stage 1 uses a(t_n), stage 2 a(t_n + dt/2).

    branches (optional, for derivative checks at the kinks only): a dict that fixes the
    side of each non-smooth choice instead of deciding it from the values, with entries
    "sign1", "sign2" (the sign taken for |U_d| at each stage, +-1 per cell) and "take_r",
    "take_l" (the limiter branch of each face and component of the right- and left-moving
    waves, see van_leer).  Missing entries are decided from the values as usual.
    """
    br = branches or {}
    fr, fl = split_fluxes(q, a_stage1, d, gamma, e_floor, br.get("sign1"))
    f1 = fr - shift(fl, d, 1)
    qh = q - 0.5 * dt * (f1 - shift(f1, d, -1))

    fr, fl = split_fluxes(qh, a_stage2, d, gamma, e_floor, br.get("sign2"))
    fr_m1, fr_p1 = shift(fr, d, -1), shift(fr, d, 1)
    fl_p1, fl_p2 = shift(fl, d, 1), shift(fl, d, 2)
    fr_face = fr + van_leer(0.5 * (fr - fr_m1), 0.5 * (fr_p1 - fr), eps, br.get("take_r"))
    fl_face = fl_p1 - van_leer(0.5 * (fl_p1 - fl), 0.5 * (fl_p2 - fl_p1), eps,
                               br.get("take_l"))
    f2 = fr_face - fl_face
    return q - dt * (f2 - shift(f2, d, -1))


# Strang order (Sec. 2.3.2): the direction order is reversed on every other step and
# rotated every two steps: XYZ ZYX | ZXY YXZ | YZX XZY, a cycle of six steps.
STRANG_ORDER = ((0, 1, 2), (2, 1, 0), (2, 0, 1), (1, 0, 2), (1, 2, 0), (0, 2, 1))


def strang_axes(step):
    return STRANG_ORDER[step % 6]


def max_signal_speed(q, a, gamma, e_floor):
    """max over cells and axes of (|U_d| + c_s)/a, the speed in the CFL condition (eq. dt)."""
    u, _, cs = primitives(q, a, gamma, e_floor)
    return float(((u.abs() + cs) / a).max())
