"""Space-time averaged Riemann fluxes at a face (Sec. II.3, Sec. V).

The wave structure is frozen at the space-time barycentre of the face: the
two barycentre states u_b (eq. 54) from the zones on either side give the
signal speeds (HLL) or the frozen eigen-system (linearized solver), and the
flux is then a fixed linear combination of the space-time averages <u> and
<F> from both sides (eq. 56).

Readings where the paper is silent:
* HLL speeds: lambda_L = min over the two barycentre states of v_n - c_f and
  lambda_R = max of v_n + c_f (c_f = sound speed for Euler, fast
  magnetosonic speed for MHD), then lambda_L <- min(lambda_L, 0) and
  lambda_R <- max(lambda_R, 0) as stated after eq. (17).
* Linearized solver (Euler): F = (<F>_L + <F>_R)/2 - R |Lambda| L (<u>_R -
  <u>_L)/2 with the eigen-system of the Euler flux Jacobian at the arithmetic
  mean of the two barycentre primitive states; no entropy fix.
* Linearized solver (ideal MHD): the same formula with |A| = R |Lambda| R^-1
  of the seven-wave system -- the conserved variables (rho, m, E, B_t1, B_t2)
  with the normal field B_n held at its frozen value -- at the mean of the two
  barycentre primitive states (rho, v, P, B).  The normal field is the
  face's own (continuous) field, so its jump, which the time evolution of the
  two sides' polynomials leaves at truncation level, is not dissipated; the
  normal-field flux is zero as in eq. (7).  Here |A| is formed from its
  definition: the flux Jacobian by complex-step differentiation of the flux
  (exact to rounding) and a library eigen-decomposition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .physics import primitives, conserved, flux, fast_speed


def hll_speeds(ubl, ubr, axis, gamma):
    """lambda_L, lambda_R from the two barycentre states, clipped at zero."""
    _, vl, _, _ = primitives(ubl, gamma)
    _, vr, _, _ = primitives(ubr, gamma)
    cl = fast_speed(ubl, axis, gamma)
    cr = fast_speed(ubr, axis, gamma)
    lam_l = np.minimum(np.minimum(vl[axis] - cl, vr[axis] - cr), 0.0)
    lam_r = np.maximum(np.maximum(vl[axis] + cl, vr[axis] + cr), 0.0)
    return lam_l, lam_r


def hll(pl, pr, axis, gamma):
    """Eq. (56) with the speeds read above; pl/pr are face-side packets
    (left = top side of the lower zone, right = bottom side of the upper)."""
    lam_l, lam_r = hll_speeds(pl['ub'], pr['ub'], axis, gamma)
    return hll_combine(pl['f'], pr['f'], pl['u'], pr['u'], lam_l, lam_r)


def hll_combine(fl, fr, ul, ur, lam_l, lam_r):
    """Eq. (17)/(56) for given speeds (already clipped at zero)."""
    return (lam_r * fl - lam_l * fr + lam_r * lam_l * (ur - ul)) / (lam_r - lam_l)


def euler_eigen_dissipation(ubl, ubr, du, axis, gamma):
    """R |Lambda| L du for the Euler Jacobian along ``axis`` frozen at the
    mean of the two barycentre primitive states."""
    rl, vl, Pl, _ = primitives(ubl, gamma)
    rr, vr, Pr, _ = primitives(ubr, gamma)
    rho = 0.5 * (rl + rr)
    v = 0.5 * (vl + vr)
    p = 0.5 * (Pl + Pr)
    c = np.sqrt(gamma * p / rho)
    q2 = (v * v).sum(axis=0)
    Hent = c * c / (gamma - 1.0) + 0.5 * q2
    t1, t2 = {0: (1, 2), 1: (0, 2), 2: (0, 1)}[axis]
    un, ua, ub = v[axis], v[t1], v[t2]
    d1 = du[0]
    dn = du[1 + axis]
    da = du[1 + t1]
    db = du[1 + t2]
    de = du[4]
    # wave strengths alpha = L du for the eigenvectors listed below
    a_a = da - ua * d1
    a_b = db - ub * d1
    de_bar = de - a_a * ua - a_b * ub
    a_2 = (gamma - 1.0) / (c * c) * (d1 * (Hent - un * un) + un * dn - de_bar)
    a_1 = (d1 * (un + c) - dn - c * a_2) / (2.0 * c)
    a_5 = d1 - a_1 - a_2
    l1 = np.abs(un - c)
    l2 = np.abs(un)
    l5 = np.abs(un + c)
    # eigenvectors (rho, m_n, m_t1, m_t2, E):
    # r1 = (1, un-c, ua, ub, H - un c), r2 = (1, un, ua, ub, q2/2),
    # r_a = (0, 0, 1, 0, ua), r_b = (0, 0, 0, 1, ub), r5 = (1, un+c, ua, ub, H + un c)
    out = np.zeros_like(du)
    w1, w2, wa, wb, w5 = l1 * a_1, l2 * a_2, l2 * a_a, l2 * a_b, l5 * a_5
    out[0] = w1 + w2 + w5
    out[1 + axis] = w1 * (un - c) + w2 * un + w5 * (un + c)
    out[1 + t1] = (w1 + w2 + w5) * ua + wa
    out[1 + t2] = (w1 + w2 + w5) * ub + wb
    out[4] = (w1 * (Hent - un * c) + w2 * 0.5 * q2 + wa * ua + wb * ub
              + w5 * (Hent + un * c))
    return out


def linearized_euler(pl, pr, axis, gamma):
    """Linearized (Roe-type) flux with frozen eigenvectors (Sec. II.3)."""
    du = pr['u'] - pl['u']
    return 0.5 * (pl['f'] + pr['f']) - 0.5 * euler_eigen_dissipation(
        pl['ub'], pr['ub'], du, axis, gamma)


# ------------------------------------------------------- linearized MHD ----

def _transverse(axis):
    return {0: (1, 2), 1: (0, 2), 2: (0, 1)}[axis]


def seven_wave_slots(axis):
    """Rows of the 8-vector (rho, m, E, B) that form the seven-wave system
    along ``axis``: (rho, m_x, m_y, m_z, E, B_t1, B_t2)."""
    t1, t2 = _transverse(axis)
    return [0, 1, 2, 3, 4, 5 + t1, 5 + t2]


def frozen_state(ubl, ubr, gamma):
    """Conserved 8-vector at the mean of the two barycentre primitive states."""
    rl, vl, Pl, Bl = primitives(ubl, gamma)
    rr, vr, Pr, Br = primitives(ubr, gamma)
    return conserved(0.5 * (rl + rr), 0.5 * (vl + vr), 0.5 * (Pl + Pr), 0.5 * (Bl + Br), gamma)


def mhd_jacobian(u8, axis, gamma, h=1e-30):
    """7x7 Jacobian d F7 / d q7 (seven-wave slots, B_n fixed) of the flux
    along ``axis`` at the states u8 (8, M): complex-step derivatives, exact
    to rounding.  Returns (M, 7, 7)."""
    slots = seven_wave_slots(axis)
    M = u8.shape[1]
    J = np.zeros((M, 7, 7))
    for k, s in enumerate(slots):
        uc = u8.astype(complex)
        uc[s] = uc[s] + 1j * h
        F = flux(uc, axis, gamma)
        J[:, :, k] = (F[slots].imag / h).T
    return J


def mhd_abs_jacobian(ubl, ubr, axis, gamma):
    """|A| = R |Lambda| R^-1 of the seven-wave Jacobian at the frozen state of
    each face; ubl, ubr (8, ...) -> (M, 7, 7) over the flattened faces."""
    u8 = frozen_state(ubl, ubr, gamma).reshape(8, -1)
    A = mhd_jacobian(u8, axis, gamma)
    lam, R = np.linalg.eig(A)
    absA = (R * np.abs(lam.real)[:, None, :]) @ np.linalg.inv(R)
    return absA.real


def mhd_dissipation(absA, du8, axis):
    """|A| du on the seven-wave slots of du8 (8, ...); the normal-field row of
    the result is zero."""
    slots = seven_wave_slots(axis)
    shape = du8.shape[1:]
    d7 = du8[slots].reshape(7, -1).T[:, :, None]
    D7 = (absA @ d7)[:, :, 0].T
    out = np.zeros_like(du8)
    out[slots] = D7.reshape((7,) + shape)
    return out


def linearized_mhd_combine(fl, fr, ul, ur, absA, axis):
    """(F_L + F_R)/2 - |A| (u_R - u_L)/2 for 8-vectors."""
    return 0.5 * (fl + fr) - 0.5 * mhd_dissipation(absA, ur - ul, axis)
