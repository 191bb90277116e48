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

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .physics import primitives, fast_speed


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
