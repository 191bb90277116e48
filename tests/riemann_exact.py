"""Exact solution of the Euler Riemann problem (ideal gas), for tests: the
star pressure from Newton's iteration on the pressure function (Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4), then
the self-similar solution sampled at x/t.  Independent of the scheme."""

import numpy as np


def _f(p, rho, pk, gamma):
    """Pressure function of one side and its derivative."""
    c = np.sqrt(gamma * pk / rho)
    if p > pk:                                   # shock
        a = 2.0 / ((gamma + 1.0) * rho)
        b = (gamma - 1.0) / (gamma + 1.0) * pk
        q = np.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + b))
    r = p / pk                                   # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    return 2.0 * c / (gamma - 1.0) * (r ** e - 1.0), r ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * c)


def star_state(left, right, gamma):
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, gamma)
        fr, dr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p_new = max(1e-12, p - dp)
        if abs(p_new - p) <= 1e-15 * p:
            p = p_new
            break
        p = p_new
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, gamma, xi):
    """(rho, u, p) at the similarity coordinates xi = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.empty((3,) + np.shape(xi))
    for idx, s in np.ndenumerate(np.asarray(xi)):
        if s <= us:                              # left of the contact
            rho, u, p, c = rl, ul, pl, np.sqrt(gamma * pl / rl)
            if ps > pl:                          # left shock
                sl = ul - c * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl
                                      + (gamma - 1.0) / (2.0 * gamma))
                val = (rl, ul, pl) if s < sl else (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:                                # left rarefaction
                cs = c * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                if s < ul - c:
                    val = (rl, ul, pl)
                elif s > us - cs:
                    val = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    uu = 2.0 / (gamma + 1.0) * (c + (gamma - 1.0) / 2.0 * ul + s)
                    cc = 2.0 / (gamma + 1.0) * (c + (gamma - 1.0) / 2.0 * (ul - s))
                    rho = rl * (cc / c) ** (2.0 / (gamma - 1.0))
                    val = (rho, uu, pl * (cc / c) ** (2.0 * gamma / (gamma - 1.0)))
        else:                                    # right of the contact
            c = np.sqrt(gamma * pr / rr)
            if ps > pr:                          # right shock
                sr = ur + c * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr
                                      + (gamma - 1.0) / (2.0 * gamma))
                val = (rr, ur, pr) if s > sr else (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:                                # right rarefaction
                cs = c * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                if s > ur + c:
                    val = (rr, ur, pr)
                elif s < us + cs:
                    val = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    uu = 2.0 / (gamma + 1.0) * (-c + (gamma - 1.0) / 2.0 * ur + s)
                    cc = 2.0 / (gamma + 1.0) * (c - (gamma - 1.0) / 2.0 * (ur - s))
                    rho = rr * (cc / c) ** (2.0 / (gamma - 1.0))
                    val = (rho, uu, pr * (cc / c) ** (2.0 * gamma / (gamma - 1.0)))
        out[(slice(None),) + idx] = val
    return out


def zone_averages_x(n, t, left, right, gamma=1.4, x0=0.5, sub=64):
    """Zone averages of (rho, rho u, E) of the exact solution on n zones of
    [0, 1] along x (sub points per zone)."""
    x = (np.arange(n * sub) + 0.5) / (n * sub)
    rho, u, p = sample(left, right, gamma, (x - x0) / t)
    cons = np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])
    return cons.reshape(3, n, sub).mean(axis=2)
