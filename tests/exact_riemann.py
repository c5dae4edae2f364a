"""Exact Riemann solver of the 1-D Euler equations for a gamma-law gas, as
derived in Toro (2009), Ch. 4: Newton iteration on the pressure function
f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0, then sampling of the self-similar
solution.  Used to pin the oracle's hydrodynamic limit (B = 0)."""
import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    pr = p / pk  # rarefaction
    f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star(L, R, g):
    rl, ul, pl = L
    rr, ur, prr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * prr / rr)
    p = max(1e-8, 0.5 * (pl + prr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, prr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, prr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, g, s):
    """Density, velocity, pressure at x/t = s (array)."""
    rl, ul, pl = L
    rr, ur, prr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * prr / rr)
    ps, us = star(L, R, g)
    s = np.asarray(s, dtype=float)
    out = np.zeros((3,) + s.shape)
    for idx, x in np.ndenumerate(s):
        if x <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if x <= sl:
                    w = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    w = (r, us, ps)
            else:  # left rarefaction
                shl = ul - cl
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - cs
                if x <= shl:
                    w = (rl, ul, pl)
                elif x >= stl:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * cl) * (ul - x)
                    r = rl * c ** (2 / (g - 1))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + x)
                    p = pl * c ** (2 * g / (g - 1))
                    w = (r, u, p)
        else:  # right of contact
            if ps > prr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / prr + (g - 1) / (2 * g))
                if x >= sr:
                    w = (rr, ur, prr)
                else:
                    r = rr * ((ps / prr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / prr + 1))
                    w = (r, us, ps)
            else:
                shr = ur + cr
                cs = cr * (ps / prr) ** ((g - 1) / (2 * g))
                str_ = us + cs
                if x >= shr:
                    w = (rr, ur, prr)
                elif x <= str_:
                    w = (rr * (ps / prr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * cr) * (ur - x)
                    r = rr * c ** (2 / (g - 1))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + x)
                    p = prr * c ** (2 * g / (g - 1))
                    w = (r, u, p)
        out[(slice(None),) + idx] = w
    return out
