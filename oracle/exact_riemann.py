"""Exact solution of the 1-D Riemann problem of the Euler equations (ideal gas).

TEST INFRASTRUCTURE: used only to pin the oracle against a closed-form
solution (the shock-tube problem). It is the classical construction -- two
nonlinear waves (shock or rarefaction) either side of a contact, the star
pressure found as the root of the pressure function by Newton iteration, then
self-similar sampling in x/t -- written from the gas-dynamics relations
themselves (Rankine-Hugoniot conditions across a shock, isentropic Riemann
invariants across a rarefaction; cf. Courant & Friedrichs 1948, Toro ch. 4).
"""
from __future__ import annotations

import math

import numpy as np


def _wave_function(p, rho, pk, gamma):
    """f_K(p) = velocity jump across the K wave to reach pressure p, and f_K'(p)."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock: Rankine-Hugoniot
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction: isentropic, constant Riemann invariant
    r = p / pk
    f = 2.0 * c / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = r ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * c)
    return f, df


def star_state(left, right, gamma, tol=1e-15, maxit=100):
    """(p*, u*) between the left and right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # start from the two-rarefaction estimate, which is exact when both waves are rarefactions
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    for _ in range(maxit):
        fl, dfl = _wave_function(p, rl, pl, gamma)
        fr, dfr = _wave_function(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(p - dp, 1e-14 * p)
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _wave_function(p, rl, pl, gamma)
    fr, _ = _wave_function(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(left, right, gamma):
    """rho*_L, rho*_R (shock adiabat or isentrope on each side)."""
    p, _ = star_state(left, right, gamma)
    out = []
    for rho, _, pk in (left, right):
        r = p / pk
        if p > pk:
            g = (gamma - 1.0) / (gamma + 1.0)
            out.append(rho * (r + g) / (g * r + 1.0))
        else:
            out.append(rho * r ** (1.0 / gamma))
    return tuple(out)


def wave_speeds(left, right, gamma):
    """Speeds of the left and right outer waves (shock speed, or rarefaction head)."""
    p, _ = star_state(left, right, gamma)
    speeds = []
    for side, (rho, u, pk) in (("L", left), ("R", right)):
        c = math.sqrt(gamma * pk / rho)
        sgn = -1.0 if side == "L" else 1.0
        if p > pk:
            speeds.append(u + sgn * c * math.sqrt((gamma + 1.0) / (2.0 * gamma) * p / pk
                                                  + (gamma - 1.0) / (2.0 * gamma)))
        else:
            speeds.append(u + sgn * c)
    return tuple(speeds)


def sample(xi, left, right, gamma):
    """(rho, u, p) at similarity coordinate xi = (x - x0)/t; xi may be an array."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    p_s, u_s = star_state(left, right, gamma)
    rho_sl, rho_sr = star_densities(left, right, gamma)
    out = np.empty((3, xi.size))
    g = gamma
    for n, s in enumerate(xi):
        if s <= u_s:
            rho, u, p = left
            c = math.sqrt(g * p / rho)
            if p_s > p:
                S = u - c * math.sqrt((g + 1) / (2 * g) * p_s / p + (g - 1) / (2 * g))
                out[:, n] = (rho, u, p) if s <= S else (rho_sl, u_s, p_s)
            else:
                head, tail = u - c, u_s - c * (p_s / p) ** ((g - 1) / (2 * g))
                if s <= head:
                    out[:, n] = (rho, u, p)
                elif s >= tail:
                    out[:, n] = (rho_sl, u_s, p_s)
                else:
                    f = 2 / (g + 1) + (g - 1) / ((g + 1) * c) * (u - s)
                    out[:, n] = (rho * f ** (2 / (g - 1)), 2 / (g + 1) * (c + 0.5 * (g - 1) * u + s),
                                 p * f ** (2 * g / (g - 1)))
        else:
            rho, u, p = right
            c = math.sqrt(g * p / rho)
            if p_s > p:
                S = u + c * math.sqrt((g + 1) / (2 * g) * p_s / p + (g - 1) / (2 * g))
                out[:, n] = (rho, u, p) if s >= S else (rho_sr, u_s, p_s)
            else:
                head, tail = u + c, u_s + c * (p_s / p) ** ((g - 1) / (2 * g))
                if s >= head:
                    out[:, n] = (rho, u, p)
                elif s <= tail:
                    out[:, n] = (rho_sr, u_s, p_s)
                else:
                    f = 2 / (g + 1) - (g - 1) / ((g + 1) * c) * (u - s)
                    out[:, n] = (rho * f ** (2 / (g - 1)), 2 / (g + 1) * (-c + 0.5 * (g - 1) * u + s),
                                 p * f ** (2 * g / (g - 1)))
    return out


def cell_averages(edges, t, x0, left, right, gamma, sub=64):
    """Cell averages of (rho, rho u, E) over cells with the given edges at time t,
    by midpoint quadrature with `sub` points per cell."""
    edges = np.asarray(edges, dtype=np.float64)
    n = edges.size - 1
    frac = (np.arange(sub) + 0.5) / sub
    pts = (edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * frac[None, :]).ravel()
    rho, u, p = sample((pts - x0) / t, left, right, gamma)
    E = p / (gamma - 1) + 0.5 * rho * u * u
    return (rho.reshape(n, sub).mean(1), (rho * u).reshape(n, sub).mean(1),
            E.reshape(n, sub).mean(1))
