"""Exact solution of the one-dimensional shallow-water Riemann problem.

Written from the classical wave-curve theory of the shallow-water equations
(not from the paper's approximate solver): across a shock of the k-wave
(star depth h > h_k)

    f_k(h) = (h - h_k) sqrt(g (h + h_k) / (2 h h_k)),

across a rarefaction (h <= h_k)

    f_k(h) = 2 (sqrt(g h) - sqrt(g h_k)),

and the star depth solves f_L(h) + f_R(h) + u_R - u_L = 0, with
u* = (u_L + u_R)/2 + (f_R(h*) - f_L(h*))/2. A dry side gives Ritter's
rarefaction reaching the dry front at u + 2a (or u - 2a).

Evaluated with mpmath at 50 digits. Used only by the tests, to pin the
oracle's wave-speed estimates and the dam-break solutions (Stoker, Ritter).
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50


def _f(h, hk, g):
    if h > hk:
        return (h - hk) * mp.sqrt(g * (h + hk) / (2 * h * hk))
    return 2 * (mp.sqrt(g * h) - mp.sqrt(g * hk))


def star_state(hL, uL, hR, uR, g=9.81):
    """Exact (h*, u*) for two wet states; h* = 0 if a vacuum forms."""
    hL, uL, hR, uR, g = map(mp.mpf, (hL, uL, hR, uR, g))
    aL, aR = mp.sqrt(g * hL), mp.sqrt(g * hR)
    if uR - uL >= 2 * (aL + aR):
        return mp.mpf(0), None
    F = lambda h: _f(h, hL, g) + _f(h, hR, g) + uR - uL  # noqa: E731
    lo, hi = mp.mpf("1e-40"), max(hL, hR)
    while F(hi) < 0:
        hi *= 2
    for _ in range(400):          # bisection, then polish
        mid = (lo + hi) / 2
        if F(mid) > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo < mp.mpf(10) ** (-45) * hi:
            break
    hs = (lo + hi) / 2
    us = (uL + uR) / 2 + (_f(hs, hR, g) - _f(hs, hL, g)) / 2
    return hs, us


def shock_speed_left(hL, uL, hs, g=9.81):
    """Speed of a left-facing shock from (hL, uL) to depth hs > hL, from the
    Rankine-Hugoniot condition on mass with the shock relation for u*."""
    hL, uL, hs, g = map(mp.mpf, (hL, uL, hs, g))
    us = uL - _f(hs, hL, g)
    return (hs * us - hL * uL) / (hs - hL)


def shock_speed_right(hR, uR, hs, g=9.81):
    hR, uR, hs, g = map(mp.mpf, (hR, uR, hs, g))
    us = uR + _f(hs, hR, g)
    return (hs * us - hR * uR) / (hs - hR)


def sample(hL, uL, hR, uR, xi, g=9.81):
    """Exact (h, u) at similarity coordinate xi = x / t. Handles a dry
    right or left side (Ritter)."""
    hL, uL, hR, uR, xi, g = map(mp.mpf, (hL, uL, hR, uR, xi, g))
    if hR == 0:
        aL = mp.sqrt(g * hL)
        if xi <= uL - aL:
            return hL, uL
        if xi >= uL + 2 * aL:
            return mp.mpf(0), mp.mpf(0)
        a = (uL + 2 * aL - xi) / 3
        return a * a / g, (uL + 2 * aL + 2 * xi) / 3
    if hL == 0:
        aR = mp.sqrt(g * hR)
        if xi >= uR + aR:
            return hR, uR
        if xi <= uR - 2 * aR:
            return mp.mpf(0), mp.mpf(0)
        a = (-uR + 2 * aR + xi) / 3
        return a * a / g, (uR - 2 * aR + 2 * xi) / 3
    hs, us = star_state(hL, uL, hR, uR, g)
    aL, aR = mp.sqrt(g * hL), mp.sqrt(g * hR)
    a_s = mp.sqrt(g * hs)
    if xi <= us:
        if hs > hL:
            s = shock_speed_left(hL, uL, hs, g)
            return (hL, uL) if xi < s else (hs, us)
        head, tail = uL - aL, us - a_s
        if xi <= head:
            return hL, uL
        if xi >= tail:
            return hs, us
        a = (uL + 2 * aL - xi) / 3
        return a * a / g, (uL + 2 * aL + 2 * xi) / 3
    if hs > hR:
        s = shock_speed_right(hR, uR, hs, g)
        return (hR, uR) if xi > s else (hs, us)
    head, tail = uR + aR, us + a_s
    if xi >= head:
        return hR, uR
    if xi <= tail:
        return hs, us
    a = (-uR + 2 * aR + xi) / 3
    return a * a / g, (uR - 2 * aR + 2 * xi) / 3


def godunov_flux(hL, uL, vL, hR, uR, vR, g=9.81):
    """Exact Godunov flux (h u, h u^2 + g h^2/2, h u v) of the state at
    x/t = 0; the passive tangential velocity is carried by the contact u*."""
    h, u = sample(hL, uL, hR, uR, 0, g)
    if hL > 0 and hR > 0:
        _, us = star_state(hL, uL, hR, uR, g)
    else:
        us = u
    v = mp.mpf(vL) if us >= 0 else mp.mpf(vR)
    g = mp.mpf(g)
    return h * u, h * u * u + g * h * h / 2, h * u * v


def profile(hL, uL, hR, uR, xi, g=9.81):
    """Vectorised exact depth and velocity at the similarity coordinates
    ``xi`` (numpy array); the star state is solved once in mpmath."""
    import numpy as np
    xi = np.asarray(xi, dtype=float)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    if hR == 0 or hL == 0:
        for k, x in enumerate(xi):
            a, b = sample(hL, uL, hR, uR, x, g)
            h[k], u[k] = float(a), float(b)
        return h, u
    hs, us = star_state(hL, uL, hR, uR, g)
    hs, us = float(hs), float(us)
    aL, aR, a_s = (np.sqrt(g * hL), np.sqrt(g * hR), np.sqrt(g * hs))
    for k, x in enumerate(xi):
        if x <= us:
            if hs > hL:
                s = float(shock_speed_left(hL, uL, hs, g))
                h[k], u[k] = (hL, uL) if x < s else (hs, us)
            elif x <= uL - aL:
                h[k], u[k] = hL, uL
            elif x >= us - a_s:
                h[k], u[k] = hs, us
            else:
                a = (uL + 2 * aL - x) / 3
                h[k], u[k] = a * a / g, (uL + 2 * aL + 2 * x) / 3
        else:
            if hs > hR:
                s = float(shock_speed_right(hR, uR, hs, g))
                h[k], u[k] = (hR, uR) if x > s else (hs, us)
            elif x >= uR + aR:
                h[k], u[k] = hR, uR
            elif x <= us + a_s:
                h[k], u[k] = hs, us
            else:
                a = (-uR + 2 * aR + x) / 3
                h[k], u[k] = a * a / g, (uR - 2 * aR + 2 * x) / 3
    return h, u
