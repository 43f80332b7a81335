"""Numpy restatements of the PDHG readings, for pinning the oracle (test helper).

Each function writes one definition out in dense numpy from the readings of
the method (the paper's Section 2 residuals and stopping measures, and the
PDLP / cuPDLP+-style readings for what the paper leaves open), so that the
oracle's C code can be checked against something other than itself.  The
oracle's traced iterates, its Ruiz factors and its evaluation log are the
inputs; nothing here calls into the oracle.

Notation: a trailing `s` marks the scaled problem A~ = D_r A D_c,
b~ = D_r b, c~ = D_c c, l~ = l / D_c; x = D_c x~, y = D_r y~.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Scaled:
    A: np.ndarray        # original dense A
    b: np.ndarray
    c: np.ndarray
    l: np.ndarray
    dr: np.ndarray
    dc: np.ndarray
    As: np.ndarray
    bs: np.ndarray
    cs: np.ndarray
    ls: np.ndarray


def scaled(lp, dr, dc, l=None) -> Scaled:
    A = lp.dense()
    l = np.zeros(lp.n) if l is None else np.asarray(l, dtype=np.float64)
    As = (dr[:, None] * A) * dc[None, :]
    return Scaled(A, lp.b, lp.c, l, dr, dc, As, dr * lp.b, dc * lp.c, l / dc)


def to_scaled(S: Scaled, x, y):
    return x / S.dc, y / S.dr


def to_unscaled(S: Scaled, xs, ys):
    return S.dc * xs, S.dr * ys


# ------------------------------------------------------------- Section 2

def kkt(S: Scaled, x, y) -> dict:
    """Relative KKT errors of an unscaled pair on the original data: the
    residuals r_P = b - Ax and r_D = A^T y + z - c with z = max(0, c - A^T y),
    the objective gap with dobj = b^T y + l^T z, each relative to 1 + norm,
    and maxresid, the largest of the three."""
    rp = S.b - S.A @ x
    d = S.c - S.A.T @ y
    z = np.maximum(0.0, d)
    rd = S.A.T @ y + z - S.c
    pobj = S.c @ x
    dobj = S.b @ y + S.l @ z
    rel_p = np.linalg.norm(rp) / (1 + np.linalg.norm(S.b))
    rel_d = np.linalg.norm(rd) / (1 + np.linalg.norm(S.c))
    rel_g = abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj))
    return dict(rel_p=rel_p, rel_d=rel_d, rel_gap=rel_g,
                maxresid=max(rel_p, rel_d, rel_g), pobj=pobj, dobj=dobj)


# ------------------------------------------------------------- the iteration

def pdhg_step(S: Scaled, xs, ys, tau, sigma):
    """One PDHG step on the scaled problem: projected primal step, then the
    dual step at the extrapolated point 2 x_new - x."""
    xn = np.maximum(S.ls, xs - tau * (S.cs - S.As.T @ ys))
    yn = ys + sigma * (S.bs - S.As @ (2.0 * xn - xs))
    return xn, yn


def kkt_omega(S: Scaled, xs, ys, omega) -> float:
    """Weighted KKT error on the scaled problem, used by the restart test:
    sqrt(w^2 ||b~ - A~x~||^2 + ||r~_D||^2 / w^2 + gap~^2), with
    r~_D = max(0, A~^T y~ - c~) and gap~ = c~^T x~ - b~^T y~ - l~^T z~."""
    rp = S.bs - S.As @ xs
    d = S.cs - S.As.T @ ys
    z = np.maximum(0.0, d)
    rd = z - d
    gap = S.cs @ xs - S.bs @ ys - S.ls @ z
    return float(np.sqrt(omega ** 2 * (rp @ rp) + (rd @ rd) / omega ** 2 + gap ** 2))


def omega_smoothed(omega, dx, dy, theta=0.5):
    """Primal weight at a restart: log w moves the fraction theta toward
    log(dy / dx); unchanged when either distance is at most 1e-10."""
    if not (dx > 1e-10 and dy > 1e-10):
        return omega
    return float(np.exp(theta * np.log(dy / dx) + (1 - theta) * np.log(omega)))


def restart_test(K, K_last, K_prev, t, k, beta=(0.2, 0.8, 0.36)):
    """Adaptive restart: sufficient decay, or necessary decay with no further
    progress since the previous check, or an artificial restart once the
    iterations since the last restart reach beta_art times the total.
    Returns (fired, reason) with reason 1, 2 or 3 (0: no restart)."""
    if K <= beta[0] * K_last:
        return True, 1
    if K <= beta[1] * K_last and K > K_prev:
        return True, 2
    if t >= beta[2] * k:
        return True, 3
    return False, 0


def halpern_lambda(t: int) -> float:
    """Halpern weight of the step taken t steps after the anchor."""
    return (t + 1.0) / (t + 2.0)


def halpern_step(S: Scaled, xs, ys, xa, ya, t, tau, sigma, rho=1.0):
    """z <- lambda ((1 + rho) T(z) - rho z) + (1 - lambda) z_a."""
    xh, yh = pdhg_step(S, xs, ys, tau, sigma)
    lam = halpern_lambda(t)
    xn = lam * ((1 + rho) * xh - rho * xs) + (1 - lam) * xa
    yn = lam * ((1 + rho) * yh - rho * ys) + (1 - lam) * ya
    return xn, yn


def close(a, b, rtol, atol=0.0):
    """Elementwise |a - b| <= rtol * max|b| + atol (vectors or scalars)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.max(np.abs(b)) if b.size else 0.0
    return bool(np.all(np.abs(a - b) <= rtol * scale + atol))
