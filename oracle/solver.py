"""Conjugate gradient for Hermitian positive-definite operators (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2: K = M^dag M is large and sparse and is inverted by an iterative
solver such as conjugate gradient.  The paper fixes no stopping rule, initial
guess or precision.  Reading: textbook Hestenes-Stiefel CG, x0 = 0, stop when
the true residual ||b - A x|| <= tol ||b|| (recomputed at exit).
"""
from __future__ import annotations

import numpy as np


def vdot(a, b) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def norm2(a) -> float:
    return float(np.vdot(a.reshape(-1), a.reshape(-1)).real)


def cg(apply_A, b, tol=1e-10, maxiter=10000):
    """Solve A x = b.  Returns (x, iterations, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = norm2(r)
    bb = norm2(b)
    if bb == 0.0:
        return x, 0, 0.0
    it = 0
    while True:
        while rr > tol * tol * bb and it < maxiter:
            Ap = apply_A(p)
            alpha = rr / vdot(p, Ap).real
            x = x + alpha * p
            r = r - alpha * Ap
            rr_new = norm2(r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            it += 1
        true_r = np.sqrt(norm2(b - apply_A(x)) / bb)
        if true_r <= tol or it >= maxiter:
            return x, it, true_r
        # iterated residual drifted below the true one: restart from x
        r = b - apply_A(x)
        p = r.copy()
        rr = norm2(r)


def cg_multishift(apply_A, b, shifts, tol=1e-10, maxiter=10000):
    """Solve (A + s) x_s = b for every shift s >= 0 in the Krylov space of A + min(s).

    The shifted systems share CG's Krylov space because A + s and A + s0 differ
    by a multiple of the identity; their residuals stay collinear with the base
    residual, r_s = zeta_s r, and zeta obeys (with the base CG's alpha_i,
    beta_i, and d = s - s0)

        zeta_{i+1} = zeta_i zeta_{i-1} alpha_{i-1}
                     / (alpha_i beta_{i-1} (zeta_{i-1} - zeta_i) + zeta_{i-1} alpha_{i-1} (1 + d alpha_i)),
        alpha_{s,i} = alpha_i zeta_{i+1} / zeta_i,      beta_{s,i} = beta_i (zeta_{i+1} / zeta_i)^2,
        x_s += alpha_{s,i} p_s,                         p_s = zeta_{i+1} r_{i+1} + beta_{s,i} p_s,

    from zeta_0 = zeta_{-1} = 1, alpha_{-1} = 1, beta_{-1} = 0 (the shifted-system
    CG of Jegerlehner, hep-lat/9612014).  A shift stops once |zeta_s|^2 |r|^2 <=
    tol^2 |b|^2; the iteration stops with the base system.  Returns
    (list of x_s in the order of ``shifts``, iterations, true relative residuals).
    """
    shifts = [float(s) for s in shifts]
    s0 = min(shifts)
    A0 = lambda v: apply_A(v) + s0 * v
    d = [s - s0 for s in shifts]
    n = len(shifts)
    xs = [np.zeros_like(b) for _ in range(n)]
    ps = [b.copy() for _ in range(n)]
    r = b.copy()
    p = b.copy()
    rr = norm2(r)
    bb = norm2(b)
    zeta_prev = [1.0] * n
    zeta = [1.0] * n
    done = [bb == 0.0] * n
    alpha_prev, beta_prev = 1.0, 0.0
    it = 0
    while rr > tol * tol * bb and it < maxiter:
        Ap = A0(p)
        alpha = rr / vdot(p, Ap).real
        zeta_next = list(zeta)
        for k in range(n):
            if done[k]:
                continue
            den = (alpha * beta_prev * (zeta_prev[k] - zeta[k])
                   + zeta_prev[k] * alpha_prev * (1.0 + d[k] * alpha))
            zeta_next[k] = zeta[k] * zeta_prev[k] * alpha_prev / den
            xs[k] = xs[k] + (alpha * zeta_next[k] / zeta[k]) * ps[k]
        r = r - alpha * Ap
        rr_new = norm2(r)
        beta = rr_new / rr
        for k in range(n):
            if done[k]:
                continue
            bk = beta * (zeta_next[k] / zeta[k]) ** 2
            ps[k] = zeta_next[k] * r + bk * ps[k]
            if zeta_next[k] ** 2 * rr_new <= tol * tol * bb:
                done[k] = True
        p = r + beta * p
        zeta_prev, zeta = zeta, zeta_next
        alpha_prev, beta_prev, rr = alpha, beta, rr_new
        it += 1
    res = [np.sqrt(norm2(b - apply_A(x) - s * x) / bb) if bb else 0.0 for x, s in zip(xs, shifts)]
    return xs, it, res
