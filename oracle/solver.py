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
