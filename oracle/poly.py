"""Chebyshev filter polynomial P_n(x) ~ 1/x on [a, b] (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2 (polynomial filtering) takes P(K) a low-order polynomial approximating
K^-1 built from Chebyshev polynomials, with the order as the only tuning
parameter; Sec. 3.3 (two filters) needs P_1 to divide P_2.  The paper does not
print the family.  Reading: the minimax-relative Chebyshev form on [a, b],

    1 - x P_n(x) = T_{n+1}(y(x)) / T_{n+1}(y0),
    y(x) = (b + a - 2x) / (b - a),   y0 = y(0) = (b + a) / (b - a),

so |1 - x P_n(x)| <= 1 / T_{n+1}(y0) on [a, b].  Its n roots are
z_k = ((b+a)/2)(1 - cos t_k) - i sqrt(ab) sin t_k, t_k = 2 pi k / (n+1),
k = 1..n (they depend on n only through n+1, hence P_{n1} | P_{n2} whenever
(n1+1) | (n2+1), matching the nested orders 4 -> 24/34/54 of Sec. 3.3).

The intermediate filter of the two-filter actions (Sec. 3.3, Q(K) = P_2/P_1;
Sec. 4.2, Q(J)) is the quotient P_{n2}/P_{n1}: the polynomial whose roots are
those of P_{n2} that are not roots of P_{n1}, with leading coefficient
c_{n2}/c_{n1}.  The functions below take n_div = n1 (0: no divisor).

Three evaluations are provided (closed form, real recurrence, root product) so
that they can be checked against each other; operator application uses the root
product, the direct consequence of the definition.
"""
from __future__ import annotations

import numpy as np


def cheb_T(m: int, y):
    """T_m(y) from its trigonometric / hyperbolic closed form."""
    y = np.asarray(y, dtype=float)
    out = np.empty_like(y)
    inside = np.abs(y) <= 1
    out[inside] = np.cos(m * np.arccos(y[inside]))
    big = y > 1
    out[big] = np.cosh(m * np.arccosh(y[big]))
    small = y < -1
    out[small] = (-1) ** m * np.cosh(m * np.arccosh(-y[small]))
    return out


def y_of_x(x, a, b):
    return (b + a - 2.0 * np.asarray(x, dtype=float)) / (b - a)


def p_closed(x, n, a, b):
    x = np.asarray(x, dtype=float)
    y0 = (b + a) / (b - a)
    return (1.0 - cheb_T(n + 1, y_of_x(x, a, b)) / cheb_T(n + 1, np.array(y0))) / x


def p_recurrence(x, n, a, b):
    """P_n(x) = (2/(b-a)) e_{n+1}(y) / T_{n+1}(y0), where
    e_m(y) = (T_m(y0) - T_m(y)) / (y0 - y) obeys
    e_{m+1} = 2 y0 e_m + 2 T_m(y) - e_{m-1}, e_0 = 0, e_1 = 1."""
    y = y_of_x(x, a, b)
    y0 = (b + a) / (b - a)
    t_prev, t_cur = np.ones_like(y), y.copy()        # T_0, T_1
    e_prev, e_cur = np.zeros_like(y), np.ones_like(y)  # e_0, e_1
    T0_prev, T0_cur = 1.0, y0
    for m in range(1, n + 1):
        e_next = 2 * y0 * e_cur + 2 * t_cur - e_prev
        t_next = 2 * y * t_cur - t_prev
        T0_next = 2 * y0 * T0_cur - T0_prev
        e_prev, e_cur = e_cur, e_next
        t_prev, t_cur = t_cur, t_next
        T0_prev, T0_cur = T0_cur, T0_next
    return (2.0 / (b - a)) * e_cur / T0_cur


def roots(n, a, b) -> np.ndarray:
    k = np.arange(1, n + 1)
    th = 2 * np.pi * k / (n + 1)
    return 0.5 * (b + a) * (1 - np.cos(th)) - 1j * np.sqrt(a * b) * np.sin(th)


def lead_coeff(n, a, b) -> float:
    """c with P_n(x) = c prod_k (x - z_k) (leading coefficient of P_n)."""
    y0 = (b + a) / (b - a)
    return (-1) ** n * 2.0 ** n * (2.0 / (b - a)) ** (n + 1) / float(cheb_T(n + 1, np.array(y0)))


def p_roots(x, n, a, b):
    x = np.asarray(x, dtype=float)
    out = lead_coeff(n, a, b) * np.ones_like(x, dtype=complex)
    for z in roots(n, a, b):
        out = out * (x - z)
    return out.real


def max_rel_error(n, a, b) -> float:
    """sup over [a, b] of |1 - x P(x)| = 1 / T_{n+1}(y0)."""
    y0 = (b + a) / (b - a)
    return 1.0 / float(cheb_T(n + 1, np.array(y0)))


# ---------------------------------------------------------------- quotients P_n / P_{n_div}
def roots_of(n, a, b, n_div=0) -> np.ndarray:
    """Roots of P_n / P_{n_div}: the roots of P_n that are not roots of P_{n_div}."""
    z = roots(n, a, b)
    if not n_div:
        return z
    if n_div >= n or (n + 1) % (n_div + 1):
        raise ValueError("P_n_div divides P_n only when (n_div + 1) | (n + 1)")
    zd = roots(n_div, a, b)
    keep = np.array([w for w in z if np.abs(zd - w).min() > 1e-9 * b])
    if len(keep) != n - n_div:
        raise ValueError("root sets do not nest")
    return keep


def lead_of(n, a, b, n_div=0) -> float:
    """Leading coefficient of P_n / P_{n_div}."""
    return lead_coeff(n, a, b) / (lead_coeff(n_div, a, b) if n_div else 1.0)


def p_quotient_roots(x, n, a, b, n_div=0):
    """P_n(x) / P_{n_div}(x) as lead * prod (x - z) over roots_of (real x)."""
    x = np.asarray(x, dtype=float)
    out = lead_of(n, a, b, n_div) * np.ones_like(x, dtype=complex)
    for z in roots_of(n, a, b, n_div):
        out = out * (x - z)
    return out.real


# ---------------------------------------------------------------- operators
def q_roots(n, a, b, n_div=0) -> np.ndarray:
    """Roots of Q with P = Q^dag Q (P = P_n / P_{n_div}): those with negative imaginary part."""
    z = roots_of(n, a, b, n_div)
    if len(z) % 2:
        raise ValueError("P = Q^dag Q needs an even number of roots")
    q = z[z.imag < 0]
    if 2 * len(q) != len(z):
        raise ValueError("roots do not come in conjugate pairs")
    return q


def apply_P(apply_J, psi, n, a, b, n_div=0):
    out = psi.astype(np.complex128)
    for z in roots_of(n, a, b, n_div):
        out = apply_J(out) - z * out
    return lead_of(n, a, b, n_div) * out


def apply_Q(apply_J, psi, n, a, b, dagger=False, n_div=0):
    out = psi.astype(np.complex128)
    for z in q_roots(n, a, b, n_div):
        zz = np.conj(z) if dagger else z
        out = apply_J(out) - zz * out
    return np.sqrt(lead_of(n, a, b, n_div)) * out


def apply_PJ(apply_J, psi, n, a, b, n_div=0):
    return apply_P(apply_J, apply_J(psi), n, a, b, n_div)
