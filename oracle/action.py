"""Pseudofermion action terms: value, heatbath and force (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2 gives the two-flavour action phi^dag K^-1 phi, its mass-preconditioned
split phi1^dag J^-1 phi1 + phi2^dag J K^-1 phi2 and the polynomial-filtered
split phi1^dag P(K) phi1 + phi2^dag [P(K) K]^-1 phi2; Sec. 4.1 combines them
(PF-MP): phi1^dag P(J) phi1 + phi2^dag [P(J) J]^-1 phi2 + phi3^dag J K^-1 phi3.
Heatbaths draw phi from Gaussian chi with density exp(-chi^dag chi).

Readings (the paper prints no formulas for these):

* every term has its operator J = K-hat(kappa) + mu^2 on the even sites: the
  paper's Hasenbusch matrix J = K(kappa') is kappa = kappa', mu^2 = 0; the
  mu^2 form shifts K-hat instead.  W = M-hat(kappa) + i mu g5 has W^dag W = J,
  and P(J), Q(J), J commute;
* a correction term J_n J_d^-1 (Sec. 2: J K^-1; Sec. 3.3: J_1 J_2^-1,
  J_2 K^-1) is taken in its Hermitian form with the same determinant:
  RATIO, phi^dag W_n J^-1 W_n^dag phi, with the numerator W_n = M-hat(kappa_n)
  + i mu_n g5 (kappa_n = kappa_num, or kappa when 0; mu_n^2 = mu2_num) and
  the term's J as denominator;
* P is P_n, or the quotient P_n / P_{n_div} of the two-filter actions
  (Sec. 3.3 Q(K) = P_2/P_1, Sec. 4.2 Q(J)); P = Q^dag Q with Q = sqrt(c)
  prod (J - z_k) over P's roots of negative imaginary part (see ``poly``).

Term kinds and heatbaths (given chi), W_d = W of the term's J:

    KINV_FULL  phi^dag K^-1 phi, full lattice     phi = M^dag chi
    KINV       phi^dag J^-1 phi                    phi = W^dag chi
    RATIO      phi^dag W_n J^-1 W_n^dag phi        phi = W_n J_n^-1 W_d^dag chi
    POLY       phi^dag P(J) phi                    phi = Q^dag P(J)^-1 chi
    POLYK_INV  phi^dag [P(J) J]^-1 phi             phi = Q^dag W^dag chi

Forces are the Lie derivatives grad^a S = d/de S(exp(i e T^a) U_mu(x))|_0,
shape [4, V, 8], from the product rule applied to each action with
``force.bilinear_grad`` as the only link-derivative primitive.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lattice as lat
from . import poly
from . import solver
from . import wilson as wl
from .force import bilinear_grad


@dataclass
class Term:
    kind: str                 # KINV_FULL | KINV | RATIO | POLY | POLYK_INV
    kappa: float
    mu2: float = 0.0
    n: int = 0                # polynomial order
    a: float = 0.001          # polynomial interval [a, b]
    b: float = 8.0
    tol: float = 1e-12        # CG tolerance of the solves inside the term
    n_div: int = 0            # P = P_n / P_{n_div} (0: P_n)
    kappa_num: float = 0.0    # RATIO numerator kappa (0: kappa)
    mu2_num: float = 0.0      # RATIO numerator shift

    @property
    def kn(self) -> float:
        return self.kappa_num or self.kappa


class Ops:
    """Operators of one lattice: U, L, t_bc bound once."""

    def __init__(self, U, L, t_bc=-1):
        self.U, self.L, self.t_bc = U, tuple(L), t_bc

    # full lattice
    def M(self, psi, kappa, dagger=False):
        return wl.M(self.U, psi, self.L, kappa, self.t_bc, dagger)

    def K(self, psi, kappa):
        return wl.K(self.U, psi, self.L, kappa, self.t_bc)

    # even sites
    def Mhat(self, psi, kappa, dagger=False):
        return wl.Mhat(self.U, psi, self.L, kappa, self.t_bc, dagger)

    def Khat(self, psi, kappa):
        return wl.Khat(self.U, psi, self.L, kappa, self.t_bc)

    def J(self, psi, kappa, mu2):
        return wl.J(self.U, psi, self.L, kappa, mu2, self.t_bc)

    def W(self, psi, kappa, mu2, dagger=False):
        return wl.W(self.U, psi, self.L, kappa, np.sqrt(mu2), self.t_bc, dagger)

    # link derivatives
    def grad_re_dMhat(self, A, B, kappa):
        """Coefficients of Re(A^dag dM-hat B), A and B on even sites.

        dM-hat = -kappa^2 (dD_eo D_oe + D_eo dD_oe), so with
        A' = A + (D^dag)_oe A and B' = B + D_oe B (odd parts added) this is
        -kappa^2 times one full-lattice bilinear.
        """
        L = self.L
        Ah = lat.embed(A, L, 0) + lat.embed(wl.hop_eo(self.U, A, L, 1, self.t_bc, dagger=True), L, 1)
        Bh = lat.embed(B, L, 0) + lat.embed(wl.hop_eo(self.U, B, L, 1, self.t_bc), L, 1)
        return -kappa ** 2 * bilinear_grad(self.U, Ah, Bh, L, self.t_bc)

    def grad_re_dJ(self, Lv, Rv, kappa):
        """Coefficients of Re(Lv^dag dJ Rv), dJ = dM-hat^dag M-hat + M-hat^dag dM-hat."""
        return (self.grad_re_dMhat(self.Mhat(Rv, kappa), Lv, kappa)
                + self.grad_re_dMhat(self.Mhat(Lv, kappa), Rv, kappa))


def _inv(apply_A, b, tol):
    x, _, _ = solver.cg(apply_A, b, tol=tol)
    return x


# ---------------------------------------------------------------- action values
def action(ops: Ops, t: Term, phi) -> float:
    k, m2 = t.kappa, t.mu2
    J = lambda v: ops.J(v, k, m2)
    if t.kind == "KINV_FULL":
        return solver.vdot(phi, _inv(lambda v: ops.K(v, k), phi, t.tol)).real
    if t.kind == "KINV":
        return solver.vdot(phi, _inv(J, phi, t.tol)).real
    if t.kind == "RATIO":
        v = ops.W(phi, t.kn, t.mu2_num, dagger=True)
        return solver.vdot(v, _inv(J, v, t.tol)).real
    if t.kind == "POLY":
        return solver.vdot(phi, poly.apply_P(J, phi, t.n, t.a, t.b, t.n_div)).real
    if t.kind == "POLYK_INV":
        Pi = lambda v: poly.apply_PJ(J, v, t.n, t.a, t.b, t.n_div)
        return solver.vdot(phi, _inv(Pi, phi, t.tol)).real
    raise ValueError(t.kind)


# ---------------------------------------------------------------- heatbaths
def heatbath(ops: Ops, t: Term, chi):
    k, m2 = t.kappa, t.mu2
    J = lambda v: ops.J(v, k, m2)
    if t.kind == "KINV_FULL":
        return ops.M(chi, k, dagger=True)
    if t.kind == "KINV":
        return ops.W(chi, k, m2, dagger=True)
    if t.kind == "RATIO":
        Jn = lambda v: ops.J(v, t.kn, t.mu2_num)
        return ops.W(_inv(Jn, ops.W(chi, k, m2, dagger=True), t.tol), t.kn, t.mu2_num)
    if t.kind == "POLY":
        Pinv_chi = _inv(lambda v: poly.apply_P(J, v, t.n, t.a, t.b, t.n_div), chi, t.tol)
        return poly.apply_Q(J, Pinv_chi, t.n, t.a, t.b, dagger=True, n_div=t.n_div)
    if t.kind == "POLYK_INV":
        return poly.apply_Q(J, ops.W(chi, k, m2, dagger=True), t.n, t.a, t.b, dagger=True, n_div=t.n_div)
    raise ValueError(t.kind)


# ---------------------------------------------------------------- forces
def _chain_grad(ops, t, right, left_top):
    """sum_k Re(L_k^dag dJ R_k) for the factors (J - z_k), k = 1..n/2, of Q:
    R_k = prod_{j<k} (J - z_j) right,  L_k = prod_{j>k} (J - conj z_j) left_top."""
    k, m2 = t.kappa, t.mu2
    J = lambda v: ops.J(v, k, m2)
    z = poly.q_roots(t.n, t.a, t.b, t.n_div)
    m = len(z)
    R = [right]
    for j in range(m - 1):
        R.append(J(R[-1]) - z[j] * R[-1])
    g = 0.0
    Lv = left_top
    for kk in range(m - 1, -1, -1):
        g = g + ops.grad_re_dJ(Lv, R[kk], k)
        Lv = J(Lv) - np.conj(z[kk]) * Lv
    return g


def force(ops: Ops, t: Term, phi) -> np.ndarray:
    """grad^a S_term, shape [4, V, 8]."""
    k, m2 = t.kappa, t.mu2
    J = lambda v: ops.J(v, k, m2)
    if t.kind == "KINV_FULL":
        X = _inv(lambda v: ops.K(v, k), phi, t.tol)
        Y = ops.M(X, k)
        # dS = -X^dag dK X = -2 Re(Y^dag dM X),  dM = -kappa dD
        return 2.0 * k * bilinear_grad(ops.U, Y, X, ops.L, ops.t_bc)
    if t.kind == "KINV":
        X = _inv(J, phi, t.tol)
        return -2.0 * ops.grad_re_dMhat(ops.Mhat(X, k), X, k)
    if t.kind == "RATIO":
        v = ops.W(phi, t.kn, t.mu2_num, dagger=True)
        X = _inv(J, v, t.tol)
        # S = v^dag X, v = W_n^dag phi:
        # dS = 2 Re(phi^dag dM-hat(kappa_n) X) - 2 Re(Y^dag dM-hat(kappa) X), Y = W X
        return (2.0 * ops.grad_re_dMhat(phi, X, t.kn)
                - 2.0 * ops.grad_re_dMhat(ops.W(X, k, m2), X, k))
    if t.kind == "POLY":
        sc = np.sqrt(poly.lead_of(t.n, t.a, t.b, t.n_div))
        psi = poly.apply_Q(J, phi, t.n, t.a, t.b, n_div=t.n_div)
        return 2.0 * sc * _chain_grad(ops, t, phi, psi)
    if t.kind == "POLYK_INV":
        sc = np.sqrt(poly.lead_of(t.n, t.a, t.b, t.n_div))
        X = _inv(lambda v: poly.apply_PJ(J, v, t.n, t.a, t.b, t.n_div), phi, t.tol)
        QX = poly.apply_Q(J, X, t.n, t.a, t.b, n_div=t.n_div)
        g = 2.0 * sc * _chain_grad(ops, t, X, J(QX)) + ops.grad_re_dJ(QX, QX, k)
        return -g
    raise ValueError(t.kind)
