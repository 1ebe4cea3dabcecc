"""Pins for the oracle's CG and Chebyshev filter polynomial."""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import poly, solver, wilson as wl


def test_cg_matches_dense_solve():
    L, kappa, mu2 = (4, 4, 2, 4), 0.155, 0.05
    U = li.random_links(L, 0.447, 31)
    Vh = li.volume(L) // 2
    b = li.gaussian_spinor((Vh, 4, 3), 2001)
    A = lambda v: wl.J(U, v, L, kappa, mu2)
    x, it, res = solver.cg(A, b, tol=1e-12)
    assert res <= 1e-12 and it > 5
    Jd = wl.dense(A, Vh)
    xd = np.linalg.solve(Jd, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_cg_maxiter_reports_nonconvergence():
    L = (4, 2, 2, 4)
    U = li.random_links(L, 0.447, 31)
    b = li.gaussian_spinor((li.volume(L) // 2, 4, 3), 1)
    x, it, res = solver.cg(lambda v: wl.Khat(U, v, L, 0.155), b, tol=1e-12, maxiter=2)
    assert it == 2 and res > 1e-12


A, B, N = 0.001, 8.0, 16


def test_three_polynomial_evaluations_agree():
    x = np.geomspace(A, B, 2001)
    pc = poly.p_closed(x, N, A, B)
    pr = poly.p_recurrence(x, N, A, B)
    pz = poly.p_roots(x, N, A, B)
    assert np.abs(pr / pc - 1).max() < 1e-11
    assert np.abs(pz / pc - 1).max() < 1e-11


def test_chebyshev_T_recurrence_vs_closed_form():
    y = np.linspace(-3, 3, 301)
    t0, t1 = np.ones_like(y), y.copy()
    for m in range(2, 20):
        t0, t1 = t1, 2 * y * t1 - t0
        assert np.allclose(poly.cheb_T(m, y), t1, rtol=1e-12, atol=1e-12)


def test_minimax_relative_error_equioscillates():
    """|1 - x P(x)| <= 1/T_{n+1}(y0) on [a, b], attained at the n+2 Chebyshev extrema."""
    bound = poly.max_rel_error(N, A, B)
    assert abs(bound - 0.931853) < 1e-6
    x = np.linspace(A, B, 200001)
    err = np.abs(1 - x * poly.p_closed(x, N, A, B))
    assert err.max() <= bound * (1 + 1e-12)
    k = np.arange(N + 2)
    xk = 0.5 * (B + A) - 0.5 * (B - A) * np.cos(np.pi * k / (N + 1))
    assert np.allclose(np.abs(1 - xk * poly.p_closed(xk, N, A, B)), bound, rtol=1e-9)


def test_positivity_and_factorisation():
    x = np.geomspace(1e-6, 50, 5001)
    P = poly.p_closed(x, N, A, B)
    assert (P > 0).all()
    c = poly.lead_coeff(N, A, B)
    assert abs(c - 3.5623e-6) / 3.5623e-6 < 1e-4
    Q = np.sqrt(c) * np.prod(x[:, None] - poly.q_roots(N, A, B)[None], axis=1)
    # against the root product everywhere; against the closed form away from
    # x -> 0, where 1 - T(y)/T(y0) cancels
    assert np.allclose(np.abs(Q) ** 2, poly.p_roots(x, N, A, B), rtol=1e-13)
    far = x > 1e-3
    assert np.allclose(np.abs(Q[far]) ** 2, P[far], rtol=1e-11)


@pytest.mark.parametrize("n2", [24, 34, 54])
def test_nested_orders_divide(n2):
    """P_4 | P_{n2} when 5 | n2 + 1 (the 2PF orders of Sec. 3.3)."""
    r4 = poly.roots(4, A, B)
    rn = poly.roots(n2, A, B)
    for z in r4:
        assert np.abs(rn - z).min() < 1e-12


def test_operator_application_matches_spectral_definition():
    """P(J) psi via roots equals V f(Lambda) V^dag psi with f the closed form."""
    L, kappa, mu2 = (4, 2, 2, 4), 0.155, 0.05
    U = li.random_links(L, 0.447, 41)
    Vh = li.volume(L) // 2
    Jop = lambda v: wl.J(U, v, L, kappa, mu2)
    Jd = wl.dense(Jop, Vh)
    lam, vec = np.linalg.eigh(Jd)
    assert lam.min() > A and lam.max() < B
    psi = li.gaussian_spinor((Vh, 4, 3), 3).reshape(-1)
    ref = vec @ (poly.p_closed(lam, N, A, B) * (vec.conj().T @ psi))
    got = poly.apply_P(Jop, psi.reshape(Vh, 4, 3), N, A, B).reshape(-1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    # P = Q^dag Q and Pi = P(J) J
    q = poly.apply_Q(Jop, psi.reshape(Vh, 4, 3), N, A, B)
    qq = poly.apply_Q(Jop, q, N, A, B, dagger=True).reshape(-1)
    assert np.linalg.norm(qq - ref) / np.linalg.norm(ref) < 1e-12
    pij = poly.apply_PJ(Jop, psi.reshape(Vh, 4, 3), N, A, B).reshape(-1)
    refpj = vec @ (lam * poly.p_closed(lam, N, A, B) * (vec.conj().T @ psi))
    assert np.linalg.norm(pij - refpj) / np.linalg.norm(refpj) < 1e-12


def test_multishift_cg_matches_dense_solves_per_shift():
    """One Krylov space for every shift: each x_s solves (A + s) x_s = b (dense solve),
    in any shift order; the smallest shift's iterate is plain CG's, bit for bit."""
    L, kappa = (4, 4, 2, 4), 0.155
    U = li.random_links(L, 0.447, 31)
    Vh = li.volume(L) // 2
    b = li.gaussian_spinor((Vh, 4, 3), 2002)
    A = lambda v: wl.Khat(U, v, L, kappa)
    shifts = [0.5, 0.0, 0.05, 0.005]
    xs, it, res = solver.cg_multishift(A, b, shifts, tol=1e-12)
    assert max(res) <= 1e-12 * 1.5 and it > 10
    Kd = wl.dense(A, Vh)
    for s, x in zip(shifts, xs):
        xd = np.linalg.solve(Kd + s * np.eye(Kd.shape[0]), b.reshape(-1)).reshape(b.shape)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10, s
    x0, it0, _ = solver.cg(A, b, tol=1e-12)
    assert it0 == it and np.array_equal(xs[1], x0)
    # a zero source gives zero solutions
    zs, zit, zres = solver.cg_multishift(A, np.zeros_like(b), shifts)
    assert zit == 0 and all(np.abs(z).max() == 0 for z in zs)
