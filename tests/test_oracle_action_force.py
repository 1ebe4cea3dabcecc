"""Pins for the oracle's action terms, heatbaths and forces.

Forces are checked against central finite differences of the oracle's own
action values along random su(3) directions of every link (the action is a
different code path: solves and products, no bilinear), against gauge
covariance, and the heatbaths against S(phi) = chi^dag chi.  The determinant
bookkeeping of the filtered actions is checked by dense log-determinants.
"""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import action as act, gauge, lattice as lat, poly, su3, wilson as wl

L4 = (4, 4, 4, 4)


def _links(L=L4, a=0.447, seed=1003):
    return li.random_links(L, a, seed)


def _rotate(U, omega, eps):
    """U_mu(x) -> exp(i eps sum_a omega^a T^a) U_mu(x) for all links."""
    R = su3.expi(eps, su3.coeffs_to_matrix(omega))
    return np.einsum("mxab,mxbc->mxac", R, U)


TERMS = {
    "KINV": act.Term("KINV", 0.155, mu2=0.05, tol=1e-14),
    "RATIO": act.Term("RATIO", 0.155, mu2=0.05, tol=1e-14),
    "POLY": act.Term("POLY", 0.155, mu2=0.05, n=4, tol=1e-14),
    "POLYK_INV": act.Term("POLYK_INV", 0.155, mu2=0.05, n=4, tol=1e-14),
}


def _phi(term, L=L4):
    V = li.volume(L)
    if term.kind == "KINV_FULL":
        return li.gaussian_spinor((V, 4, 3), 2001)
    return li.gaussian_spinor((V // 2, 4, 3), 2001)


@pytest.mark.parametrize("name", ["KINV_FULL", "KINV", "RATIO", "POLY", "POLYK_INV"])
def test_force_matches_finite_differences(name):
    if name == "KINV_FULL":
        term = act.Term("KINV_FULL", 0.12, tol=1e-14)
        U = _links(a=0.3)
    else:
        term = TERMS[name]
        U = _links()
    phi = _phi(term)
    F = act.force(act.Ops(U, L4), term, phi)
    omega = np.random.default_rng(7).standard_normal((4, li.volume(L4), 8))
    eps = 1e-5
    Sp = act.action(act.Ops(_rotate(U, omega, eps), L4), term, phi)
    Sm = act.action(act.Ops(_rotate(U, omega, -eps), L4), term, phi)
    fd = (Sp - Sm) / (2 * eps)
    an = float(np.sum(omega * F))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # single link, single generator: a local check that the sum above does not mask
    om1 = np.zeros_like(omega)
    om1[3, 17, 5] = 1.0          # a time link
    om1[3, 17 + 64 * 3, 2] = 0.7  # a time link crossing the antiperiodic wrap
    Sp = act.action(act.Ops(_rotate(U, om1, eps), L4), term, phi)
    Sm = act.action(act.Ops(_rotate(U, om1, -eps), L4), term, phi)
    assert abs((Sp - Sm) / (2 * eps) - np.sum(om1 * F)) <= 1e-6 * max(1.0, np.abs(F).max())


def test_gauge_force_matches_finite_differences_and_vanishes_at_unit_links():
    U = _links(a=0.447)
    beta = 5.6
    F = gauge.force(U, L4, beta)
    omega = np.random.default_rng(8).standard_normal(F.shape)
    eps = 1e-5
    fd = (gauge.action(_rotate(U, omega, eps), L4, beta) - gauge.action(_rotate(U, omega, -eps), L4, beta)) / (2 * eps)
    assert abs(fd - np.sum(omega * F)) <= 1e-6 * abs(fd)
    assert np.abs(gauge.force(li.unit_links(L4), L4, beta)).max() == 0.0


def test_force_gauge_covariance():
    """U -> G U G(x+mu)^dag, phi -> G phi: F_mu(x) -> G(x) F_mu(x) G(x)^dag."""
    L = (4, 4, 2, 4)
    U = _links(L)
    term = act.Term("RATIO", 0.155, mu2=0.05, tol=1e-14)
    phi = _phi(term, L)
    V = li.volume(L)
    G = li.random_su3_field(V, 12)
    Ug = np.stack([np.einsum("xab,xbc,xdc->xad", G, U[m], np.conj(lat.shift(G, L, m, +1))) for m in range(4)])
    Ge = G[lat.parity_sites(L, 0)]
    F0 = su3.coeffs_to_matrix(act.force(act.Ops(U, L), term, phi))
    F1 = su3.coeffs_to_matrix(act.force(act.Ops(Ug, L), term, np.einsum("xab,xsb->xsa", Ge, phi)))
    rot = np.einsum("xab,mxbc,xdc->mxad", G, F0, np.conj(G))
    assert np.abs(F1 - rot).max() < 1e-10 * np.abs(F0).max()


@pytest.mark.parametrize("name", ["KINV", "RATIO", "POLY", "POLYK_INV"])
def test_heatbath_gives_S_equal_chi_norm(name):
    term = TERMS[name]
    U = _links()
    ops = act.Ops(U, L4)
    chi = li.gaussian_spinor((li.volume(L4) // 2, 4, 3), 3001)
    phi = act.heatbath(ops, term, chi)
    S = act.action(ops, term, phi)
    assert abs(S - np.vdot(chi, chi).real) < 1e-10 * S


def test_heatbath_full_lattice_two_flavour():
    U = _links(a=0.3)
    ops = act.Ops(U, L4)
    term = act.Term("KINV_FULL", 0.12, tol=1e-14)
    chi = li.gaussian_spinor((li.volume(L4), 4, 3), 3002)
    S = act.action(ops, term, act.heatbath(ops, term, chi))
    assert abs(S - np.vdot(chi, chi).real) < 1e-10 * S


def test_filtered_actions_reproduce_det_Khat():
    """PF-MP bookkeeping (Sec. 4.1): det P(J)^-1 det[P(J) J] det(W K^-1 W^dag)^-1 = det K-hat
    (the Gaussian integral of exp(-phi^dag A phi) gives 1/det A)."""
    L, kappa, mu2, n = (2, 2, 2, 4), 0.155, 0.05, 6
    U = _links(L, seed=77)
    Vh = li.volume(L) // 2
    ops = act.Ops(U, L)
    J = lambda v: ops.J(v, kappa, mu2)
    dP = np.linalg.slogdet(wl.dense(lambda v: poly.apply_P(J, v, n, 0.001, 8.0), Vh))[1]
    dPJ = np.linalg.slogdet(wl.dense(lambda v: poly.apply_PJ(J, v, n, 0.001, 8.0), Vh))[1]
    Kh = wl.dense(lambda v: ops.Khat(v, kappa), Vh)
    Wd = wl.dense(lambda v: ops.W(v, kappa, mu2), Vh)
    dR = np.linalg.slogdet(Wd @ np.linalg.inv(Kh) @ Wd.conj().T)[1]
    dK = np.linalg.slogdet(Kh)[1]
    assert abs((-dP + dPJ - dR) - dK) < 1e-9 * abs(dK) + 1e-9
    # W^dag W = J
    Jd = wl.dense(J, Vh)
    assert np.abs(Wd.conj().T @ Wd - Jd).max() < 1e-13
