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
    "RATIO": act.Term("RATIO", 0.155, mu2_num=0.05, tol=1e-14),
    "POLY": act.Term("POLY", 0.155, mu2=0.05, n=4, tol=1e-14),
    "POLYK_INV": act.Term("POLYK_INV", 0.155, mu2=0.05, n=4, tol=1e-14),
    # the paper's kappa' form J = K-hat(kappa') and the nested / two-filter terms
    "RATIO_KAPPA": act.Term("RATIO", 0.155, kappa_num=0.150, tol=1e-14),        # J K^-1
    "RATIO_NESTED": act.Term("RATIO", 0.150, kappa_num=0.145, tol=1e-14),       # J_1 J_2^-1
    "RATIO_SHIFTS": act.Term("RATIO", 0.155, mu2=0.005, mu2_num=0.05, tol=1e-14),
    "POLY_QUOTIENT": act.Term("POLY", 0.150, n=24, n_div=4, tol=1e-12),         # Q(J) = P_24 / P_4
    "POLYK_INV_KAPPA": act.Term("POLYK_INV", 0.150, n=4, tol=1e-14),
}


def _phi(term, L=L4):
    V = li.volume(L)
    if term.kind == "KINV_FULL":
        return li.gaussian_spinor((V, 4, 3), 2001)
    return li.gaussian_spinor((V // 2, 4, 3), 2001)


@pytest.mark.parametrize("name", ["KINV_FULL"] + list(TERMS))
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
    term = act.Term("RATIO", 0.155, mu2_num=0.05, tol=1e-14)
    phi = _phi(term, L)
    V = li.volume(L)
    G = li.random_su3_field(V, 12)
    Ug = np.stack([np.einsum("xab,xbc,xdc->xad", G, U[m], np.conj(lat.shift(G, L, m, +1))) for m in range(4)])
    Ge = G[lat.parity_sites(L, 0)]
    F0 = su3.coeffs_to_matrix(act.force(act.Ops(U, L), term, phi))
    F1 = su3.coeffs_to_matrix(act.force(act.Ops(Ug, L), term, np.einsum("xab,xsb->xsa", Ge, phi)))
    rot = np.einsum("xab,mxbc,xdc->mxad", G, F0, np.conj(G))
    assert np.abs(F1 - rot).max() < 1e-10 * np.abs(F0).max()


@pytest.mark.parametrize("name", list(TERMS))
def test_heatbath_gives_S_equal_chi_norm(name):
    term = TERMS[name]
    L = L4 if name in ("KINV", "RATIO", "POLY", "POLYK_INV") else (4, 2, 2, 4)
    U = _links(L)
    ops = act.Ops(U, L)
    chi = li.gaussian_spinor((li.volume(L) // 2, 4, 3), 3001)
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


# ---------------------------------------------------------------- the paper's actions
K, KP, K1, K2, MU2 = 0.155, 0.150, 0.145, 0.150, 0.05


def T(kind, kappa, **kw):
    return act.Term(kind, kappa, tol=1e-13, **kw)


# Sec. 2 (MP, PF), Sec. 3.3 (2PF, 2MP), Sec. 4.1 (PF-MP, kappa' and mu^2 forms),
# Sec. 4.2 (1PF-2MP, 2PF-1MP); kappa' < kappa (the reading of Sec. 4.1's sign)
PAPER_ACTIONS = {
    "MP": [T("KINV", KP), T("RATIO", K, kappa_num=KP)],
    "PF": [T("POLY", K, n=4), T("POLYK_INV", K, n=4)],
    "2PF": [T("POLY", K, n=4), T("POLY", K, n=24, n_div=4), T("POLYK_INV", K, n=24)],
    "2MP": [T("KINV", K1), T("RATIO", K2, kappa_num=K1), T("RATIO", K, kappa_num=K2)],
    "PF-MP": [T("POLY", KP, n=4), T("POLYK_INV", KP, n=4), T("RATIO", K, kappa_num=KP)],
    "PF-MP-mu2": [T("POLY", K, mu2=MU2, n=4), T("POLYK_INV", K, mu2=MU2, n=4), T("RATIO", K, mu2_num=MU2)],
    "1PF-2MP": [T("POLY", K1, n=4), T("POLYK_INV", K1, n=4), T("RATIO", K2, kappa_num=K1),
                T("RATIO", K, kappa_num=K2)],
    "2PF-1MP": [T("POLY", KP, n=4), T("POLY", KP, n=24, n_div=4), T("POLYK_INV", KP, n=24),
                T("RATIO", K, kappa_num=KP)],
}


def _dense_term(ops, t, Vh):
    """The term's kernel A (S = phi^dag A phi) from dense operator matrices; polynomials
    through the eigendecomposition of J and the closed form of P_n (not its roots)."""
    Jd = wl.dense(lambda v: ops.J(v, t.kappa, t.mu2), Vh)
    if t.kind == "KINV":
        return np.linalg.inv(Jd)
    if t.kind == "RATIO":
        Wn = wl.dense(lambda v: ops.W(v, t.kappa_num or t.kappa, t.mu2_num), Vh)
        return Wn @ np.linalg.inv(Jd) @ Wn.conj().T
    lam, Vec = np.linalg.eigh(Jd)
    p = poly.p_closed(lam, t.n, t.a, t.b)
    if t.n_div:
        p = p / poly.p_closed(lam, t.n_div, t.a, t.b)
    if t.kind == "POLY":
        return (Vec * p) @ Vec.conj().T
    if t.kind == "POLYK_INV":
        return (Vec / (p * lam)) @ Vec.conj().T
    raise ValueError(t.kind)


@pytest.mark.parametrize("name", list(PAPER_ACTIONS))
def test_paper_actions_reproduce_det_Khat(name):
    """Each action's Gaussian integral gives det K-hat(kappa): sum_i log det A_i = -log det K-hat,
    and the oracle's matrix-free action values equal phi^dag A_i phi."""
    L = (2, 2, 2, 4)
    U = _links(L, seed=77)
    Vh = li.volume(L) // 2
    ops = act.Ops(U, L)
    dK = np.linalg.slogdet(wl.dense(lambda v: ops.Khat(v, K), Vh))[1]
    total = 0.0
    phi = li.gaussian_spinor((Vh, 4, 3), 2101)
    for t in PAPER_ACTIONS[name]:
        A = _dense_term(ops, t, Vh)
        sign, ld = np.linalg.slogdet(A)
        assert abs(sign - 1) < 1e-9          # Hermitian positive definite
        total += ld
        S_dense = np.vdot(phi.reshape(-1), A @ phi.reshape(-1)).real
        assert abs(act.action(ops, t, phi) - S_dense) <= 1e-9 * abs(S_dense), (name, t.kind)
    assert abs(total + dK) <= 1e-8 * abs(dK), (total, -dK)


def test_quotient_polynomial_closed_form_and_roots():
    """P_24 / P_4 (Sec. 3.3 nesting): 20 roots, in conjugate pairs, values equal the quotient
    of the closed forms, and |Q(x)|^2 = P(x) on the real axis."""
    a, b = 0.001, 8.0
    z = poly.roots_of(24, a, b, 4)
    assert len(z) == 20 and len(poly.q_roots(24, a, b, 4)) == 10
    assert max(np.abs(z - np.conj(w)).min() for w in z) < 1e-12
    x = np.geomspace(2e-3, 7.9, 401)
    ref = poly.p_closed(x, 24, a, b) / poly.p_closed(x, 4, a, b)
    assert np.abs(poly.p_quotient_roots(x, 24, a, b, 4) / ref - 1).max() < 1e-10
    q = np.sqrt(poly.lead_of(24, a, b, 4)) * np.prod([x - w for w in poly.q_roots(24, a, b, 4)], axis=0)
    assert np.abs(np.abs(q) ** 2 / ref - 1).max() < 1e-10
    with pytest.raises(ValueError):
        poly.roots_of(24, a, b, 6)       # 7 does not divide 25


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 10)])
def test_bilinear_at_sampled_links_matches_whole_lattice(L):
    """The link-by-link evaluation (used on large lattices at sampled links) equals the
    whole-lattice bilinear derivative at every link, time wrap included."""
    from oracle import force as ofo
    U = _links(L)
    V = li.volume(L)
    A = li.gaussian_spinor((V, 4, 3), 71)
    C = li.gaussian_spinor((V, 4, 3), 72)
    whole = ofo.bilinear_grad(U, A, C, L)
    links = [(mu, x) for mu in range(4) for x in range(V)]
    at = ofo.bilinear_grad_at(U, A, C, L, links).reshape(4, V, 8)
    assert np.max(np.abs(at - whole)) <= 1e-13 * np.max(np.abs(whole))


def test_bilinear_at_matches_finite_differences_of_the_hop():
    """d/de Re(A^dag D(U') C), U'_mu(x) = exp(i e T^a) U_mu(x) at single links (one of
    them crossing the antiperiodic time edge), by central differences of the oracle's
    hop: pins the per-link evaluation on its own."""
    from oracle import force as ofo
    L = L4
    U = _links(L)
    V = li.volume(L)
    A = li.gaussian_spinor((V, 4, 3), 73)
    C = li.gaussian_spinor((V, 4, 3), 74)
    T = lat.generators()
    x_edge = 1 + L[0] * (2 + L[1] * (3 + L[2] * (L[3] - 1)))   # t = Lt - 1: its t link wraps
    links = [(0, 5), (1, 77), (2, 130), (3, 200), (3, x_edge)]
    got = ofo.bilinear_grad_at(U, A, C, L, links)
    eps = 1e-6
    for i, (mu, x) in enumerate(links):
        for a in (0, 3, 7):
            vals = []
            for s in (+1, -1):
                Up = U.copy()
                Up[mu][x] = su3.expi(s * eps, T[a]) @ U[mu][x]
                vals.append(np.vdot(A, wl.hop(Up, C, L)).real)
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - got[i, a]) <= 1e-6 * max(1.0, abs(got[i, a])), (mu, x, a, fd, got[i, a])
