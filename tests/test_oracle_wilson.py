"""Pins for the oracle's Wilson operator, even-odd Schur complement and K-hat.

Each test checks the oracle against something the mathematics fixes:
free-field closed forms, gamma5-hermiticity, gauge covariance, the norm
bound, the Schur-complement determinant identity and the adjoint.
"""
import itertools

import numpy as np
import pytest

import lattice_inputs as li
from oracle import lattice as lat, wilson as wl


def plane_wave(L, n, u):
    """psi(x) = exp(i p.x) u with p_mu = 2 pi n_mu / L_mu (space), (2 n_t + 1) pi / Lt (time)."""
    x, y, z, t = lat.coords(L)
    p = np.array([2 * np.pi * n[0] / L[0], 2 * np.pi * n[1] / L[1], 2 * np.pi * n[2] / L[2],
                  (2 * n[3] + 1) * np.pi / L[3]])
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[:, None, None] * u[None], p


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 2, 6, 8), (16, 16, 16, 32)])
def test_free_field_plane_wave(L):
    """U = 1: D e^{ipx} u = sum_mu (2 cos p_mu - 2 i g_mu sin p_mu) u e^{ipx} (antiperiodic t)."""
    rng = np.random.default_rng(5)
    U = li.unit_links(L)
    g = lat.gammas()
    for _ in range(2 if L[0] < 16 else 1):
        n = [int(rng.integers(0, L[m])) for m in range(4)]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p = plane_wave(L, n, u)
        Dk = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * g[m] for m in range(4))
        expect = np.einsum("st,xtc->xsc", Dk, psi)
        got = wl.hop(U, psi, L, t_bc=-1)
        assert np.abs(got - expect).max() < 1e-12


def _free_momenta(L):
    for n in itertools.product(*[range(l) for l in L]):
        yield np.array([2 * np.pi * n[0] / L[0], 2 * np.pi * n[1] / L[1], 2 * np.pi * n[2] / L[2],
                        (2 * n[3] + 1) * np.pi / L[3]])


def test_free_field_spectrum_full_K():
    """eig K = (1 - 2 kappa sum cos p)^2 + 4 kappa^2 sum sin^2 p, 12-fold."""
    L, kappa = (4, 2, 2, 4), 0.12
    U = li.unit_links(L)
    V = li.volume(L)
    Kd = wl.dense(lambda v: wl.K(U, v, L, kappa), V)
    ev = np.linalg.eigvalsh(Kd)
    closed = []
    for p in _free_momenta(L):
        closed += [(1 - 2 * kappa * np.cos(p).sum()) ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum()] * 12
    assert np.abs(np.sort(closed) - ev).max() < 1e-13


def test_free_field_spectrum_even_odd_Khat():
    """eig K-hat = |1 - 4 kappa^2 (c +- i |s|)^2|^2, 6-fold per sign, p ~ p + (pi,pi,pi,pi)."""
    L, kappa = (4, 4, 2, 4), 0.155
    U = li.unit_links(L)
    Kd = wl.dense(lambda v: wl.Khat(U, v, L, kappa), li.volume(L) // 2)
    ev = np.linalg.eigvalsh(Kd)
    closed = []
    for p in _free_momenta(L):
        c, s = np.cos(p).sum(), np.sqrt((np.sin(p) ** 2).sum())
        for sg in (+1, -1):
            closed += [abs(1 - 4 * kappa ** 2 * (c + sg * 1j * s) ** 2) ** 2] * 6
    assert np.abs(np.sort(closed) - np.repeat(ev, 2)).max() < 1e-13


def test_gamma5_hermiticity_and_adjoint():
    L = (4, 4, 4, 4)
    U = li.random_links(L, 0.3, 1001)
    V = li.volume(L)
    eta = li.gaussian_spinor((V, 4, 3), 1)
    psi = li.gaussian_spinor((V, 4, 3), 2)
    g5 = lat.gamma5()
    Mpsi = wl.M(U, psi, L, 0.12)
    Mdag_eta = wl.M(U, eta, L, 0.12, dagger=True)
    # adjoint: <eta, M psi> = <M^dag eta, psi>
    assert abs(np.vdot(eta, Mpsi) - np.vdot(Mdag_eta, psi)) < 1e-11
    # gamma5-hermiticity: M^dag = g5 M g5
    g5Mg5 = lat.apply_spin(g5, wl.M(U, lat.apply_spin(g5, eta), L, 0.12))
    assert np.abs(g5Mg5 - Mdag_eta).max() < 1e-13
    # the same on the even-odd Schur complement
    e = li.gaussian_spinor((V // 2, 4, 3), 3)
    lhs = wl.Mhat(U, e, L, 0.155, dagger=True)
    rhs = lat.apply_spin(g5, wl.Mhat(U, lat.apply_spin(g5, e), L, 0.155))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_gauge_covariance():
    """U_mu(x) -> G(x) U_mu(x) G(x+mu)^dag, psi -> G psi  gives  D psi -> G D psi."""
    L = (4, 4, 2, 6)
    V = li.volume(L)
    U = li.random_links(L, 0.5, 3)
    G = li.random_su3_field(V, 4)
    psi = li.gaussian_spinor((V, 4, 3), 5)
    Ug = np.stack([np.einsum("xab,xbc,xdc->xad", G, U[m], np.conj(lat.shift(G, L, m, +1)))
                   for m in range(4)])
    lhs = wl.hop(Ug, np.einsum("xab,xsb->xsa", G, psi), L)
    rhs = np.einsum("xab,xsb->xsa", G, wl.hop(U, psi, L))
    assert np.abs(lhs - rhs).max() < 1e-12


def test_norm_bound_and_Khat_spectrum():
    """||D|| <= 8, hence spec K-hat in [0, (1 + 64 kappa^2)^2]."""
    L, kappa = (4, 4, 4, 4), 0.155
    U = li.random_links(L, 0.447, 9)
    V = li.volume(L)
    v = li.gaussian_spinor((V, 4, 3), 1)
    for _ in range(60):
        w = wl.hop(U, wl.hop(U, v, L), L, dagger=True)
        lam = np.sqrt(np.vdot(w, w).real / np.vdot(v, v).real)
        v = w / np.linalg.norm(w)
    assert lam <= 64 + 1e-9
    L = (4, 4, 2, 4)
    U = li.random_links(L, 0.447, 9)
    Kd = wl.dense(lambda e: wl.Khat(U, e, L, kappa), li.volume(L) // 2)
    ev = np.linalg.eigvalsh(Kd)
    assert ev.min() > 0 and ev.max() <= (1 + 64 * kappa ** 2) ** 2


def test_schur_complement_determinant_and_inverse():
    """det M = det M-hat and (M^-1)_ee = M-hat^-1 (even-odd preconditioning, Sec. 3.1)."""
    L, kappa = (4, 2, 2, 4), 0.155
    U = li.random_links(L, 0.447, 21)
    V = li.volume(L)
    Md = wl.dense(lambda v: wl.M(U, v, L, kappa), V)
    Mh = wl.dense(lambda v: wl.Mhat(U, v, L, kappa), V // 2)
    s1, l1 = np.linalg.slogdet(Md)
    s2, l2 = np.linalg.slogdet(Mh)
    assert abs(l1 - l2) < 1e-11 and abs(s1 - s2) < 1e-11
    ev = lat.parity_sites(L, 0)
    idx = (ev[:, None] * 12 + np.arange(12)[None]).reshape(-1)
    Minv_ee = np.linalg.inv(Md)[np.ix_(idx, idx)]
    assert np.abs(Minv_ee - np.linalg.inv(Mh)).max() < 1e-12


@pytest.mark.parametrize("L", [(4, 4, 2, 6), (6, 2, 4, 4)])
def test_hop_at_sampled_sites_equals_full_hop(L):
    """The per-site evaluation (used at full sizes) agrees with the whole-lattice hop,
    both parities, dagger, across the antiperiodic time wrap."""
    U = li.random_links(L, 0.447, 5)
    Vh = li.volume(L) // 2
    rng = np.random.default_rng(3)
    for p in (0, 1):
        psi = li.gaussian_spinor((Vh, 4, 3), 40 + p)
        sites = rng.choice(Vh, 17, replace=False)
        for dagger in (False, True):
            full = wl.hop_eo(U, psi, L, p, t_bc=-1, dagger=dagger)
            at = wl.hop_eo_at(U, psi, L, p, sites, t_bc=-1, dagger=dagger)
            assert np.abs(at - full[sites]).max() < 1e-13


def test_J_at_matches_whole_lattice_J():
    """The sampled-site J (used at full sizes) agrees with the whole-lattice J, at
    sites including ones whose neighbourhoods wrap in every direction."""
    L = (4, 4, 6, 8)
    U = li.random_links(L, 0.447, 6)
    Vh = li.volume(L) // 2
    psi = li.gaussian_spinor((Vh, 4, 3), 41)
    sites = np.sort(np.random.default_rng(4).choice(Vh, 11, replace=False))
    full = wl.J(U, psi, L, 0.156, 0.05)
    at = wl.J_at(U, psi, L, 0.156, 0.05, sites)
    assert np.abs(at - full[sites]).max() < 1e-12 * np.abs(full).max()
