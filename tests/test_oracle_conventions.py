"""Pins for the oracle's conventions: gamma matrices, generators, links, shifts."""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import gauge, lattice as lat, su3


def test_clifford_algebra_and_gamma5():
    g = lat.gammas()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            anti = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(anti, 2 * (m == n) * np.eye(4), atol=0)
    assert np.allclose(lat.gamma5(), np.diag([1, 1, -1, -1]), atol=0)


def test_generators_normalisation_and_structure_constants():
    T = lat.generators()
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15
    # [T1, T2] = i T3 and [T4, T5] = i (T3 + sqrt3 T8)/2: f_123 = 1, f_458 = sqrt3/2
    assert np.allclose(T[0] @ T[1] - T[1] @ T[0], 1j * T[2])
    assert np.allclose(T[3] @ T[4] - T[4] @ T[3], 1j * (0.5 * T[2] + np.sqrt(3) / 2 * T[7]))


def test_coefficient_maps_roundtrip():
    p = np.random.default_rng(0).standard_normal((10, 8))
    P = su3.coeffs_to_matrix(p)
    assert np.allclose(su3.matrix_to_coeffs(P), p)
    # sum tr P^2 = (1/2) sum p^2 (momentum normalisation of Sec. 2)
    assert np.allclose(np.einsum("nij,nji->n", P, P).real, 0.5 * (p * p).sum(-1))


def test_random_links_are_su3():
    U = li.random_links((4, 4, 4, 4), 0.3, 7)
    I = np.einsum("mxab,mxcb->mxac", U, U.conj())
    assert np.abs(I - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_gauge_transforms_are_su3():
    G = li.random_su3_field(100, 3)
    assert np.abs(np.einsum("xab,xcb->xac", G, G.conj()) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(G) - 1).max() < 1e-14


def test_hermitian_noise_law_of_link_generator():
    """h^a = 2 tr(T^a H) ~ N(0, 1): the link generator's traceless Hermitian draw."""
    rng = np.random.default_rng(11)
    H = li._gaussian_traceless_hermitian(rng, 200000)
    h = su3.matrix_to_coeffs(H)
    assert np.allclose(h.mean(0), 0, atol=0.01)
    assert np.allclose(h.var(0), 1, atol=0.02)


@pytest.mark.parametrize("a,target,L", [(0.3, 0.785, (4, 4, 4, 4)),
                                        (0.447, 0.58, (8, 8, 8, 8)),
                                        (0.432, 0.60, (8, 8, 8, 8))])
def test_plaquette_of_synthetic_links(a, target, L):
    """Independent links: <plaquette> = u0^4 with u0 = <Re tr U>/3 (E[U] = u0 * 1
    by conjugation invariance of the law of H)."""
    U = li.random_links(L, a, 1)
    u0 = np.einsum("mxaa->", U).real / (3 * U.shape[0] * U.shape[1])
    plaq = gauge.mean_plaquette(U, L)
    assert abs(plaq - u0 ** 4) < 0.01
    assert abs(plaq - target) < 0.01


def test_shift_roundtrip_and_antiperiodic_wrap():
    L = (4, 2, 2, 6)
    f = np.random.default_rng(1).standard_normal((li.volume(L), 4, 3))
    for mu in range(4):
        g = lat.shift(lat.shift(f, L, mu, +1, -1), L, mu, -1, -1)
        assert np.array_equal(g, f)
    g = f
    for _ in range(L[3]):
        g = lat.shift(g, L, 3, +1, -1)
    assert np.array_equal(g, -f)
    # x + 1 in the flat index convention s = x + Lx (y + Ly (z + Lz t))
    x, y, z, t = lat.coords(L)
    s = np.arange(li.volume(L))
    sx = lat.shift(s.astype(float), L, 0, +1)
    assert np.array_equal(sx, ((x + 1) % L[0] + L[0] * (y + L[1] * (z + L[2] * t))).astype(float))
