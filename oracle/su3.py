"""su(3) algebra helpers: coefficient maps, exp(i eps P), reunitarisation (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2: the momentum P is distributed as exp(-sum tr P^2) and the time step
T[eps] maps U -> exp(i eps P) U.  Reading: P = sum_a p^a T^a, Hermitian and
traceless, T^a = lambda^a / 2; exp(i eps P) by Hermitian eigendecomposition;
reunitarisation by Gram-Schmidt on the first two rows, third row the complex
conjugate of their cross product.

The Lie derivative of a real function S of the link U along T^a is
grad^a S = d/de S(exp(i e T^a) U)|_0; for S = Re tr(i T^a G)-type linear
forms this is ``grad_from_matrix``.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat


def coeffs_to_matrix(p: np.ndarray) -> np.ndarray:
    """[..., 8] real -> [..., 3, 3] Hermitian traceless sum_a p^a T^a."""
    return np.einsum("...a,aij->...ij", p, lat.generators())


def matrix_to_coeffs(P: np.ndarray) -> np.ndarray:
    """Inverse of coeffs_to_matrix on Hermitian traceless input: p^a = 2 tr(T^a P)."""
    return 2.0 * np.einsum("aij,...ji->...a", lat.generators(), P).real


def grad_from_matrix(G: np.ndarray) -> np.ndarray:
    """Coefficients Re(i tr(T^a G)) for [..., 3, 3] complex G."""
    tr = np.einsum("aij,...ji->...a", lat.generators(), G)
    return (1j * tr).real


def expi(eps: float, P: np.ndarray) -> np.ndarray:
    """exp(i eps P) for Hermitian P [..., 3, 3]."""
    w, v = np.linalg.eigh(P)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * eps * w), np.conj(v))


def reunitarize(U: np.ndarray) -> np.ndarray:
    shp = U.shape
    u = U.reshape(-1, 3, 3)
    r1 = u[:, 0, :] / np.linalg.norm(u[:, 0, :], axis=-1, keepdims=True)
    r2 = u[:, 1, :] - np.sum(np.conj(r1) * u[:, 1, :], axis=-1, keepdims=True) * r1
    r2 = r2 / np.linalg.norm(r2, axis=-1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=1).reshape(shp)


def dagger(U: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(U, -1, -2))
