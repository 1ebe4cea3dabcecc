"""Wilson plaquette gauge action S_G and its force (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2 writes S = S_G[U] + S_F without fixing S_G.  Reading (Wilson plaquette
action, beta as in the HMC workload):

    S_G = beta sum_{x, mu<nu} (1 - Re tr U_munu(x) / 3),
    U_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,

periodic in all directions (the fermion time phase is not part of S_G).
Force coefficients grad^a S_G = d/de S_G(exp(i e T^a) U_mu(x))|_0
= -(beta/3) Re(i tr(T^a U_mu(x) A_mu(x))), A the sum of the six staples.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat
from . import su3


def _mm(a, b):
    return np.einsum("xab,xbc->xac", a, b)


def plaquette_field(U, L, mu, nu):
    Uf_nu = lat.shift(U[nu], L, mu, +1)      # U_nu(x + mu)
    Uf_mu = lat.shift(U[mu], L, nu, +1)      # U_mu(x + nu)
    return _mm(_mm(_mm(U[mu], Uf_nu), su3.dagger(Uf_mu)), su3.dagger(U[nu]))


def mean_plaquette(U, L) -> float:
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            tot += np.trace(plaquette_field(U, L, mu, nu), axis1=1, axis2=2).real.sum() / 3.0
    return tot / (6 * lat.volume(L))


def action(U, L, beta) -> float:
    return beta * 6 * lat.volume(L) * (1.0 - mean_plaquette(U, L))


def staples(U, L, mu):
    A = np.zeros_like(U[mu])
    for nu in range(4):
        if nu == mu:
            continue
        Uf_nu = lat.shift(U[nu], L, mu, +1)                          # U_nu(x+mu)
        Uf_mu = lat.shift(U[mu], L, nu, +1)                          # U_mu(x+nu)
        A += _mm(_mm(Uf_nu, su3.dagger(Uf_mu)), su3.dagger(U[nu]))
        # lower staple: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        lower = _mm(_mm(su3.dagger(Uf_nu), su3.dagger(U[mu])), U[nu])  # evaluated at x' = x - nu
        A += lat.shift(lower, L, nu, -1)
    return A


def force(U, L, beta) -> np.ndarray:
    """grad^a S_G, shape [4, V, 8]."""
    F = np.zeros((4, lat.volume(L), 8))
    for mu in range(4):
        F[mu] = -(beta / 3.0) * su3.grad_from_matrix(_mm(U[mu], staples(U, L, mu)))
    return F
