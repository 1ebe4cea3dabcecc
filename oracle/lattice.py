"""Lattice geometry, gamma matrices and su(3) generators (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper (Sec. 2-3.1) fixes a 4D lattice with gauge links U, Wilson fermions
and even-odd preconditioning, but no indexing, gamma basis or generator
normalisation.  The readings taken here:

* flat site index s = x + Lx*(y + Ly*(z + Lz*t)); mu = 0..3 is x, y, z, t;
* parity (x + y + z + t) mod 2, even = 0;
* periodic boundaries in space; the fermion fields see an extra phase
  ``t_bc`` (-1: antiperiodic) on every hop that wraps in time; the gauge
  action never sees it;
* Hermitian chiral gamma matrices with gamma_5 = g1 g2 g3 g4 = diag(1,1,-1,-1);
* su(3) generators T^a = lambda^a / 2 (Gell-Mann), tr T^a T^b = delta^ab / 2.
"""
from __future__ import annotations

import numpy as np

# direction mu -> axis of the [t, z, y, x] grid view of a flat field
AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def volume(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


def grid_shape(L):
    return (L[3], L[2], L[1], L[0])


def coords(L):
    """x, y, z, t of every flat site index."""
    s = np.arange(volume(L))
    x = s % L[0]
    y = (s // L[0]) % L[1]
    z = (s // (L[0] * L[1])) % L[2]
    t = s // (L[0] * L[1] * L[2])
    return x, y, z, t


def parity(L) -> np.ndarray:
    x, y, z, t = coords(L)
    return (x + y + z + t) % 2


def shift(f: np.ndarray, L, mu: int, sign: int, t_bc: int = 1) -> np.ndarray:
    """g(x) = f(x + sign * mu_hat); a time wrap multiplies by t_bc.

    ``f`` is a flat field with the site index first.
    """
    g = f.reshape(grid_shape(L) + f.shape[1:])
    g = np.roll(g, -sign, axis=AXIS[mu])
    if mu == 3 and t_bc != 1:
        g = g.copy()
        edge = L[3] - 1 if sign > 0 else 0
        g[edge] *= t_bc
    return g.reshape(f.shape)


def link_phase(L, mu: int, t_bc: int) -> np.ndarray:
    """Per-site factor that the fermion operator attaches to U_mu(x).

    The hop from x to x + mu_hat crosses the time boundary exactly when
    mu = t and t(x) = Lt - 1.
    """
    ph = np.ones(volume(L))
    if mu == 3 and t_bc != 1:
        _, _, _, t = coords(L)
        ph[t == L[3] - 1] = t_bc
    return ph


# ---------------------------------------------------------------- gammas
def gammas() -> np.ndarray:
    """gamma_1..gamma_4 (index 0..3 = x, y, z, t), Hermitian chiral basis."""
    i = 1j
    g1 = np.array([[0, 0, 0, -i], [0, 0, -i, 0], [0, i, 0, 0], [i, 0, 0, 0]])
    g2 = np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=complex)
    g3 = np.array([[0, 0, -i, 0], [0, 0, 0, i], [i, 0, 0, 0], [0, -i, 0, 0]])
    g4 = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=complex)
    return np.stack([g1, g2, g3, g4]).astype(np.complex128)


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def apply_spin(m: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to a spinor field [..., 4, 3]."""
    return np.einsum("st,...tc->...sc", m, psi)


# ---------------------------------------------------------------- su(3)
def gellmann() -> np.ndarray:
    """lambda^1 .. lambda^8."""
    i = 1j
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -i, i
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -i, i
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -i, i
    l[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return l


def generators() -> np.ndarray:
    """T^a = lambda^a / 2."""
    return 0.5 * gellmann()


# ---------------------------------------------------------------- parity fields
def parity_sites(L, p: int) -> np.ndarray:
    """Flat indices of the parity-p sites in lexicographic order."""
    return np.nonzero(parity(L) == p)[0]


def embed(psi_h: np.ndarray, L, p: int) -> np.ndarray:
    """Half-lattice field (parity-p sites, lexicographic) -> full field, zero elsewhere."""
    full = np.zeros((volume(L),) + psi_h.shape[1:], dtype=psi_h.dtype)
    full[parity_sites(L, p)] = psi_h
    return full


def restrict(psi: np.ndarray, L, p: int) -> np.ndarray:
    return psi[parity_sites(L, p)]
