"""Wilson fermion operator, even-odd preconditioning and K = M^dag M (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2 names the fermion matrix M and K = M^dag M; Sec. 3.1 fixes Wilson
fermions with hopping parameter kappa and even-odd preconditioning, but prints
no formula.  The reading (standard hopping-parameter form):

    M = 1 - kappa D,
    (D psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x + mu)
                      + (1 + g_mu) U_mu(x - mu)^dag psi(x - mu),

with the time-boundary phase of ``lattice.shift``.  D^dag is written out from
the definition of the adjoint (the projectors swap), not through gamma_5; the
gamma_5-hermiticity D^dag = g5 D g5 is a test, not an assumption.

Even-odd: with M_ee = M_oo = 1 the Schur complement on the even sites is
M-hat = 1 - kappa^2 D_eo D_oe, and K-hat = M-hat^dag M-hat.  The Hasenbusch
shift is J = K-hat + mu^2 (mass-preconditioner in the mu^2 form).
Half-lattice fields are [V/2, 4, 3] arrays of one parity's sites in
lexicographic order.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat


def hop(U, psi, L, t_bc=-1, dagger=False):
    """Full-lattice D psi (or D^dag psi).  U: [4,V,3,3], psi: [V,4,3]."""
    g = lat.gammas()
    one = np.eye(4)
    s = -1.0 if dagger else 1.0
    out = np.zeros_like(psi)
    for mu in range(4):
        fwd = lat.shift(psi, L, mu, +1, t_bc)                      # psi(x + mu)
        u_fwd = np.einsum("xab,xsb->xsa", U[mu], fwd)               # U_mu(x) psi(x + mu)
        out += lat.apply_spin(one - s * g[mu], u_fwd)
        udag_psi = np.einsum("xba,xsb->xsa", np.conj(U[mu]), psi)   # U_mu(x)^dag psi(x)
        bwd = lat.shift(udag_psi, L, mu, -1, t_bc)                  # ... at x - mu
        out += lat.apply_spin(one + s * g[mu], bwd)
    return out


def M(U, psi, L, kappa, t_bc=-1, dagger=False):
    return psi - kappa * hop(U, psi, L, t_bc, dagger)


def K(U, psi, L, kappa, t_bc=-1):
    """K = M^dag M on the full lattice (Sec. 2)."""
    return M(U, M(U, psi, L, kappa, t_bc), L, kappa, t_bc, dagger=True)


# ---------------------------------------------------------------- even-odd
def hop_eo(U, psi_h, L, out_parity, t_bc=-1, dagger=False):
    """The parity block of D (or D^dag) that maps parity 1-p to parity p."""
    full = lat.embed(psi_h, L, 1 - out_parity)
    return lat.restrict(hop(U, full, L, t_bc, dagger), L, out_parity)


def Mhat(U, psi_e, L, kappa, t_bc=-1, dagger=False):
    """M-hat = 1 - kappa^2 D_eo D_oe on even sites (or its adjoint)."""
    odd = hop_eo(U, psi_e, L, 1, t_bc, dagger)
    return psi_e - kappa ** 2 * hop_eo(U, odd, L, 0, t_bc, dagger)


def Khat(U, psi_e, L, kappa, t_bc=-1):
    return Mhat(U, Mhat(U, psi_e, L, kappa, t_bc), L, kappa, t_bc, dagger=True)


def J(U, psi_e, L, kappa, mu2, t_bc=-1):
    """Hasenbusch-shifted operator J = K-hat + mu^2."""
    return Khat(U, psi_e, L, kappa, t_bc) + mu2 * psi_e


def W(U, psi_e, L, kappa, mu, t_bc=-1, dagger=False):
    """W = M-hat + i mu g5 (W^dag W = J, derived from g5-hermiticity)."""
    g5 = lat.gamma5()
    s = -1.0 if dagger else 1.0
    return Mhat(U, psi_e, L, kappa, t_bc, dagger) + s * 1j * mu * lat.apply_spin(g5, psi_e)


def neighbours_h(L, p_from, sites_h) -> np.ndarray:
    """Half-lattice indices (parity 1 - p_from) of the 8 nearest neighbours of the
    listed parity-p_from sites (half-lattice indices), sorted, without repeats."""
    full = lat.parity_sites(L, p_from)[np.asarray(sites_h)]
    other = lat.parity_sites(L, 1 - p_from)
    c = np.stack(np.unravel_index(full, tuple(reversed(L)))[::-1], axis=1)
    out = []
    for mu in range(4):
        for d in (1, -1):
            y = c.copy()
            y[:, mu] = (y[:, mu] + d) % L[mu]
            out.append(np.searchsorted(other, y[:, 0] + L[0] * (y[:, 1] + L[1] * (y[:, 2] + L[2] * y[:, 3]))))
    return np.unique(np.concatenate(out))


def J_at(U, psi_e, L, kappa, mu2, sites_h, t_bc=-1) -> np.ndarray:
    """(J psi)(s) at the listed even sites only: M-hat and its adjoint written out
    as in Mhat, each hop evaluated by hop_eo_at on just the sites the four nested
    hops reach from the listed ones (for large lattices).  Returns [n, 4, 3]."""
    Vh = psi_e.shape[0]
    s0 = np.asarray(sites_h)
    n1 = neighbours_h(L, 0, s0)                    # odd sites of D_oe^dag y read at s0
    s2 = np.union1d(neighbours_h(L, 1, n1), s0)    # even sites of y = M-hat psi read there
    n3 = neighbours_h(L, 0, s2)                    # odd sites of D_oe psi read at s2
    o = np.zeros((Vh,) + psi_e.shape[1:], dtype=np.complex128)
    o[n3] = hop_eo_at(U, psi_e, L, 1, n3, t_bc)
    y = np.zeros_like(o)
    y[s2] = psi_e[s2] - kappa ** 2 * hop_eo_at(U, o, L, 0, s2, t_bc)
    o = np.zeros_like(o)
    o[n1] = hop_eo_at(U, y, L, 1, n1, t_bc, dagger=True)
    return y[s0] - kappa ** 2 * hop_eo_at(U, o, L, 0, s0, t_bc, dagger=True) + mu2 * psi_e[s0]


def dense(op, n_sites, dtype=np.complex128):
    """Dense matrix of a linear map on [n_sites, 4, 3] fields (brute force, tiny lattices)."""
    n = n_sites * 12
    A = np.zeros((n, n), dtype=dtype)
    e = np.zeros(n, dtype=dtype)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = op(e.reshape(n_sites, 4, 3)).reshape(n)
    return A


def hop_eo_at(U, psi_h, L, out_parity, sites_h, t_bc=-1, dagger=False):
    """hop_eo evaluated only at the listed output sites (half-lattice indices of
    parity out_parity), from the definition of D term by term: for large
    lattices, where a few sampled sites check a full-size result.
    psi_h: half field of parity 1 - out_parity.  Returns [len(sites_h), 4, 3]."""
    g = lat.gammas()
    one = np.eye(4)
    s = -1.0 if dagger else 1.0
    full_out = lat.parity_sites(L, out_parity)[np.asarray(sites_h)]
    full_in = lat.parity_sites(L, 1 - out_parity)
    x = np.stack(np.unravel_index(full_out, tuple(reversed(L)))[::-1], axis=1)   # (x, y, z, t) per site

    def flat(c):
        return c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))

    out = np.zeros((len(full_out), 4, 3), dtype=np.complex128)
    for mu in range(4):
        for sign in (+1, -1):
            y = x.copy()
            y[:, mu] += sign
            wrap = (y[:, mu] < 0) | (y[:, mu] >= L[mu])
            y[:, mu] %= L[mu]
            ph = np.where(wrap & (mu == 3), float(t_bc), 1.0)
            psi_y = psi_h[np.searchsorted(full_in, flat(y))]                     # psi(x +- mu)
            if sign > 0:
                v = np.einsum("nab,nsb->nsa", U[mu][full_out], psi_y)           # U_mu(x) psi(x + mu)
                out += ph[:, None, None] * lat.apply_spin(one - s * g[mu], v)
            else:
                v = np.einsum("nba,nsb->nsa", np.conj(U[mu][flat(y)]), psi_y)   # U_mu(x - mu)^dag psi(x - mu)
                out += ph[:, None, None] * lat.apply_spin(one + s * g[mu], v)
    return out
