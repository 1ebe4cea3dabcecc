"""Link derivative of the Wilson hopping bilinear (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2 gives the fermion force as the U-derivative of phi^dag K^-1 phi, which
by the product rule reduces to derivatives of bilinears Re(A^dag D C).  The
paper prints no formula; derived here from the definition of D (see
``wilson.hop``).  For the link U_mu(x) (with its fermion boundary phase) and
y = x + mu, only two terms of Re(A^dag D C) contain it:

    Re A(x)^dag (1 - g_mu) U C(y)  +  Re A(y)^dag (1 + g_mu) U^dag C(x).

Under U -> exp(i e T^a) U their derivative is Re(i tr(T^a W)) with

    W = U Xi - Theta U^dag,
    Xi    = sum_spin C(y) [(1 - g_mu) A(x)]^dag   (3x3 colour matrix),
    Theta = sum_spin C(x) [(1 + g_mu) A(y)]^dag.

Written with the full 4x4 spin matrices, no projector shortcuts.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat
from . import su3


def bilinear_grad(U, A, C, L, t_bc=-1) -> np.ndarray:
    """g[mu, x, a] = d/de Re(A^dag D(U') C) at e = 0, U'_mu(x) = exp(i e T^a) U_mu(x)."""
    g = lat.gammas()
    one = np.eye(4)
    out = np.zeros((4, lat.volume(L), 8))
    for mu in range(4):
        Ub = U[mu] * lat.link_phase(L, mu, t_bc)[:, None, None]
        Cy = lat.shift(C, L, mu, +1)
        Ay = lat.shift(A, L, mu, +1)
        PA = lat.apply_spin(one - g[mu], A)
        PAy = lat.apply_spin(one + g[mu], Ay)
        Xi = np.einsum("xsa,xsb->xab", Cy, np.conj(PA))
        Theta = np.einsum("xsa,xsb->xab", C, np.conj(PAy))
        Wm = np.einsum("xab,xbc->xac", Ub, Xi) - np.einsum("xab,xbc->xac", Theta, su3.dagger(Ub))
        out[mu] = su3.grad_from_matrix(Wm)
    return out


def bilinear_grad_at(U, A, C, L, links, t_bc=-1) -> np.ndarray:
    """bilinear_grad evaluated only at the listed links, written link by link from the
    same definition (the two terms of Re(A^dag D C) that hold U_mu(x)): for large
    lattices, where sampled links check a full-size force.

    links: sequence of (mu, x), x a flat full-lattice site index.  Returns [n, 8]."""
    g = lat.gammas()
    one = np.eye(4)
    out = np.zeros((len(links), 8))
    for i, (mu, x) in enumerate(links):
        c = [x % L[0], (x // L[0]) % L[1], (x // (L[0] * L[1])) % L[2], x // (L[0] * L[1] * L[2])]
        c[mu] += 1
        wrapped = c[mu] == L[mu]
        c[mu] %= L[mu]
        y = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))
        ph = float(t_bc) if (wrapped and mu == 3) else 1.0
        Ub = ph * U[mu][x]                                   # U_mu(x) with its fermion phase
        PAx = (one - g[mu]) @ A[x]                           # [(1 - g_mu) A(x)], 4 x 3
        PAy = (one + g[mu]) @ A[y]                           # [(1 + g_mu) A(y)]
        Xi = sum(np.outer(C[y][s], np.conj(PAx[s])) for s in range(4))
        Theta = sum(np.outer(C[x][s], np.conj(PAy[s])) for s in range(4))
        Wm = Ub @ Xi - Theta @ np.conj(Ub.T)
        out[i] = su3.grad_from_matrix(Wm)
    return out
