"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module draws random numbers and nothing else of the method: it builds no
Dirac operator, no action, no force and no integrator step.  Every random input
of a run (gauge links, sources, pseudofermion noise, momenta, gauge
transformations, Metropolis uniforms) comes from here, on the host, from
``numpy.random.default_rng`` (PCG64), so the oracle and the GPU library see the
same arrays.

Conventions fixed here (the paper gives none; Sec. 2 only names the fields):

* lattice extents ``L = (Lx, Ly, Lz, Lt)``; flat site index
  ``s = x + Lx*(y + Ly*(z + Lz*t))``; directions mu = 0..3 are x, y, z, t;
* spinor fields: complex128 ``[V, 4 spin, 3 colour]``;
* gauge links: complex128 ``[4 mu, V, 3, 3]`` (row, column);
* su(3) coefficient fields (momenta): float64 ``[4 mu, V, 8]``, the eight
  real coefficients of P = sum_a p^a T^a with T^a = lambda^a / 2;
* Gaussian noise chi with density exp(-chi^dag chi) (Sec. 2): real and
  imaginary parts of every complex component are N(0, 1/2);
* momenta with density exp(-sum tr P^2) (Sec. 2): with tr T^a T^b = delta/2,
  each coefficient p^a is N(0, 1).

Synthetic gauge links are U = exp(i a H) with H a Gaussian traceless Hermitian
3x3 matrix whose coefficients h^a in the T^a basis are N(0, 1), followed by an
SU(3) projection (Gram-Schmidt on the first two rows, third row the complex
conjugate of their cross product).  H is drawn as the traceless part of
(A + A^dag)/2 with A a standard complex Gaussian matrix, which has exactly
that law, so no generator matrices are needed here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "volume", "random_links", "unit_links",
    "gaussian_spinor", "gaussian_momenta", "random_su3_field", "uniforms",
    "seed_links", "seed_source", "seed_md", "seed_metropolis",
]


def volume(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


# --------------------------------------------------------------------------
# seeds: one stream per input kind, so that adding an input never shifts another
def seed_links(config_index: int) -> int:
    return 1001 + int(config_index)


def seed_source(j: int) -> int:
    return 2001 + int(j)


def seed_md(trajectory: int, term: int) -> int:
    """Momenta (term = 15) and pseudofermion noise (term = action-term index)."""
    return 3001 + 16 * int(trajectory) + int(term)


def seed_metropolis(trajectory: int) -> int:
    return 4001 + int(trajectory)


# --------------------------------------------------------------------------
def _gaussian_traceless_hermitian(rng: np.random.Generator, n: int) -> np.ndarray:
    a = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h -= tr[:, None, None] * np.eye(3)[None]
    return h


def _project_su3(u: np.ndarray) -> np.ndarray:
    r1 = u[:, 0, :]
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = u[:, 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1, keepdims=True) * r1
    r2 = r2 / np.linalg.norm(r2, axis=-1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=1)


def _expi_hermitian(h: np.ndarray, a: float) -> np.ndarray:
    """exp(i a H) for a stack of traceless Hermitian 3x3 matrices [N, 3, 3].

    Eigenvalues from the trigonometric solution of l^3 - p l - q = 0
    (p = tr H^2 / 2, q = det H), then Lagrange interpolation on them:
    exp(i a H) = sum_k e^{i a l_k} prod_{j != k} (H - l_j) / (l_k - l_j)
               = f2 H^2 + f1 H + f0 1.
    Vectorised over N with one batched product (H^2); eigenvalue gaps of
    Gaussian Hermitian matrices are repelled, so the divisions are benign.
    """
    H = np.moveaxis(h, 0, -1)                      # [3, 3, N]
    H2 = np.empty_like(H)
    for i in range(3):
        for k in range(3):
            H2[i, k] = H[i, 0] * H[0, k] + H[i, 1] * H[1, k] + H[i, 2] * H[2, k]
    p = 0.5 * (H2[0, 0] + H2[1, 1] + H2[2, 2]).real
    q = (H[0, 0] * (H[1, 1] * H[2, 2] - H[1, 2] * H[2, 1])
         - H[0, 1] * (H[1, 0] * H[2, 2] - H[1, 2] * H[2, 0])
         + H[0, 2] * (H[1, 0] * H[2, 1] - H[1, 1] * H[2, 0])).real
    r = np.sqrt(np.maximum(p, 1e-300) / 3.0)
    th = np.arccos(np.clip(q / (2.0 * r ** 3), -1.0, 1.0))
    lam = [2.0 * r * np.cos((th - 2.0 * np.pi * k) / 3.0) for k in range(3)]
    f0 = np.zeros(H.shape[-1], dtype=np.complex128)
    f1 = np.zeros_like(f0)
    f2 = np.zeros_like(f0)
    for k in range(3):
        j, l = (k + 1) % 3, (k + 2) % 3
        w = np.exp(1j * a * lam[k]) / ((lam[k] - lam[j]) * (lam[k] - lam[l]))
        f2 += w
        f1 -= w * (lam[j] + lam[l])
        f0 += w * (lam[j] * lam[l])
    U = f2 * H2 + f1 * H
    for i in range(3):
        U[i, i] += f0
    return np.moveaxis(U, -1, 0)


def random_links(L, a: float, seed: int) -> np.ndarray:
    """U_mu(x) = SU(3)-projected exp(i a H), H Gaussian traceless Hermitian."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    h = _gaussian_traceless_hermitian(rng, 4 * V)
    u = _project_su3(np.ascontiguousarray(_expi_hermitian(h, a)))
    return np.ascontiguousarray(u.reshape(4, V, 3, 3))


def unit_links(L) -> np.ndarray:
    V = volume(L)
    u = np.zeros((4, V, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3_field(n: int, seed: int) -> np.ndarray:
    """n independent Haar-random SU(3) matrices (gauge transformations)."""
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return _project_su3(q)


def gaussian_spinor(shape, seed: int) -> np.ndarray:
    """Complex Gaussian with density exp(-|z|^2) per component: Re, Im ~ N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    z = rng.standard_normal(shape + (2,)) * np.sqrt(0.5)
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def gaussian_momenta(L, seed: int) -> np.ndarray:
    """Coefficients p^a ~ N(0,1), shape [4, V, 8]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4, volume(L), 8))


def uniforms(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(n)


# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    """A synthetic workload: lattice, hopping parameter and link spread."""
    name: str
    L: Tuple[int, int, int, int]
    kappa: float
    link_spread: float           # the a of U = exp(i a H)
    t_bc: int = -1               # antiperiodic in time
    nrhs: int = 1
    mu2: Tuple[float, ...] = (0.0,)
    tol: float = 1e-10
    beta: float = 5.6
    poly_degree: int = 16
    poly_interval: Tuple[float, float] = (0.001, 8.0)
    hasenbusch_mu2: float = 0.05
    config_index: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return volume(self.L)

    def links(self) -> np.ndarray:
        return random_links(self.L, self.link_spread, seed_links(self.config_index))


# Link spreads: a = 0.3 as stated for the 4^4 case; a = 0.447 and a = 0.432
# give a plaquette of about 0.58 and 0.60 (the oracle's plaquette test checks
# both at the configured seeds).
WORKLOADS = {
    "small_4x4": Workload("wilson 4^4 kappa=0.12 full-K FP64", (4, 4, 4, 4), 0.12, 0.3,
                          config_index=0),
    "eo_16x32": Workload("wilson 16^3x32 kappa=0.155 even-odd", (16, 16, 16, 32), 0.155, 0.447,
                         config_index=1),
    "multirhs_16x32": Workload("wilson 16^3x32 kappa=0.155 8 rhs shifted", (16, 16, 16, 32), 0.155,
                               0.447, nrhs=8, mu2=(0.0, 0.005, 0.05, 0.5, 0.0, 0.005, 0.05, 0.5),
                               config_index=2),
    "hmc_16x32": Workload("PF-MP HMC 16^3x32 kappa=0.155 beta=5.6", (16, 16, 16, 32), 0.155, 0.447,
                          config_index=3),
    "large_32x64": Workload("wilson 32^3x64 kappa=0.156 4 rhs", (32, 32, 32, 64), 0.156, 0.432,
                            nrhs=4, mu2=(0.0, 0.0, 0.0, 0.0), config_index=4),
}
