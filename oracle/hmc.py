"""One HMC trajectory with Metropolis accept/reject (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 2: pseudofermions phi are drawn from Gaussian noise chi, momenta P from
exp(-sum tr P^2); H = sum tr P^2 + S is integrated with T[eps]: U ->
exp(i eps P) U and S[eps]: P -> P - eps F, F the force; the end point is
accepted with probability min(1, exp(-dH)).  With P = sum_a p^a T^a,
sum tr P^2 = (1/2) sum (p^a)^2 and F = sum_a (grad^a S) T^a, so the momentum
update is p^a -> p^a - eps grad^a S.  Links are reunitarised after every
T step (FP64).  Terms are placed on time scales by ``integrator.merge``
(Sec. 3.2); the gauge action is the last scale.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import action as act
from . import gauge
from . import integrator
from . import su3


@dataclass
class HMCParams:
    terms: List[act.Term]
    beta: float
    nsteps: List[int]           # per term, then the gauge action
    scheme: str = "omelyan"     # or "leapfrog"
    tau: float = 1.0
    t_bc: int = -1


@dataclass
class HMCResult:
    U: np.ndarray
    P: np.ndarray
    dH: float
    H0: float
    H1: float
    S0: list = field(default_factory=list)
    S1: list = field(default_factory=list)
    accepted: bool = False


def hamiltonian(U, P, L, params: HMCParams, phis):
    ops = act.Ops(U, L, params.t_bc)
    S = [act.action(ops, t, phi) for t, phi in zip(params.terms, phis)]
    S.append(gauge.action(U, L, params.beta))
    return 0.5 * float(np.sum(P * P)) + sum(S), S


def force(U, L, params: HMCParams, phis, i):
    if i == len(params.terms):
        return gauge.force(U, L, params.beta)
    ops = act.Ops(U, L, params.t_bc)
    return act.force(ops, params.terms[i], phis[i])


def integrate(U, P, L, params: HMCParams, phis):
    schemes = [integrator.scheme_events(params.scheme, n) for n in params.nsteps]
    for step in integrator.merge(schemes):
        if step[0] == "T":
            eps = float(step[1]) * params.tau
            U = su3.reunitarize(np.einsum("mxab,mxbc->mxac", su3.expi(eps, su3.coeffs_to_matrix(P)), U))
        else:
            _, i, w = step
            P = P - float(w) * params.tau * force(U, L, params, phis, i)
    return U, P


def trajectory(U, P, L, params: HMCParams, chis, u_metropolis: float) -> HMCResult:
    ops = act.Ops(U, L, params.t_bc)
    phis = [act.heatbath(ops, t, chi) for t, chi in zip(params.terms, chis)]
    H0, S0 = hamiltonian(U, P, L, params, phis)
    U1, P1 = integrate(U, P, L, params, phis)
    H1, S1 = hamiltonian(U1, P1, L, params, phis)
    dH = H1 - H0
    acc = bool(u_metropolis < np.exp(-dH))
    return HMCResult(U1 if acc else U, P1, dH, H0, H1, S0, S1, acc)
