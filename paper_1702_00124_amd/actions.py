"""The actions the paper compares, as lists of pseudofermion terms.

Sec. 2: mass preconditioning (MP) phi1^dag J^-1 phi1 + phi2^dag J K^-1 phi2 and
polynomial filtering (PF) phi1^dag P(K) phi1 + phi2^dag [P(K) K]^-1 phi2;
Sec. 3.3: two filters, 2PF with P_1, Q = P_2 / P_1, [P_2 K]^-1 and 2MP with
J_1^-1, J_1 J_2^-1, J_2 K^-1; Sec. 4.1: PF-MP with P(J), [P(J) J]^-1, J K^-1;
Sec. 4.2: 1PF-2MP and 2PF-1MP.  J = K-hat(kappa') (kappa' < kappa, the reading
of Sec. 4.1's sign), correction terms in their Hermitian RATIO form.  Terms are
listed from the cheapest (finest integration scale) to the most expensive.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

# (kind, kappa or the name of a kappa, extra Term fields)
Spec = List[Tuple[str, str, dict]]

PAPER_ACTIONS: Dict[str, Spec] = {
    "MP": [("KINV", "kp", {}), ("RATIO", "k", {"kappa_num": "kp"})],
    "PF": [("POLY", "k", {"degree": 16}), ("POLYK_INV", "k", {"degree": 16})],
    "2PF": [("POLY", "k", {"degree": 4}), ("POLY", "k", {"degree": 24, "degree_div": 4}),
            ("POLYK_INV", "k", {"degree": 24})],
    "2MP": [("KINV", "k1", {}), ("RATIO", "k2", {"kappa_num": "k1"}), ("RATIO", "k", {"kappa_num": "k2"})],
    "PF-MP": [("POLY", "kp", {"degree": 4}), ("POLYK_INV", "kp", {"degree": 4}), ("RATIO", "k", {"kappa_num": "kp"})],
    "1PF-2MP": [("POLY", "k1", {"degree": 4}), ("POLYK_INV", "k1", {"degree": 4}), ("RATIO", "k2", {"kappa_num": "k1"}),
                ("RATIO", "k", {"kappa_num": "k2"})],
    "2PF-1MP": [("POLY", "kp", {"degree": 4}), ("POLY", "kp", {"degree": 24, "degree_div": 4}),
                ("POLYK_INV", "kp", {"degree": 24}), ("RATIO", "k", {"kappa_num": "kp"})],
}


def build_terms(name: str, kappas: Dict[str, float], cg, a: float = 0.001, b: float = 8.0):
    """Term objects of one action; kappas maps 'k', 'kp', 'k1', 'k2' to values."""
    from .lattice import Term
    terms = []
    for kind, kname, kw in PAPER_ACTIONS[name]:
        fields = {f: (kappas[v] if f == "kappa_num" else v) for f, v in kw.items()}
        terms.append(Term(kind, kappas[kname], a=a, b=b, cg=cg, **fields))
    return terms


def default_nsteps(nterms: int, first: int = 40, rest: int = 20, gauge: int = 80) -> List[int]:
    """Steps per scale: the cheapest term, every other term, then the gauge action."""
    return [first] + [rest] * (nterms - 1) + [gauge]


# The HMC workload on the 16^3 x 32 lattice: kappa 0.155, Wilson gauge action
# beta 5.6, PF-MP in the mu^2 form (Sec. 4.1 with J = K-hat + mu^2):
# POLY(J) + POLYK_INV(J) + RATIO (numerator shift mu^2), Chebyshev order 16 on
# [0.001, 8], Omelyan, tau = 1.  Steps per scale (poly, poly-K inverse, ratio,
# gauge): the ratio term, the most expensive, is the outer scale with 20
# steps; the others are set by their forces.  Measured on this lattice from
# one set of momenta and noise, doubling one scale at a time from
# 40 / 20 / 20 / 80 (dH 17.7 at the synthetic start, -1.83 after an MP
# thermalisation): only the poly-K inverse term moves dH (to 3.5 / -0.47),
# so it takes 40 steps; doubling the poly, ratio or gauge scale changes
# dH by under 10%.
WORKLOAD = {"kappa": 0.155, "beta": 5.6, "mu2": 0.05, "degree": 16, "a": 0.001, "b": 8.0}
WORKLOAD_NSTEPS = [40, 40, 20, 80]


def workload_terms(cg_md, cg_poly, kappa=WORKLOAD["kappa"], mu2=WORKLOAD["mu2"], degree=WORKLOAD["degree"],
                   a=WORKLOAD["a"], b=WORKLOAD["b"]):
    """POLY(J), POLYK_INV(J) and RATIO of the HMC workload: the polynomial terms
    solve with cg_poly, the ratio term with cg_md."""
    from .lattice import Term
    return [Term("POLY", kappa, mu2=mu2, degree=degree, a=a, b=b, cg=cg_poly),
            Term("POLYK_INV", kappa, mu2=mu2, degree=degree, a=a, b=b, cg=cg_poly),
            Term("RATIO", kappa, mu2_num=mu2, cg=cg_md)]


def thermalise(lat, ntraj, kappa=WORKLOAD["kappa"], beta=WORKLOAD["beta"], nsteps=(60, 30, 120), traj0=100000,
               cg=None, log=None):
    """ntraj HMC trajectories with Metropolis of the MP action (kappa' = kappa - 0.005)
    from the lattice's current links, which they leave thermalised.  Every exact
    action samples the same distribution det K-hat exp(-S_G), so the cheap,
    well-accepted MP chain serves any of them.  Seeded per trajectory index
    (traj0 + k).  Returns rows (dH, accepted, plaquette, seconds)."""
    import time

    import torch

    import lattice_inputs as li
    from .lattice import CG
    cg = cg or CG(tol=1e-10, inner="f32", chunk=8, delta=0.003)
    terms = build_terms("MP", {"k": kappa, "kp": round(kappa - 0.005, 6), "k1": 0.0, "k2": 0.0}, cg)
    L, Vh = lat.L, lat.Vh
    u = li.uniforms(max(ntraj, 1), li.seed_metropolis(traj0))
    rows = []
    for k in range(ntraj):
        t = traj0 + k
        P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(L, li.seed_md(t, 15))))
        chi = torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(t, i))))
                         for i in range(len(terms))])
        t0 = time.perf_counter()
        r = lat.hmc_trajectory(terms, list(nsteps), P, chi, float(u[k]), beta=beta, tau=1.0, integrator="omelyan")
        rows.append((r.dH, bool(r.accepted), r.plaquette, time.perf_counter() - t0))
        if log:
            log(f"thermalisation {k}: dH {r.dH:.4f} accepted {int(r.accepted)} plaquette {r.plaquette:.5f} "
                f"({rows[-1][3]:.2f} s)")
    return rows
