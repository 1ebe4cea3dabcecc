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
