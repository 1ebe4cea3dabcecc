"""Pins for the oracle's integrator schedule, SU(3) exponential and HMC trajectory."""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import lattice_inputs as li
from oracle import action as act, hmc, integrator, su3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "generalized_integrator_example.txt")


def _read_golden():
    steps = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        kind, term, w = line.split()
        w = Fraction(w)
        steps.append(("T", w) if kind == "T" else ("S", int(term) - 1, w))
    return steps


def test_merge_reproduces_paper_example():
    """Sec. 3.2: I_1 (2-step leapfrog) overlaid with I_2 (3-step leapfrog)."""
    got = integrator.merge([integrator.scheme_events("leapfrog", 2),
                            integrator.scheme_events("leapfrog", 3)])
    assert got == _read_golden()


@pytest.mark.parametrize("kind", ["leapfrog", "omelyan"])
def test_schedule_weights_sum_to_tau(kind):
    ns = [20, 40, 80, 7]
    sched = integrator.merge([integrator.scheme_events(kind, n) for n in ns])
    assert sum((s[1] for s in sched if s[0] == "T"), Fraction(0)) == 1
    for i in range(len(ns)):
        assert sum(float(s[2]) for s in sched if s[0] == "S" and s[1] == i) == pytest.approx(1.0, abs=1e-13)
    # time-reversal symmetry of the whole schedule
    assert [s[0] for s in sched] == [s[0] for s in reversed(sched)]


def test_su3_exponential():
    p = np.random.default_rng(3).standard_normal((50, 8))
    P = su3.coeffs_to_matrix(p)
    E = su3.expi(0.37, P)
    ref = np.stack([scipy.linalg.expm(0.37j * m) for m in P])
    assert np.abs(E - ref).max() < 1e-14
    assert np.abs(np.einsum("nab,ncb->nac", E, E.conj()) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(E) - 1).max() < 1e-14
    assert np.abs(np.einsum("nab,nbc->nac", E, su3.expi(-0.37, P)) - np.eye(3)).max() < 1e-14


L4 = (4, 4, 4, 4)


def _setup(nsteps, scheme="omelyan", tau=1.0):
    terms = [act.Term("POLY", 0.155, mu2=0.05, n=4, tol=1e-14),
             act.Term("POLYK_INV", 0.155, mu2=0.05, n=4, tol=1e-14),
             act.Term("RATIO", 0.155, mu2_num=0.05, tol=1e-14)]
    params = hmc.HMCParams(terms=terms, beta=5.6, nsteps=nsteps, scheme=scheme, tau=tau)
    U = li.random_links(L4, 0.447, 1003)
    P = li.gaussian_momenta(L4, li.seed_md(0, 15))
    Vh = li.volume(L4) // 2
    chis = [li.gaussian_spinor((Vh, 4, 3), li.seed_md(0, i)) for i in range(len(terms))]
    return U, P, params, chis


@pytest.mark.slow
def test_trajectory_is_reversible():
    U, P, params, chis = _setup([2, 1, 1, 3], tau=0.2)
    ops = act.Ops(U, L4)
    phis = [act.heatbath(ops, t, c) for t, c in zip(params.terms, chis)]
    U1, P1 = hmc.integrate(U, P, L4, params, phis)
    U2, P2 = hmc.integrate(U1, -P1, L4, params, phis)
    assert np.abs(U2 - U).max() < 1e-11
    assert np.abs(P2 + P).max() < 1e-10


@pytest.mark.slow
def test_energy_violation_scales_as_step_squared():
    dh = []
    for k in (1, 2):
        U, P, params, chis = _setup([2 * k, 1 * k, 1 * k, 4 * k], scheme="leapfrog", tau=0.2)
        r = hmc.trajectory(U, P, L4, params, chis, 0.5)
        dh.append(r.dH)
    ratio = dh[0] / dh[1]
    assert 3.0 < ratio < 5.0, dh
