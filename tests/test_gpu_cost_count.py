"""GPU: the cost count N_mat of Sec. 3.1 (fermion-matrix K multiplications per
trajectory) against the counting rule stated with wl_counters.

* Per trajectory, for every term kind: the library's n_kmat equals the count
  derived from the rule, from the per-solve log (iterations and FP64 residual
  applications of each CG, and the K multiplications of one operator
  application: 1 for J or K, the polynomial's own count for P(J) and P(J) J)
  and from the integrator schedule (the number of force evaluations of the
  term): solves + heatbath Q^dag (q) + two actions P (n, or 2q for a quotient)
  for POLY, and Q + 2(q - 1) chain multiplications per POLY force, Q + 1 +
  2(q - 1) per POLY-K-inverse force.  The number of logged solves and their
  multiplications per application are checked against the term's structure.
* Independently of the library's bookkeeping, CG counting against the hop
  launch counter: with one rhs and one iteration per convergence check,
  every iteration and every FP64 residual is one J = four hop launches, in
  the inner precision and in FP64 respectively.
"""
import pytest
import torch

import lattice_inputs as li
from paper_1702_00124_amd.lattice import CG, Term, integrator_schedule
from tests.gpu_common import full_noise, half_noise, make_lattice, say

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)


def _q(n, ndiv=0):
    """Root factors of Q for P_n, or of the quotient P_n / P_ndiv."""
    r = (n + 1) // (ndiv + 1) if ndiv else 0
    return len([k for k in range(1, n // 2 + 1) if not (r and k % r == 0)])


def _terms(inner):
    cg = CG(tol=1e-11, inner=inner, chunk=4, delta=0.01)
    return {
        "KINV_FULL": Term("KINV_FULL", 0.12, cg=cg),
        "KINV": Term("KINV", 0.155, mu2=0.05, cg=cg),
        "RATIO": Term("RATIO", 0.155, mu2_num=0.05, cg=cg),
        "RATIO_KAPPA": Term("RATIO", 0.155, kappa_num=0.150, cg=cg),
        "POLY": Term("POLY", 0.155, mu2=0.05, degree=4, cg=cg),
        "POLY_QUOTIENT": Term("POLY", 0.150, degree=24, degree_div=4, cg=cg),
        "POLYK_INV": Term("POLYK_INV", 0.155, mu2=0.05, degree=4, cg=cg),
        "POLYK_INV_16": Term("POLYK_INV", 0.155, mu2=0.05, degree=16, cg=cg),
    }


@pytest.mark.parametrize("inner", ["f64", "f32"])
@pytest.mark.parametrize("name", list(_terms("f64")))
def test_trajectory_n_mat_follows_the_counting_rule(name, inner):
    term = _terms(inner)[name]
    say("N_mat rule", name, inner)
    lat, _ = make_lattice(L4, a=0.3 if term.kind == "KINV_FULL" else 0.447)
    nsteps = [3, 6]
    chi = full_noise(L4, 3100) if term.full else half_noise(L4, 3100)
    chib = lat.import_full(torch.from_numpy(chi)) if term.full else lat.import_spinor(torch.from_numpy(chi))
    P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(L4, 3101)))
    lat.solve_log(True)
    r = lat.hmc_trajectory([term], nsteps, P, chib, 0.5, tau=0.2, integrator="omelyan", no_metropolis=True)
    log = lat.solve_log_read()
    lat.solve_log(False)
    nforce = sum(1 for e in integrator_schedule(nsteps, "omelyan") if e[0] == "S" and e[1] == 0)
    solves = sum((it + res) * jpa for it, res, jpa in log)
    q = _q(term.degree, term.degree_div) if term.kind in ("POLY", "POLYK_INV") else 0
    pc = 2 * q if term.degree_div else term.degree
    if term.kind == "POLY":
        extra = q + 2 * pc + nforce * (q + 2 * (q - 1))
        shape = [(pc,)]                                     # heatbath: CG on P(J)
    elif term.kind == "POLYK_INV":
        extra = q + nforce * (q + 1 + 2 * (q - 1))
        shape = [(pc + 1,)] * (2 + nforce)                  # two actions and the forces: CG on P(J) J
    elif term.kind == "RATIO":
        extra = 0
        shape = [(1,)] * (3 + nforce)                       # heatbath, two actions, forces
    else:
        extra = 0
        shape = [(1,)] * (2 + nforce)
    say(f"  {len(log)} solves, {sum(it for it, _, _ in log)} iterations, forces {nforce}: "
        f"n_kmat {r.n_kmat} = solves {solves} + {extra}")
    assert [(jpa,) for _, _, jpa in log] == shape
    assert all(it > 0 and res >= 1 for it, res, _ in log)
    assert r.n_kmat == solves + extra
    # the trajectory's CG iteration count leaves out the heatbath's solve
    hb = 1 if term.kind in ("RATIO", "POLY") else 0
    assert r.cg_iters == sum(it for it, _, _ in log[hb:])


@pytest.mark.parametrize("kind", ["KINV", "POLYK_INV", "POLY"])
@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_count_matches_hop_launches(kind, inner):
    """One rhs, convergence checked every iteration: the operator applications the
    count records are exactly the hop launches made, four per J."""
    lat, _ = make_lattice(L4)
    say("N_mat vs hop launches", kind, inner)
    term = Term(kind, 0.155, mu2=0.05, degree=4 if kind != "KINV" else 0, cg=CG(tol=1e-11, inner=inner, chunk=1))
    phi = lat.import_spinor(torch.from_numpy(half_noise(L4, 3200)))
    torch.cuda.synchronize()
    h0, k0 = lat.hop_counts(), lat.counters()[1]
    lat.solve_log(True)
    lat.action(term, phi)
    log = lat.solve_log_read()
    lat.solve_log(False)
    h1, k1 = lat.hop_counts(), lat.counters()[1]
    dk = k1 - k0
    dh = {p: h1[p] - h0[p] for p in h1}
    say(f"  n_kmat {dk}, hops {dh}, log {log}")
    if kind == "POLY":      # no solve: P_4(J) = 4 J
        assert log == [] and dk == 4 and dh["f64"] == 16
        return
    (it, res, jpa), = log
    assert dk == (it + res) * jpa
    ip = inner
    if ip == "f64":
        assert dh["f64"] == 4 * dk
    else:                   # iterations in the inner precision, residuals in FP64
        assert dh[ip] == 4 * it * jpa and dh["f64"] == 4 * res * jpa
