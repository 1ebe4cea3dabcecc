"""GPU parity: CG (FP64, mixed precision, batched, graph-captured) against the FP64 oracle.

Protocol (solutions are only tolerance-accurate): both sides solve to a
relative true residual tol; the difference of solutions is bounded by
cond(A) * (r_gpu + r_cpu) <= cond * 2 tol.  With cond(K) < 100 on these
lattices, tol = 1e-12 gives <= 2e-10, asserted as 1e-9.
"""
import numpy as np
import pytest
import torch

from oracle import solver as osol, wilson as ow
from paper_1702_00124_amd.lattice import CG
from paper_1702_00124_amd import _lib as W
from tests.gpu_common import full_noise, half_noise, make_lattice, need_gpu, rel, say, to_np

pytestmark = pytest.mark.gpu


def test_cg_full_lattice_small_workload():
    """4^4, kappa = 0.12, full K = M^dag M, FP64 (the small two-flavour workload)."""
    L, kappa = (4, 4, 4, 4), 0.12
    say("cg full K", L)
    lat, U = make_lattice(L, a=0.3, seed=1001)
    b = full_noise(L, 2001)
    x, st, rc = lat.cg_solve(lat.import_full(torch.from_numpy(b)), kappa, "K", params=CG(tol=1e-12))
    assert rc == 0 and st[0].converged and st[0].true_rel_res <= 1e-12
    xg = to_np(lat.export_full(x))
    xr, _, _ = osol.cg(lambda v: ow.K(U, v, L, kappa), b, tol=1e-12)
    assert rel(xg, xr) <= 1e-9
    assert rel(ow.K(U, xg, L, kappa), b) <= 1e-11


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("inner", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("graph", [False, True])
def test_cg_even_odd_precisions(inner, graph, variant):
    """Both hop variants: the fused <p, J p> partials of each feed the CG."""
    L, kappa, mu2 = (8, 8, 8, 8), 0.155, 0.0
    say("cg J", inner, "graph" if graph else "eager", "variant", variant)
    lat, U = make_lattice(L, variant=variant)
    b = half_noise(L, 2002)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), kappa, "J", mu2=[mu2],
                             params=CG(tol=1e-10, inner=inner, use_graph=graph))
    say(f"  iters {st[0].iters} reliable {st[0].reliable_updates} true res {st[0].true_rel_res:.2e}")
    assert rc == 0 and st[0].converged and st[0].true_rel_res <= 1e-10
    xg = to_np(lat.export_spinor(x))
    assert rel(ow.J(U, xg, L, kappa, mu2), b) <= 1e-10 * 1.01
    xr, _, _ = osol.cg(lambda v: ow.J(U, v, L, kappa, mu2), b, tol=1e-10)
    assert rel(xg, xr) <= 200 * 2e-10


@pytest.mark.parametrize("variant,passes", [(0, 1), (0, 2), (1, 1), (1, 2), (1, 4)])
def test_cg_batched_shifts_match_single(variant, passes):
    """8 rhs, rhs j with shift mu2[j mod 4] (the batched multi-rhs workload's
    pairing), for each multi-rhs hop layout: thread per site, and the
    direction-parallel kernel with 1, 2 or 4 rhs passes per link load (for the
    site kernel, passes >= 2 means two rhs per thread)."""
    L, kappa = (6, 4, 4, 10), 0.155
    mu2 = [0.0, 0.005, 0.05, 0.5] * 2
    say("cg batched 8 rhs, variant", variant, "passes", passes)
    lat, U = make_lattice(L, variant=variant)
    for prec in ("f64", "f32", "bf16"):
        lat.set_hop_config(prec, -1, npass=passes)
    b = half_noise(L, 2010, nrhs=8)
    for inner in ("f64", "f32"):
        x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), kappa, "J", mu2=mu2, nrhs=8,
                                 params=CG(tol=1e-10, inner=inner, use_graph=True))
        assert rc == 0
        xg = to_np(lat.export_spinor(x, "f64", 8))
        for j in range(8):
            assert st[j].converged and st[j].true_rel_res <= 1e-10
            assert rel(ow.J(U, xg[j], L, kappa, mu2[j]), b[j]) <= 1.01e-10
        its = [s.iters for s in st]
        say(f"  {inner}: iterations per rhs {its}")
        # heavier shifts converge faster
        assert its[3] < its[0]


def test_cg_nonconvergence_and_zero_rhs():
    L = (4, 4, 4, 4)
    say("cg edge cases")
    lat, U = make_lattice(L)
    b = half_noise(L, 3)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", params=CG(tol=1e-10, maxiter=1, chunk=1))
    assert rc == -5 and not st[0].converged and st[0].iters == 1
    z = np.zeros_like(b)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(z)), 0.155, "J")
    assert rc == 0 and st[0].iters == 0 and np.abs(to_np(lat.export_spinor(x))).max() == 0.0


def test_multishift_cg_matches_oracle():
    """8 sources x 4 Hasenbusch shifts (given unsorted) in one Krylov space per source:
    every solution against the oracle's multi-shift CG and its own true residual."""
    from oracle import solver as osl
    L, kappa = (6, 4, 4, 10), 0.155
    shifts = [0.5, 0.0, 0.05, 0.005]
    nrhs = 8
    say("multi-shift cg", nrhs, "sources", shifts)
    lat, U = make_lattice(L)
    b = half_noise(L, 2020, nrhs=nrhs)
    x, st, rc = lat.cg_multishift(lat.import_spinor(torch.from_numpy(b)), kappa, shifts, nrhs,
                                  CG(tol=1e-11, chunk=4))
    assert rc == 0
    A = lambda v: ow.Khat(U, v, L, kappa)
    for s, sh in enumerate(shifts):
        xg = to_np(lat.export_spinor(lat.shift_block(x, s, nrhs), "f64", nrhs))
        say(f"  shift {sh}: iterations {[c.iters for c in st[s]]}")
        for r in range(nrhs):
            assert st[s][r].converged and st[s][r].true_rel_res <= 1e-11
            assert rel(ow.J(U, xg[r], L, kappa, sh), b[r]) <= 1.01e-11
        xr, _, _ = osl.cg_multishift(A, b[0], shifts, tol=1e-11)
        assert rel(xg[0], xr[s]) <= 100 * 2e-11
    # heavier shifts freeze earlier
    assert st[0][0].iters < st[1][0].iters


def test_multishift_refinement_and_edges():
    """A base run cut short by maxiter is finished by per-system refinement; a zero
    source gives zero solutions; too many systems is an error."""
    L, kappa = (4, 4, 4, 4), 0.155
    lat, U = make_lattice(L)
    b = half_noise(L, 2021, nrhs=2)
    b[1] = 0.0
    shifts = [0.0, 0.05]
    x, st, rc = lat.cg_multishift(lat.import_spinor(torch.from_numpy(b)), kappa, shifts, 2,
                                  CG(tol=1e-10, maxiter=8, chunk=4))
    assert rc == 0
    for s, sh in enumerate(shifts):
        xg = to_np(lat.export_spinor(lat.shift_block(x, s, 2), "f64", 2))
        assert st[s][0].reliable_updates == 1 and st[s][0].converged
        assert rel(ow.J(U, xg[0], L, kappa, sh), b[0]) <= 1.01e-10
        assert np.abs(xg[1]).max() == 0.0 and st[s][1].converged
    with pytest.raises(Exception):
        lat.cg_multishift(lat.import_spinor(torch.from_numpy(half_noise(L, 1, nrhs=16))), kappa, [0.0] * 5, 16)


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_cg_initial_guess(inner):
    """use_x0: the solution itself as x0 takes no iteration and is kept; a
    perturbed solution converges to the same tolerance in fewer iterations
    than x0 = 0; a zero source with a non-zero x0 returns x = 0."""
    L, kappa, mu2 = (8, 8, 8, 8), 0.155, 0.0
    say("cg initial guess", inner)
    lat, U = make_lattice(L)
    b = half_noise(L, 2101)
    bg = lat.import_spinor(torch.from_numpy(b))
    x, st, rc = lat.cg_solve(bg, kappa, "J", mu2=[mu2], params=CG(tol=1e-10, inner=inner))
    cold = st[0].iters
    assert rc == 0 and st[0].converged
    xs = to_np(lat.export_spinor(x))
    # exact solution as the guess
    x1 = x.clone()
    _, st1, rc1 = lat.cg_solve(bg, kappa, "J", mu2=[mu2], params=CG(tol=1e-10, inner=inner, use_x0=True), x=x1)
    assert rc1 == 0 and st1[0].converged and st1[0].iters == 0
    assert torch.equal(x1, x)
    # perturbed guess
    pert = xs + 1e-4 * np.linalg.norm(xs) / np.sqrt(xs.size) * half_noise(L, 2102)
    x2 = lat.import_spinor(torch.from_numpy(pert))
    _, st2, rc2 = lat.cg_solve(bg, kappa, "J", mu2=[mu2], params=CG(tol=1e-10, inner=inner, use_x0=True), x=x2)
    say(f"  iters cold {cold}, from perturbed guess {st2[0].iters}")
    assert rc2 == 0 and st2[0].converged and st2[0].true_rel_res <= 1e-10
    assert 0 < st2[0].iters < cold
    xg = to_np(lat.export_spinor(x2))
    assert rel(ow.J(U, xg, L, kappa, mu2), b) <= 1e-10 * 1.01
    # zero source
    x3 = x.clone()
    _, st3, rc3 = lat.cg_solve(lat.new_field("f64").zero_(), kappa, "J", mu2=[mu2],
                               params=CG(tol=1e-10, inner=inner, use_x0=True), x=x3)
    assert rc3 == 0 and st3[0].iters == 0 and not torch.any(x3)


def test_cg_initial_guess_full_lattice_and_batched():
    """use_x0 on the full-lattice K and on a 4-rhs batch whose guesses are
    mixed: exact, perturbed, zero, exact."""
    L, kappa = (4, 4, 4, 4), 0.12
    say("cg initial guess, full K and batched J")
    lat, U = make_lattice(L, a=0.3, seed=1001)
    b = full_noise(L, 2103)
    bg = lat.import_full(torch.from_numpy(b))
    x, st, _ = lat.cg_solve(bg, kappa, "K", params=CG(tol=1e-12))
    x1 = x.clone()
    _, st1, rc1 = lat.cg_solve(bg, kappa, "K", params=CG(tol=1e-12, use_x0=True), x=x1)
    assert rc1 == 0 and st1[0].iters == 0 and torch.equal(x1, x)

    L, kappa = (6, 4, 4, 10), 0.155
    lat, U = make_lattice(L)
    bs = [half_noise(L, 2110 + j) for j in range(4)]
    bg = torch.cat([lat.import_spinor(torch.from_numpy(v)) for v in bs])
    mu2 = [0.0, 0.01, 0.05, 0.2]
    x, st, rc = lat.cg_solve(bg, kappa, "J", mu2=mu2, nrhs=4, params=CG(tol=1e-11))
    assert rc == 0
    fb = lat.field_bytes("f64")
    x0 = x.clone()
    xs1 = to_np(lat.export_spinor(x[fb:2 * fb]))
    x0[fb:2 * fb] = lat.import_spinor(torch.from_numpy(xs1 + 1e-3 * half_noise(L, 2120)))
    x0[2 * fb:3 * fb] = 0
    _, st0, rc0 = lat.cg_solve(bg, kappa, "J", mu2=mu2, nrhs=4, params=CG(tol=1e-11, use_x0=True), x=x0)
    say(f"  iters cold {[s.iters for s in st]}, guessed {[s.iters for s in st0]}")
    assert rc0 == 0 and all(s.converged for s in st0)
    assert st0[0].iters == 0 and st0[3].iters == 0
    assert 0 < st0[1].iters < st[1].iters and st0[2].iters == st[2].iters
    assert torch.equal(x0[:fb], x[:fb]) and torch.equal(x0[3 * fb:], x[3 * fb:])
    for j in range(4):
        xg = to_np(lat.export_spinor(x0[j * fb:(j + 1) * fb]))
        assert rel(ow.J(U, xg, L, kappa, mu2[j]), bs[j]) <= 1e-11 * 1.01


def test_multishift_rejects_initial_guess():
    from paper_1702_00124_amd import _lib as W
    L = (4, 4, 4, 4)
    lat, U = make_lattice(L)
    b = lat.import_spinor(torch.from_numpy(half_noise(L, 2130)))
    with pytest.raises(W.WilsonError):
        lat.cg_multishift(b, 0.155, [0.0, 0.1], params=CG(use_x0=True))


def test_cg_rejects_non_finite_source():
    """A NaN or Inf in b is reported as WL_EINVAL before any iteration."""
    from paper_1702_00124_amd import _lib as W
    L = (4, 4, 4, 4)
    lat, U = make_lattice(L)
    for bad in (np.nan, np.inf):
        b = half_noise(L, 2140)
        b[7, 1, 2] = bad
        with pytest.raises(W.WilsonError) as e:
            lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", params=CG(inner="f32"))
        assert e.value.code == W.WL_EINVAL and "non-finite" in str(e.value)


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_cg_breakdown_terminates(inner):
    """J = K-hat - 10 is negative definite (spec K-hat lies in [0, (1 + 64 kappa^2)^2]):
    <p, J p> < 0 breaks the iteration at once; the solver restarts, then gives
    up with WL_ENOCONV instead of looping, leaving a finite x."""
    L = (4, 4, 4, 4)
    lat, U = make_lattice(L)
    b = half_noise(L, 2150)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", mu2=[-10.0],
                             params=CG(tol=1e-10, inner=inner, maxiter=1000, chunk=4))
    say(f"  {inner}: rc {rc}, iters {st[0].iters}, reliable updates {st[0].reliable_updates}")
    assert rc == W.WL_ENOCONV and not st[0].converged
    assert np.isfinite(to_np(lat.export_spinor(x))).all()


def test_cg_graph_recaptured_after_workspace_grows():
    """Regression: on a fresh lattice a graph-captured FP32-inner CG whose first
    FP64 reliable update comes after the capture (threshold 0.001, chunks of 2)
    grows the operator's workspace in that update; the chunk graph is captured
    again instead of being replayed with the freed buffers."""
    L, kappa = (8, 8, 8, 8), 0.155
    lat, U = make_lattice(L)
    b = half_noise(L, 2160)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), kappa, "J", mu2=[0.0],
                             params=CG(tol=1e-10, inner="f32", delta=0.001, chunk=2, use_graph=True))
    say(f"  iters {st[0].iters}, reliable updates {st[0].reliable_updates}")
    assert rc == 0 and st[0].converged
    assert rel(ow.J(U, to_np(lat.export_spinor(x)), L, kappa, 0.0), b) <= 1.01e-10


def test_kappa_zero_degenerate():
    """kappa = 0, where the hopping term drops out of M = 1 - kappa D and
    M-hat = 1 - kappa^2 D_eo D_oe (Sec. 2): M, M^dag, K, M-hat and M-hat^dag are
    the identity bit for bit in FP64 and J = (1 + mu2) times it; CG on J stops
    after one iteration at b / (1 + mu2); the filter's four forms are the oracle's
    polynomials of the number 1 + mu2 (n = 16 on [0.001, 8]); an action term with
    kappa = 0 is refused."""
    from oracle import poly as opoly
    from paper_1702_00124_amd.lattice import Term
    L = (6, 4, 4, 10)
    mu2 = 0.05
    lat, _ = make_lattice(L)
    psi = half_noise(L, 81)
    full = full_noise(L, 82)
    x = lat.import_spinor(torch.from_numpy(psi))
    xf = lat.import_full(torch.from_numpy(full))
    for op in ("MHAT", "MHAT_DAG"):
        assert np.array_equal(to_np(lat.export_spinor(lat.apply_K(x, 0.0, op=op))), psi), op
    for op in ("M", "MDAG", "K"):
        assert np.array_equal(to_np(lat.export_full(lat.apply_K(xf, 0.0, op=op))), full), op
    assert rel(to_np(lat.export_spinor(lat.apply_K(x, 0.0, op="J", mu2=(mu2,)))), (1 + mu2) * psi) <= 1e-15
    sol, st, rc = lat.cg_solve(x, 0.0, "J", mu2=(mu2,))
    assert rc == 0 and st[0].iters == 1 and st[0].true_rel_res <= 1e-14
    assert rel(to_np(lat.export_spinor(sol)), psi / (1 + mu2)) <= 1e-14
    scale = lambda v: (1 + mu2) * v
    for mode, ref in (("P", opoly.apply_P(scale, psi, 16, 0.001, 8.0)),
                      ("PJ", opoly.apply_PJ(scale, psi, 16, 0.001, 8.0)),
                      ("Q", opoly.apply_Q(scale, psi, 16, 0.001, 8.0)),
                      ("QDAG", opoly.apply_Q(scale, psi, 16, 0.001, 8.0, dagger=True))):
        got = to_np(lat.export_spinor(lat.poly_filter_apply(x, 0.0, mu2, 16, 0.001, 8.0, mode)))
        say(f"kappa = 0, filter {mode}: relative difference {rel(got, ref):.2e}")
        assert rel(got, ref) <= 1e-12, mode
    with pytest.raises(W.WilsonError):
        lat.heatbath(Term("KINV", 0.0, mu2), lat.import_spinor(torch.from_numpy(psi)))
    lat.close()
