"""GPU parity of the mixed-volume batch (several lattices' hops in one
persistent launch; J and CG on top) against the FP64 oracle and against the
single-lattice path.

Two batches: the workload's volumes 8^3x16, 12^3x24 and 16^3x32 (kappa 0.155,
0.150, 0.145; own links each), and small ragged ones (4^4, 6x4x4x10 with a
half-empty last tile, 8^4).  Bounds as in the single-lattice tests: FP64 hop
1e-12, FP32 1e-6, BF16 2e-2; solves by their FP64 true residual under the
oracle's J, and solutions against single-lattice solutions to cond * 2 tol.
"""
import numpy as np
import pytest
import torch

from oracle import wilson as ow
from paper_1702_00124_amd import _lib as W
from paper_1702_00124_amd.lattice import CG, WilsonBatch
from tests.gpu_common import check_prec, half_noise, make_lattice, rel, say, to_np

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16": 2e-2}
WORKLOAD = [((8, 8, 8, 16), 0.155, 0.0), ((12, 12, 12, 24), 0.150, 0.005), ((16, 16, 16, 32), 0.145, 0.05)]
RAGGED = [((4, 4, 4, 4), 0.155, 0.0), ((6, 4, 4, 10), 0.150, 0.05), ((8, 8, 8, 8), 0.145, 0.5)]


def _batch(spec, seed0):
    lats, links = [], []
    for i, (L, _, _) in enumerate(spec):
        lat, U = make_lattice(L, seed=seed0 + i)
        lats.append(lat)
        links.append(U)
    return WilsonBatch(lats), lats, links


@pytest.fixture(scope="module", params=["workload", "ragged"])
def batch(request):
    spec = WORKLOAD if request.param == "workload" else RAGGED
    say("batch", request.param, [s[0] for s in spec])
    B, lats, links = _batch(spec, 1500 if request.param == "workload" else 1600)
    yield spec, B, lats, links
    B.close()
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_batch_dslash_matches_oracle(batch, prec):
    spec, B, lats, links = batch
    for parity, dagger in ((0, False), (1, False), (0, True)):
        psi = [half_noise(L, 700 + 10 * i + parity) for i, (L, _, _) in enumerate(spec)]
        out = B.unpack(B.dslash(B.pack([torch.from_numpy(p) for p in psi], prec), parity, dagger, prec), prec)
        for i, (L, _, _) in enumerate(spec):
            ref = ow.hop_eo(links[i], psi[i], L, parity, t_bc=-1, dagger=dagger)
            err, emax = check_prec(to_np(out[i]), ref, prec, (parity, dagger, L))
            say(f"  {prec} parity {parity} dagger {dagger} {L}: {err:.2e} (max element {emax:.2e})")


def test_batch_J_matches_single_lattice_and_oracle(batch):
    spec, B, lats, links = batch
    kappa = [s[1] for s in spec]
    mu2 = [s[2] for s in spec]
    psi = [half_noise(L, 800 + i) for i, (L, _, _) in enumerate(spec)]
    out = B.unpack(B.apply_J(B.pack([torch.from_numpy(p) for p in psi]), kappa, mu2))
    for i, (L, k, m) in enumerate(spec):
        single = to_np(lats[i].export_spinor(lats[i].apply_K(lats[i].import_spinor(torch.from_numpy(psi[i])), k, "J",
                                                             mu2=[m])))
        got = to_np(out[i])
        assert rel(got, single) <= 1e-14, L
        assert rel(got, ow.J(links[i], psi[i], L, k, m)) <= 1e-12, L


@pytest.mark.parametrize("inner,graph", [("f64", False), ("f32", True), ("bf16", True)])
def test_batch_cg_matches_oracle_residual_and_single_solves(batch, inner, graph):
    spec, B, lats, links = batch
    kappa = [s[1] for s in spec]
    mu2 = [s[2] for s in spec]
    b = [half_noise(L, 900 + i) for i, (L, _, _) in enumerate(spec)]
    say("batch cg", inner, "graph" if graph else "eager")
    x, st, rc = B.cg_solve(B.pack([torch.from_numpy(v) for v in b]), kappa, mu2,
                           CG(tol=1e-10, inner=inner, use_graph=graph))
    say(f"  iterations {[s.iters for s in st]}, reliable updates {st[0].reliable_updates}")
    assert rc == 0
    xs = B.unpack(x)
    for i, (L, k, m) in enumerate(spec):
        assert st[i].converged and st[i].true_rel_res <= 1e-10
        xg = to_np(xs[i])
        assert rel(ow.J(links[i], xg, L, k, m), b[i]) <= 1.01e-10, L
        xsingle, s1, rc1 = lats[i].cg_solve(lats[i].import_spinor(torch.from_numpy(b[i])), k, "J", mu2=[m],
                                            params=CG(tol=1e-10, inner=inner))
        assert rc1 == 0
        assert rel(xg, to_np(lats[i].export_spinor(xsingle))) <= 200 * 2e-10, L


MAX8 = [(4, 4, 4, 4), (6, 4, 4, 10), (4, 4, 4, 6), (8, 4, 4, 4), (4, 6, 4, 4), (4, 4, 6, 8), (6, 6, 4, 4),
        (8, 8, 8, 8)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_of_eight_lattices(prec):
    """The largest batch: 8 lattices, 63 tiles of 64 sites, two with a ragged last
    tile, so the eighths of the tile range that the XCDs walk straddle lattice
    boundaries; each lattice's hop against the oracle.  A ninth lattice is refused."""
    say("batch of 8", prec)
    lats, links = [], []
    for i, L in enumerate(MAX8):
        lat, U = make_lattice(L, seed=1700 + i)
        lats.append(lat)
        links.append(U)
    B = WilsonBatch(lats)
    psi = [half_noise(L, 720 + i) for i, L in enumerate(MAX8)]
    for parity, dagger in ((0, False), (1, True)):
        out = B.unpack(B.dslash(B.pack([torch.from_numpy(p) for p in psi], prec), parity, dagger, prec), prec)
        for i, L in enumerate(MAX8):
            check_prec(to_np(out[i]), ow.hop_eo(links[i], psi[i], L, parity, t_bc=-1, dagger=dagger), prec,
                       (parity, dagger, L))
    extra, _ = make_lattice((4, 4, 4, 4), seed=1799)
    with pytest.raises(W.WilsonError):
        WilsonBatch(lats + [extra])
    B.close()
    for lat in lats + [extra]:
        lat.close()


def test_batch_of_one_and_errors():
    L = (6, 4, 4, 10)
    lat, U = make_lattice(L)
    B = WilsonBatch([lat])
    b = half_noise(L, 950)
    x, st, rc = B.cg_solve(B.pack([torch.from_numpy(b)]), [0.155], [0.0], CG(tol=1e-12))
    assert rc == 0 and rel(ow.J(U, to_np(B.unpack(x)[0]), L, 0.155, 0.0), b) <= 1.01e-12
    with pytest.raises(W.WilsonError):
        B.cg_solve(B.pack([torch.from_numpy(b)]), [0.155], [0.0], CG(use_x0=True))
    import ctypes as C
    h = C.c_void_p()
    assert W.load().wl_batch_create(C.byref(h), None, 0) == W.WL_EINVAL
    B.close()
    lat.close()
