"""GPU parity on the other volumes of the batched multi-rhs workload, after the
autotuner has picked each launch configuration:

* 8^3 x 16: V_h = 4096, 64 hop tiles and 16 site-kernel blocks (XCD order on);
* 12^3 x 24: V_h = 20736, 324 hop tiles and 81 site-kernel blocks, neither a
  multiple of the 8 XCDs, so the plain workgroup order.

The hop in every precision for 1 and 8 rhs against the oracle's whole-lattice
hop (bounds as in the small-lattice hop tests), and the 8-rhs batched CG over
the four shifts mu2 in {0, 0.005, 0.05, 0.5} (rhs j with shift j mod 4), FP32
and BF16 inner with FP64 reliable updates, by its FP64 true residual under the
oracle's J.
"""
import pytest
import torch

from oracle import wilson as ow
from paper_1702_00124_amd.lattice import CG
from tests.gpu_common import check_prec, half_noise, make_lattice, rel, say, to_np

pytestmark = pytest.mark.gpu

KAPPA = 0.155
SHIFTS = [0.0, 0.005, 0.05, 0.5]
TOL = {"f64": 1e-12, "f32": 1e-6, "bf16": 2e-2}


@pytest.fixture(scope="module", params=[(8, 8, 8, 16), (12, 12, 12, 24)], ids=["8x16", "12x24"])
def tuned(request):
    L = request.param
    say("volume", L, "autotune")
    lat, U = make_lattice(L)
    lat.autotune()
    say("  kept:", {p: [lat.hop_config(p, k) for k in range(3)] for p in ("f64", "f32", "bf16")})
    yield L, lat, U
    lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 8])
def test_hop_matches_oracle(tuned, prec, nrhs):
    L, lat, U = tuned
    for parity in (0, 1):
        say("hop", L, prec, "nrhs", nrhs, "parity", parity)
        psi = half_noise(L, 300 + parity, nrhs=nrhs)
        out = lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), parity, prec=prec, nrhs=nrhs)
        got = to_np(lat.export_spinor(out, prec, nrhs)).reshape(psi.shape)
        for r in range(nrhs):
            ref = ow.hop_eo(U, psi[r], L, parity, t_bc=-1)
            check_prec(got[r], ref, prec, (nrhs, parity, r))


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_batched_cg_over_shifts(tuned, inner):
    L, lat, U = tuned
    say("batched cg", L, inner)
    mu2 = [SHIFTS[j % 4] for j in range(8)]
    b = half_noise(L, 400, nrhs=8)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), KAPPA, "J", mu2=mu2, nrhs=8,
                             params=CG(tol=1e-10, inner=inner, use_graph=True))
    say(f"  iterations {[s.iters for s in st]}, reliable updates {st[0].reliable_updates}")
    assert rc == 0
    xg = to_np(lat.export_spinor(x, "f64", 8))
    for j in range(8):
        assert st[j].converged and st[j].true_rel_res <= 1e-10
        assert rel(ow.J(U, xg[j], L, KAPPA, mu2[j]), b[j]) <= 1.01e-10
