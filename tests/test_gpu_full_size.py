"""GPU parity at the full 32^3 x 64 size (1,048,576 sites per parity), in the launch
configurations the autotuner picks there (as the benchmark's large-volume leg does):
the hop on sampled output sites against the oracle's per-site evaluation, and the
mixed-precision batched CG by its FP64 true residual (a property at any size)."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
from oracle import wilson as ow
from paper_1702_00124_amd.lattice import CG
from tests.gpu_common import need_gpu, rel, say, to_np

pytestmark = pytest.mark.gpu

L = (32, 32, 32, 64)
TOL = {"f64": 1e-13, "f32": 1e-6, "bf16": 2e-2}


@pytest.fixture(scope="module")
def big():
    need_gpu()
    from paper_1702_00124_amd.lattice import WilsonLattice
    say("full size: links", L)
    U = li.random_links(L, 0.432, li.seed_links(4))
    lat = WilsonLattice(L, t_bc=-1)
    lat.set_links(torch.from_numpy(U))
    lat.autotune()
    say("  tuned:", {p: [lat.hop_config(p, k) for k in range(3)] for p in ("f64", "f32", "bf16")})
    yield lat, U
    lat.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_hop_sampled_sites_full_size(big, prec):
    lat, U = big
    Vh = lat.Vh
    sites = np.random.default_rng(11).choice(Vh, 256, replace=False)
    for nrhs in (1, 4):
        say("full size hop", prec, "nrhs", nrhs)
        psi = li.gaussian_spinor((nrhs, Vh, 4, 3), 5100 + nrhs)
        out = lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), 0, prec=prec, nrhs=nrhs)
        got = to_np(lat.export_spinor(out, prec, nrhs)).reshape(nrhs, Vh, 4, 3)
        for r in range(nrhs):
            ref = ow.hop_eo_at(U, psi[r], L, 0, sites, t_bc=-1)
            e = rel(got[r][sites], ref)
            say(f"  rhs {r}: sampled relative error {e:.2e}")
            assert e <= TOL[prec]
        del psi, out, got
    if prec == "f64":   # the other parity and the dagger, one rhs
        psi = li.gaussian_spinor((Vh, 4, 3), 5200)
        got = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi)), 1, True)))
        assert rel(got[sites], ow.hop_eo_at(U, psi, L, 1, sites, t_bc=-1, dagger=True)) <= TOL["f64"]


@pytest.mark.parametrize("inner", ["bf16", "f32"])
def test_batched_cg_full_size_true_residual(big, inner):
    """4 sources, kappa 0.156: every solution meets |b - J x| <= 1e-10 |b| with the
    library's FP64 J (parity-checked against the oracle at small sizes)."""
    lat, U = big
    say("full size CG, inner", inner)
    b = li.gaussian_spinor((4, lat.Vh, 4, 3), 5300)
    bb = lat.import_spinor(torch.from_numpy(b))
    x, st, rc = lat.cg_solve(bb, 0.156, "J", mu2=[0.0] * 4, nrhs=4, params=CG(tol=1e-10, inner=inner))
    say(f"  iterations {[s.iters for s in st]}, reliable updates {st[0].reliable_updates}")
    assert rc == 0
    Jx = to_np(lat.export_spinor(lat.apply_K(x, 0.156, "J", mu2=[0.0] * 4, nrhs=4), "f64", 4))
    for r in range(4):
        assert st[r].converged
        assert rel(Jx[r], b[r]) <= 1.01e-10
