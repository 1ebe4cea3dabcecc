"""GPU: apply_K_noalloc, the allocation-free variant of apply_K (intermediates in the
library's fixed device scratch), against apply_K on the same inputs and against the
FP64 oracle.

The two entry points run the same kernels with the same launch configuration on the
same inputs, so their outputs must be bit-identical; the FP64 results also meet the
1e-12 oracle bar of the operator tests.  Two calls in a row, the second on a smaller
input (fewer rhs, then a smaller lattice), check that the scratch the first call left
does not leak into the second.  A request beyond the scratch limit is refused before
anything is launched.
"""
import numpy as np
import pytest
import torch

from oracle import wilson as ow
from tests.gpu_common import full_noise, half_noise, make_lattice, rel, say, to_np

pytestmark = pytest.mark.gpu

KAPPA = 0.155


def _pair(lat, buf, op, prec, nrhs, mu2, full=False):
    ref = lat.apply_K(buf, KAPPA, op, mu2=mu2, prec=prec, nrhs=nrhs)
    out = lat.new_field(prec, nrhs, full=full)
    out.fill_(0x7F)   # stale bytes: the entry point must overwrite every site
    lat.apply_K_noalloc(buf, out, KAPPA, op, mu2=mu2, prec=prec, nrhs=nrhs)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_noalloc_matches_apply_K_two_calls(prec):
    # first call: 8^3 x 16, 4 rhs; second: 4^4, 1 rhs (smaller), on the same device scratch
    for L, nrhs, seed in (((8, 8, 8, 16), 4, 61), ((4, 4, 4, 4), 1, 62)):
        say("noalloc", prec, L, "nrhs", nrhs)
        lat, U = make_lattice(L)
        e = half_noise(L, seed, nrhs=nrhs)
        buf = lat.import_spinor(torch.from_numpy(e), prec)
        mu2 = [0.0, 0.005, 0.05, 0.5][:nrhs]
        for op in ("J", "MHAT", "MHAT_DAG"):
            ref, got = _pair(lat, buf, op, prec, nrhs, mu2)
            # the sites as the canonical export gives them (exact in every precision)
            r_c = lat.export_spinor(ref, prec, nrhs)
            g_c = lat.export_spinor(got, prec, nrhs)
            assert torch.equal(r_c, g_c), (op, L, nrhs)
            if prec == "f64":
                g = to_np(g_c).reshape(nrhs, -1, 4, 3)
                for r in range(nrhs):
                    want = (ow.J(U, e.reshape(nrhs, -1, 4, 3)[r], L, KAPPA, mu2[r]) if op == "J" else
                            ow.Mhat(U, e.reshape(nrhs, -1, 4, 3)[r], L, KAPPA, dagger=(op == "MHAT_DAG")))
                    assert rel(g[r], want) <= 1e-12, (op, r)
        if prec == "f64":
            f = full_noise(L, seed + 10)
            fb = lat.import_full(torch.from_numpy(f))
            for op, want in (("K", ow.K(U, f, L, 0.12)), ("M", ow.M(U, f, L, 0.12))):
                ref = lat.apply_K(fb, 0.12, op)
                out = lat.new_field("f64", 1, full=True)
                out.fill_(0x7F)
                lat.apply_K_noalloc(fb, out, 0.12, op)
                torch.cuda.synchronize()
                assert torch.equal(lat.export_full(ref), lat.export_full(out)), op
                assert rel(to_np(lat.export_full(out)), want) <= 1e-12, op
        lat.close()


def test_noalloc_refuses_beyond_scratch_limit():
    from paper_1702_00124_amd import WilsonError
    L = (16, 16, 16, 32)
    say("noalloc limit", L)
    lat, _ = make_lattice(L)
    # J on 16 FP64 rhs needs 2 x 16 fields of 12.7 MB: above the 256 MiB scratch
    buf = lat.new_field("f64", 16)
    out = lat.new_field("f64", 16)
    with pytest.raises(WilsonError, match="scratch"):
        lat.apply_K_noalloc(buf, out, KAPPA, "J", mu2=[0.0] * 16, nrhs=16)
    # one FP64 rhs fits, and matches apply_K
    e = half_noise(L, 63)
    b1 = lat.import_spinor(torch.from_numpy(e))
    o1 = lat.new_field("f64", 1)
    lat.apply_K_noalloc(b1, o1, KAPPA, "J", mu2=[0.05])
    ref = lat.apply_K(b1, KAPPA, "J", mu2=[0.05])
    torch.cuda.synchronize()
    assert torch.equal(lat.export_spinor(ref), lat.export_spinor(o1))
    lat.close()
