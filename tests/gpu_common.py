"""Shared helpers of the GPU parity tests (seeded inputs, oracle comparisons)."""
import sys

import numpy as np
import pytest
import torch

import lattice_inputs as li
from oracle import lattice as olat


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def make_lattice(L, a=0.447, seed=1003, unit=False, variant=None):
    from paper_1702_00124_amd.lattice import WilsonLattice
    need_gpu()
    lat = WilsonLattice(L, t_bc=-1)
    if variant is not None:
        for prec in ("f64", "f32", "bf16"):
            lat.set_hop_variant(prec, variant)
    U = li.unit_links(L) if unit else li.random_links(L, a, seed)
    lat.set_links(torch.from_numpy(U))
    return lat, U


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    """max |a - b| / max |b|: catches an error confined to a few sites that the l2
    norm over the whole field would average away."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# Storage-precision bounds of one operator application against the FP64 result.
# l2: unit roundoff (FP32 2^-24, BF16 storage 2^-9) times the O(10) growth of one
# stencil application.  Max element (relative to the largest entry): the same
# roundoff on each entry's eight terms, whose largest lie within a few times the
# field's largest entry: FP32 1e-5, BF16 5e-2.  FP64 is held to the FP64 bar.
LOWP_L2 = {"f64": 1e-12, "f32": 1e-6, "bf16": 2e-2}
LOWP_MAX = {"f64": 1e-12, "f32": 1e-5, "bf16": 5e-2}


def check_prec(got, ref, prec, what=""):
    """Assert both bounds of LOWP_L2 / LOWP_MAX; returns (l2, max) errors."""
    e2, em = rel(got, ref), rel_max(got, ref)
    assert e2 <= LOWP_L2[prec], (what, prec, "l2", e2)
    assert em <= LOWP_MAX[prec], (what, prec, "max", em)
    return e2, em


def to_np(t):
    return t.detach().cpu().numpy()


def half_noise(L, seed, nrhs=None):
    Vh = li.volume(L) // 2
    shape = (Vh, 4, 3) if nrhs is None else (nrhs, Vh, 4, 3)
    return li.gaussian_spinor(shape, seed)


def full_noise(L, seed):
    return li.gaussian_spinor((li.volume(L), 4, 3), seed)


def su3_internal_to_canon(lat, F):
    return to_np(lat.export_su3(F))


def embed_parity(L, psi_h, p):
    return olat.embed(psi_h, L, p)
