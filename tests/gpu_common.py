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
