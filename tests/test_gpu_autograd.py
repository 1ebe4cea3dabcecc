"""GPU: the autograd.Function whose backward is the force kernel, against the
FP64 oracle's force and central finite differences of the library's own
action (solves at tol 1e-13 on both sides)."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
from oracle import action as oact
from paper_1702_00124_amd.autograd import pseudofermion_action
from paper_1702_00124_amd.lattice import CG, Term
from tests.gpu_common import half_noise, make_lattice, rel, say, to_np

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)


@pytest.mark.parametrize("kind", ["RATIO", "POLYK_INV"])
def test_backward_is_force_and_matches_finite_differences(kind):
    say("autograd", kind)
    lat, U = make_lattice(L4)
    shift = dict(mu2_num=0.05) if kind == "RATIO" else dict(mu2=0.05)
    term = Term(kind, 0.155, degree=4, cg=CG(tol=1e-13), **shift)
    phi_np = half_noise(L4, 4001)
    phi = lat.import_spinor(torch.from_numpy(phi_np))
    omega = torch.zeros((4, lat.V, 8), dtype=torch.float64, device=lat.device, requires_grad=True)
    S = pseudofermion_action(omega, phi, lat, term)
    S.backward()
    g = to_np(omega.grad)
    ref = oact.force(oact.Ops(U, L4), oact.Term(kind, 0.155, n=4, tol=1e-13, **shift), phi_np)
    assert rel(g, ref) <= 1e-9
    # links restored, and central differences along a random direction
    assert np.array_equal(to_np(lat.get_links()), U)
    v = torch.from_numpy(np.random.default_rng(3).standard_normal((4, lat.V, 8))).to(lat.device)
    eps = 1e-5
    with torch.no_grad():
        sp = pseudofermion_action(eps * v, phi, lat, term).item()
        sm = pseudofermion_action(-eps * v, phi, lat, term).item()
    fd = (sp - sm) / (2 * eps)
    an = float((omega.grad * v).sum())
    say(f"  fd {fd:.8f} analytic {an:.8f}")
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
