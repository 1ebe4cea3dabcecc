"""GPU: the cost-metric driver (the paper's C = N_mat / P_acc) on a tiny lattice:
bookkeeping only (C = N_mat / P_acc per action, every action present)."""
import pytest

from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def test_cost_driver_bookkeeping():
    need_gpu()
    from paper_1702_00124_amd import cost
    say("cost driver 4^4")
    out = cost.run((4, 4, 4, 4), 0.155, 5.6, ntherm=2, ntraj=3, actions=["MP", "2PF-1MP"], steps=(4, 2, 8),
                   log=lambda *a: say(*a))
    assert set(out["actions"]) == {"MP", "2PF-1MP"}
    for name, r in out["actions"].items():
        assert r["N_mat"] > 0 and 0.0 <= r["P_acc"] <= 1.0
        if r["P_acc"] > 0:
            assert abs(r["C"] - r["N_mat"] / r["P_acc"]) <= 0.1 + 1e-6 * r["C"]
