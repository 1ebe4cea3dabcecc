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
                   therm_steps=(6, 3, 10), log=lambda *a: say(*a))
    assert set(out["actions"]) == {"MP", "2PF-1MP"}
    assert out["steps_rule"] == [4, 2, 8] and out["therm_steps_rule"] == [6, 3, 10]
    assert out["actions"]["2PF-1MP"]["nsteps"] == [4, 2, 2, 2, 8]
    for name, r in out["actions"].items():
        assert r["N_mat"] > 0 and 0.0 <= r["P_acc"] <= 1.0
        if r["P_acc"] > 0:
            assert abs(r["C"] - r["N_mat"] / r["P_acc"]) <= 0.1 + 1e-6 * r["C"]


def test_cost_driver_checkpoint_resume_is_bit_exact(tmp_path):
    """The chains stopped every 3 trajectories and resumed from the checkpoint
    give the uninterrupted run's numbers exactly (same launch configurations
    through the autotuner cache; every random input derived from the
    trajectory index)."""
    need_gpu()
    from paper_1702_00124_amd import cost
    tune = str(tmp_path / "tune.json")
    kw = dict(ntherm=2, ntraj=3, actions=["MP", "PF-MP"], steps=(4, 2, 8), tune_cache=tune,
              log=lambda *a: say(*a))
    say("cost driver checkpoint / resume 4^4")
    full = cost.run((4, 4, 4, 4), 0.155, 5.6, **kw)
    ck = str(tmp_path / "ck")
    calls, out = 0, None
    while out is None:
        out = cost.run((4, 4, 4, 4), 0.155, 5.6, checkpoint=ck, max_traj=3, **kw)
        calls += 1
        assert calls <= 5
    assert calls == 3   # 2 + 3 + 3 trajectories in calls of at most 3
    assert out["thermalised_plaquette"] == full["thermalised_plaquette"]
    for name, a in full["actions"].items():
        b = out["actions"][name]
        for key in ("C", "P_acc", "N_mat", "cg_iters", "exp_minus_dH", "dH_rms", "plaquette"):
            assert a[key] == b[key], (name, key)
    with pytest.raises(ValueError):
        cost.run((4, 4, 4, 4), 0.150, 5.6, checkpoint=ck, **kw)
