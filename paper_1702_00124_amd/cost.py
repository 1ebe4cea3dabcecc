"""The paper's cost metric C = N_mat / P_acc (Sec. 3.1) for each of its actions.

    python -m paper_1702_00124_amd.cost [--lattice 8,8,8,16] [--kappa 0.155] [--beta 5.6]
        [--therm 60] [--traj 40] [--actions MP,PF-MP,...] [--steps 20,10,40] [--therm-steps 60,30,120]

N_mat is the number of fermion-matrix multiplications (K-hat and J applications,
including heatbath and action solves) per trajectory and P_acc the Metropolis
acceptance rate.  Seeded synthetic links (exp(i a H), a = 0.447) are first
thermalised by HMC with the MP action: every exact action samples the same
distribution det K-hat exp(-S_G), so one thermalised configuration serves all.
Each action then runs its own Markov chain of --traj trajectories from it, with
Omelyan steps (--steps: the cheapest term, every other term, the gauge action)
on tau = 1 (--therm-steps: the thermalisation's own rule, by default the same),
MD solves FP32 inner / FP64 reliable updates to 1e-10.  Reported per
action: C, P_acc, mean N_mat and CG iterations, <exp(-dH)> (1 in equilibrium, a
check of the integrator and the chain), plaquette, seconds per trajectory.

Every step runs in libwilson_hmc on the GPU; this module draws the host random
numbers (lattice_inputs) and does the bookkeeping.

Checkpoint and resume (--checkpoint DIR): between trajectories the chain state
(current links as canonical complex128, the thermalised links, the next
trajectory index, the rows of the current chain and the finished actions) is
written to DIR (state.json plus .npy arrays, each replaced atomically).  Every
random input is derived from the trajectory index, so a resumed run continues
the same chains bit for bit, given the same launch configurations (pass the
same --tune-cache to both runs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time


class Checkpoint:
    """Chain state between trajectories in a directory (JSON header + .npy arrays)."""

    def __init__(self, path):
        self.path = path
        os.makedirs(path, exist_ok=True)

    def _file(self, name):
        return os.path.join(self.path, name)

    def save_array(self, name, a):
        import numpy as np
        tmp = self._file(name + ".tmp.npy")
        np.save(tmp, a)
        os.replace(tmp, self._file(name + ".npy"))

    def load_array(self, name):
        import numpy as np
        return np.load(self._file(name + ".npy"))

    def save_state(self, state):
        tmp = self._file("state.json.tmp")
        with open(tmp, "w") as f:
            json.dump(state, f)
        os.replace(tmp, self._file("state.json"))

    def load_state(self):
        try:
            with open(self._file("state.json")) as f:
                return json.load(f)
        except OSError:
            return None


def run(L=(8, 8, 8, 16), kappa=0.155, beta=5.6, ntherm=60, ntraj=40, actions=None, steps=(20, 10, 40),
        log=print, checkpoint=None, max_traj=None, tune_cache=None, therm_steps=None):
    """checkpoint: directory for checkpoint / resume; max_traj: stop (returning
    None) after that many trajectories in this call, the state saved;
    tune_cache: autotuner cache file; therm_steps: the step rule of the
    thermalisation (default: steps)."""
    import numpy as np
    import torch

    import lattice_inputs as li
    from .actions import PAPER_ACTIONS, build_terms
    from .lattice import CG, WilsonLattice

    kappas = {"k": kappa, "kp": round(kappa - 0.005, 6), "k1": round(kappa - 0.010, 6),
              "k2": round(kappa - 0.005, 6)}
    names = list(actions or PAPER_ACTIONS)
    V = li.volume(L)
    Vh = V // 2
    lat = WilsonLattice(L, t_bc=-1)
    lat.set_links(torch.from_numpy(li.random_links(L, 0.447, li.seed_links(7))))
    lat.autotune(cache=tune_cache)
    cg = CG(tol=1e-10, inner="f32", chunk=8)
    ck = Checkpoint(checkpoint) if checkpoint else None
    run_key = {"lattice": list(L), "kappa": kappa, "beta": beta, "therm": ntherm, "traj": ntraj,
               "steps": list(steps), "therm_steps": list(therm_steps or steps), "actions": names}
    state = ck.load_state() if ck else None
    if state is not None:
        if state["run"] != run_key:
            lat.close()
            raise ValueError(f"checkpoint {checkpoint} belongs to another run: {state['run']}")
        lat.set_links(torch.from_numpy(ck.load_array("links")))
        log(f"resuming at phase {state['phase']}, trajectory {state['k']}")
    else:
        state = {"run": run_key, "phase": "therm", "k": 0, "rows": [], "done": {}}
    budget = [max_traj if max_traj is not None else -1]

    def nsteps_for(n, st):
        return [st[0]] + [st[1]] * (n - 1) + [st[2]]

    def chain(name, count, traj0, st=steps):
        """Trajectories state['k']..count-1 of one chain; None if the budget ran out."""
        terms = build_terms(name, kappas, cg)
        ns = nsteps_for(len(terms), st)
        u = li.uniforms(count, li.seed_metropolis(traj0))
        rows = [tuple(r) for r in state["rows"]]
        for k in range(state["k"], count):
            if budget[0] == 0:
                return None, ns
            budget[0] -= 1
            t = traj0 + k
            P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(L, li.seed_md(t, 15))))
            chi = torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(t, i))))
                             for i in range(len(terms))])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lat.hmc_trajectory(terms, ns, P, chi, float(u[k]), beta=beta, tau=1.0, integrator="omelyan")
            torch.cuda.synchronize()
            rows.append((r.dH, bool(r.accepted), int(r.n_kmat), int(r.cg_iters), r.plaquette,
                         time.perf_counter() - t0))
            log(f"{name} {k}: dH {r.dH:.4f} accepted {int(r.accepted)} n_mat {r.n_kmat} cg {r.cg_iters} "
                f"plaquette {r.plaquette:.5f} ({rows[-1][5]:.2f} s)")
            if ck:
                ck.save_array("links", lat.get_links().cpu().numpy())
                state["k"], state["rows"] = k + 1, rows
                ck.save_state(state)
        return rows, ns

    def next_phase(phase):
        state["phase"], state["k"], state["rows"] = phase, 0, []
        if ck:
            ck.save_state(state)

    t_start = time.time()
    if state["phase"] == "therm":
        rows, ns = chain("MP", ntherm, 100000, tuple(therm_steps or steps))
        if rows is None:
            lat.close()
            return None
        plaq = [r[4] for r in rows]
        log(f"thermalisation: {ntherm} MP trajectories, plaquette {plaq[0]:.4f} -> {plaq[-1]:.4f}, "
            f"acceptance {np.mean([r[1] for r in rows]):.2f} ({time.time() - t_start:.0f} s)")
        state["thermalised_plaquette"] = round(plaq[-1], 5)
        if ck:
            ck.save_array("links_therm", lat.get_links().cpu().numpy())
        next_phase(names[0] if names else "end")
    U0 = (torch.from_numpy(ck.load_array("links_therm")) if ck else lat.get_links().clone())
    out = {"lattice": list(L), "kappa": kappa, "kappas": kappas, "beta": beta, "therm": ntherm, "traj": ntraj,
           "steps_rule": list(steps), "therm_steps_rule": list(therm_steps or steps),
           "thermalised_plaquette": state["thermalised_plaquette"], "actions": {}}
    for ai, name in enumerate(names):
        if name in state["done"]:
            out["actions"][name] = state["done"][name]
            continue
        if state["k"] == 0:
            lat.set_links(U0)
        rows, ns = chain(name, ntraj, 200000 + 10000 * ai)
        if rows is None:
            lat.close()
            return None
        dH = np.array([r[0] for r in rows])
        acc = np.array([r[1] for r in rows], dtype=float)
        nmat = np.array([r[2] for r in rows], dtype=float)
        pacc = float(acc.mean())
        # binomial standard error of P_acc, propagated to C
        pe = math.sqrt(max(pacc * (1 - pacc), 1e-12) / len(rows))
        C = float(nmat.mean() / pacc) if pacc > 0 else float("inf")
        res = {"C": round(C, 1), "C_err": round(C * pe / pacc, 1) if pacc > 0 else None,
               "P_acc": round(pacc, 3), "N_mat": round(float(nmat.mean()), 1),
               "cg_iters": round(float(np.mean([r[3] for r in rows])), 1),
               "exp_minus_dH": round(float(np.mean(np.exp(-dH))), 3),
               "exp_minus_dH_err": round(float(np.std(np.exp(-dH)) / math.sqrt(len(rows))), 3),
               "dH_rms": round(float(np.sqrt(np.mean(dH ** 2))), 4),
               "plaquette": round(float(np.mean([r[4] for r in rows])), 5),
               "seconds_per_traj": round(float(np.mean([r[5] for r in rows])), 3), "nsteps": ns}
        out["actions"][name] = res
        state["done"][name] = res
        next_phase(names[ai + 1] if ai + 1 < len(names) else "end")
        log(f"{name}: " + json.dumps(res))
    lat.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--lattice", default="8,8,8,16")
    ap.add_argument("--kappa", type=float, default=0.155)
    ap.add_argument("--beta", type=float, default=5.6)
    ap.add_argument("--therm", type=int, default=60)
    ap.add_argument("--traj", type=int, default=40)
    ap.add_argument("--actions", default=None, help="comma-separated subset of the paper's actions")
    ap.add_argument("--steps", default="20,10,40", help="steps: cheapest term, other terms, gauge")
    ap.add_argument("--therm-steps", default=None, help="the same rule for the thermalisation (default: --steps)")
    ap.add_argument("--checkpoint", default=None, help="directory for checkpoint / resume")
    ap.add_argument("--max-traj", type=int, default=None, help="stop after this many trajectories (state saved)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (same launch configurations on resume)")
    args = ap.parse_args(argv)
    L = tuple(int(v) for v in args.lattice.split(","))
    steps = tuple(int(v) for v in args.steps.split(","))
    therm_steps = tuple(int(v) for v in args.therm_steps.split(",")) if args.therm_steps else None
    out = run(L, args.kappa, args.beta, args.therm, args.traj,
              args.actions.split(",") if args.actions else None, steps,
              log=lambda *a: print("[cost]", *a, file=sys.stderr, flush=True),
              checkpoint=args.checkpoint, max_traj=args.max_traj, tune_cache=args.tune_cache,
              therm_steps=therm_steps)
    if out is None:
        print(json.dumps({"stopped": True, "checkpoint": args.checkpoint}), flush=True)
    else:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
