"""Benchmark of the MI355X Wilson-fermion HMC hot path (one GPU).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--therm N] [--no-cpu] [--quick]

Workload: 16^3 x 32 lattice, kappa = 0.155, antiperiodic in time, synthetic
links exp(i a H) with a = 0.447 (plaquette ~0.58), seeded, first thermalised
by N (default 30) untimed HMC trajectories of the MP action.  One step is one
HMC trajectory, with Metropolis, of the PF-MP action (polynomial filter on
top of a Hasenbusch mass preconditioner) with the Wilson plaquette gauge
action beta = 5.6: POLY(J) + POLYK_INV(J) + RATIO, J = K-hat + 0.05,
Chebyshev order 16 on [0.001, 8], Omelyan, tau = 1, steps 40 / 40 / 20 / 80
(poly, poly-K inverse, ratio, gauge); the warmup and timed steps continue one
Markov chain from the thermalised configuration.  A trajectory runs every
hot-path stage: hops, K-hat / J, CG solves (FP32 inner with FP64 reliable
updates to a true residual 1e-10), the polynomial filter, fermion and gauge
forces, link and momentum updates, FP64 energies and the Metropolis step.
Momenta, noise and Metropolis uniforms for every trajectory are generated and
uploaded before the timed region.

value = algorithmic Dslash bytes moved per second over the timed steps (hop
applications x bytes per hop application / wall time), GB/s.  The JSON line
also carries the acceptance and <exp(-dH)> of the chain, the HBM roofline of
the hop on the 32^3 x 64 lattice (BF16 storage, 4 rhs: the large-volume
workload's own kernel; FP64 one rhs beside it; the 16^3 x 32 lattice fits the
256 MB last-level cache, so the trajectory's own hop is reported separately as
cache-resident), the CG time-to-1e-10 of FP64 vs mixed precision single-rhs
and of 8 sequential FP64 solves vs one batched mixed solve over the shifts
{0, 0.005, 0.05, 0.5}, and the FP64 oracle timed on host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s (% HBM peak); CG time-to-1e-10 mixed multi-RHS vs FP64"
HBM_PEAK_GBS = 8000.0
L = (16, 16, 16, 32)
KAPPA = 0.155
LINK_SPREAD = 0.447
BETA = 5.6
MU2_HASENBUSCH = 0.05
POLY_N, POLY_A, POLY_B = 16, 0.001, 8.0
NSTEPS = [40, 40, 20, 80]   # poly, poly-K inverse, ratio, gauge (see actions.WORKLOAD_NSTEPS)
SHIFTS = [0.0, 0.005, 0.05, 0.5, 0.0, 0.005, 0.05, 0.5]
# reliable-update threshold of the mixed-precision CG comparisons: 0.01 measured faster than 0.1 at 16^3x32
# and 32^3x64 (fewer FP64 applications, same iterations and FP64 true residual)
MIXED_DELTA = 0.01
# algorithmic bytes of one hop application per output site: 8 two-row links + input
# spinor read once + output spinor written once (perfect on-chip reuse)
HOP_BYTES_PER_SITE = {"f64": 8 * 96 + 2 * 192, "f32": 8 * 48 + 2 * 96, "bf16": 8 * 24 + 2 * 48}
# conventional flop count of one Wilson hop per output site and rhs (8 projections,
# 8 SU(3) x half-spinor products, 7 accumulations), the third-row rebuild not counted
HOP_FLOPS_PER_SITE = 1320


def hop_gflops(nrhs: int, sites: int, us: float) -> float:
    return round(HOP_FLOPS_PER_SITE * nrhs * sites / (us * 1e-6) / 1e9, 1)


# HBM traffic of one hop launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, median over dispatches 6-50 of each configuration of
# `bench.py --kernels-only --kernels-volume 32,32,32,64 --kernels-nrhs N`), scaled by
# the same counters' reading for a plain 1 GiB device copy (FETCH_SIZE read
# 524300 KiB -> x2.0; WRITE_SIZE read 1048576 KiB -> x1.0).  Keyed by
# "precision:nrhs:variant:npass:use_xcd:stream" on the 32^3 x 64 lattice.  Valid
# only for the hop kernel source they were taken on (hash of the hop kernel
# sources); otherwise `traffic` is reported as null.
PMC_FETCH_SCALE, PMC_WRITE_SCALE = 2.0, 1.0
PMC_COUNTERS = {
    "source_sha256": "5063c072b14150bb65eb8535bea70a7f8634373753568b4357ff7000fe3ffd51",
    "per_launch_kib": {
        "f64:1:0:1:1:0": {"fetch": 912761.6, "write": 196608.0},
        "f64:1:0:1:1:1": {"fetch": 743422.4, "write": 196608.0},
        "f64:1:0:1:0:0": {"fetch": 1015627.2, "write": 196608.0},
        "f64:1:0:1:0:1": {"fetch": 884423.9, "write": 196608.0},
        "f64:1:0:1:2:0": {"fetch": 867505.6, "write": 196608.0},
        "f64:1:0:1:2:1": {"fetch": 675855.1, "write": 196608.0},
        "f64:1:1:1:1:0": {"fetch": 689258.7, "write": 196608.0},
        "f64:1:1:1:1:1": {"fetch": 689024.5, "write": 196608.0},
        "f64:1:1:1:0:0": {"fetch": 558467.4, "write": 196608.0},
        "f64:1:1:1:0:1": {"fetch": 543881.8, "write": 196608.0},
        "f64:1:1:1:2:0": {"fetch": 568300.5, "write": 196608.0},
        "f64:1:1:1:2:1": {"fetch": 568156.5, "write": 196608.0},
        "f32:1:0:1:1:0": {"fetch": 370858.2, "write": 98304.0},
        "f32:1:0:1:1:1": {"fetch": 302604.6, "write": 98304.2},
        "f32:1:0:1:0:0": {"fetch": 488200.2, "write": 98304.0},
        "f32:1:0:1:0:1": {"fetch": 420665.9, "write": 98304.0},
        "f32:1:0:1:2:0": {"fetch": 396858.7, "write": 98304.0},
        "f32:1:0:1:2:1": {"fetch": 308342.5, "write": 98304.0},
        "f32:1:1:1:1:0": {"fetch": 344631.5, "write": 98304.0},
        "f32:1:1:1:1:1": {"fetch": 343257.4, "write": 98304.0},
        "f32:1:1:1:0:0": {"fetch": 272795.9, "write": 98304.0},
        "f32:1:1:1:0:1": {"fetch": 271975.6, "write": 98304.0},
        "f32:1:1:1:2:0": {"fetch": 284160.5, "write": 98304.0},
        "f32:1:1:1:2:1": {"fetch": 283824.0, "write": 98304.0},
        "bf16:1:0:1:1:0": {"fetch": 155811.5, "write": 49152.0},
        "bf16:1:0:1:1:1": {"fetch": 130996.9, "write": 49152.0},
        "bf16:1:0:1:0:0": {"fetch": 213565.9, "write": 49152.0},
        "bf16:1:0:1:0:1": {"fetch": 185421.6, "write": 49152.0},
        "bf16:1:0:1:2:0": {"fetch": 159725.4, "write": 49152.0},
        "bf16:1:0:1:2:1": {"fetch": 139411.4, "write": 49152.0},
        "bf16:1:1:1:1:0": {"fetch": 172094.5, "write": 49152.0},
        "bf16:1:1:1:1:1": {"fetch": 129134.5, "write": 49152.0},
        "bf16:1:1:1:0:0": {"fetch": 136048.7, "write": 49152.0},
        "bf16:1:1:1:0:1": {"fetch": 136045.8, "write": 49152.0},
        "bf16:1:1:1:2:0": {"fetch": 142121.1, "write": 49152.0},
        "bf16:1:1:1:2:1": {"fetch": 137862.2, "write": 49152.0},
        "f64:4:0:1:1:0": {"fetch": 2264036.4, "write": 786432.0},
        "f64:4:0:1:1:1": {"fetch": 2574642.4, "write": 786432.0},
        "f64:4:0:1:0:0": {"fetch": 2396478.8, "write": 786432.0},
        "f64:4:0:1:0:1": {"fetch": 2797765.6, "write": 786433.0},
        "f64:4:0:1:2:0": {"fetch": 1966202.1, "write": 786432.0},
        "f64:4:0:1:2:1": {"fetch": 2112441.2, "write": 786432.0},
        "f64:4:2:1:1:0": {"fetch": 2158536.9, "write": 786432.0},
        "f64:4:2:1:1:1": {"fetch": 1904074.4, "write": 786432.0},
        "f64:4:2:1:0:0": {"fetch": 1797211.6, "write": 786432.0},
        "f64:4:2:1:0:1": {"fetch": 1550027.0, "write": 786449.0},
        "f64:4:2:1:2:0": {"fetch": 1737927.8, "write": 786432.0},
        "f64:4:2:1:2:1": {"fetch": 1491612.8, "write": 786434.4},
        "f64:4:1:1:1:0": {"fetch": 1618731.6, "write": 786432.0},
        "f64:4:1:1:1:1": {"fetch": 1671151.6, "write": 786432.0},
        "f64:4:1:1:0:0": {"fetch": 1769876.9, "write": 786432.0},
        "f64:4:1:1:0:1": {"fetch": 1797876.7, "write": 786432.0},
        "f64:4:1:1:2:0": {"fetch": 1096789.6, "write": 786432.0},
        "f64:4:1:1:2:1": {"fetch": 1126431.4, "write": 786432.0},
        "f64:4:1:2:1:0": {"fetch": 1670566.1, "write": 786432.0},
        "f64:4:1:2:1:1": {"fetch": 1712691.2, "write": 786432.0},
        "f64:4:1:2:0:0": {"fetch": 1770383.0, "write": 786432.0},
        "f64:4:1:2:0:1": {"fetch": 1820200.6, "write": 786432.0},
        "f64:4:1:2:2:0": {"fetch": 1107671.4, "write": 786432.0},
        "f64:4:1:2:2:1": {"fetch": 1201626.8, "write": 786432.0},
        "f64:4:1:4:1:0": {"fetch": 1758755.5, "write": 786432.0},
        "f64:4:1:4:1:1": {"fetch": 1654775.1, "write": 786432.0},
        "f64:4:1:4:0:0": {"fetch": 1748037.0, "write": 786432.0},
        "f64:4:1:4:0:1": {"fetch": 1639506.3, "write": 786432.0},
        "f64:4:1:4:2:0": {"fetch": 1122551.8, "write": 786432.0},
        "f64:4:1:4:2:1": {"fetch": 1096926.2, "write": 786432.0},
        "f32:4:0:1:1:0": {"fetch": 1051158.1, "write": 393216.0},
        "f32:4:0:1:1:1": {"fetch": 1197997.7, "write": 393216.2},
        "f32:4:0:1:0:0": {"fetch": 1192784.7, "write": 393216.0},
        "f32:4:0:1:0:1": {"fetch": 1384213.9, "write": 393216.2},
        "f32:4:0:1:2:0": {"fetch": 861312.9, "write": 393216.0},
        "f32:4:0:1:2:1": {"fetch": 928345.4, "write": 393216.2},
        "f32:4:0:2:1:0": {"fetch": 824000.7, "write": 393216.0},
        "f32:4:0:2:1:1": {"fetch": 820299.1, "write": 393217.5},
        "f32:4:0:2:0:0": {"fetch": 1020628.6, "write": 393216.0},
        "f32:4:0:2:0:1": {"fetch": 1021245.2, "write": 393216.4},
        "f32:4:0:2:2:0": {"fetch": 575228.8, "write": 393216.0},
        "f32:4:0:2:2:1": {"fetch": 559885.4, "write": 393216.2},
        "f32:4:2:1:1:0": {"fetch": 891856.6, "write": 393216.0},
        "f32:4:2:1:1:1": {"fetch": 824560.2, "write": 393224.2},
        "f32:4:2:1:0:0": {"fetch": 722026.6, "write": 393216.0},
        "f32:4:2:1:0:1": {"fetch": 618821.4, "write": 393238.9},
        "f32:4:2:1:2:0": {"fetch": 670180.8, "write": 393216.0},
        "f32:4:2:1:2:1": {"fetch": 576731.2, "write": 393220.9},
        "f32:4:1:1:1:0": {"fetch": 788425.9, "write": 393216.0},
        "f32:4:1:1:1:1": {"fetch": 796077.4, "write": 393216.0},
        "f32:4:1:1:0:0": {"fetch": 698201.7, "write": 393216.0},
        "f32:4:1:1:0:1": {"fetch": 528833.2, "write": 393216.0},
        "f32:4:1:1:2:0": {"fetch": 546436.9, "write": 393216.0},
        "f32:4:1:1:2:1": {"fetch": 552026.3, "write": 393216.0},
        "f32:4:1:2:1:0": {"fetch": 795093.5, "write": 393216.0},
        "f32:4:1:2:1:1": {"fetch": 790177.7, "write": 393216.0},
        "f32:4:1:2:0:0": {"fetch": 658807.9, "write": 393216.0},
        "f32:4:1:2:0:1": {"fetch": 519848.8, "write": 393216.0},
        "f32:4:1:2:2:0": {"fetch": 548756.8, "write": 393216.0},
        "f32:4:1:2:2:1": {"fetch": 546735.8, "write": 393216.0},
        "f32:4:1:4:1:0": {"fetch": 795022.7, "write": 393216.0},
        "f32:4:1:4:1:1": {"fetch": 790152.8, "write": 393216.0},
        "f32:4:1:4:0:0": {"fetch": 658870.3, "write": 393216.0},
        "f32:4:1:4:0:1": {"fetch": 519884.2, "write": 393216.0},
        "f32:4:1:4:2:0": {"fetch": 548726.4, "write": 393216.0},
        "f32:4:1:4:2:1": {"fetch": 546736.8, "write": 393216.0},
        "bf16:4:0:1:1:0": {"fetch": 417760.2, "write": 196608.0},
        "bf16:4:0:1:1:1": {"fetch": 477404.0, "write": 196608.0},
        "bf16:4:0:1:0:0": {"fetch": 523169.4, "write": 196608.0},
        "bf16:4:0:1:0:1": {"fetch": 565987.1, "write": 196608.0},
        "bf16:4:0:1:2:0": {"fetch": 294195.1, "write": 196608.0},
        "bf16:4:0:1:2:1": {"fetch": 346531.1, "write": 196608.0},
        "bf16:4:0:2:1:0": {"fetch": 395547.1, "write": 196608.0},
        "bf16:4:0:2:1:1": {"fetch": 395407.8, "write": 196608.0},
        "bf16:4:0:2:0:0": {"fetch": 448498.9, "write": 196608.0},
        "bf16:4:0:2:0:1": {"fetch": 419367.3, "write": 196608.0},
        "bf16:4:0:2:2:0": {"fetch": 273536.3, "write": 196608.0},
        "bf16:4:0:2:2:1": {"fetch": 273946.0, "write": 196608.0},
        "bf16:4:2:1:1:0": {"fetch": 395309.1, "write": 196608.0},
        "bf16:4:2:1:1:1": {"fetch": 394389.8, "write": 196608.0},
        "bf16:4:2:1:0:0": {"fetch": 257784.8, "write": 196608.0},
        "bf16:4:2:1:0:1": {"fetch": 249163.4, "write": 196608.0},
        "bf16:4:2:1:2:0": {"fetch": 274031.8, "write": 196608.0},
        "bf16:4:2:1:2:1": {"fetch": 273263.6, "write": 196608.0},
        "bf16:4:1:1:1:0": {"fetch": 394154.9, "write": 196608.0},
        "bf16:4:1:1:1:1": {"fetch": 401118.4, "write": 196608.0},
        "bf16:4:1:1:0:0": {"fetch": 249383.1, "write": 196608.0},
        "bf16:4:1:1:0:1": {"fetch": 253829.8, "write": 196608.0},
        "bf16:4:1:1:2:0": {"fetch": 273292.9, "write": 196608.0},
        "bf16:4:1:1:2:1": {"fetch": 280851.9, "write": 196608.0},
        "bf16:4:1:2:1:0": {"fetch": 394309.2, "write": 196608.0},
        "bf16:4:1:2:1:1": {"fetch": 394267.1, "write": 196608.0},
        "bf16:4:1:2:0:0": {"fetch": 251040.4, "write": 196608.0},
        "bf16:4:1:2:0:1": {"fetch": 249121.5, "write": 196608.0},
        "bf16:4:1:2:2:0": {"fetch": 273424.2, "write": 196608.0},
        "bf16:4:1:2:2:1": {"fetch": 273402.5, "write": 196608.0},
        "bf16:4:1:4:1:0": {"fetch": 394310.0, "write": 196608.0},
        "bf16:4:1:4:1:1": {"fetch": 394267.1, "write": 196608.0},
        "bf16:4:1:4:0:0": {"fetch": 251062.6, "write": 196608.0},
        "bf16:4:1:4:0:1": {"fetch": 249120.9, "write": 196608.0},
        "bf16:4:1:4:2:0": {"fetch": 273424.9, "write": 196608.0},
        "bf16:4:1:4:2:1": {"fetch": 273402.5, "write": 196608.0},
    },
}


def hop_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("dslash.hip", "wl_device.h"):
        with open(os.path.join(ROOT, "paper_1702_00124_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _host_cores():
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return os.cpu_count(), aff


def cpu_leg(spec: dict) -> dict:
    """Runs in a child process started by cpu_baseline (threads fixed by its
    environment): the FP64 oracle on the 16^3 x 32 workload.
      kind "single": median of 3 of one D_eo and one K-hat application, then CG
        on J = K-hat + mu2 for `cg_iters` iterations (0: to the true residual 1e-10);
      kind "rhs": CG on rhs j (shift SHIFTS[j]) for `cg_iters` iterations."""
    import statistics

    import numpy as np

    import lattice_inputs as li
    from oracle import solver as osol, wilson as ow
    Lc = tuple(spec["L"])
    U = li.random_links(Lc, LINK_SPREAD, li.seed_links(1))
    Vh = li.volume(Lc) // 2
    out = {}
    if spec["kind"] == "single":
        psi = li.gaussian_spinor((Vh, 4, 3), li.seed_source(0))
        th, tk = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            ow.hop_eo(U, psi, Lc, 0, t_bc=-1)
            th.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            ow.Khat(U, psi, Lc, KAPPA, t_bc=-1)
            tk.append(time.perf_counter() - t0)
        out["hop_s"] = statistics.median(th)
        out["khat_s"] = statistics.median(tk)
        j = 0
    else:
        j = spec["rhs"]
    b = li.gaussian_spinor((Vh, 4, 3), li.seed_source(j))
    mu2 = SHIFTS[j]
    n = spec["cg_iters"]
    t0 = time.perf_counter()
    _, it, res = osol.cg(lambda v: ow.J(U, v, Lc, KAPPA, mu2, t_bc=-1), b, tol=1e-10,
                         maxiter=n if n > 0 else 10000)
    out.update({"cg_s": time.perf_counter() - t0, "cg_iters": it, "cg_true_rel_res": res})
    return out


def _run_cpu_leg(spec: dict, threads: int = 1, timeout: float = 3600):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OPENBLAS_NUM_THREADS=str(threads),
               MKL_NUM_THREADS=str(threads))
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", json.dumps(spec)],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)


def _collect(proc, timeout: float = 3600) -> dict:
    out, err = proc.communicate(timeout=timeout)
    if proc.returncode != 0:
        raise RuntimeError(err[-2000:])
    return json.loads(out.strip().splitlines()[-1])


def cpu_baseline(gpu_iters: int = 93, gpu_iters8=(93, 86, 58, 24, 93, 86, 58, 24), full: bool = False,
                 sample_iters: int = 4):
    """The FP64 oracle on the host: one core (threads pinned to 1) for D_eo, K-hat
    (median of 3) and the CG of the single-rhs workload, and all cores (one worker
    process per rhs, up to the 8 rhs of the batched workload) for the 8-rhs CG.
    Bounded by default: the CGs run `sample_iters` iterations and are extrapolated
    to the GPU's iteration count; full=True runs them to the true residual 1e-10."""
    cores, aff = _host_cores()
    t_all = time.perf_counter()
    single = _collect(_run_cpu_leg({"kind": "single", "L": L, "cg_iters": 0 if full else sample_iters}))
    nw = max(1, min(8, aff))
    t0 = time.perf_counter()
    procs = []
    results = []
    for j in range(8):   # at most nw workers at a time
        procs.append(_run_cpu_leg({"kind": "rhs", "L": L, "rhs": j, "cg_iters": 0 if full else sample_iters}))
        if len(procs) == nw:
            results += [_collect(p) for p in procs]
            procs = []
    results += [_collect(p) for p in procs]
    wall8 = time.perf_counter() - t0
    Vh = L[0] * L[1] * L[2] * L[3] // 2
    gbs = HOP_BYTES_PER_SITE["f64"] * Vh / single["hop_s"] / 1e9
    # a CG run ends with one more operator application for its true residual (about
    # one K-hat): per-iteration time without it
    per_it = max(single["cg_s"] - single["khat_s"], 0.0) / max(single["cg_iters"], 1)
    cg_single = single["cg_s"] if full else per_it * gpu_iters
    it8 = [r["cg_iters"] for r in results]
    # all-core 8-rhs time: measured wall, or each worker's per-iteration time scaled
    # to the GPU's iteration count of its rhs (the workers run in waves of nw)
    if full:
        cg8 = wall8
    else:   # waves of nw workers; a wave lasts as long as its slowest rhs at the GPU's iteration counts
        per8 = [max(r["cg_s"] - single["khat_s"], 0.0) / max(r["cg_iters"], 1) * gpu_iters8[j]
                for j, r in enumerate(results)]
        cg8 = sum(max(per8[w:w + nw]) for w in range(0, 8, nw))
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 oracle (NumPy) on the 16^3x32 workload: one D_eo {single['hop_s']:.2f} s and one "
                       f"K-hat {single['khat_s']:.2f} s (median of 3, one thread); CG on J "
                       + (f"to 1e-10 in {single['cg_iters']} iterations" if full else
                          f"for {single['cg_iters']} iterations, extrapolated to the GPU's {gpu_iters}")
                       + f"; the 8-rhs CG on {nw} worker processes (one thread each)"),
            "host_cpu_count": cores, "host_affinity": aff,
            "hop_s": round(single["hop_s"], 3), "khat_s": round(single["khat_s"], 3),
            "cg_single_rhs_s": round(cg_single, 2), "cg_single_rhs_measured": full,
            "cg_s_per_iteration": round(per_it, 3), "cg_sample_iterations": single["cg_iters"],
            "all_cores": {"workers": nw, "rhs": 8, "cg_iters": it8,
                          "seconds": round(cg8, 2), "measured_to_convergence": full,
                          "wall_sample_s": round(wall8, 2)},
            "leg_seconds": round(time.perf_counter() - t_all, 1)}


# kappas of the paper's actions on the bench lattice: kappa_1 = 0.145 < kappa' =
# kappa_2 = 0.150 < kappa = 0.155 (the action lists live in the package)
ACTION_KAPPAS = {"k": KAPPA, "kp": 0.150, "k1": 0.145, "k2": 0.150}


def paper_actions(lat, U, li, torch, Term, CG, L, Vh):
    """One trajectory of each of the paper's actions on the bench lattice: Omelyan,
    tau = 1, 40 steps for the first (cheapest) term, 20 for every other, 80 for the
    gauge action; MD solves FP32 inner / FP64 reliable updates to 1e-10.  Reports the
    paper's cost numerator N_mat (K-hat and J applications per trajectory), CG
    iterations, dH and the wall time (acceptance needs an equilibrated ensemble)."""
    from paper_1702_00124_amd.actions import PAPER_ACTIONS, build_terms, default_nsteps
    cg = CG(tol=1e-10, inner="f32", chunk=8)
    out = {}
    for name in PAPER_ACTIONS:
        lat.set_links(torch.from_numpy(U))
        terms = build_terms(name, ACTION_KAPPAS, cg)
        nsteps = default_nsteps(len(terms))
        P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(L, li.seed_md(50, 15))))
        chi = torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(50, i))))
                         for i in range(len(terms))])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.hmc_trajectory(terms, nsteps, P, chi, 0.5, beta=BETA, tau=1.0, integrator="omelyan")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"n_mat": int(r.n_kmat), "cg_iters": int(r.cg_iters), "dH": round(r.dH, 4),
                     "seconds": round(dt, 3), "nsteps": nsteps}
        log("paper action", name, json.dumps(out[name]))
    lat.set_links(torch.from_numpy(U))
    return out


def chrono_guess(lat, U, li, torch, terms, nsteps, L, Vh):
    """The bench trajectory from the same links, momenta and noise, force solves
    from x0 = 0 vs from each term's previous force solution (chronological
    guess): CG iterations, K applications, wall time and dH of each."""
    out = {}
    for chrono in (False, True):
        lat.set_links(torch.from_numpy(U))
        P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(L, li.seed_md(60, 15))))
        chi = torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(60, i))))
                         for i in range(len(terms))])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.hmc_trajectory(terms, nsteps, P, chi, 0.5, beta=BETA, tau=1.0, integrator="omelyan",
                               no_metropolis=True, chrono=chrono)
        torch.cuda.synchronize()
        out["chronological" if chrono else "cold"] = {
            "cg_iters": int(r.cg_iters), "n_mat": int(r.n_kmat), "seconds": round(time.perf_counter() - t0, 3),
            "dH": round(r.dH, 6)}
    lat.set_links(torch.from_numpy(U))
    log("chronological guess", json.dumps(out))
    return out


def _best_time(torch, fn, reps=3):
    best, out = 1e30, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best, out


def mixed_volume(li, torch, CG, WilsonLattice, WilsonBatch):
    """The batched workload's mixed-volume case: 8^3x16, 12^3x24 and 16^3x32
    (kappa 0.155, own links at plaquette ~0.58 each, shifts mu2 = 0.005, 0.05, 0)
    solved to true residual 1e-10 by one CG over the batch, every hop of the
    three lattices one launch, vs the three single-lattice solves (each lattice
    autotuned) one after the other; FP32 inner iterations with FP64 reliable
    updates, graph-captured chunks, in both."""
    vols = [(8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32)]
    lats = []
    for i, Lv in enumerate(vols):
        lat = WilsonLattice(Lv, t_bc=-1)
        lat.set_links(torch.from_numpy(li.random_links(Lv, LINK_SPREAD, li.seed_links(10 + i))))
        lat.autotune()
        lats.append(lat)
    B = WilsonBatch(lats)
    kappa, mu2 = [KAPPA] * 3, [0.005, 0.05, 0.0]
    bs = [li.gaussian_spinor((li.volume(Lv) // 2, 4, 3), li.seed_source(200 + i)) for i, Lv in enumerate(vols)]
    bb = B.pack([torch.from_numpy(v) for v in bs])
    singles = [lat.import_spinor(torch.from_numpy(v)) for lat, v in zip(lats, bs)]
    prm = CG(tol=1e-10, inner="f32", delta=MIXED_DELTA, use_graph=True)

    def seq():
        return [lat.cg_solve(b1, kappa[i], "J", mu2=[mu2[i]], params=prm)[1][0]
                for i, (lat, b1) in enumerate(zip(lats, singles))]
    tb, (_, sb, rcb) = _best_time(torch, lambda: B.cg_solve(bb, kappa, mu2, prm))
    ts, ss = _best_time(torch, seq)
    out = {"volumes": [list(v) for v in vols], "batch_ms": round(tb * 1e3, 2), "sequential_ms": round(ts * 1e3, 2),
           "speedup": round(ts / tb, 3), "batch_iters": [s.iters for s in sb],
           "sequential_iters": [s.iters for s in ss], "batch_true_res_max": max(s.true_rel_res for s in sb),
           "rc": rcb}
    log("mixed-volume batch", json.dumps(out))
    B.close()
    for lat in lats:
        lat.close()
    return out


LARGE_L, LARGE_KAPPA, LARGE_SPREAD = (32, 32, 32, 64), 0.156, 0.432
# 2 spinors x 24 + 4 links x 12 (two rows) + 32 coefficients read and written, FP64
BILINEAR_BYTES_PER_SITE = 8 * (2 * 24 + 4 * 12 + 2 * 32)
VARIANT_NAMES = ["thread-per-site", "direction-parallel", "thread-per-site, links shared in LDS"]
ORDER_NAMES = ["round-robin", "XCD-contiguous", "z-blocked round-robin"]
SPINOR_BYTES = {"f64": 192, "f32": 96, "bf16": 48}
LINK_BYTES = {"f64": 96, "f32": 48, "bf16": 24}


def hop_bytes(prec: str, nrhs: int, sites: int) -> int:
    """Algorithmic bytes of one hop launch: 8 two-row links per output site read once
    (shared by the rhs), each rhs's input spinor read once and output written once."""
    return (8 * LINK_BYTES[prec] + 2 * nrhs * SPINOR_BYTES[prec]) * sites


def large_lattice(li, torch, WilsonLattice, tune_cache=None):
    """The large-volume workload's lattice: 32^3 x 64, kappa 0.156, links with
    plaquette ~0.60, hop configurations autotuned on it."""
    t0 = time.time()
    U = li.random_links(LARGE_L, LARGE_SPREAD, li.seed_links(4))
    log(f"large volume: links in {time.time() - t0:.1f}s")
    lat = WilsonLattice(LARGE_L, t_bc=-1)
    lat.set_links(torch.from_numpy(U))
    del U
    tune = lat.autotune(cache=tune_cache)
    log("large volume hop autotune (us per launch, C API order):",
        json.dumps({p: [round(x, 1) for x in v] for p, v in tune.items()}))
    return lat


def _traffic(prec, nrhs, cfg):
    kib = PMC_COUNTERS["per_launch_kib"].get(f"{prec}:{nrhs}:" + ":".join(map(str, cfg)))
    if kib and PMC_COUNTERS["source_sha256"] == hop_source_hash():
        return int(1024 * (kib["fetch"] * PMC_FETCH_SCALE + kib["write"] * PMC_WRITE_SCALE))
    return None


def hbm_roofline(lat):
    """The hop of the large-volume workload at 32^3 x 64 (working set far beyond the
    256 MB last-level cache): BF16 storage with 4 rhs, and FP64 with one rhs beside
    it, each in its tuned configuration, timed as a burst of 500 back-to-back
    launches with HIP events on the library stream (each launch reads the previous
    one's output)."""
    Vh = lat.Vh
    out = {}
    for prec, nrhs in (("bf16", 4), ("f64", 1)):
        cfg = lat.hop_config(prec, 0 if nrhs == 1 else (1 if nrhs <= 4 else 2))
        us = lat.time_hop(prec, nrhs, 500)
        byt = hop_bytes(prec, nrhs, Vh)
        gbs = byt / (us * 1e-6) / 1e9
        variant, npass, use_xcd, stream = cfg
        out[f"{prec}_x{nrhs}"] = {
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": _traffic(prec, nrhs, cfg),
            "kernel": f"hop {prec} x{nrhs} rhs on {'x'.join(map(str, LARGE_L))} "
                      f"({VARIANT_NAMES[variant]}, npass {npass}, "
                      f"{ORDER_NAMES[use_xcd]} workgroup order, "
                      f"{'streaming' if stream else 'cached'} access)",
            "config": list(cfg), "avg_launch_us": round(us, 2), "algorithmic_bytes_per_launch": byt,
            "launches": 500, "gflops": hop_gflops(nrhs, Vh, us)}
        log(f"hbm roofline {prec} x{nrhs}:", json.dumps(out[f"{prec}_x{nrhs}"]))
    return out


def large_volume(lat, li, torch, np, CG):
    """32^3 x 64, kappa = 0.156, links with plaquette ~0.60, 4 Gaussian rhs:
    hop bandwidth per precision, CG to true residual 1e-10 with FP64 single rhs
    vs BF16-storage / FP32-arithmetic inner iterations on the 4-rhs batch (FP64
    reliable updates), and the force bilinear's throughput."""
    Vh = lat.Vh
    kappa = LARGE_KAPPA
    out = {"lattice": list(LARGE_L), "kappa": kappa, "plaquette": round(lat.plaquette(), 5)}
    out["hop"] = {}
    for p in ("f64", "f32", "bf16"):
        for nrhs in (1, 4):
            us = lat.time_hop(p, nrhs, 200)
            byt = hop_bytes(p, nrhs, Vh)
            out["hop"][f"{p}_x{nrhs}"] = {"us": round(us, 1), "us_per_rhs": round(us / nrhs, 1),
                                          "GBs": round(byt / (us * 1e-6) / 1e9, 1),
                                          "GFLOPs": hop_gflops(nrhs, Vh, us)}
    out["copy_f64_hop_bytes_gbs"] = round(lat.stream_copy(HOP_BYTES_PER_SITE["f64"] * Vh // 2 // 16 * 16, 50), 1)
    log("large volume hop", json.dumps(out["hop"]), "copy of the FP64 hop's bytes:", out["copy_f64_hop_bytes_gbs"])
    bs = [li.gaussian_spinor((Vh, 4, 3), li.seed_source(100 + j)) for j in range(4)]
    b1 = lat.import_spinor(torch.from_numpy(bs[0]))
    b4 = lat.import_spinor(torch.from_numpy(np.stack(bs)))
    res = {}
    for name, b, nrhs, inner in (("f64_x1", b1, 1, "f64"), ("bf16_x4", b4, 4, "bf16"), ("f32_x4", b4, 4, "f32")):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st, rc = lat.cg_solve(b, kappa, "J", mu2=[0.0] * nrhs, nrhs=nrhs,
                                 params=CG(tol=1e-10, inner=inner, maxiter=20000,
                                           delta=MIXED_DELTA if inner != "f64" else 0.1))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[name] = {"ms": round(dt * 1e3, 1), "ms_per_rhs": round(dt * 1e3 / nrhs, 1),
                     "iters": [s.iters for s in st], "reliable_updates": st[0].reliable_updates,
                     "max_true_rel_res": max(s.true_rel_res for s in st), "rc": rc}
        log("large volume cg", name, json.dumps(res[name]))
    res["bf16_x4_speedup_per_rhs"] = round(res["f64_x1"]["ms"] / res["bf16_x4"]["ms_per_rhs"], 3)
    res["f32_x4_speedup_per_rhs"] = round(res["f64_x1"]["ms"] / res["f32_x4"]["ms_per_rhs"], 3)
    out["cg"] = res
    # force bilinear: 2 full FP64 spinors, 4 two-row FP64 links, read and write of 32
    # force coefficients per site; two distinct spinor fields
    A = lat.new_field("f64", 1, full=True)
    A.fill_(0.5)
    Cf = lat.new_field("f64", 1, full=True)
    Cf.fill_(0.25)
    F = lat.new_su3()
    for _ in range(2):
        lat.force_bilinear(A, Cf, F)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        lat.force_bilinear(A, Cf, F)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / 10 * 1e3
    fb = BILINEAR_BYTES_PER_SITE * 2 * Vh
    # the same with every link counted as a full 3x3 matrix (18 reals, 1472 B per site)
    fb_full = (BILINEAR_BYTES_PER_SITE + 8 * 4 * 6) * 2 * Vh
    out["force_bilinear"] = {"us": round(us, 1), "GBs": round(fb / (us * 1e-6) / 1e9, 1),
                             "frac": round(fb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": fb,
                             "frac_full_links": round(fb_full / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    out["hop_config"] = {p: [lat.hop_config(p, k) for k in range(3)] for p in ("f64", "f32", "bf16")}
    return out


KERNELS_ONLY_CONFIGS = [(v, x, st) for v in (0, 1) for x in (1, 0, 2) for st in (0, 1)]   # (variant, order, stream)


def kernels_only_configs(prec: str, nrhs: int):
    """(variant, npass, order, stream) tried per precision by --kernels-only: one rhs
    takes KERNELS_ONLY_CONFIGS; several rhs take every candidate the autotuner times
    for their class (site npass 1 and, for FP32 / BF16, 2; the shared-link variant;
    direction-parallel npass 1, 2, 4), each per (order, stream).  Configurations the
    lattice does not allow (the z-blocked order 2) are skipped at launch time and left
    out of the logged list."""
    if nrhs == 1:
        return [(v, 1, x, st) for v, x, st in KERNELS_ONLY_CONFIGS]
    cands = [(0, 1)] + ([(0, 2)] if prec != "f64" else []) + [(2, 1), (1, 1), (1, 2), (1, 4)]
    return [(v, n, x, st) for v, n in cands for x in (1, 0, 2) for st in (0, 1)]


def kernels_only(lat, Vh, li, torch, nrhs: int = 1):
    """Hop launches for kernel-trace and counter runs: 50 launches of nrhs
    right-hand sides for every configuration of kernels_only_configs, for f64,
    f32, bf16 in that order, then a plain copy of known size whose FETCH_SIZE
    / WRITE_SIZE calibrate the counters."""
    import numpy as np
    psi = li.gaussian_spinor((Vh, 4, 3) if nrhs == 1 else (nrhs, Vh, 4, 3), li.seed_source(0))
    from paper_1702_00124_amd import WilsonError
    kind = {1: 0}.get(nrhs, 1 if nrhs <= 4 else 2)
    launched = []
    for prec in ("f64", "f32", "bf16"):
        b = lat.import_spinor(torch.from_numpy(np.ascontiguousarray(psi)), prec)
        out = lat.new_field(prec, nrhs)
        for variant, npass, xcd, stream in kernels_only_configs(prec, nrhs):
            try:
                lat.set_hop_config(prec, kind, variant=variant, npass=npass, use_xcd=xcd, stream=stream)
            except WilsonError:
                continue
            launched.append([prec, variant, npass, xcd, stream])
            for _ in range(50):
                lat.dslash(b, 0, prec=prec, nrhs=nrhs, out=out)
        del b, out
    torch.cuda.synchronize()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"kernels-only done: 50 hop launches of {nrhs} rhs for each [precision, variant, npass, order, stream] "
        "in KERNELS_LAUNCHED " + json.dumps(launched) + " then 5 copies of 1 GiB")


def solver_kernels(lat, Vh, li, torch, CG, WilsonLattice, WilsonBatch):
    """Launches of the solver and force kernels for kernel-trace and counter
    runs, on the given lattice: three FP32-inner CG solves of J x = b (mu2
    0.05, to 1e-10, threshold 0.01, eager launches: the CG update and xpay
    kernels once per iteration, fused with the scalar steps where the
    reduction rows are short), 50 FP32 batched hops over the 8^3x16 +
    12^3x24 + 16^3x32 mixed-volume batch (one launch each), 50 force bilinears,
    then 5 device copies of 1 GiB for the counter calibration."""
    b = lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_source(0))))
    prm = CG(tol=1e-10, inner="f32", delta=MIXED_DELTA)
    for _ in range(3):
        _, st, rc = lat.cg_solve(b, KAPPA, "J", mu2=[MU2_HASENBUSCH], params=prm)
        assert rc == 0
    vols = [(8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32)]
    lats = []
    for i, Lv in enumerate(vols):
        lt = WilsonLattice(Lv, t_bc=-1)
        lt.set_links(torch.from_numpy(li.random_links(Lv, LINK_SPREAD, li.seed_links(10 + i))))
        lats.append(lt)
    B = WilsonBatch(lats)
    bb = B.pack([torch.from_numpy(li.gaussian_spinor((li.volume(Lv) // 2, 4, 3), li.seed_source(200 + i)))
                 for i, Lv in enumerate(vols)], "f32")
    for _ in range(50):
        B.dslash(bb, 0, prec="f32")
    A = lat.new_field("f64", 1, full=True)
    A.fill_(0.5)
    Cf = lat.new_field("f64", 1, full=True)
    Cf.fill_(0.25)
    F = lat.new_su3()
    for _ in range(50):
        lat.force_bilinear(A, Cf, F)
    torch.cuda.synchronize()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"solver-kernels done: 3 FP32-inner CG solves ({st[0].iters} iterations each), 50 batched FP32 hops over",
        vols, "50 force bilinears, 5 copies of 1 GiB")
    B.close()
    for lt in lats:
        lt.close()


def precision_errors_md(lat, U_start, li, torch, terms_of, nsteps, Vh):
    """Errors of the trajectory's mixed-precision solves against FP64 solves on the
    same inputs: each workload term's force (FP32 inner iterations with FP64
    reliable updates at threshold 0.003 vs FP64 CG, both to the true residual
    1e-10) and dH of one trajectory (same links, momenta and noise)."""
    from paper_1702_00124_amd.lattice import CG
    mixed = terms_of(CG(tol=1e-10, inner="f32", chunk=8, delta=0.003), CG(tol=1e-10, inner="f32", chunk=2, delta=0.003))
    fp64 = terms_of(CG(tol=1e-10, inner="f64", chunk=8), CG(tol=1e-10, inner="f64", chunk=2))
    out = {}
    lat.set_links(U_start)
    for i, name in enumerate(("poly", "polyk_inv", "ratio")):
        phi = lat.heatbath(fp64[i], lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3),
                                                                                         li.seed_md(70, i)))))
        F64 = lat.fermion_force(fp64[i], phi)
        F32 = lat.fermion_force(mixed[i], phi)
        d = F32 - F64
        out[f"force_{name}_f32_inner_vs_f64"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(F64))
        out[f"force_{name}_f32_inner_vs_f64_max"] = float(d.abs().max() / F64.abs().max())
    dh = {}
    for tag, terms in (("f32", mixed), ("f64", fp64)):
        lat.set_links(U_start)
        P = lat.import_su3(torch.from_numpy(li.gaussian_momenta(lat.L, li.seed_md(71, 15))))
        chi = torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(71, i))))
                         for i in range(3)])
        r = lat.hmc_trajectory(terms, nsteps, P, chi, 0.5, beta=BETA, tau=1.0, integrator="omelyan",
                               no_metropolis=True)
        dh[tag] = r.dH
    out["dH_f32_inner"] = dh["f32"]
    out["dH_f64"] = dh["f64"]
    out["dH_f32_inner_minus_f64"] = dh["f32"] - dh["f64"]
    lat.set_links(U_start)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--therm", type=int, default=30,
                    help="untimed MP trajectories that thermalise the synthetic links before the warmup")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline leg")
    ap.add_argument("--cpu-full", action="store_true",
                    help="run the oracle CGs of cpu_baseline to convergence (minutes of host time) "
                         "instead of a bounded sample extrapolated to the GPU's iteration counts")
    ap.add_argument("--quick", action="store_true", help="skip the CG comparison and large-volume legs")
    ap.add_argument("--md-delta", type=float, default=0.003,
                    help="reliable-update threshold of the trajectory's FP32-inner solves")
    ap.add_argument("--md-poly-chunk", type=int, default=2,
                    help="iterations between convergence checks of the polynomial terms' solves")
    ap.add_argument("--md-poly-inner", default="f32", choices=("f32", "bf16"),
                    help="storage precision of the polynomial terms' inner iterations")
    ap.add_argument("--cg-graph", action="store_true",
                    help="the trajectory's solves replay each chunk of CG iterations as a captured HIP graph")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of hop autotuning results (keyed by lattice, device and build): read on a "
                         "hit, written otherwise (a profiled run takes the configurations an unprofiled run tuned)")
    ap.add_argument("--md-steps", default=",".join(map(str, NSTEPS)),
                    help="integrator steps per scale (poly, poly-K inverse, ratio, gauge); profiling runs shorten them")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the hop kernels (50 per configuration and precision) and a 1 GiB copy, "
                         "for counter runs")
    ap.add_argument("--kernels-nrhs", type=int, default=1,
                    help="right-hand sides of the --kernels-only launches (1: the one-rhs configurations; "
                         "2-16: every candidate of that rhs class)")
    ap.add_argument("--solver-kernels", action="store_true",
                    help="only launch the fused CG kernels (three FP32-inner solves), the mixed-volume batch hop "
                         "and the force bilinear, and a 1 GiB copy, for counter runs")
    ap.add_argument("--kernels-volume", default=None,
                    help="Lx,Ly,Lz,Lt of the --kernels-only or --solver-kernels lattice (default the trajectory's "
                         "16,16,16,32; 32,32,32,64 is the large-volume lattice with plaquette ~0.60 links)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only build the 32^3x64 lattice and time the HBM-roofline hop bursts (for a kernel trace "
                         "of the same launches)")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_leg:
        print(json.dumps(cpu_leg(json.loads(args.cpu_leg))), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is a design only; nothing here uses a second GPU.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lattice_inputs as li
    from paper_1702_00124_amd.actions import thermalise, workload_terms
    from paper_1702_00124_amd.lattice import CG, Term, WilsonBatch, WilsonLattice

    torch.cuda.set_device(0)
    if (args.kernels_only or args.solver_kernels) and args.kernels_volume:
        Lk = tuple(int(v) for v in args.kernels_volume.split(","))
        assert len(Lk) == 4
        lat = WilsonLattice(Lk, t_bc=-1)
        lat.set_links(torch.from_numpy(li.random_links(Lk, 0.432, li.seed_links(4))))
        log(f"{'kernels-only' if args.kernels_only else 'solver-kernels'} lattice {Lk}, "
            f"plaquette {lat.plaquette():.4f}")
        if args.kernels_only:
            kernels_only(lat, li.volume(Lk) // 2, li, torch, args.kernels_nrhs)
        else:
            solver_kernels(lat, li.volume(Lk) // 2, li, torch, CG, WilsonLattice, WilsonBatch)
        return
    if args.roofline_only:
        big = large_lattice(li, torch, WilsonLattice, args.tune_cache)
        print(json.dumps({"hbm_roofline": hbm_roofline(big), "source_sha256": hop_source_hash()}), flush=True)
        return
    Vh = L[0] * L[1] * L[2] * L[3] // 2
    nsteps = [int(v) for v in args.md_steps.split(",")]
    assert len(nsteps) == 4
    t0 = time.time()
    U = li.random_links(L, LINK_SPREAD, li.seed_links(1))
    log(f"links generated in {time.time() - t0:.1f}s")
    lat = WilsonLattice(L, t_bc=-1)
    lat.set_links(torch.from_numpy(U))
    plaq0 = lat.plaquette()
    log(f"plaquette {plaq0:.4f}")
    if args.kernels_only:
        kernels_only(lat, Vh, li, torch, args.kernels_nrhs)
        return
    if args.solver_kernels:
        solver_kernels(lat, Vh, li, torch, CG, WilsonLattice, WilsonBatch)
        return
    if args.tune_cache:
        from paper_1702_00124_amd import _lib as W
        from paper_1702_00124_amd.lattice import tune_cache_key, tune_cache_read, tune_device_id
        key = tune_cache_key(L, tune_device_id(0), W.LIB_PATH)
        hit = tune_cache_read(args.tune_cache, key) is not None
        log(f"hop tuning cache {args.tune_cache}: key {key}, {'hit' if hit else 'miss (tuning now)'}")
    tune = lat.autotune(cache=args.tune_cache)
    log(f"hop autotune (us per launch, candidates in the C API order): {tune}")
    log("hop configurations kept (variant, npass, use_xcd, stream) for 1, 2-4, 5-16 rhs:",
        {p: [lat.hop_config(p, k) for k in range(3)] for p in ("f64", "f32", "bf16")})

    # thermalisation: MP chain from the synthetic links (untimed)
    t0 = time.time()
    therm_rows = thermalise(lat, args.therm, kappa=KAPPA, beta=BETA, log=lambda m: log(m)) if args.therm else []
    plaq_therm = lat.plaquette()
    log(f"thermalised by {args.therm} MP trajectories in {time.time() - t0:.0f}s: plaquette {plaq0:.5f} -> "
        f"{plaq_therm:.5f}, acceptance {np.mean([r[1] for r in therm_rows]) if therm_rows else float('nan'):.2f}")
    U_therm = lat.get_links().clone()

    cg_md = CG(tol=1e-10, inner="f32", chunk=8, delta=args.md_delta, use_graph=args.cg_graph)
    # the polynomial solve's operator is degree + 1 J applications: check convergence more often
    cg_poly = CG(tol=1e-10, inner=args.md_poly_inner, chunk=args.md_poly_chunk, delta=args.md_delta)
    terms = workload_terms(cg_md, cg_poly, kappa=KAPPA, mu2=MU2_HASENBUSCH, degree=POLY_N, a=POLY_A, b=POLY_B)
    ntraj = args.warmup + args.steps
    P, chi, u = [], [], li.uniforms(ntraj, li.seed_metropolis(0))
    for k in range(ntraj):
        P.append(lat.import_su3(torch.from_numpy(li.gaussian_momenta(L, li.seed_md(k, 15)))))
        chi.append(torch.cat([lat.import_spinor(torch.from_numpy(li.gaussian_spinor((Vh, 4, 3), li.seed_md(k, i))))
                              for i in range(len(terms))]))
    torch.cuda.synchronize()

    def trajectory(k):
        return lat.hmc_trajectory(terms, nsteps, P[k], chi[k], float(u[k]), beta=BETA, tau=1.0,
                                  integrator="omelyan")

    chain = []
    for k in range(args.warmup):
        r = trajectory(k)
        chain.append(r)
        log(f"warmup trajectory {k}: dH {r.dH:.5f} accepted {r.accepted} plaquette {r.plaquette:.5f}")
    torch.cuda.synchronize()
    hop0 = lat.hop_counts()
    lat.profile(True)
    results = []
    t_start = time.perf_counter()
    for k in range(args.warmup, ntraj):
        ts = time.perf_counter()
        r = trajectory(k)
        results.append(r)
        log(f"trajectory {k}: dH {r.dH:.5f} accepted {r.accepted} n_kmat {r.n_kmat} "
            f"cg_iters {r.cg_iters} plaquette {r.plaquette:.5f} ({time.perf_counter() - ts:.2f}s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prof = lat.profile_read()
    lat.profile(False)
    hop1 = lat.hop_counts()
    chain += results
    n_hop = {p: hop1[p] - hop0[p] for p in hop1}
    bytes_per_hop = {p: b * Vh for p, b in HOP_BYTES_PER_SITE.items()}
    value = sum(n_hop[p] * bytes_per_hop[p] for p in n_hop) / wall / 1e9

    # the trajectory's dominant kernel: the hop precision with the most time in the
    # timed steps (applications x sampled in-situ duration), one rhs on 16^3 x 32,
    # whose working set fits the 256 MB last-level cache: cache-resident bandwidth,
    # from a burst of back-to-back launches with HIP events on the library's stream
    dom = max(prof, key=lambda p: n_hop[p] * prof[p][0])
    avg_us = lat.time_hop(dom, 1, 500)
    variant, _, use_xcd, stream = lat.hop_config(dom, 0)
    trajectory_hop = {
        "bound": "llc", "achieved": round(bytes_per_hop[dom] / (avg_us * 1e-6) / 1e9, 1), "unit": "GB/s",
        "frac_of_hbm_peak": round(bytes_per_hop[dom] / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
        "kernel": f"hop {dom} on 16x16x16x32 ({VARIANT_NAMES[variant]}, "
                  f"{ORDER_NAMES[use_xcd]} workgroup order, "
                  f"{'streaming' if stream else 'cached'} access)",
        "avg_launch_us": round(avg_us, 2), "in_situ_avg_us": round(prof[dom][0], 2),
        "in_situ_samples": prof[dom][1], "algorithmic_bytes_per_launch": bytes_per_hop[dom],
        "gflops": hop_gflops(1, Vh, avg_us),
        "note": "working set (links and two fields) inside the 256 MB last-level cache: not an HBM figure"}
    ex = np.exp(-np.array([r.dH for r in chain]))
    extra = {"hop_gflops_sustained": round(sum(n_hop.values()) * HOP_FLOPS_PER_SITE * Vh / wall / 1e9, 1),
             "hop_avg_us": {p: round(v[0], 2) for p, v in prof.items()},
             "hop_gbs": {p: round(bytes_per_hop[p] / (v[0] * 1e-6) / 1e9, 1) if v[0] > 0 else None
                         for p, v in prof.items()},
             "trajectory_hop": trajectory_hop,
             "thermalisation": {"mp_trajectories": args.therm, "plaquette_synthetic": round(plaq0, 5),
                                "plaquette_thermalised": round(plaq_therm, 5),
                                "acceptance": round(float(np.mean([r[1] for r in therm_rows])), 3)
                                if therm_rows else None},
             "chain": {"trajectories": len(chain), "acceptance": round(float(np.mean([r.accepted for r in chain])), 3),
                       "exp_minus_dH": round(float(ex.mean()), 4),
                       "exp_minus_dH_err": round(float(ex.std(ddof=1) / np.sqrt(len(ex))), 4) if len(ex) > 1 else None,
                       "dH_rms": round(float(np.sqrt(np.mean([r.dH ** 2 for r in chain]))), 4)},
             "dH": [round(r.dH, 5) for r in results], "accepted": [int(r.accepted) for r in results],
             "dH_warmup": [round(r.dH, 5) for r in chain[:args.warmup]],
             "n_kmat_per_traj": [int(r.n_kmat) for r in results],
             "cg_iters_per_traj": [int(r.cg_iters) for r in results],
             "plaquette_start": round(plaq_therm, 5), "plaquette_end": round(results[-1].plaquette, 5),
             "md_steps": nsteps,
             "hop_config": {p: [lat.hop_config(p, k) for k in range(3)] for p in ("f64", "f32", "bf16")}}
    log("chain", json.dumps(extra["chain"]))

    gpu_iters, gpu_iters8 = 93, (93, 86, 58, 24, 93, 86, 58, 24)
    if not args.quick:
        # CG time-to-1e-10: FP64 vs mixed single rhs, 8 sequential FP64 vs one batched mixed
        lat.set_links(torch.from_numpy(U))
        bs = [li.gaussian_spinor((Vh, 4, 3), li.seed_source(j)) for j in range(8)]
        b1 = lat.import_spinor(torch.from_numpy(bs[0]))
        b8 = lat.import_spinor(torch.from_numpy(np.stack(bs)))
        bj = [lat.import_spinor(torch.from_numpy(b)) for b in bs]

        def timed(fn, reps=3):
            best, out = 1e30, None
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                out = fn()
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            return best, out

        t64, (x64, s64, _) = timed(lambda: lat.cg_solve(b1, KAPPA, "J", mu2=[0.0], params=CG(tol=1e-10, inner="f64")))
        t32, (x32, s32, _) = timed(lambda: lat.cg_solve(b1, KAPPA, "J", mu2=[0.0],
                                                       params=CG(tol=1e-10, inner="f32", delta=MIXED_DELTA)))
        _, (x16, _, _) = timed(lambda: lat.cg_solve(b1, KAPPA, "J", mu2=[0.0],
                                                    params=CG(tol=1e-10, inner="bf16", delta=MIXED_DELTA)),
                               reps=1)

        def rel_err(a, b):
            return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

        def max_err(a, b):
            return float((a - b).abs().max() / b.abs().max())
        # storage-precision errors against the FP64 path on the same input (relative l2, and the
        # largest element's error relative to the largest element)
        src = torch.from_numpy(bs[0])
        ref_hop = lat.export_spinor(lat.dslash(lat.import_spinor(src), 1))
        ref_k = lat.export_spinor(lat.apply_K(lat.import_spinor(src), KAPPA, "J"))
        prec_err = {"cg_solution_f32_inner_vs_f64": rel_err(lat.export_spinor(x32), lat.export_spinor(x64)),
                    "cg_solution_bf16_inner_vs_f64": rel_err(lat.export_spinor(x16), lat.export_spinor(x64))}
        for pr in ("f32", "bf16"):
            hop = lat.export_spinor(lat.dslash(lat.import_spinor(src, pr), 1, prec=pr), pr)
            kj = lat.export_spinor(lat.apply_K(lat.import_spinor(src, pr), KAPPA, "J", prec=pr), pr)
            prec_err[f"hop_{pr}_vs_f64"] = rel_err(hop, ref_hop)
            prec_err[f"hop_{pr}_vs_f64_max"] = max_err(hop, ref_hop)
            prec_err[f"khat_{pr}_vs_f64"] = rel_err(kj, ref_k)
            prec_err[f"khat_{pr}_vs_f64_max"] = max_err(kj, ref_k)
        prec_err.update(precision_errors_md(
            lat, U_therm, li, torch,
            lambda cm, cp: workload_terms(cm, cp, kappa=KAPPA, mu2=MU2_HASENBUSCH, degree=POLY_N, a=POLY_A,
                                          b=POLY_B), nsteps, Vh))
        extra["precision_errors"] = {k: float(f"{v:.4g}") for k, v in prec_err.items()}
        log("precision errors", json.dumps(extra["precision_errors"]))

        def seq64():
            return [lat.cg_solve(bj[j], KAPPA, "J", mu2=[SHIFTS[j]], params=CG(tol=1e-10, inner="f64"))[1][0]
                    for j in range(8)]
        lat.set_links(torch.from_numpy(U))
        tseq, sseq = timed(seq64, reps=2)
        tbat, (_, sbat, _) = timed(lambda: lat.cg_solve(b8, KAPPA, "J", mu2=SHIFTS, nrhs=8,
                                                        params=CG(tol=1e-10, inner="f32", delta=MIXED_DELTA)),
                                   reps=2)
        # the same batch with other inner settings, each to the same FP64 true residual
        variants = {}
        for name, prm in (("f32_graph", CG(tol=1e-10, inner="f32", delta=MIXED_DELTA, use_graph=True)),
                          ("f32_delta0.1", CG(tol=1e-10, inner="f32", delta=0.1)),
                          ("bf16", CG(tol=1e-10, inner="bf16", delta=MIXED_DELTA)),
                          ("bf16_graph", CG(tol=1e-10, inner="bf16", delta=MIXED_DELTA, use_graph=True))):
            tv, (_, sv, rcv) = timed(lambda: lat.cg_solve(b8, KAPPA, "J", mu2=SHIFTS, nrhs=8, params=prm), reps=2)
            variants[name] = {"ms": round(tv * 1e3, 2), "iters_max": max(v.iters for v in sv),
                              "reliable_updates": sv[0].reliable_updates,
                              "true_res_max": max(v.true_rel_res for v in sv), "rc": rcv,
                              "speedup_vs_sequential_f64": round(tseq / tv, 3)}
        # 8 sources x the 4 shifts = 32 systems: one multi-shift FP64 solve (one Krylov
        # space per source) vs two batched FP32-inner solves of 16 systems each
        SH4 = SHIFTS[:4]
        tms, (_, sms, rcms) = timed(lambda: lat.cg_multishift(b8, KAPPA, SH4, 8, CG(tol=1e-10)), reps=2)
        mu16 = [m for m in SH4 for _ in range(4)]

        def two_batches():
            out = []
            for h in range(2):
                # systems (source j, shift k) for j in 4h..4h+3, every k: 16 rhs
                src = torch.cat([bj[4 * h + j] for k in range(4) for j in range(4)])
                out += lat.cg_solve(src, KAPPA, "J", mu2=mu16, nrhs=16,
                                    params=CG(tol=1e-10, inner="f32", delta=MIXED_DELTA))[1]
            return out
        t32x, s32x = timed(two_batches, reps=2)
        gpu_iters, gpu_iters8 = s64[0].iters, [s.iters for s in sseq]
        extra["cg"] = {
            "single_rhs_f64_ms": round(t64 * 1e3, 2), "single_rhs_f64_iters": s64[0].iters,
            "single_rhs_mixed_f32_ms": round(t32 * 1e3, 2), "single_rhs_mixed_iters": s32[0].iters,
            "single_rhs_mixed_reliable_updates": s32[0].reliable_updates,
            "single_rhs_speedup": round(t64 / t32, 3),
            "true_rel_res_f64": s64[0].true_rel_res, "true_rel_res_mixed": s32[0].true_rel_res,
            "eight_rhs_sequential_f64_ms": round(tseq * 1e3, 2),
            "eight_rhs_batched_mixed_ms": round(tbat * 1e3, 2),
            "multi_rhs_speedup": round(tseq / tbat, 3),
            "eight_rhs_batched_variants": variants,
            "eight_rhs_iters_f64": [s.iters for s in sseq], "eight_rhs_iters_batched": [s.iters for s in sbat],
            "eight_rhs_true_res_max": max(s.true_rel_res for s in sbat),
            "multishift_32_systems_f64_ms": round(tms * 1e3, 2),
            "multishift_base_iters": max(c.iters for c in sms[0]),
            "multishift_true_res_max": max(c.true_rel_res for row in sms for c in row),
            "multishift_refined": sum(c.reliable_updates for row in sms for c in row),
            "batched_32_systems_mixed_ms": round(t32x * 1e3, 2),
            "batched_32_true_res_max": max(c.true_rel_res for c in s32x),
            "multishift_speedup_vs_batched": round(t32x / tms, 3),
        }
        log("cg", json.dumps(extra["cg"]))
        extra["paper_actions"] = paper_actions(lat, U, li, torch, Term, CG, L, Vh)
        extra["chrono"] = chrono_guess(lat, U, li, torch, terms, nsteps, L, Vh)
        extra["mixed_volume"] = mixed_volume(li, torch, CG, WilsonLattice, WilsonBatch)
    lat.close()
    torch.cuda.empty_cache()
    big = large_lattice(li, torch, WilsonLattice, args.tune_cache)
    hbm = hbm_roofline(big)
    if not args.quick:
        extra["large_volume"] = large_volume(big, li, torch, np, CG)
    big.close()
    torch.cuda.empty_cache()
    extra["hbm_roofline_fp64_x1"] = hbm["f64_x1"]

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer", "data": "synthetic",
        "config": {"workload": "PF-MP HMC trajectory with Metropolis on a thermalised chain, wilson 16^3x32 "
                               "kappa=0.155 beta=5.6, cheb n=16 [0.001,8], mu2=0.05, omelyan tau=1 steps "
                               + "/".join(map(str, nsteps)),
                   "lattice": list(L), "kappa": KAPPA, "link_spread": LINK_SPREAD, "md_steps": nsteps,
                   "thermalisation_mp_trajectories": args.therm, "parallelism": "single GPU"},
        "roofline": hbm["bf16_x4"],
        "hop_applications": n_hop,
        "extra": extra,
    }
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(gpu_iters, gpu_iters8, full=args.cpu_full)
        except Exception as e:  # the baseline must not hide the GPU result
            out["cpu_baseline"] = {"error": str(e)[:200]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
