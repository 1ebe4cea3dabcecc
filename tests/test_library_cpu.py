"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, the header compiles as C, and the host-side integrator schedule
matches the paper's worked example and the oracle (no GPU needed)."""
import ctypes
import os
import re
import subprocess
from fractions import Fraction

import pytest

from oracle import integrator as oint

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wilson_hmc.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)))


def _lib():
    from paper_1702_00124_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwilson_hmc.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = _declared_functions()
    assert len(names) >= 30
    for n in ("wilson_dslash", "apply_K", "cg_solve", "poly_filter_apply", "fermion_force", "hmc_trajectory"):
        assert n in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # every declared symbol has a ctypes signature in the binding
    from paper_1702_00124_amd import _lib as W
    assert sorted(W.SIGNATURES) == names


def test_header_compiles_as_c(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "wilson_hmc.h"\nint main(void) { return WL_OK; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c", str(c), "-o",
                        str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_error_reporting_without_device():
    lib = _lib()
    from paper_1702_00124_amd import _lib as W
    n = ctypes.c_int()
    assert lib.wl_integrator_schedule(None, 0, 0, 0.0, None, None, None, 0, ctypes.byref(n)) == W.WL_EINVAL
    assert b"bad arguments" in lib.wl_last_error()
    assert lib.wl_destroy(None) == W.WL_OK


def _to_fractions(sched):
    out = []
    for e in sched:
        if e[0] == "T":
            out.append(("T", Fraction(e[1]).limit_denominator(10000)))
        else:
            out.append(("S", e[1], Fraction(e[2]).limit_denominator(10000)))
    return out


def test_library_schedule_reproduces_paper_example():
    _lib()
    from paper_1702_00124_amd.lattice import integrator_schedule
    from tests.test_oracle_integrator_hmc import _read_golden
    got = _to_fractions(integrator_schedule([2, 3], "leapfrog"))
    assert got == _read_golden()


@pytest.mark.parametrize("kind", ["leapfrog", "omelyan"])
def test_library_schedule_matches_oracle(kind):
    _lib()
    from paper_1702_00124_amd.lattice import integrator_schedule
    ns = [40, 20, 20, 80]
    lib_s = integrator_schedule(ns, kind)
    ora_s = oint.merge([oint.scheme_events(kind, n) for n in ns])
    assert len(lib_s) == len(ora_s)
    for a, b in zip(lib_s, ora_s):
        assert a[0] == b[0]
        if a[0] == "S":
            assert a[1] == b[1] and abs(a[2] - float(b[2])) < 1e-15
        else:
            assert abs(a[1] - float(b[1])) < 1e-15


def test_binding_structs_match_header_layout(tmp_path):
    """Every ctypes struct of the binding has the header struct's size and
    member offsets (a C probe compiled against the header prints them)."""
    from paper_1702_00124_amd import _lib as W
    structs = {"wl_cg_params": W.CgParams, "wl_cg_stats": W.CgStats, "wl_poly": W.Poly, "wl_term": W.Term,
               "wl_hmc_params": W.HmcParams, "wl_hmc_result": W.HmcResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "wilson_hmc.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_autotune_cache_file_round_trip(tmp_path):
    """The autotuner cache: key from extents, device and library build; entries
    added one by one to one JSON file; a missing or corrupt file reads as empty."""
    from paper_1702_00124_amd import _lib as W
    from paper_1702_00124_amd.lattice import tune_cache_key, tune_cache_read, tune_cache_write
    k1 = tune_cache_key((16, 16, 16, 32), "gpu", W.LIB_PATH)
    k2 = tune_cache_key((8, 8, 8, 16), "gpu", W.LIB_PATH)
    assert k1 != k2 and k1.startswith("16x16x16x32|gpu|")
    path = str(tmp_path / "tune.json")
    assert tune_cache_read(path, k1) is None
    e1 = {"configs": {"f64": [[0, 1, 1, 0]] * 3}, "us": {"f64": [1.0] * 48}}
    e2 = {"configs": {"f32": [[1, 4, 0, 1]] * 3}, "us": {"f32": [2.0] * 48}}
    tune_cache_write(path, k1, e1)
    tune_cache_write(path, k2, e2)
    assert tune_cache_read(path, k1) == e1 and tune_cache_read(path, k2) == e2
    (tmp_path / "bad.json").write_text("{not json")
    assert tune_cache_read(str(tmp_path / "bad.json"), k1) is None


def test_cost_checkpoint_files_round_trip(tmp_path):
    """Checkpoint state and arrays survive a write / read cycle exactly; no state reads as None."""
    import numpy as np
    from paper_1702_00124_amd.cost import Checkpoint
    ck = Checkpoint(str(tmp_path / "ck"))
    assert ck.load_state() is None
    U = (np.arange(24, dtype=np.float64) * (1 + 0.5j)).reshape(2, 3, 4)
    ck.save_array("links", U)
    st = {"run": {"lattice": [4, 4, 4, 4]}, "phase": "MP", "k": 2, "rows": [[0.1, True, 5, 6, 0.5, 1.0]],
          "done": {}}
    ck.save_state(st)
    assert np.array_equal(ck.load_array("links"), U) and ck.load_array("links").dtype == np.complex128
    assert ck.load_state() == st


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(HEADER), "..", "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_bench_counter_table_covers_the_kernels_only_launches():
    """bench.py's 32^3 x 64 HBM traffic table (FETCH_SIZE / WRITE_SIZE per launch) has an
    entry for every configuration its --kernels-only leg launches with 1 and 4 rhs, in
    every precision: every configuration the autotuner can keep for the roofline launches
    (the thread-per-site kernel with one or two rhs per thread, its shared-link variant
    and the direction-parallel passes, in the three workgroup orders, cached and
    streaming), so the bench line's traffic is never missing for a tuned choice."""
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(HEADER), ".."))
    import bench
    kib = bench.PMC_COUNTERS["per_launch_kib"]
    for nrhs in (1, 4):
        for prec in ("f64", "f32", "bf16"):
            cfgs = bench.kernels_only_configs(prec, nrhs)
            variants = {c[0] for c in cfgs}
            assert variants == ({0, 1} if nrhs == 1 else {0, 1, 2}), (prec, nrhs)
            for cfg in cfgs:
                key = f"{prec}:{nrhs}:" + ":".join(map(str, cfg))
                assert key in kib, key
                assert kib[key]["fetch"] > 0 and kib[key]["write"] > 0
