"""GPU parity: layout round trips, the hop kernel and the operators, against the FP64 oracle.

FP64 bar: relative l2 error <= 1e-12 (the operator is a fixed sum of a few
hundred products per site; observed errors are ~1e-16).  FP32 / BF16 storage
is compared to the FP64 oracle with the error stated in each test: unit
roundoff times the O(10) growth of one stencil application (FP32: 2^-24 ->
bound 1e-6; BF16 storage of links and spinors: 2^-9 -> bound 2e-2).
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
from oracle import wilson as ow
from paper_1702_00124_amd.lattice import CG
from tests.gpu_common import LOWP_MAX, full_noise, half_noise, make_lattice, need_gpu, rel, rel_max, say, to_np

pytestmark = pytest.mark.gpu

# 4^4: one partial workgroup; 6x4x4x10: two workgroups, ragged tail;
# 8^4: eight workgroups (XCD-aware tile order active)
SHAPES = [(4, 4, 4, 4), (6, 4, 4, 10), (8, 8, 8, 8)]


@pytest.mark.parametrize("L", SHAPES)
def test_layout_roundtrips(L):
    say("layout roundtrip", L)
    lat, U = make_lattice(L)
    assert np.array_equal(to_np(lat.get_links()), U)
    psi = half_noise(L, 1, nrhs=3)
    for prec in ("f64", "f32", "bf16"):
        back = to_np(lat.export_spinor(lat.import_spinor(torch.from_numpy(psi), prec), prec, 3))
        tol = {"f64": 0.0, "f32": 1e-7, "bf16": 8e-3}[prec]
        assert rel(back, psi) <= tol, prec
    f = full_noise(L, 2)
    assert np.array_equal(to_np(lat.export_full(lat.import_full(torch.from_numpy(f)))), f)
    p = li.gaussian_momenta(L, 3)
    assert np.array_equal(to_np(lat.export_su3(lat.import_su3(torch.from_numpy(p)))), p)


VARIANTS = [0, 1, 2]   # thread per site, direction-parallel, thread per site with the links shared in LDS


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("L", SHAPES)
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("dagger", [False, True])
def test_dslash_f64_matches_oracle(L, parity, dagger, variant):
    say("dslash f64", L, parity, dagger, "variant", variant)
    lat, U = make_lattice(L, variant=variant)
    psi = half_noise(L, 10 + parity)
    got = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi)), parity, dagger)))
    ref = ow.hop_eo(U, psi, L, parity, t_bc=-1, dagger=dagger)
    assert rel(got, ref) <= 1e-12


def test_dslash_free_field_plane_wave_at_full_size():
    """U = 1 at 16^3 x 32: D maps each plane wave to its closed-form momentum-space image."""
    L = (16, 16, 16, 32)
    say("free-field plane wave", L)
    lat, U = make_lattice(L, unit=True)
    from oracle import lattice as olat
    g = olat.gammas()
    x, y, z, t = olat.coords(L)
    n = (3, 5, 7, 2)
    p = np.array([2 * np.pi * n[0] / L[0], 2 * np.pi * n[1] / L[1], 2 * np.pi * n[2] / L[2], (2 * n[3] + 1) * np.pi / L[3]])
    u = li.gaussian_spinor((4, 3), 4)
    psi = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[:, None, None] * u[None]
    Dk = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * g[m] for m in range(4))
    expect = np.einsum("st,xtc->xsc", Dk, psi)
    ev, od = olat.parity_sites(L, 0), olat.parity_sites(L, 1)
    got_e = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi[od])), 0)))
    got_o = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi[ev])), 1)))
    assert rel(got_e, expect[ev]) <= 1e-13
    assert rel(got_o, expect[od]) <= 1e-13


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("bf16", 2e-2)])
def test_dslash_low_precision_error(prec, tol, variant):
    L = (8, 8, 8, 8)
    say("dslash", prec, L, "variant", variant)
    lat, U = make_lattice(L, variant=variant)
    psi = half_noise(L, 21, nrhs=4)
    got = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), 0, prec=prec, nrhs=4),
                                  prec, 4))
    for r in range(4):
        ref = ow.hop_eo(U, psi[r], L, 0)
        e = rel(got[r], ref)
        em = rel_max(got[r], ref)
        say(f"  rhs {r}: relative error vs FP64 oracle {e:.3e}, max element {em:.3e}")
        assert e <= tol
        assert em <= LOWP_MAX[prec]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [2, 3, 4])
def test_dslash_multi_rhs_equals_single(nrhs, prec, variant):
    """Batched rhs give bit-identical results to one-at-a-time (same arithmetic per rhs)."""
    L = (6, 4, 4, 10)
    say("dslash multi-rhs", nrhs, prec, "variant", variant)
    lat, U = make_lattice(L, variant=variant)
    psi = half_noise(L, 31, nrhs=nrhs)
    multi = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), 1, prec=prec,
                                               nrhs=nrhs), prec, nrhs))
    for r in range(nrhs):
        single = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi[r]), prec), 1, prec=prec),
                                         prec))
        assert np.array_equal(multi[r], single)


def test_variants_agree_and_autotune():
    L = (8, 8, 8, 8)
    say("variants agree / autotune")
    lat, U = make_lattice(L)
    psi = half_noise(L, 33)
    outs = []
    for v in VARIANTS:
        lat.set_hop_variant("f64", v)
        outs.append(to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi)), 0))))
    assert rel(outs[0], outs[1]) <= 1e-14 and np.array_equal(outs[0], outs[2])
    res = lat.autotune()
    say(f"  autotune us per launch: {res}")
    # 8^4 fits the last-level cache: streaming candidates are not timed; a z plane of
    # 32 half sites holds no whole tile, so the z-blocked order is not a candidate either
    # classes 1 and 2: site 1, site 2, shared, dp 1, dp 2, dp 4 per (stream, order)
    for v in res.values():
        assert len(v) == 84
        assert min(v[0:4]) > 0 and v[4:12] == [0.0] * 8                # class 0
        for c0 in (12, 48):                                             # classes 1 and 2
            assert min(v[c0:c0 + 12]) > 0 and v[c0 + 12:c0 + 36] == [0.0] * 24
    for prec in ("f64", "f32", "bf16"):
        assert all(lat.hop_config(prec, k)[3] == 0 for k in range(3))
    for prec in ("f64", "f32", "bf16"):
        say(f"  kept {prec}: {[lat.hop_config(prec, k) for k in range(3)]}")
    # the tuned choice still gives the oracle's hop, one rhs and several
    psi4 = half_noise(L, 34, nrhs=4)
    got = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi4)), 0, nrhs=4), "f64", 4))
    for r in range(4):
        assert rel(got[r], ow.hop_eo(U, psi4[r], L, 0)) <= 1e-12


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 10)])
def test_operators_match_oracle(L):
    say("operators", L)
    kappa = 0.155
    lat, U = make_lattice(L)
    e = half_noise(L, 41)
    eb = lat.import_spinor(torch.from_numpy(e))
    got = to_np(lat.export_spinor(lat.apply_K(eb, kappa, "MHAT")))
    assert rel(got, ow.Mhat(U, e, L, kappa)) <= 1e-12
    got = to_np(lat.export_spinor(lat.apply_K(eb, kappa, "MHAT_DAG")))
    assert rel(got, ow.Mhat(U, e, L, kappa, dagger=True)) <= 1e-12
    for mu2 in (0.0, 0.05):
        got = to_np(lat.export_spinor(lat.apply_K(eb, kappa, "J", mu2=[mu2])))
        assert rel(got, ow.J(U, e, L, kappa, mu2)) <= 1e-12
    f = full_noise(L, 42)
    fb = lat.import_full(torch.from_numpy(f))
    assert rel(to_np(lat.export_full(lat.apply_K(fb, 0.12, "M"))), ow.M(U, f, L, 0.12)) <= 1e-12
    assert rel(to_np(lat.export_full(lat.apply_K(fb, 0.12, "MDAG"))), ow.M(U, f, L, 0.12, dagger=True)) <= 1e-12
    assert rel(to_np(lat.export_full(lat.apply_K(fb, 0.12, "K"))), ow.K(U, f, L, 0.12)) <= 1e-12


def test_shifted_operator_batch_per_rhs_shift():
    L = (6, 4, 4, 10)
    say("J batch with per-rhs shifts")
    lat, U = make_lattice(L)
    mu2 = [0.0, 0.005, 0.05, 0.5]
    e = half_noise(L, 51, nrhs=4)
    got = to_np(lat.export_spinor(lat.apply_K(lat.import_spinor(torch.from_numpy(e)), 0.155, "J", mu2=mu2, nrhs=4),
                                  "f64", 4))
    for r in range(4):
        assert rel(got[r], ow.J(U, e[r], L, 0.155, mu2[r])) <= 1e-12


def test_errors_are_reported():
    need_gpu()
    from paper_1702_00124_amd import WilsonError
    from paper_1702_00124_amd.lattice import WilsonLattice
    with pytest.raises(WilsonError):
        WilsonLattice((5, 4, 4, 4))
    lat, _ = make_lattice((4, 4, 4, 4))
    b = lat.new_field()
    with pytest.raises(WilsonError):
        lat.dslash(b, 0, nrhs=17)
    with pytest.raises(WilsonError):
        lat.apply_K(b, 0.1, "J", out=b)


@pytest.mark.parametrize("passes", [1, 2, 4])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [5, 8, 12, 16])
def test_dslash_link_reuse_passes_equal_single(nrhs, prec, passes):
    """Direction-parallel kernel holding each link across 1, 2 or 4 rhs passes:
    bit-identical to one rhs at a time, dagger included; 16 = the rhs limit."""
    L = (6, 4, 4, 10)
    say("dslash link-reuse passes", passes, prec, "nrhs", nrhs)
    lat, U = make_lattice(L, variant=1)
    lat.set_hop_config(prec, -1, npass=passes)
    psi = half_noise(L, 35, nrhs=nrhs)
    for dagger in (False, True):
        multi = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), 0, dagger,
                                                   prec=prec, nrhs=nrhs), prec, nrhs))
        for r in range(nrhs):
            single = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(psi[r]), prec), 0, dagger,
                                                        prec=prec), prec))
            assert np.array_equal(multi[r], single), (r, dagger)
        if prec == "f64":
            assert rel(multi[nrhs - 1], ow.hop_eo(U, psi[nrhs - 1], L, 0, t_bc=-1, dagger=dagger)) <= 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
def test_dslash_zblocked_order_invariance(variant):
    """The z-blocked workgroup order (32x32 z planes of 8 columns of 64 half
    sites, Lz = 16: two blocks of 8 planes) changes no output bit against the
    other two orders, with one rhs, four and eight (the rhs groups of a tile on
    one XCD), in every storage precision; a CG whose J hops take it (with the
    fused <p, Jp> partials per 64-site tile) converges to the oracle's J."""
    L = (32, 32, 16, 4)
    say("dslash z-blocked order", "variant", variant)
    lat, U = make_lattice(L, variant=variant)
    psi = half_noise(L, 38, nrhs=8)
    for prec in ("f64", "f32", "bf16"):
        for nrhs in (1, 4, 8):
            src = psi[0] if nrhs == 1 else psi[:nrhs]
            outs = {}
            for xcd in (1, 0, 2):
                lat.set_hop_config(prec, -1, use_xcd=xcd)
                outs[xcd] = to_np(lat.export_spinor(lat.dslash(lat.import_spinor(torch.from_numpy(src), prec), 0,
                                                               prec=prec, nrhs=nrhs), prec, nrhs))
            assert np.array_equal(outs[0], outs[1]), (prec, nrhs)
            assert np.array_equal(outs[2], outs[1]), (prec, nrhs)
            if prec == "f64" and nrhs > 1:
                assert rel(outs[2][nrhs - 1], ow.hop_eo(U, psi[nrhs - 1], L, 0)) <= 1e-12
    b = half_noise(L, 39)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", params=CG(tol=1e-10, inner="f32"))
    assert rc == 0 and st[0].true_rel_res <= 1e-10
    assert rel(ow.J(U, to_np(lat.export_spinor(x)), L, 0.155, 0.0), b) <= 1.01e-10


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (6, 4, 4, 10)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_dslash_launch_config_invariance(variant, L):
    """Rhs per pass or thread, passes per link load and workgroup order change
    no output bit of a variant, streaming access at most one rounding; 8^4
    spans 32 64-site tiles per parity, 6x4x4x10 a ragged 7.5 (and 1.9 blocks of
    the thread-per-site kernel, whose round-robin grid is padded to 8)."""
    say("dslash launch configurations", "variant", variant, L)
    lat, U = make_lattice(L, variant=variant)
    psi = half_noise(L, 36, nrhs=4)
    outs = {}
    for npass in (1, 2, 4):
        for xcd in (1, 0):
            for stream in (0, 1):
                for prec in ("f64", "bf16"):
                    lat.set_hop_config(prec, -1, npass=npass, use_xcd=xcd, stream=stream)
                    outs[(npass, xcd, stream, prec)] = to_np(lat.export_spinor(
                        lat.dslash(lat.import_spinor(torch.from_numpy(psi), prec), 1, prec=prec, nrhs=4), prec, 4))
    # same code path: bit-identical; streaming access compiles to other load
    # and store instructions, where the compiler may contract products into
    # FMAs differently: one rounding of the storage precision at most
    for k, v in outs.items():
        ref = outs[(1, 1, k[2], k[3])]
        assert np.array_equal(v, ref), k
        other = outs[(1, 1, 1 - k[2], k[3])]
        e = rel(v, other)
        if e:
            say(f"  {k}: streaming vs cached relative difference {e:.2e}")
        assert e <= (1e-15 if k[3] == "f64" else 4e-3), k
    assert rel(outs[(1, 1, 0, "f64")][2], ow.hop_eo(U, psi[2], L, 1)) <= 1e-12
    lat.set_hop_config("f32", -1, npass=2, use_xcd=0, stream=1)
    b = half_noise(L, 37)
    x, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", params=CG(tol=1e-10, inner="f32"))
    assert rc == 0 and st[0].true_rel_res <= 1e-10
    assert rel(ow.J(U, to_np(lat.export_spinor(x)), L, 0.155, 0.0), b) <= 1.01e-10
    with pytest.raises(Exception):
        lat.set_hop_config("f64", 0, npass=3)


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (6, 4, 4, 10)])
def test_shared_link_variant_matches_site_kernel(L):
    """The shared-link variant (a workgroup takes one 64-site tile for four rhs
    and reads the tile's links into LDS once) gives the thread-per-site
    kernel's output bit for bit: every precision, 4, 5, 8 and 16 rhs (5: a partly
    idle last group of four), both output parities and the dagger, every workgroup
    order, and with the fused epilogue (J with per-rhs shifts); a batched CG
    whose J hops take it (with the fused <p, Jp> partials) converges to the
    oracle's J."""
    say("shared-link variant", L)
    lat, U = make_lattice(L)
    psi = half_noise(L, 91, nrhs=16)
    shifts = [0.0, 0.005, 0.05, 0.5] * 4
    for prec in ("f64", "f32", "bf16"):
        for nrhs in (4, 5, 8, 16):
            x = lat.import_spinor(torch.from_numpy(psi[:nrhs]), prec)
            outs = {}
            for variant, xcd in ((0, 1), (2, 1), (2, 0)):
                lat.set_hop_config(prec, -1, variant=variant, npass=1, use_xcd=xcd, stream=0)
                for parity in (0, 1):
                    for dag in (False, True):
                        outs[(variant, xcd, parity, dag)] = to_np(lat.export_spinor(
                            lat.dslash(x, parity, dagger=dag, prec=prec, nrhs=nrhs), prec, nrhs))
                outs[(variant, xcd, "J")] = to_np(lat.export_spinor(
                    lat.apply_K(x, 0.155, op="J", mu2=shifts[:nrhs], prec=prec, nrhs=nrhs), prec, nrhs))
            for k, v in outs.items():
                assert np.array_equal(v, outs[(0, 1) + k[2:]]), (prec, nrhs, k)
    lat.set_hop_config("f32", -1, variant=2, npass=1, use_xcd=0, stream=0)
    b = half_noise(L, 92, nrhs=4)
    xs, st, rc = lat.cg_solve(lat.import_spinor(torch.from_numpy(b)), 0.155, "J", mu2=shifts[:4], nrhs=4,
                              params=CG(tol=1e-10, inner="f32"))
    assert rc == 0 and all(s.true_rel_res <= 1e-10 for s in st)
    xr = to_np(lat.export_spinor(xs, "f64", 4))
    for r in range(4):
        assert rel(ow.J(U, xr[r], L, 0.155, shifts[r]), b[r]) <= 1.01e-10
    lat.close()


def test_autotune_cache_hit_sets_same_configurations(tmp_path):
    """A second lattice of the same shape takes the cached configurations without timing."""
    L = (8, 8, 8, 8)
    path = str(tmp_path / "tune.json")
    lat1, _ = make_lattice(L)
    us1 = lat1.autotune(cache=path)
    lat2, _ = make_lattice(L)
    for prec in ("f64", "f32", "bf16"):
        lat2.set_hop_config(prec, -1, variant=0 if lat1.hop_config(prec, 0)[0] else 1)
    us2 = lat2.autotune(cache=path)
    assert us2 == us1
    for prec in ("f64", "f32", "bf16"):
        assert [lat2.hop_config(prec, k) for k in range(3)] == [lat1.hop_config(prec, k) for k in range(3)]
