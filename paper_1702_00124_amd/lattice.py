"""Python binding of libwilson_hmc: torch tensors for device memory and streams.

Argument marshalling only.  Every computation (layout packing, hops,
operators, solves, polynomial filter, forces, HMC) runs in the HIP library;
torch allocates the buffers and supplies the stream.

Field conventions (see include/wilson_hmc.h): canonical spinors are complex128
``[nrhs, V/2, 4, 3]`` (one parity, lexicographic) or ``[V, 4, 3]`` (full);
links complex128 ``[4, V, 3, 3]``; su(3) fields float64 ``[4, V, 8]``.  Internal
fields are opaque uint8 device tensors of ``field_bytes`` bytes.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _lib as W

PREC = {"f64": W.WL_F64, "f32": W.WL_F32, "bf16": W.WL_BF16}
TERM_KIND = {"KINV_FULL": W.WL_TERM_KINV_FULL, "KINV": W.WL_TERM_KINV, "RATIO": W.WL_TERM_RATIO,
             "POLY": W.WL_TERM_POLY, "POLYK_INV": W.WL_TERM_POLYK_INV}
POLY_MODE = {"P": W.WL_POLY_P, "PJ": W.WL_POLY_PJ, "Q": W.WL_POLY_Q, "QDAG": W.WL_POLY_QDAG}
OPS = {"M": W.WL_OP_M, "MDAG": W.WL_OP_MDAG, "K": W.WL_OP_K, "MHAT": W.WL_OP_MHAT,
       "MHAT_DAG": W.WL_OP_MHAT_DAG, "J": W.WL_OP_J}


def _ptr(t: torch.Tensor) -> C.c_void_p:
    if not t.is_cuda:
        raise ValueError("libwilson_hmc takes device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _host_ptr(t: torch.Tensor) -> C.c_void_p:
    if t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous host tensor")
    return C.c_void_p(t.data_ptr())


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def _need(t: torch.Tensor, nbytes: int, what: str = "buffer"):
    """Reject device buffers smaller than the library will touch (it sees plain pointers)."""
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what} has {have} bytes, needs {nbytes}")


@dataclass
class CG:
    tol: float = 1e-10
    maxiter: int = 10000
    inner: str = "f64"
    delta: float = 0.1
    chunk: int = 8
    use_graph: bool = False
    use_x0: bool = False       # cg_solve: the x passed in holds the initial guess

    def c(self) -> W.CgParams:
        return W.CgParams(self.tol, self.maxiter, _prec(self.inner), self.delta, self.chunk, int(self.use_graph),
                          int(self.use_x0))


@dataclass
class Term:
    """A pseudofermion action term (kinds: KINV_FULL, KINV, RATIO, POLY, POLYK_INV).

    (kappa, mu2) define the term's J = K-hat(kappa) + mu2; RATIO's numerator is
    M-hat(kappa_num or kappa) + i sqrt(mu2_num) g5; degree_div > 0 makes the
    polynomial the quotient P_degree / P_degree_div."""
    kind: str
    kappa: float
    mu2: float = 0.0
    degree: int = 0
    a: float = 0.001
    b: float = 8.0
    cg: CG = field(default_factory=CG)
    degree_div: int = 0
    kappa_num: float = 0.0
    mu2_num: float = 0.0

    def c(self) -> W.Term:
        return W.Term(TERM_KIND[self.kind], self.kappa, self.mu2, W.Poly(self.degree, self.a, self.b, self.degree_div),
                      self.cg.c(), self.kappa_num, self.mu2_num)

    @property
    def full(self) -> bool:
        return self.kind == "KINV_FULL"


@dataclass
class CgResult:
    iters: int
    reliable_updates: int
    converged: bool
    true_rel_res: float


class WilsonLattice:
    """One lattice context: geometry, packed links, workspace (owned by the library)."""

    def __init__(self, L: Sequence[int], t_bc: int = -1, device: Optional[torch.device] = None):
        self.lib = W.load()
        dev = torch.device(device or "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        torch.cuda.set_device(self.device)
        self.L = tuple(int(x) for x in L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.Vh = self.V // 2
        self.t_bc = t_bc
        h = C.c_void_p()
        arr = (C.c_int32 * 4)(*self.L)
        W.check(self.lib.wl_create(C.byref(h), arr, t_bc, self._stream()))
        self.h = h

    def _stream(self) -> C.c_void_p:
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        W.check(self.lib.wl_set_stream(self.h, self._stream()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.wl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- memory
    def field_bytes(self, prec="f64", nrhs: int = 1) -> int:
        n = C.c_size_t()
        W.check(self.lib.wl_field_bytes(self.h, _prec(prec), nrhs, C.byref(n)))
        return n.value

    def new_field(self, prec="f64", nrhs: int = 1, full: bool = False) -> torch.Tensor:
        n = self.field_bytes(prec, nrhs) * (2 if full else 1)
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def new_su3(self) -> torch.Tensor:
        # [2 parity][4 mu][8][V/2] float64
        return torch.zeros(32 * self.V, dtype=torch.float64, device=self.device)

    # ---------------------------------------------------------------- links / fields
    def set_links(self, U: torch.Tensor):
        """Canonical complex128 [4, V, 3, 3] links; a CPU tensor is handed over as a host
        array (the library stages it), a device tensor as a device array."""
        on_device = U.device.type != "cpu"
        U = (U.to(device=self.device) if on_device else U).to(dtype=torch.complex128).contiguous()
        assert U.shape == (4, self.V, 3, 3)
        W.check(self.lib.wl_set_links(self.h, _ptr(U) if on_device else _host_ptr(U), int(on_device)))

    def get_links(self, host: bool = False) -> torch.Tensor:
        """The links as canonical complex128 [4, V, 3, 3] (host=True: into a CPU tensor)."""
        U = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device="cpu" if host else self.device)
        W.check(self.lib.wl_get_links(self.h, _host_ptr(U) if host else _ptr(U), int(not host)))
        return U

    def import_spinor(self, psi: torch.Tensor, prec="f64") -> torch.Tensor:
        psi = psi.to(device=self.device, dtype=torch.complex128).contiguous()
        nrhs = 1 if psi.dim() == 3 else psi.shape[0]
        assert psi.shape[-3:] == (self.Vh, 4, 3)
        out = self.new_field(prec, nrhs)
        W.check(self.lib.wl_import_spinor(self.h, _ptr(out), _ptr(psi), _prec(prec), nrhs))
        return out

    def export_spinor(self, buf: torch.Tensor, prec="f64", nrhs: int = 1) -> torch.Tensor:
        _need(buf, self.field_bytes(prec, nrhs), "internal field")
        out = torch.empty((nrhs, self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        W.check(self.lib.wl_export_spinor(self.h, _ptr(out), _ptr(buf), _prec(prec), nrhs))
        return out[0] if nrhs == 1 else out

    def import_full(self, psi: torch.Tensor) -> torch.Tensor:
        psi = psi.to(device=self.device, dtype=torch.complex128).contiguous()
        assert psi.shape == (self.V, 4, 3)
        out = self.new_field("f64", 1, full=True)
        W.check(self.lib.wl_import_full(self.h, _ptr(out), _ptr(psi)))
        return out

    def export_full(self, buf: torch.Tensor) -> torch.Tensor:
        _need(buf, 2 * self.field_bytes("f64"), "internal field")
        out = torch.empty((self.V, 4, 3), dtype=torch.complex128, device=self.device)
        W.check(self.lib.wl_export_full(self.h, _ptr(out), _ptr(buf)))
        return out

    def import_su3(self, p: torch.Tensor) -> torch.Tensor:
        p = p.to(device=self.device, dtype=torch.float64).contiguous()
        assert p.shape == (4, self.V, 8)
        out = self.new_su3()
        W.check(self.lib.wl_import_su3(self.h, _ptr(out), _ptr(p)))
        return out

    def export_su3(self, buf: torch.Tensor) -> torch.Tensor:
        _need(buf, 256 * self.V, "internal su(3) field")
        out = torch.empty((4, self.V, 8), dtype=torch.float64, device=self.device)
        W.check(self.lib.wl_export_su3(self.h, _ptr(out), _ptr(buf)))
        return out

    # ---------------------------------------------------------------- operators
    def dslash(self, buf: torch.Tensor, out_parity: int, dagger: bool = False, prec="f64", nrhs: int = 1,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_field(prec, nrhs) if out is None else out
        if 1 <= nrhs <= 16:
            _need(buf, self.field_bytes(prec, nrhs), "input")
            _need(out, self.field_bytes(prec, nrhs), "output")
        W.check(self.lib.wilson_dslash(self.h, _ptr(out), _ptr(buf), out_parity, int(dagger), _prec(prec), nrhs))
        return out

    def apply_K(self, buf: torch.Tensor, kappa: float, op: str = "J", mu2: Sequence[float] = (0.0,),
                prec="f64", nrhs: int = 1, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        full = op in ("M", "MDAG", "K")
        out = self.new_field(prec, nrhs, full=full) if out is None else out
        if 1 <= nrhs <= 16:
            need = self.field_bytes(prec, nrhs) * (2 if full else 1)
            _need(buf, need, "input")
            _need(out, need, "output")
        m = (C.c_double * max(nrhs, 1))(*list(mu2)[:nrhs]) if mu2 is not None else None
        W.check(self.lib.apply_K(self.h, _ptr(out), _ptr(buf), kappa, m, nrhs, OPS[op], _prec(prec)))
        return out

    def apply_K_noalloc(self, buf: torch.Tensor, out: torch.Tensor, kappa: float, op: str = "J",
                        mu2: Sequence[float] = (0.0,), prec="f64", nrhs: int = 1) -> torch.Tensor:
        """apply_K with the operator's intermediates in the library's fixed device
        scratch: no device allocation in the call (the caller passes out)."""
        full = op in ("M", "MDAG", "K")
        if 1 <= nrhs <= 16:
            need = self.field_bytes(prec, nrhs) * (2 if full else 1)
            _need(buf, need, "input")
            _need(out, need, "output")
        m = (C.c_double * max(nrhs, 1))(*list(mu2)[:nrhs]) if mu2 is not None else None
        W.check(self.lib.apply_K_noalloc(self.h, _ptr(out), _ptr(buf), kappa, m, nrhs, OPS[op], _prec(prec)))
        return out

    def cg_solve(self, b: torch.Tensor, kappa: float, op: str = "J", mu2: Sequence[float] = (0.0,), nrhs: int = 1,
                 params: Optional[CG] = None, x: Optional[torch.Tensor] = None):
        params = params or CG()
        full = op == "K"
        x = self.new_field("f64", nrhs, full=full) if x is None else x
        if 1 <= nrhs <= 16:
            need = self.field_bytes("f64", nrhs) * (2 if full else 1)
            _need(b, need, "rhs")
            _need(x, need, "solution")
        m = (C.c_double * nrhs)(*[float(v) for v in list(mu2)[:nrhs]]) if mu2 is not None else None
        st = (W.CgStats * nrhs)()
        prm = params.c()
        rc = W.check(self.lib.cg_solve(self.h, _ptr(x), _ptr(b), kappa, m, nrhs, OPS[op], C.byref(prm), st))
        res = [CgResult(s.iters, s.reliable_updates, bool(s.converged), s.true_rel_res) for s in st]
        return x, res, rc

    def cg_multishift(self, b: torch.Tensor, kappa: float, shifts: Sequence[float], nrhs: int = 1,
                      params: Optional[CG] = None):
        """x[s * nrhs + r] = (K-hat + shifts[s])^-1 b_r for every shift at once (FP64);
        returns (x, [[CgResult per rhs] per shift], rc)."""
        params = params or CG()
        ns = len(shifts)
        x = torch.empty(self.field_bytes("f64") * ns * nrhs, dtype=torch.uint8, device=self.device)
        _need(b, self.field_bytes("f64", nrhs), "rhs")
        sh = (C.c_double * ns)(*[float(v) for v in shifts])
        st = (W.CgStats * (ns * nrhs))()
        prm = params.c()
        rc = W.check(self.lib.cg_multishift(self.h, _ptr(x), _ptr(b), kappa, sh, ns, nrhs, C.byref(prm), st))
        res = [[CgResult(st[s * nrhs + r].iters, st[s * nrhs + r].reliable_updates, bool(st[s * nrhs + r].converged),
                         st[s * nrhs + r].true_rel_res) for r in range(nrhs)] for s in range(ns)]
        return x, res, rc

    def shift_block(self, x: torch.Tensor, s: int, nrhs: int) -> torch.Tensor:
        """The nrhs solutions of shift s inside a cg_multishift result."""
        fb = self.field_bytes("f64")
        return x[s * nrhs * fb:(s + 1) * nrhs * fb]

    def poly_filter_apply(self, buf: torch.Tensor, kappa: float, mu2: float, degree: int, a: float, b: float,
                          mode: str = "P", out: Optional[torch.Tensor] = None, degree_div: int = 0,
                          nrhs: int = 1, prec="f64") -> torch.Tensor:
        out = self.new_field(prec, nrhs) if out is None else out
        if 1 <= nrhs <= 16:
            _need(buf, self.field_bytes(prec, nrhs), "input")
            _need(out, self.field_bytes(prec, nrhs), "output")
        p = W.Poly(degree, a, b, degree_div)
        W.check(self.lib.poly_filter_apply(self.h, _ptr(out), _ptr(buf), kappa, mu2, C.byref(p), POLY_MODE[mode],
                                           nrhs, _prec(prec)))
        return out

    # ---------------------------------------------------------------- action terms / forces
    def heatbath(self, term: Term, chi: torch.Tensor) -> torch.Tensor:
        phi = self.new_field("f64", 1, full=term.full)
        _need(chi, phi.numel(), "noise")
        t = term.c()
        W.check(self.lib.wl_heatbath(self.h, _ptr(phi), C.byref(t), _ptr(chi)))
        return phi

    def action(self, term: Term, phi: torch.Tensor) -> float:
        s = C.c_double()
        _need(phi, self.field_bytes("f64") * (2 if term.full else 1), "pseudofermion")
        t = term.c()
        W.check(self.lib.wl_action(self.h, C.byref(t), _ptr(phi), C.byref(s)))
        return s.value

    def fermion_force(self, term: Term, phi: torch.Tensor, F: Optional[torch.Tensor] = None,
                      coeff: float = 1.0) -> torch.Tensor:
        F = self.new_su3() if F is None else F
        _need(F, 256 * self.V, "force")
        _need(phi, self.field_bytes("f64") * (2 if term.full else 1), "pseudofermion")
        t = term.c()
        W.check(self.lib.fermion_force(self.h, _ptr(F), C.byref(t), _ptr(phi), coeff, None))
        return F

    def force_bilinear(self, A_full: torch.Tensor, C_full: torch.Tensor, F: Optional[torch.Tensor] = None,
                       coeff: float = 1.0) -> torch.Tensor:
        F = self.new_su3() if F is None else F
        _need(F, 256 * self.V, "force")
        _need(A_full, 2 * self.field_bytes("f64"), "A")
        _need(C_full, 2 * self.field_bytes("f64"), "C")
        W.check(self.lib.wl_force_bilinear(self.h, _ptr(F), _ptr(A_full), _ptr(C_full), coeff))
        return F

    def gauge_force(self, beta: float, F: Optional[torch.Tensor] = None, coeff: float = 1.0) -> torch.Tensor:
        F = self.new_su3() if F is None else F
        _need(F, 256 * self.V, "force")
        W.check(self.lib.wl_gauge_force(self.h, _ptr(F), beta, coeff))
        return F

    def plaquette(self) -> float:
        p = C.c_double()
        W.check(self.lib.wl_plaquette(self.h, C.byref(p)))
        return p.value

    def link_update(self, P: torch.Tensor, eps: float):
        _need(P, 256 * self.V, "momenta")
        W.check(self.lib.wl_link_update(self.h, _ptr(P), eps))

    def hmc_trajectory(self, terms: List[Term], nsteps: Sequence[int], P: torch.Tensor, chi: torch.Tensor,
                       u: float, beta: float = 5.6, tau: float = 1.0, integrator: str = "omelyan",
                       no_metropolis: bool = False, omelyan_lambda: float = 0.0,
                       phi_given: bool = False, chrono: bool = False, chrono_depth: int = 0) -> W.HmcResult:
        prm = W.HmcParams()
        prm.beta, prm.tau, prm.omelyan_lambda = beta, tau, omelyan_lambda
        prm.integrator = W.WL_INT_OMELYAN if integrator == "omelyan" else W.WL_INT_LEAPFROG
        prm.nterms = len(terms)
        for i, t in enumerate(terms):
            prm.terms[i] = t.c()
        for i, n in enumerate(nsteps):
            prm.nsteps[i] = int(n)
        prm.flags = ((W.WL_HMC_NO_METROPOLIS if no_metropolis else 0) | (W.WL_HMC_PHI_GIVEN if phi_given else 0)
                     | (W.WL_HMC_CHRONO if chrono else 0))
        prm.chrono_depth = int(chrono_depth)
        _need(P, 256 * self.V, "momenta")
        _need(chi, sum(self.field_bytes("f64") * (2 if t.full else 1) for t in terms), "noise")
        res = W.HmcResult()
        W.check(self.lib.hmc_trajectory(self.h, C.byref(prm), _ptr(P), _ptr(chi), u, C.byref(res)))
        return res

    HOP_KINDS = (1, 4, 8)  # rhs counts the autotuner times classes 0, 1, 2 at (1, 2-4, 5-16 rhs)

    def hop_config(self, prec, kind: int):
        """(variant, npass, use_xcd, stream) of one precision and rhs class (0: 1 rhs, 1: 2-4, 2: 5-16)."""
        v = [C.c_int() for _ in range(4)]
        W.check(self.lib.wl_get_hop_config(self.h, _prec(prec), int(kind), *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_hop_config(self, prec, kind: int = -1, variant=None, npass=None, use_xcd=None, stream=None):
        """Set fields of the hop configuration (None keeps a field) of one rhs class or all (-1)."""
        for k in (range(3) if kind == -1 else (kind,)):
            cur = self.hop_config(prec, k)
            new = [cur[i] if v is None else int(v) for i, v in enumerate((variant, npass, use_xcd, stream))]
            W.check(self.lib.wl_set_hop_config(self.h, _prec(prec), k, *new))

    def set_hop_variant(self, prec, variant: int):
        """0: thread per site; 1: direction-parallel; 2: thread per site with the links
        shared in LDS across four rhs (from 4 rhs; below that variant 0 runs); for every
        rhs class."""
        self.set_hop_config(prec, -1, variant=variant)

    def autotune(self, cache: Optional[str] = None):
        """Time the hop configurations per precision and rhs class and keep the fastest.

        Returns {prec: [84 microsecond timings]} in the order the C API documents:
        class 0 (site, dp), then classes 1 and 2 (site 1, site 2, site with shared
        links, dp 1, dp 2, dp 4), each per (stream, order) = (0, 1), (0, 0), (0, 2),
        (1, 1), (1, 0), (1, 2) (0 where not a candidate).

        cache: a JSON file of earlier results keyed by lattice extents, device
        (ISA, compute units, memory) and library build; on a hit the stored configurations are set and
        their timings returned without timing anything, else the tuning result
        is added to the file."""
        key = tune_cache_key(self.L, tune_device_id(self.device), W.LIB_PATH) if cache else None
        if key:
            hit = tune_cache_read(cache, key)
            if hit is not None:
                for prec, cfgs in hit["configs"].items():
                    for k, c in enumerate(cfgs):
                        W.check(self.lib.wl_set_hop_config(self.h, _prec(prec), k, *c))
                return hit["us"]
        us = (C.c_double * 252)()
        W.check(self.lib.wl_autotune(self.h, us))
        res = {name: list(us[84 * i:84 * i + 84]) for name, i in PREC.items()}
        if key:
            tune_cache_write(cache, key, {"configs": {p: [list(self.hop_config(p, k)) for k in range(3)] for p in PREC},
                                          "us": res})
        return res

    def time_hop(self, prec="f64", nrhs: int = 1, nlaunch: int = 200) -> float:
        """Average microseconds per hop launch over a back-to-back burst."""
        us = C.c_double()
        W.check(self.lib.wl_time_hop(self.h, _prec(prec), nrhs, nlaunch, C.byref(us)))
        return us.value

    def stream_copy(self, nbytes: int = 1 << 30, reps: int = 10) -> float:
        """GB/s (read + write) of a plain device copy: the practical HBM ceiling."""
        g = C.c_double()
        W.check(self.lib.wl_stream_copy(self.h, nbytes, reps, C.byref(g)))
        return g.value

    def profile(self, enable: bool = True):
        W.check(self.lib.wl_profile(self.h, int(enable)))

    def profile_read(self):
        """{prec: (average hop launch duration in us, samples)} of the sampled launches."""
        us = (C.c_double * 3)()
        n = (C.c_longlong * 3)()
        W.check(self.lib.wl_profile_read(self.h, us, n))
        return {name: (us[i], n[i]) for name, i in PREC.items()}

    def hop_counts(self):
        """{prec: hop applications since create} (single-rhs units)."""
        n = (C.c_longlong * 3)()
        W.check(self.lib.wl_hop_counts(self.h, n))
        return {name: n[i] for name, i in PREC.items()}

    def solve_log(self, enable: bool = True):
        """Start (clearing) or stop the log of every CG this context runs."""
        W.check(self.lib.wl_solve_log(self.h, int(enable)))

    def solve_log_read(self, max_solves: int = 100000):
        """[(iterations summed over rhs, FP64 residual applications, K multiplications
        per operator application)] of the logged solves, in order."""
        n = C.c_int()
        it = (C.c_longlong * max_solves)()
        rs = (C.c_longlong * max_solves)()
        jp = (C.c_longlong * max_solves)()
        W.check(self.lib.wl_solve_log_read(self.h, max_solves, C.byref(n), it, rs, jp))
        return [(it[i], rs[i], jp[i]) for i in range(n.value)]

    def counters(self):
        a, b = C.c_longlong(), C.c_longlong()
        W.check(self.lib.wl_counters(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value


def tune_device_id(device) -> str:
    """The device as the tuning cache knows it: ISA, compute units and memory
    size (the marketing name can read empty, e.g. under a profiler)."""
    pr = torch.cuda.get_device_properties(device)
    arch = getattr(pr, "gcnArchName", "") or pr.name
    return f"{arch.split(':')[0]}/{pr.multi_processor_count}cu/{pr.total_memory >> 30}GiB"


def tune_cache_key(L: Sequence[int], device_name: str, lib_path: str) -> str:
    """Autotuner cache key: lattice extents, device and the library build (its bytes' sha256)."""
    import hashlib
    with open(lib_path, "rb") as f:
        build = hashlib.sha256(f.read()).hexdigest()[:16]
    return f"{'x'.join(str(int(v)) for v in L)}|{device_name}|{build}"


def tune_cache_read(path: str, key: str):
    import json
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def tune_cache_write(path: str, key: str, entry) -> None:
    """Add one entry (written to a temporary file, then renamed over the cache)."""
    import json
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[key] = entry
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, path)


class WilsonBatch:
    """Mixed-volume batch of lattices (one device, one stream) whose hops run as
    one launch: batch fields are one slot per lattice, slot l holding lattice
    l's internal even-site field and zeros past it.  Keep the lattices alive
    while the batch is in use."""

    def __init__(self, lattices: Sequence[WilsonLattice]):
        self.lib = W.load()
        self.lattices = list(lattices)
        arr = (C.c_void_p * len(self.lattices))(*[lat.h for lat in self.lattices])
        h = C.c_void_p()
        W.check(self.lib.wl_batch_create(C.byref(h), arr, len(self.lattices)))
        self.h = h
        self.device = self.lattices[0].device

    def close(self):
        if getattr(self, "h", None):
            self.lib.wl_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def slot_bytes(self, prec="f64") -> int:
        n = C.c_size_t()
        W.check(self.lib.wl_batch_slot_bytes(self.h, _prec(prec), C.byref(n)))
        return n.value

    def new_field(self, prec="f64") -> torch.Tensor:
        return torch.zeros(self.slot_bytes(prec) * len(self.lattices), dtype=torch.uint8, device=self.device)

    def slot(self, buf: torch.Tensor, l: int, prec="f64") -> torch.Tensor:
        sb = self.slot_bytes(prec)
        return buf[l * sb:(l + 1) * sb]

    def pack(self, fields: Sequence[torch.Tensor], prec="f64") -> torch.Tensor:
        """Batch field from one canonical (V_h, 4, 3) even-site field per lattice
        (imported into the zeroed slots: the import writes the lattice's sites only)."""
        out = self.new_field(prec)
        for l, (lat, f) in enumerate(zip(self.lattices, fields)):
            f = f.to(device=self.device, dtype=torch.complex128).contiguous()
            assert f.shape == (lat.Vh, 4, 3)
            W.check(self.lib.wl_import_spinor(lat.h, _ptr(self.slot(out, l, prec)), _ptr(f), _prec(prec), 1))
        return out

    def unpack(self, buf: torch.Tensor, prec="f64") -> List[torch.Tensor]:
        """Canonical (V_h, 4, 3) field of every lattice from a batch field."""
        res = []
        for l, lat in enumerate(self.lattices):
            out = torch.empty((lat.Vh, 4, 3), dtype=torch.complex128, device=self.device)
            W.check(self.lib.wl_export_spinor(lat.h, _ptr(out), _ptr(self.slot(buf, l, prec)), _prec(prec), 1))
            res.append(out)
        return res

    def dslash(self, buf: torch.Tensor, out_parity: int, dagger: bool = False, prec="f64") -> torch.Tensor:
        out = self.new_field(prec)
        _need(buf, out.numel(), "input")
        W.check(self.lib.wl_batch_dslash(self.h, _ptr(out), _ptr(buf), out_parity, int(dagger), _prec(prec)))
        return out

    def apply_J(self, buf: torch.Tensor, kappa: Sequence[float], mu2: Optional[Sequence[float]] = None,
                prec="f64") -> torch.Tensor:
        n = len(self.lattices)
        out = self.new_field(prec)
        _need(buf, out.numel(), "input")
        k = (C.c_double * n)(*[float(v) for v in kappa])
        m = (C.c_double * n)(*[float(v) for v in mu2]) if mu2 is not None else None
        W.check(self.lib.wl_batch_apply_J(self.h, _ptr(out), _ptr(buf), k, m, _prec(prec)))
        return out

    def cg_solve(self, b: torch.Tensor, kappa: Sequence[float], mu2: Optional[Sequence[float]] = None,
                 params: Optional[CG] = None):
        """x (batch field) with J_l x_l = b_l for every lattice; (x, [CgResult], rc)."""
        params = params or CG()
        n = len(self.lattices)
        x = self.new_field("f64")
        _need(b, x.numel(), "rhs")
        k = (C.c_double * n)(*[float(v) for v in kappa])
        m = (C.c_double * n)(*[float(v) for v in mu2]) if mu2 is not None else None
        st = (W.CgStats * n)()
        prm = params.c()
        rc = W.check(self.lib.wl_batch_cg_solve(self.h, _ptr(x), _ptr(b), k, m, C.byref(prm), st))
        return x, [CgResult(s.iters, s.reliable_updates, bool(s.converged), s.true_rel_res) for s in st], rc


def integrator_schedule(nsteps: Sequence[int], integrator: str = "omelyan", omelyan_lambda: float = 0.0):
    """The library's overlaid integrator schedule (host only): list of
    ('S', scale, weight) and ('T', weight), weights in units of tau."""
    lib = W.load()
    ns = (C.c_int * len(nsteps))(*[int(n) for n in nsteps])
    n = C.c_int()
    cap = 4 * sum(int(v) for v in nsteps) + 8
    kinds, terms, w = (C.c_int * cap)(), (C.c_int * cap)(), (C.c_double * cap)()
    sch = W.WL_INT_OMELYAN if integrator == "omelyan" else W.WL_INT_LEAPFROG
    W.check(lib.wl_integrator_schedule(ns, len(nsteps), sch, omelyan_lambda, kinds, terms, w, cap, C.byref(n)))
    return [("T", w[k]) if kinds[k] == 1 else ("S", terms[k], w[k]) for k in range(n.value)]
