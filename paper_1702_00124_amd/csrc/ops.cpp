// Fermion operators from hop launches with fused epilogues (Sec. 2 and 3.1):
//   M-hat psi  = psi - kappa^2 D_eo (D_oe psi)                      2 hops
//   K-hat psi  = g5 M-hat g5 M-hat psi  (gamma5-hermiticity)         4 hops
//   J psi      = K-hat psi + mu2 psi, with <psi, J psi> fused into the last hop
//   full M     = 1 - kappa D on (even, odd) halves; K = M^dag M
#include "wl_ops.h"

namespace wl {

void copy_dev(wl_lattice* L, void* dst, const void* src, size_t bytes) {
  if (dst == src || bytes == 0) return;
  WL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, L->stream));
}

void zero_dev(wl_lattice* L, void* dst, size_t bytes) { WL_HIP(hipMemsetAsync(dst, 0, bytes, L->stream)); }

size_t op_scratch_bytes(const wl_lattice* L, int op, Prec prec, int nrhs) {
  const size_t fb = spinor_bytes(prec, L->Vh) * size_t(nrhs);
  switch (op) {
    case WL_OP_J: return 2 * fb;                              // odd and even intermediates
    case WL_OP_MHAT: case WL_OP_MHAT_DAG: return fb;          // odd intermediate
    case WL_OP_K: return 2 * spinor_bytes(prec, L->Vh);       // full-lattice M in
    default: return 0;
  }
}

void op_mhat(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, int dagger, int nrhs,
             const OpScratch* scr) {
  void* odd = scr ? scr->odd : ws_get(L, "op_odd", spinor_bytes(prec, L->Vh) * nrhs);
  HopEpi e1;
  launch_hop(L, prec, odd, in, 1, dagger, nrhs, e1);
  HopEpi e2;
  e2.x = in;
  e2.a = -kappa * kappa;
  launch_hop(L, prec, out, odd, 0, dagger, nrhs, e2);
}

void op_j(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, const double* mu2, int nrhs,
          const DotOut& dot, const ChebStep* cheb, const double* lin, const OpScratch* scr) {
  WL_REQUIRE(!lin || (!cheb && !dot.partials), WL_EINVAL, "op_j: lin takes no dot or step");
  const size_t fb = spinor_bytes(prec, L->Vh) * nrhs;
  void* odd = scr ? scr->odd : ws_get(L, "op_odd", fb);
  void* v = scr ? scr->even : ws_get(L, "op_even", fb);
  HopEpi e;
  launch_hop(L, prec, odd, in, 1, 0, nrhs, e);  // D_oe in
  e.x = in;
  e.a = -kappa * kappa;
  e.g5 = 1;
  launch_hop(L, prec, v, odd, 0, 0, nrhs, e);   // v = g5 M-hat in
  HopEpi e3;
  launch_hop(L, prec, odd, v, 1, 0, nrhs, e3);  // D_oe v
  HopEpi e4;
  e4.x = v;
  e4.a = -kappa * kappa;
  e4.g5 = 1;
  bool shift = false;
  for (int r = 0; r < nrhs; ++r) {
    e4.by[r] = mu2 ? mu2[r] : 0.0;
    shift = shift || e4.by[r] != 0.0;
  }
  if (shift) e4.y = in;
  if (lin) {  // lin0 (g5 M-hat v + mu2 in) + lin1 in
    e4.cx = lin[0];
    e4.a = -kappa * kappa * lin[0];
    for (int r = 0; r < nrhs; ++r) e4.by[r] = lin[0] * e4.by[r] + lin[1];
    e4.y = in;
  }
  if (dot.partials) {
    e4.dot = 1;
    e4.dotv = in;
    e4.partials = dot.partials;
    e4.part_stride = dot.stride;
  }
  if (cheb) {  // the Chebyshev step consumes J in instead of storing it
    e4.cheb_t = in;
    e4.cheb_tprev = cheb->tprev;
    e4.cheb_e = cheb->e;
    e4.cheb_eprev = cheb->eprev;
    e4.cheb_ct = cheb->ct;
    e4.cheb_cw = cheb->cw;
    e4.cheb_ce = cheb->ce;
    out = cheb->tprev;  // never written in this mode
  }
  launch_hop(L, prec, out, odd, 0, 0, nrhs, e4);  // g5 M-hat v + mu2 in
  L->n_kmat += nrhs;
}

void op_m_full(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, int dagger) {
  const size_t hb = spinor_bytes(prec, L->Vh);
  const char* ie = static_cast<const char*>(in);
  const char* io = ie + hb;
  char* oe = static_cast<char*>(out);
  char* oo = oe + hb;
  HopEpi e;
  e.a = -kappa;
  e.x = ie;
  launch_hop(L, prec, oe, io, 0, dagger, 1, e);
  e.x = io;
  launch_hop(L, prec, oo, ie, 1, dagger, 1, e);
}

void op_k_full(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, const DotOut& dot,
               const OpScratch* scr) {
  const size_t hb = spinor_bytes(prec, L->Vh);
  char* t = static_cast<char*>(scr ? scr->odd : ws_get(L, "op_full", 2 * hb));
  op_m_full(L, prec, t, in, kappa, 0);
  const char* ie = static_cast<const char*>(in);
  char* oe = static_cast<char*>(out);
  HopEpi e;
  e.a = -kappa;
  e.x = t;
  if (dot.partials) {
    e.dot = 1;
    e.dotv = ie;
    e.partials = dot.partials;
    e.part_stride = dot.stride;
    e.part_off = 0;
  }
  launch_hop(L, prec, oe, t + hb, 0, 1, 1, e);
  e.x = t + hb;
  e.dotv = ie + hb;
  e.part_off = hop_tiles(L, prec);
  launch_hop(L, prec, oe + hb, t, 1, 1, 1, e);
  L->n_kmat += 1;
}

void op_apply(wl_lattice* L, int op, Prec prec, void* out, const void* in, double kappa, const double* mu2,
              int nrhs, const DotOut& dot, const OpScratch* scr) {
  switch (op) {
    case WL_OP_J: op_j(L, prec, out, in, kappa, mu2, nrhs, dot, nullptr, nullptr, scr); break;
    case WL_OP_K:
      WL_REQUIRE(nrhs == 1, WL_EUNSUPPORTED, "full-lattice K takes one rhs");
      op_k_full(L, prec, out, in, kappa, dot, scr);
      break;
    case WL_OP_MHAT: op_mhat(L, prec, out, in, kappa, 0, nrhs, scr); break;
    case WL_OP_MHAT_DAG: op_mhat(L, prec, out, in, kappa, 1, nrhs, scr); break;
    case WL_OP_M:
      WL_REQUIRE(nrhs == 1, WL_EUNSUPPORTED, "full-lattice M takes one rhs");
      op_m_full(L, prec, out, in, kappa, 0);
      break;
    case WL_OP_MDAG:
      WL_REQUIRE(nrhs == 1, WL_EUNSUPPORTED, "full-lattice M takes one rhs");
      op_m_full(L, prec, out, in, kappa, 1);
      break;
    default: throw Error(WL_EINVAL, "unknown operator");
  }
}

void norm2_host(wl_lattice* L, const void* x, int nrhs, double* out, int nhalves) {
  const int nb = blas_blocks(L);
  ensure_partials(L, size_t(nb) * nhalves * nrhs);
  const size_t hb = spinor_bytes(F64, L->Vh);
  // halves of a full field are one logical rhs; partials rows = rhs, columns = blocks of every half
  for (int q = 0; q < nhalves; ++q)
    for (int r = 0; r < nrhs; ++r)
      launch_dot_partials(L, static_cast<const char*>(x) + (size_t(q) * nrhs + r) * hb, nullptr, 1,
                          L->partials + size_t(r) * nb * nhalves + size_t(q) * nb, 0, 0);
  launch_finish_sum(L, L->partials, nb * nhalves, nb * nhalves, nrhs, L->dscal);
  WL_HIP(hipMemcpyAsync(L->hscal, L->dscal, sizeof(double) * nrhs, hipMemcpyDeviceToHost, L->stream));
  WL_HIP(hipStreamSynchronize(L->stream));
  for (int r = 0; r < nrhs; ++r) out[r] = L->hscal[r];
}

void cdot_host(wl_lattice* L, const void* x, const void* y, int nrhs, double* out, int nhalves) {
  const int nb = blas_blocks(L);
  ensure_partials(L, size_t(nb) * nhalves * 2 * nrhs);
  const size_t hb = spinor_bytes(F64, L->Vh);
  const int row = nb * nhalves;
  for (int q = 0; q < nhalves; ++q)
    for (int r = 0; r < nrhs; ++r) {
      const size_t off = (size_t(q) * nrhs + r) * hb;
      // rows 2r (re) and 2r+1 (im); this half's blocks start at column q * nb
      launch_dot_partials(L, static_cast<const char*>(x) + off, static_cast<const char*>(y) + off, 1,
                          L->partials + size_t(2 * r) * row + size_t(q) * nb, row, 1);
    }
  launch_finish_sum(L, L->partials, row, row, 2 * nrhs, L->dscal);
  WL_HIP(hipMemcpyAsync(L->hscal, L->dscal, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, L->stream));
  WL_HIP(hipStreamSynchronize(L->stream));
  for (int r = 0; r < 2 * nrhs; ++r) out[r] = L->hscal[r];
}

}  // namespace wl
