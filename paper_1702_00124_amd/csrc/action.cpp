// Pseudofermion action terms: heatbath, action value and force (Sec. 2: the
// two-flavour action phi^dag (M^dag M)^-1 phi and its force; mass
// preconditioning phi1^dag J^-1 phi1 + phi2^dag J K^-1 phi2; polynomial
// filtering phi1^dag P phi1 + phi2^dag [P K]^-1 phi2; Sec. 3.3: two filters;
// Sec. 4.1: PF-MP; Sec. 4.2: three filters).
//
// Each term's J = K-hat(kappa) + mu2 and W = M-hat(kappa) + i mu g5 (W^dag W = J
// by gamma5-hermiticity); RATIO's numerator W_n = M-hat(kappa_n) + i mu_n g5,
// J_n = W_n^dag W_n; P may be the quotient P_n / P_m of the two-filter actions.
//
//   term        S(phi)                        heatbath from chi
//   KINV_FULL   phi^dag K^-1 phi (full)       phi = M^dag chi
//   KINV        phi^dag J^-1 phi              phi = W^dag chi
//   RATIO       phi^dag W_n J^-1 W_n^dag phi  phi = W_n J_n^-1 W^dag chi
//   POLY        phi^dag P(J) phi              phi = Q^dag P(J)^-1 chi
//   POLYK_INV   phi^dag [P(J) J]^-1 phi       phi = Q^dag W^dag chi
//
// Forces are the Lie derivatives grad^a S along exp(i e T^a) U_mu(x), by the
// product rule down to the single link-derivative primitive
//   grad Re(A^dag D C)   (bilinear kernel, full-lattice fields),
// with Re(A^dag dM-hat B) = -kappa^2 grad Re(A'^dag D B'),
//   A' = (A, (D^dag)_oe A),  B' = (B, D_oe B),
// and Re(L^dag dJ R) = Re((M-hat R)^dag dM-hat L) + Re((M-hat L)^dag dM-hat R).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <functional>
#include <vector>

#include "wl_ops.h"

namespace wl {

namespace {

size_t hbytes(const wl_lattice* L) { return spinor_bytes(F64, L->Vh); }

PolyDesc pdesc(const wl_term& t) { return PolyDesc{t.poly.degree, t.poly.a, t.poly.b, t.poly.degree_div}; }

// RATIO numerator kappa
double kappa_n(const wl_term& t) { return t.kappa_num > 0.0 ? t.kappa_num : t.kappa; }

void check_term(const wl_term& t) {
  WL_REQUIRE(t.kind >= WL_TERM_KINV_FULL && t.kind <= WL_TERM_POLYK_INV, WL_EINVAL, "unknown term kind");
  WL_REQUIRE(t.kappa > 0.0 && t.kappa_num >= 0.0, WL_EINVAL, "kappa must be positive");
  WL_REQUIRE(t.mu2 >= 0.0 && t.mu2_num >= 0.0, WL_EINVAL, "mu2 must be non-negative");
  WL_REQUIRE(t.kind != WL_TERM_KINV_FULL || t.mu2 == 0.0, WL_EUNSUPPORTED, "full-lattice term takes mu2 = 0");
  if (t.kind == WL_TERM_POLY || t.kind == WL_TERM_POLYK_INV) check_poly(pdesc(t));
}

// out = W in (dagger: W^dag in), W = M-hat + i mu g5
void op_w(wl_lattice* L, void* out, const void* in, double kappa, double mu2, int dagger) {
  void* t = ws_get(L, "act_wtmp", hbytes(L));
  op_mhat(L, F64, t, in, kappa, dagger, 1);
  const double one[2] = {1.0, 0.0};
  const double imu[2] = {0.0, (dagger ? -1.0 : 1.0) * std::sqrt(mu2)};
  launch_caxpby(L, out, one, t, imu, in, 1, 1);
}

using ApplyF64 = std::function<void(void* out, const void* in)>;

// Cholesky solve of the m x m Hermitian system G c = r (G row-major, c holds r
// on entry); false if G is not numerically positive definite.
bool hpd_solve(int m, std::vector<std::complex<double>>& G, std::vector<std::complex<double>>& c) {
  for (int j = 0; j < m; ++j) {
    double d = G[j * m + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(G[j * m + k]);
    if (!(d > 1e-14 * std::abs(G[j * m + j].real()))) return false;
    d = std::sqrt(d);
    G[j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      std::complex<double> s = G[i * m + j];
      for (int k = 0; k < j; ++k) s -= G[i * m + k] * std::conj(G[j * m + k]);
      G[i * m + j] = s / d;
    }
  }
  for (int i = 0; i < m; ++i) {  // L y = r
    for (int k = 0; k < i; ++k) c[i] -= G[i * m + k] * c[k];
    c[i] /= G[i * m + i].real();
  }
  for (int i = m - 1; i >= 0; --i) {  // L^dag c = y
    for (int k = i + 1; k < m; ++k) c[i] -= std::conj(G[k * m + i]) * c[k];
    c[i] /= G[i * m + i].real();
  }
  return true;
}

// Chronological initial guess (minimal-residual extrapolation): x0 is the
// vector of the span S of the term's stored solutions that minimises the
// A-norm of the error, i.e. x0 = V (V^dag A V)^-1 V^dag b with V an
// orthonormal basis of S (modified Gram-Schmidt, newest solution first;
// vectors already in the span are dropped).  No stored solution, or a basis
// whose Gram matrix is not positive definite, leaves x0 = 0.
void chrono_in(wl_lattice* L, ChronoSlot* ch, void* x, const void* b, const ApplyF64& A, wl_cg_params& cg) {
  cg.use_x0 = 0;
  if (!ch || ch->count == 0) return;
  const size_t fb = ch->fb;
  const int nh = ch->nh;
  auto fld = [&](char* base, int i) { return base + size_t(i) * fb; };
  auto axpy = [&](void* out, std::complex<double> a, const void* y, std::complex<double> bc, const void* z) {
    double ca[2 * 2], cb[2 * 2];
    for (int q = 0; q < nh; ++q) {
      ca[2 * q] = a.real();
      ca[2 * q + 1] = a.imag();
      cb[2 * q] = bc.real();
      cb[2 * q + 1] = bc.imag();
    }
    launch_caxpby(L, out, ca, y, z ? cb : nullptr, z, 0, nh);
  };
  int m = 0;
  for (int k = 0; k < ch->count; ++k) {
    const int j = (ch->next - 1 - k + 2 * ch->depth) % ch->depth;
    char* v = fld(ch->basis, m);
    copy_dev(L, v, fld(ch->ring, j), fb);
    double n0 = 0.0, n1 = 0.0;
    norm2_host(L, v, 1, &n0, nh);
    if (!(n0 > 0.0)) continue;
    for (int i = 0; i < m; ++i) {
      double c[2];
      cdot_host(L, fld(ch->basis, i), v, 1, c, nh);
      axpy(v, 1.0, v, std::complex<double>(-c[0], -c[1]), fld(ch->basis, i));
    }
    norm2_host(L, v, 1, &n1, nh);
    if (!(n1 > 1e-20 * n0)) continue;
    axpy(v, 1.0 / std::sqrt(n1), v, 0.0, nullptr);
    ++m;
  }
  if (m == 0) return;
  std::vector<std::complex<double>> G(m * m), c(m);
  for (int j = 0; j < m; ++j) A(fld(ch->abasis, j), fld(ch->basis, j));
  for (int i = 0; i < m; ++i) {
    double d[2];
    for (int j = i; j < m; ++j) {
      cdot_host(L, fld(ch->basis, i), fld(ch->abasis, j), 1, d, nh);
      G[i * m + j] = std::complex<double>(d[0], d[1]);
      G[j * m + i] = std::conj(G[i * m + j]);
    }
    G[i * m + i] = G[i * m + i].real();
    cdot_host(L, fld(ch->basis, i), b, 1, d, nh);
    c[i] = std::complex<double>(d[0], d[1]);
  }
  if (!hpd_solve(m, G, c)) return;
  axpy(x, c[0], fld(ch->basis, 0), 0.0, nullptr);
  for (int i = 1; i < m; ++i) axpy(x, 1.0, x, c[i], fld(ch->basis, i));
  cg.use_x0 = 1;
}

// keep the new solution, dropping the oldest once depth are stored
void chrono_out(wl_lattice* L, ChronoSlot* ch, const void* x) {
  if (!ch) return;
  copy_dev(L, ch->ring + size_t(ch->next) * ch->fb, x, ch->fb);
  ch->next = (ch->next + 1) % ch->depth;
  ch->count = std::min(ch->count + 1, ch->depth);
}

int solve_j(wl_lattice* L, void* x, const void* b, double kappa, double mu2, const wl_cg_params& cg_in,
            long long* iters, ChronoSlot* ch = nullptr) {
  wl_cg_stats st{};
  wl_cg_params cg = cg_in;
  chrono_in(L, ch, x, b, [&](void* out, const void* in) { op_j(L, F64, out, in, kappa, &mu2, 1); }, cg);
  const int rc = cg_run(L, x, b, kappa, &mu2, 1, WL_OP_J, cg, &st);
  chrono_out(L, ch, x);
  if (iters) *iters += st.iters;
  WL_REQUIRE(rc == WL_OK, rc, "inner CG did not converge");
  return rc;
}

void solve_poly(wl_lattice* L, void* x, const void* b, const wl_term& t, int mode, long long* iters,
                ChronoSlot* ch = nullptr) {
  wl_cg_stats st{};
  const PolyDesc pd = pdesc(t);
  auto apply = [&](Prec pr, void* out, const void* in) { poly_apply(L, mode, out, in, t.kappa, t.mu2, pd, pr); };
  wl_cg_params cg = t.cg;
  // the guess needs the operator on each stored solution: in FP32 when the
  // solve iterates in lower precision (the guess is only a starting point;
  // convergence is still judged on the FP64 residual)
  const Prec gp = Prec(cg.inner) == F64 ? F64 : F32;
  auto apply_guess = [&](void* out, const void* in) {
    if (gp == F64) {
      apply(F64, out, in);
      return;
    }
    void* a = ws_get(L, "pg_in", spinor_bytes(gp, L->Vh));
    void* o = ws_get(L, "pg_out", spinor_bytes(gp, L->Vh));
    launch_convert(L, gp, a, F64, in, 1);
    apply(gp, o, a);
    launch_convert(L, F64, out, gp, o, 1);
  };
  chrono_in(L, ch, x, b, apply_guess, cg);
  const int rc = cg_run_generic(L, x, b, apply, cg, &st, poly_j_count(mode, pd));
  chrono_out(L, ch, x);
  if (iters) *iters += st.iters;
  WL_REQUIRE(rc == WL_OK, rc, "polynomial CG did not converge");
}

double re_dot(wl_lattice* L, const void* x, const void* y, int nhalves = 1) {
  double d[2];
  cdot_host(L, x, y, 1, d, nhalves);
  return d[0];
}

// F += coeff * grad Re(A^dag dM-hat B)
void grad_re_dmhat(wl_lattice* L, double* F, const void* A, const void* B, double kappa, double coeff) {
  void* Ao = ws_get(L, "gm_Ao", hbytes(L));
  void* Bo = ws_get(L, "gm_Bo", hbytes(L));
  HopEpi e;
  launch_hop(L, F64, Ao, A, 1, 1, 1, e);  // (D^dag)_oe A
  launch_hop(L, F64, Bo, B, 1, 0, 1, e);  // D_oe B
  launch_bilinear(L, F, A, Ao, B, Bo, -kappa * kappa * coeff);
}

// The pieces of M-hat v that Re(L^dag dJ R) and J v share: D_oe v, M-hat v
// = v - kappa^2 D_eo D_oe v and (D^dag)_oe M-hat v.
struct HatParts {
  void* odd;
  void* m;
  void* ao;
};

HatParts hat_ws(wl_lattice* L, const std::string& name) {
  const size_t hb = hbytes(L);
  return HatParts{ws_get(L, name + "_o", hb), ws_get(L, name + "_m", hb), ws_get(L, name + "_a", hb)};
}

// three hops
void hat_parts(wl_lattice* L, const void* v, double kappa, const HatParts& p) {
  const HopEpi plain;
  HopEpi mh;
  mh.x = v;
  mh.a = -kappa * kappa;
  launch_hop(L, F64, p.odd, v, 1, 0, 1, plain);  // D_oe v
  launch_hop(L, F64, p.m, p.odd, 0, 0, 1, mh);   // M-hat v
  launch_hop(L, F64, p.ao, p.m, 1, 1, 1, plain);  // (D^dag)_oe M-hat v
}

// jv = J v = M-hat^dag (M-hat v) + mu2 v from v's parts: one hop, counted as
// one multiplication by J in the cost count
void j_from_parts(wl_lattice* L, void* jv, const void* v, const HatParts& p, double kappa, double mu2) {
  HopEpi e;
  e.x = p.m;
  e.a = -kappa * kappa;
  e.y = v;
  e.by[0] = mu2;
  launch_hop(L, F64, jv, p.ao, 0, 1, 1, e);
  L->n_kmat += 1;
}

// F += coeff * grad Re(Lv^dag dJ Rv)
//   = grad Re((M-hat Rv)^dag dM-hat Lv) + grad Re((M-hat Lv)^dag dM-hat Rv),
// two bilinears on the two fields' parts
void grad_re_dj_parts(wl_lattice* L, double* F, const void* Lv, const HatParts& lp, const void* Rv,
                      const HatParts& rp, double kappa, double coeff) {
  const double c = -kappa * kappa * coeff;
  launch_bilinear(L, F, rp.m, rp.ao, Lv, lp.odd, c);
  launch_bilinear(L, F, lp.m, lp.ao, Rv, rp.odd, c);
}

// the same from the fields alone: six hops, three when Lv and Rv are one
// field (whose two terms agree)
void grad_re_dj(wl_lattice* L, double* F, const void* Lv, const void* Rv, double kappa, double coeff) {
  const HatParts lp = hat_ws(L, "gj_l");
  hat_parts(L, Lv, kappa, lp);
  if (Lv == Rv) {
    launch_bilinear(L, F, lp.m, lp.ao, Lv, lp.odd, -2.0 * kappa * kappa * coeff);
    return;
  }
  const HatParts rp = hat_ws(L, "gj_r");
  hat_parts(L, Rv, kappa, rp);
  grad_re_dj_parts(L, F, Lv, lp, Rv, rp, kappa, coeff);
}

// the chain keeps every R_k's parts from building R_{k+1} while they fit in
// 16 GiB (or the byte count in the environment variable WL_CHAIN_KEEP_BYTES);
// past it they are recomputed per term (three more hops per root factor)
size_t chain_keep_bytes() {
  const char* v = std::getenv("WL_CHAIN_KEEP_BYTES");
  if (v && *v) {
    char* end = nullptr;
    const unsigned long long n = std::strtoull(v, &end, 10);
    if (end && *end == '\0') return size_t(n);
  }
  return size_t(16) << 30;
}

// F += coeff * sum_k grad Re(L_k^dag dJ R_k) over the factors (J - z_k) of Q:
// R_k = prod_{j<k} (J - z_j) right,  L_k = prod_{j>k} (J - conj z_j) left_top
void chain_grad(wl_lattice* L, double* F, const wl_term& t, const void* right, const void* left_top, double coeff) {
  const PolyDesc pd = pdesc(t);
  std::vector<double> zr, zi;
  poly_q_roots(pd, zr, zi);
  const int m = int(zr.size());
  const size_t fb = hbytes(L);
  const bool keep = size_t(3) * size_t(m) * fb <= chain_keep_bytes();
  std::vector<void*> R(m);
  std::vector<HatParts> P(keep ? m : 1);
  for (int j = 0; j < m; ++j) R[j] = ws_get(L, "ch_R" + std::to_string(j), fb);
  for (size_t j = 0; j < P.size(); ++j) P[j] = hat_ws(L, "ch_P" + std::to_string(j));
  auto parts = [&](int j) -> const HatParts& { return P[keep ? j : 0]; };
  const HatParts lp = hat_ws(L, "ch_PL");
  void* w = ws_get(L, "ch_w", fb);
  void* Lv = ws_get(L, "ch_L", fb);
  const double one[2] = {1.0, 0.0};
  copy_dev(L, R[0], right, fb);
  for (int j = 0; j + 1 < m; ++j) {
    hat_parts(L, R[j], t.kappa, parts(j));
    j_from_parts(L, w, R[j], parts(j), t.kappa, t.mu2);
    const double mz[2] = {-zr[j], -zi[j]};
    launch_caxpby(L, R[j + 1], one, w, mz, R[j], 0, 1);
  }
  copy_dev(L, Lv, left_top, fb);
  for (int k = m - 1; k >= 0; --k) {
    if (!keep || k == m - 1) hat_parts(L, R[k], t.kappa, parts(k));
    hat_parts(L, Lv, t.kappa, lp);
    grad_re_dj_parts(L, F, Lv, lp, R[k], parts(k), t.kappa, coeff);
    if (k > 0) {
      j_from_parts(L, w, Lv, lp, t.kappa, t.mu2);  // w = J Lv
      const double mzc[2] = {-zr[k], zi[k]};
      launch_caxpby(L, Lv, one, w, mzc, Lv, 0, 1);
    }
  }
}

}  // namespace

void term_heatbath(wl_lattice* L, const wl_term& t, void* phi, const void* chi) {
  check_term(t);
  const size_t fb = hbytes(L);
  switch (t.kind) {
    case WL_TERM_KINV_FULL: op_m_full(L, F64, phi, chi, t.kappa, 1); break;
    case WL_TERM_KINV: op_w(L, phi, chi, t.kappa, t.mu2, 1); break;
    case WL_TERM_RATIO: {
      void* a = ws_get(L, "hb_a", fb);
      void* x = ws_get(L, "hb_x", fb);
      op_w(L, a, chi, t.kappa, t.mu2, 1);
      solve_j(L, x, a, kappa_n(t), t.mu2_num, t.cg, nullptr);
      op_w(L, phi, x, kappa_n(t), t.mu2_num, 0);
      break;
    }
    case WL_TERM_POLY: {
      void* x = ws_get(L, "hb_x", fb);
      solve_poly(L, x, chi, t, WL_POLY_P, nullptr);
      poly_apply(L, WL_POLY_QDAG, phi, x, t.kappa, t.mu2, pdesc(t));
      break;
    }
    case WL_TERM_POLYK_INV: {
      void* a = ws_get(L, "hb_a", fb);
      op_w(L, a, chi, t.kappa, t.mu2, 1);
      poly_apply(L, WL_POLY_QDAG, phi, a, t.kappa, t.mu2, pdesc(t));
      break;
    }
  }
}

double term_action(wl_lattice* L, const wl_term& t, const void* phi, long long* iters) {
  check_term(t);
  const size_t fb = hbytes(L);
  switch (t.kind) {
    case WL_TERM_KINV_FULL: {
      void* x = ws_get(L, "ac_xf", 2 * fb);
      wl_cg_stats st{};
      const int rc = cg_run(L, x, phi, t.kappa, nullptr, 1, WL_OP_K, t.cg, &st);
      if (iters) *iters += st.iters;
      WL_REQUIRE(rc == WL_OK, rc, "inner CG did not converge");
      return re_dot(L, phi, x, 2);
    }
    case WL_TERM_KINV: {
      void* x = ws_get(L, "ac_x", fb);
      solve_j(L, x, phi, t.kappa, t.mu2, t.cg, iters);
      return re_dot(L, phi, x);
    }
    case WL_TERM_RATIO: {
      void* v = ws_get(L, "ac_v", fb);
      void* x = ws_get(L, "ac_x", fb);
      op_w(L, v, phi, kappa_n(t), t.mu2_num, 1);
      solve_j(L, x, v, t.kappa, t.mu2, t.cg, iters);
      return re_dot(L, v, x);
    }
    case WL_TERM_POLY: {
      void* x = ws_get(L, "ac_x", fb);
      poly_apply(L, WL_POLY_P, x, phi, t.kappa, t.mu2, pdesc(t));
      return re_dot(L, phi, x);
    }
    case WL_TERM_POLYK_INV: {
      void* x = ws_get(L, "ac_x", fb);
      solve_poly(L, x, phi, t, WL_POLY_PJ, iters);
      return re_dot(L, phi, x);
    }
  }
  return 0.0;
}

void term_force(wl_lattice* L, const wl_term& t, double* F, const void* phi, double coeff, long long* iters,
                ChronoSlot* ch) {
  check_term(t);
  const size_t fb = hbytes(L);
  switch (t.kind) {
    case WL_TERM_KINV_FULL: {
      // dS = -X^dag dK X = 2 kappa grad Re(Y^dag D X), X = K^-1 phi, Y = M X
      char* x = static_cast<char*>(ws_get(L, "fo_xf", 2 * fb));
      char* y = static_cast<char*>(ws_get(L, "fo_yf", 2 * fb));
      wl_cg_stats st{};
      wl_cg_params cg = t.cg;
      chrono_in(L, ch, x, phi, [&](void* out, const void* in) { op_k_full(L, F64, out, in, t.kappa, DotOut()); },
                cg);
      const int rc = cg_run(L, x, phi, t.kappa, nullptr, 1, WL_OP_K, cg, &st);
      chrono_out(L, ch, x);
      if (iters) *iters += st.iters;
      WL_REQUIRE(rc == WL_OK, rc, "inner CG did not converge");
      op_m_full(L, F64, y, x, t.kappa, 0);
      launch_bilinear(L, F, y, y + fb, x, x + fb, 2.0 * t.kappa * coeff);
      break;
    }
    case WL_TERM_KINV: {
      // dS = -2 Re(Y^dag dM-hat X), X = J^-1 phi, Y = M-hat X
      void* x = ws_get(L, "fo_x", fb);
      void* y = ws_get(L, "fo_y", fb);
      solve_j(L, x, phi, t.kappa, t.mu2, t.cg, iters, ch);
      op_mhat(L, F64, y, x, t.kappa, 0, 1);
      grad_re_dmhat(L, F, y, x, t.kappa, -2.0 * coeff);
      break;
    }
    case WL_TERM_RATIO: {
      // S = v^dag X, v = W_n^dag phi, X = J^-1 v:
      // dS = 2 Re(phi^dag dM-hat(kappa_n) X) - 2 Re(Y^dag dM-hat(kappa) X), Y = M-hat X
      // (the i mu g5 parts of W_n and W drop out of both real parts); with
      // kappa_n = kappa the two bilinears merge into one
      void* v = ws_get(L, "fo_v", fb);
      void* x = ws_get(L, "fo_x", fb);
      void* y = ws_get(L, "fo_y", fb);
      op_w(L, v, phi, kappa_n(t), t.mu2_num, 1);
      solve_j(L, x, v, t.kappa, t.mu2, t.cg, iters, ch);
      op_mhat(L, F64, y, x, t.kappa, 0, 1);
      if (kappa_n(t) == t.kappa) {
        const double one[2] = {1.0, 0.0}, mone[2] = {-1.0, 0.0};
        launch_caxpby(L, y, one, phi, mone, y, 0, 1);
        grad_re_dmhat(L, F, y, x, t.kappa, 2.0 * coeff);
      } else {
        grad_re_dmhat(L, F, phi, x, kappa_n(t), 2.0 * coeff);
        grad_re_dmhat(L, F, y, x, t.kappa, -2.0 * coeff);
      }
      break;
    }
    case WL_TERM_POLY: {
      // S = |Q phi|^2: dS = 2 sqrt(c) sum_k Re(L_k^dag dJ R_k), R from phi, L from Q phi
      void* psi = ws_get(L, "fo_psi", fb);
      poly_apply(L, WL_POLY_Q, psi, phi, t.kappa, t.mu2, pdesc(t));
      chain_grad(L, F, t, phi, psi, 2.0 * std::sqrt(poly_lead(pdesc(t))) * coeff);
      break;
    }
    case WL_TERM_POLYK_INV: {
      // S = phi^dag (Q^dag J Q)^-1 phi, X = S's solution:
      // dS = -[2 sqrt(c) sum_k Re(L_k^dag dJ R_k) + Re((QX)^dag dJ (QX))], R from X, L from J Q X
      void* x = ws_get(L, "fo_x", fb);
      void* qx = ws_get(L, "fo_qx", fb);
      void* jqx = ws_get(L, "fo_jqx", fb);
      solve_poly(L, x, phi, t, WL_POLY_PJ, iters, ch);
      poly_apply(L, WL_POLY_Q, qx, x, t.kappa, t.mu2, pdesc(t));
      op_j(L, F64, jqx, qx, t.kappa, &t.mu2, 1);
      chain_grad(L, F, t, x, jqx, -2.0 * std::sqrt(poly_lead(pdesc(t))) * coeff);
      grad_re_dj(L, F, qx, qx, t.kappa, -coeff);
      break;
    }
  }
}

}  // namespace wl
