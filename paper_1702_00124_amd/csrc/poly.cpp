// Chebyshev filter polynomial applied to J = K-hat + mu2 (Sec. 2, polynomial
// filtering: P(K) a low-order polynomial approximating K^-1, Chebyshev, order
// the only parameter).  Reading of the family (see include/wilson_hmc.h):
//
//   1 - x P_n(x) = T_{n+1}(y(x)) / T_{n+1}(y0),  y(x) = (b + a - 2x)/(b - a),  y0 = y(0).
//
// P_n(J) psi runs the real three-term recurrence
//   t_{m+1} = 2 y(J) t_m - t_{m-1}        (t_m = T_m(y(J)) psi)
//   e_{m+1} = 2 y0 e_m + 2 t_m - e_{m-1}  (e_m = (T_m(y0) - T_m(y(J)))/(y0 - y(J)) psi)
// so that P_n(J) psi = (2/(b-a)) e_{n+1} / T_{n+1}(y0): n J applications, t_1
// and each later step of the recurrence fused into the last hop of its J
// application, the start vectors and the scaled last step one kernel each.  Q(J), with P = Q^dag Q, is the product
// over the n/2 roots z_k = ((b+a)/2)(1 - cos t_k) - i sqrt(ab) sin t_k,
// t_k = 2 pi k/(n+1), times sqrt(c), c the leading coefficient of P_n.
//
// The quotient P_n / P_m of the two-filter actions (Sec. 3.3, 4.2; (m+1) | (n+1)):
// the roots of P_m are those of P_n at the indices k divisible by
// r = (n+1)/(m+1), so the quotient's Q runs over k = 1..n/2 with k % r != 0,
// its leading coefficient is c_n / c_m, and P = Q^dag Q is applied as such.
#include <cmath>

#include "wl_ops.h"

namespace wl {

static double cheb_T_above_one(int m, double y) { return std::cosh(m * std::acosh(y)); }

// leading coefficient of P_n (Chebyshev form above)
static double lead_n(int n, double a, double b) {
  const double y0 = (b + a) / (b - a);
  const double sgn = (n % 2) ? -1.0 : 1.0;
  return sgn * std::pow(2.0, n) * std::pow(2.0 / (b - a), n + 1) / cheb_T_above_one(n + 1, y0);
}

double poly_lead(const PolyDesc& pd) {
  return lead_n(pd.n, pd.a, pd.b) / (pd.ndiv > 0 ? lead_n(pd.ndiv, pd.a, pd.b) : 1.0);
}

void poly_q_roots(const PolyDesc& pd, std::vector<double>& re, std::vector<double>& im) {
  re.clear();
  im.clear();
  const int r = pd.ndiv > 0 ? (pd.n + 1) / (pd.ndiv + 1) : 0;
  for (int k = 1; k <= pd.n / 2; ++k) {
    if (r > 0 && k % r == 0) continue;  // a root of the divisor
    const double th = 2.0 * M_PI * k / (pd.n + 1);
    re.push_back(0.5 * (pd.b + pd.a) * (1.0 - std::cos(th)));
    im.push_back(-std::sqrt(pd.a * pd.b) * std::sin(th));
  }
}

long long poly_j_count(int mode, const PolyDesc& pd) {
  std::vector<double> zr, zi;
  poly_q_roots(pd, zr, zi);
  const long long q = (long long)zr.size();
  const long long p = pd.ndiv > 0 ? 2 * q : pd.n;
  switch (mode) {
    case WL_POLY_P: return p;
    case WL_POLY_PJ: return p + 1;
    default: return q;
  }
}

void check_poly(const PolyDesc& pd) {
  WL_REQUIRE(pd.n >= 1 && pd.n <= 512, WL_EINVAL, "polynomial degree out of range");
  WL_REQUIRE(pd.a > 0.0 && pd.b > pd.a, WL_EINVAL, "polynomial interval needs 0 < a < b");
  WL_REQUIRE(pd.ndiv >= 0, WL_EINVAL, "negative divisor order");
  if (pd.ndiv > 0) {
    WL_REQUIRE(pd.ndiv < pd.n && (pd.n + 1) % (pd.ndiv + 1) == 0, WL_EINVAL,
               "divisor order m needs (m + 1) | (degree + 1)");
    WL_REQUIRE(pd.n % 2 == 0 && pd.ndiv % 2 == 0, WL_EINVAL, "quotient filters need even orders");
  }
}

// out = P_n(J) in by the recurrence, nrhs fields, storage precision pr
static void poly_P(wl_lattice* L, void* out, const void* in, double kappa, double mu2, const PolyDesc& pd, Prec pr,
                   int nrhs) {
  const size_t fb = spinor_bytes(pr, L->Vh) * nrhs;
  std::vector<double> shifts(nrhs, mu2);
  void* tA = ws_get(L, "pl_tA", fb);
  void* tB = ws_get(L, "pl_tB", fb);
  void* eA = ws_get(L, "pl_eA", fb);
  void* eB = ws_get(L, "pl_eB", fb);
  const double a = pd.a, b = pd.b;
  const double y0 = (b + a) / (b - a);
  const double ct = 2.0 * (b + a) / (b - a), cw = -4.0 / (b - a);
  // t0 = in, e0 = 0, e1 = in; t1 = y(J) in = c1 in + c2 J in from J's epilogue
  launch_cheb_init(L, in, tA, eA, eB, pr, nrhs);
  const double lin[2] = {-2.0 / (b - a), (b + a) / (b - a)};
  op_j(L, pr, tB, in, kappa, shifts.data(), nrhs, DotOut(), nullptr, lin);
  for (int m = 1; m < pd.n; ++m) {
    // J t_m and the step in one pass: tA <- t_{m+1}, eA <- e_{m+1}
    const ChebStep cs{tA, eB, eA, ct, cw, 2.0 * y0};
    op_j(L, pr, nullptr, tB, kappa, shifts.data(), nrhs, DotOut(), &cs);
    std::swap(tA, tB);
    std::swap(eA, eB);
  }
  // out = s e_{n+1}, e_{n+1} = 2 y0 e_n + 2 t_n - e_{n-1}
  launch_cheb_last(L, tB, eB, eA, out, 2.0 * y0, (2.0 / (b - a)) / cheb_T_above_one(pd.n + 1, y0), pr, nrhs);
}

// out = sqrt(c) prod_k (J - z_k) in   (conjugate roots for Q^dag)
static void poly_Q(wl_lattice* L, void* out, const void* in, double kappa, double mu2, const PolyDesc& pd,
                   int dagger, Prec pr, int nrhs) {
  WL_REQUIRE(pd.n % 2 == 0, WL_EINVAL, "P = Q^dag Q needs an even degree");
  const size_t fb = spinor_bytes(pr, L->Vh) * nrhs;
  void* v = ws_get(L, "pl_qv", fb);
  void* w = ws_get(L, "pl_w", fb);
  std::vector<double> zr, zi, shifts(nrhs, mu2);
  poly_q_roots(pd, zr, zi);
  copy_dev(L, v, in, fb);
  for (size_t k = 0; k < zr.size(); ++k) {
    op_j(L, pr, w, v, kappa, shifts.data(), nrhs);
    std::vector<double> one(2 * nrhs), mz(2 * nrhs);
    for (int r = 0; r < nrhs; ++r) {
      one[2 * r] = 1.0;
      one[2 * r + 1] = 0.0;
      mz[2 * r] = -zr[k];
      mz[2 * r + 1] = dagger ? zi[k] : -zi[k];
    }
    launch_caxpby(L, v, one.data(), w, mz.data(), v, 0, nrhs, pr);
  }
  std::vector<double> sc(2 * nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) sc[2 * r] = std::sqrt(poly_lead(pd));
  launch_caxpby(L, out, sc.data(), v, nullptr, nullptr, 0, nrhs, pr);
}

// P(J) in: the recurrence for P_n, Q^dag Q for a quotient
static void poly_full(wl_lattice* L, void* out, const void* in, double kappa, double mu2, const PolyDesc& pd,
                      Prec pr, int nrhs) {
  if (pd.ndiv == 0) {
    poly_P(L, out, in, kappa, mu2, pd, pr, nrhs);
    return;
  }
  void* q = ws_get(L, "pl_qq", spinor_bytes(pr, L->Vh) * nrhs);
  poly_Q(L, q, in, kappa, mu2, pd, 0, pr, nrhs);
  poly_Q(L, out, q, kappa, mu2, pd, 1, pr, nrhs);
}

void poly_apply(wl_lattice* L, int mode, void* out, const void* in, double kappa, double mu2, const PolyDesc& pd,
                Prec pr, int nrhs) {
  check_poly(pd);
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs must be 1..16");
  switch (mode) {
    case WL_POLY_P: poly_full(L, out, in, kappa, mu2, pd, pr, nrhs); break;
    case WL_POLY_PJ: {
      void* jin = ws_get(L, "pl_jin", spinor_bytes(pr, L->Vh) * nrhs);
      std::vector<double> shifts(nrhs, mu2);
      op_j(L, pr, jin, in, kappa, shifts.data(), nrhs);
      poly_full(L, out, jin, kappa, mu2, pd, pr, nrhs);
      break;
    }
    case WL_POLY_Q: poly_Q(L, out, in, kappa, mu2, pd, 0, pr, nrhs); break;
    case WL_POLY_QDAG: poly_Q(L, out, in, kappa, mu2, pd, 1, pr, nrhs); break;
    default: throw Error(WL_EINVAL, "unknown polynomial mode");
  }
}

}  // namespace wl
