// HMC trajectory (Sec. 2) with the generalised multi-time-scale integrator
// (Sec. 3.2).
//
// Sec. 2: pseudofermions from Gaussian noise, momenta from exp(-sum tr P^2),
// H = sum tr P^2 + S integrated with T[eps]: U -> exp(i eps P) U and
// S[eps]: P -> P - eps F, then a Metropolis step.  With P = sum_a p^a T^a,
// sum tr P^2 = (1/2) sum (p^a)^2 and the space step is p^a -= eps grad^a S.
//
// Sec. 3.2: each action term i has its own second-order scheme with n_i
// steps on [0, tau]; its S_i updates are placed at their times t and the
// schemes are overlaid, with T[dt] for the gaps between consecutive distinct
// times.  Times are kept exact as integers over the common denominator
// 2 lcm(n_i).  Updates at one time commute (they change P only); they are
// ordered by ascending term index before the trajectory midpoint and by
// descending index after it, so the schedule is its own time reverse.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "wl_ops.h"

namespace wl {

struct Event {
  int kind;    // 0: S update of `term`, 1: T step
  int term;
  double w;    // step in units of tau
};

std::vector<Event> merge_schedule(const std::vector<int>& nsteps, int scheme, double lam);

static long long lcm_ll(long long a, long long b) { return a / std::gcd(a, b) * b; }

std::vector<Event> merge_schedule(const std::vector<int>& nsteps, int scheme, double lam) {
  long long D = 2;
  for (int n : nsteps) D = lcm_ll(D, 2LL * n);
  struct Ev {
    long long t;
    int term;
    double w;
  };
  std::vector<Ev> ev;
  for (int i = 0; i < int(nsteps.size()); ++i) {
    const int n = nsteps[i];
    const long long h = D / n;
    const double hw = 1.0 / n;
    if (scheme == WL_INT_LEAPFROG) {
      ev.push_back({0, i, 0.5 * hw});
      for (int k = 1; k < n; ++k) ev.push_back({k * h, i, hw});
      ev.push_back({D, i, 0.5 * hw});
    } else {
      ev.push_back({0, i, lam * hw});
      for (int k = 0; k < n; ++k) {
        ev.push_back({k * h + h / 2, i, (1.0 - 2.0 * lam) * hw});
        if (k < n - 1) ev.push_back({(k + 1) * h, i, 2.0 * lam * hw});
      }
      ev.push_back({D, i, lam * hw});
    }
  }
  std::stable_sort(ev.begin(), ev.end(), [&](const Ev& a, const Ev& b) {
    if (a.t != b.t) return a.t < b.t;
    return (2 * a.t > D) ? a.term > b.term : a.term < b.term;
  });
  std::vector<Event> out;
  long long prev = 0;
  for (const Ev& e : ev) {
    if (e.t > prev) {
      out.push_back({1, -1, double(e.t - prev) / double(D)});
      prev = e.t;
    }
    out.push_back({0, e.term, e.w});
  }
  if (prev < D) out.push_back({1, -1, double(D - prev) / double(D)});
  return out;
}

static double sumsq_host(wl_lattice* L, const double* P) {
  const int nb = site_blocks(L->Vh);
  ensure_partials(L, nb);
  launch_su3_sumsq_partials(L, P, L->partials);
  launch_finish_sum(L, L->partials, nb, nb, 1, L->dscal);
  WL_HIP(hipMemcpyAsync(L->hscal, L->dscal, sizeof(double), hipMemcpyDeviceToHost, L->stream));
  WL_HIP(hipStreamSynchronize(L->stream));
  return L->hscal[0];
}

double plaquette_host(wl_lattice* L) {
  const int nb = site_blocks(L->Vh);
  ensure_partials(L, 2 * nb);
  launch_plaquette_partials(L, L->partials);
  launch_finish_sum(L, L->partials, 2 * nb, 2 * nb, 1, L->dscal);
  WL_HIP(hipMemcpyAsync(L->hscal, L->dscal, sizeof(double), hipMemcpyDeviceToHost, L->stream));
  WL_HIP(hipStreamSynchronize(L->stream));
  return L->hscal[0] / (6.0 * L->V);
}

int hmc_run(wl_lattice* L, const wl_hmc_params& prm, double* P, const void* chi, double u, wl_hmc_result* res) {
  const int nt = prm.nterms;
  WL_REQUIRE(nt >= 0 && nt <= 8, WL_EINVAL, "nterms must be 0..8");
  WL_REQUIRE(prm.tau > 0.0, WL_EINVAL, "tau must be positive");
  WL_REQUIRE(prm.integrator == WL_INT_LEAPFROG || prm.integrator == WL_INT_OMELYAN, WL_EINVAL, "unknown integrator");
  for (int i = 0; i <= nt; ++i) WL_REQUIRE(prm.nsteps[i] >= 1, WL_EINVAL, "nsteps must be >= 1");
  const double lam = prm.omelyan_lambda > 0.0 ? prm.omelyan_lambda : 0.1931833275037836;
  const size_t hb = spinor_bytes(F64, L->Vh);
  const long long kmat0 = L->n_kmat;
  long long cg_iters = 0;

  // keep the starting links for a rejection
  const size_t ub = full_links_bytes(L->Vh);
  void* Ubak = ws_get(L, "hmc_Ubak", ub);
  copy_dev(L, Ubak, L->Ufull, ub);

  // heatbath
  std::vector<void*> phi(nt);
  const char* c = static_cast<const char*>(chi);
  for (int i = 0; i < nt; ++i) {
    const size_t fb = (prm.terms[i].kind == WL_TERM_KINV_FULL ? 2 : 1) * hb;
    phi[i] = ws_get(L, "hmc_phi" + std::to_string(i), fb);
    if (prm.flags & WL_HMC_PHI_GIVEN) copy_dev(L, phi[i], c, fb);
    else term_heatbath(L, prm.terms[i], phi[i], c);
    c += fb;
  }

  auto hamiltonian = [&](double* S) {
    double H = 0.5 * sumsq_host(L, P);
    for (int i = 0; i < nt; ++i) {
      S[i] = term_action(L, prm.terms[i], phi[i], &cg_iters);
      H += S[i];
    }
    S[nt] = prm.beta * 6.0 * L->V * (1.0 - plaquette_host(L));
    return H + S[nt];
  };

  wl_hmc_result r{};
  r.H0 = hamiltonian(r.S0);

  // chronological initial guesses: one slot per term, empty at the start
  std::vector<ChronoSlot> chrono(nt);
  if (prm.flags & WL_HMC_CHRONO) {
    const int depth = prm.chrono_depth > 0 ? prm.chrono_depth : 4;
    WL_REQUIRE(depth <= 8, WL_EINVAL, "chrono_depth must be at most 8");
    for (int i = 0; i < nt; ++i) {
      ChronoSlot& c = chrono[i];
      c.nh = prm.terms[i].kind == WL_TERM_KINV_FULL ? 2 : 1;
      c.fb = c.nh * hb;
      c.depth = depth;
      char* buf = static_cast<char*>(ws_get(L, "hmc_chrono" + std::to_string(i), 3 * size_t(depth) * c.fb));
      c.ring = buf;
      c.basis = buf + size_t(depth) * c.fb;
      c.abasis = buf + 2 * size_t(depth) * c.fb;
    }
  }

  std::vector<int> ns(prm.nsteps, prm.nsteps + nt + 1);
  for (const Event& e : merge_schedule(ns, prm.integrator, lam)) {
    const double eps = e.w * prm.tau;
    if (e.kind == 1) {
      launch_link_update(L, P, eps);
    } else if (e.term < nt) {
      term_force(L, prm.terms[e.term], P, phi[e.term], -eps, &cg_iters,
                 (prm.flags & WL_HMC_CHRONO) ? &chrono[e.term] : nullptr);
    } else {
      // grad S_G = -(beta/3) Re(i tr(T^a U A)); P -= eps grad S_G
      launch_gauge_force(L, P, eps * prm.beta / 3.0);
    }
  }

  r.H1 = hamiltonian(r.S1);
  r.dH = r.H1 - r.H0;
  r.accepted = (prm.flags & WL_HMC_NO_METROPOLIS) ? 1 : (u < std::exp(-r.dH) ? 1 : 0);
  if (!r.accepted) copy_dev(L, L->Ufull, Ubak, ub);
  L->lowp_valid = false;
  r.plaquette = plaquette_host(L);
  r.n_kmat = L->n_kmat - kmat0;
  r.cg_iters = cg_iters;
  if (res) *res = r;
  return WL_OK;
}

}  // namespace wl
