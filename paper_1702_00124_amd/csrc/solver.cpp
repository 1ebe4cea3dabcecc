// Conjugate gradient on J = K-hat + mu2 (even sites, batched rhs) or on the
// full-lattice K = M^dag M (Sec. 2: K is inverted by an iterative solver such
// as CG; Sec. 3.1: even-odd preconditioning).
//
// Textbook CG from x0 = 0 (or a given initial guess); every scalar (alpha, beta, |r|^2, the per-rhs
// convergence flag) lives on the device, so an iteration is five kernels and
// no host round trip.  The host looks at the state once per chunk of
// iterations; a converged rhs is frozen on the device (alpha = 0) while the
// others continue.  The stop rule is the FP64 true residual
// |b - A x| <= tol |b|, checked whenever the iterated residual says so.
//
// Mixed precision: the inner iteration keeps r, p and A p in FP32 (or BF16)
// storage with FP32 arithmetic; x accumulates in FP64 and every dot product
// is accumulated in FP64.  A reliable update r = b - A x in FP64 replaces the
// iterated residual whenever it fell below delta times its largest value since
// the previous update (checked at chunk boundaries), and before exit.
//
// Optionally each chunk is captured once as a hipGraph on a side stream and
// replayed on the context stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "wl_ops.h"
#include "wl_solver_state.h"

namespace wl {

namespace {

struct CgGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long long ws_gen = -1;  // the lattice's workspace generation the capture saw
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~CgGraph() { reset(); }
};

}  // namespace


// CG core.  apply_lp: inner-precision operator with fused Re<in, out>
// partials (rows of nbrow); apply64: FP64 operator for true residuals.
// Fields hold nrhs right-hand sides of nh halves each.  With jpa > 0 the
// cost counter is set to what the solve needed: jpa K multiplications per
// operator application, one application per iteration of each rhs up to its
// convergence and one per rhs for each FP64 residual b - A x (applications a
// chunk issues past a rhs's convergence are not counted); jpa = 0 leaves the
// counter to the operator's own launches.
static int cg_core(wl_lattice* L, void* x, const void* b, int nrhs, int nh, int nbrow, size_t hb64, size_t hbi,
                   const ApplyLowp& apply_lp, const Apply64& apply64, const wl_cg_params& prm,
                   wl_cg_stats* stats, long long jpa) {
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs && nrhs * nh <= kMaxRhs, WL_EINVAL, "nrhs out of range");
  WL_REQUIRE(prm.tol > 0.0 && prm.maxiter > 0, WL_EINVAL, "cg: tol and maxiter must be positive");
  const Prec ip = Prec(prm.inner);
  WL_REQUIRE(ip == F64 || ip == F32 || ip == BF16, WL_EINVAL, "cg: unknown inner precision");
  const bool mixed = ip != F64;
  const double delta = prm.delta > 0.0 ? prm.delta : 0.1;
  const int chunk = prm.chunk > 0 ? prm.chunk : 8;
  const size_t fb64 = hb64 * nh * nrhs;
  const size_t fbi = hbi * nh * nrhs;

  void* r = ws_get(L, "cg_r", fbi);
  void* p = ws_get(L, "cg_p", fbi);
  void* Ap = ws_get(L, "cg_Ap", fbi);
  void* r64 = ws_get(L, "cg_r64", fb64);
  void* Ax64 = ws_get(L, "cg_Ax64", fb64);
  // a mixed CG accumulates its iterations' steps in FP32 and folds them into the
  // FP64 x before each FP64 true residual (so the update moves half the bytes of x)
  const Prec xp = mixed ? F32 : F64;
  void* xa = mixed ? ws_get(L, "cg_x32", spinor_bytes(F32, L->Vh) * nh * nrhs) : x;
  ensure_partials(L, size_t(nrhs) * nbrow * 3 + 64);
  double* st = L->dscal + kCgState;
  const long long kmat0 = L->n_kmat;
  long long kmat_extra = 0;

  // true residual r64 = b - A x (FP64); rr_true[r] = |r64|^2
  std::vector<double> rr_true(nrhs), bb(nrhs);
  auto true_residual = [&]() {
    if (mixed) launch_cg_fold(L, x, xa, nrhs * nh);
    apply64(Ax64, x);
    ++kmat_extra;
    double ca[2 * kMaxRhs] = {0}, cb[2 * kMaxRhs] = {0};
    for (int f = 0; f < nrhs * nh; ++f) {
      ca[2 * f] = 1.0;
      cb[2 * f] = -1.0;
    }
    launch_caxpby(L, r64, ca, b, cb, Ax64, 0, nrhs * nh);
    norm2_host(L, r64, nrhs, rr_true.data(), nh);
  };

  // ---- initial state: x = x0 (0 unless given), r = b - A x0, p = r
  if (mixed) zero_dev(L, xa, spinor_bytes(F32, L->Vh) * nh * nrhs);
  norm2_host(L, b, nrhs, bb.data(), nh);
  for (int i = 0; i < nrhs; ++i) WL_REQUIRE(std::isfinite(bb[i]), WL_EINVAL, "cg: non-finite right-hand side");
  if (prm.use_x0) {
    for (int i = 0; i < nrhs; ++i)  // a zero source has the zero solution
      if (bb[i] == 0.0) zero_dev(L, static_cast<char*>(x) + size_t(i) * nh * hb64, nh * hb64);
    true_residual();
    if (mixed) launch_convert(L, ip, r, F64, r64, nrhs * nh);
    else copy_dev(L, r, r64, fb64);
  } else {
    zero_dev(L, x, fb64);
    if (mixed) launch_convert(L, ip, r, F64, b, nrhs * nh);
    else copy_dev(L, r, b, fb64);
    for (int i = 0; i < nrhs; ++i) rr_true[i] = bb[i];
  }
  copy_dev(L, p, r, fbi);
  std::vector<double> hs(CG_NROWS * kMaxRhs, 0.0);
  auto S = [&](int row, int rr) -> double& { return hs[row * kMaxRhs + rr]; };
  std::vector<char> verified(nrhs, 0);
  for (int i = 0; i < nrhs; ++i) {
    S(CG_RR, i) = rr_true[i];
    S(CG_BB, i) = bb[i];
    S(CG_TOL2, i) = prm.tol * prm.tol;
    S(CG_MAXRR, i) = rr_true[i];
    if (bb[i] == 0.0 || rr_true[i] <= prm.tol * prm.tol * bb[i]) {
      S(CG_DONE, i) = 1.0;
      verified[i] = 1;
      if (bb[i] == 0.0) rr_true[i] = 0.0;
    }
  }
  auto push_state = [&]() {
    std::memcpy(L->hscal + kCgState, hs.data(), sizeof(double) * hs.size());
    WL_HIP(hipMemcpyAsync(st, L->hscal + kCgState, sizeof(double) * hs.size(), hipMemcpyHostToDevice, L->stream));
  };
  auto pull_state = [&]() {
    WL_HIP(hipMemcpyAsync(L->hscal + kCgState, st, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, L->stream));
    WL_HIP(hipStreamSynchronize(L->stream));
    std::memcpy(hs.data(), L->hscal + kCgState, sizeof(double) * hs.size());
  };
  push_state();

  // rows of nbrow partials: the operator writes nbrow of <p, A p> per rhs;
  // the update writes nh * blas_blocks of |r|^2 (never more than nbrow)
  const int nb_upd = nh * blas_blocks(L);
  WL_REQUIRE(nb_upd <= nbrow, WL_EINVAL, "cg: reduction row too narrow");
  // Fused scalars (alpha in the update kernel, beta in the p update) save two
  // launches per iteration but make every block re-read a partial-sum row:
  // worth it while those re-reads (blocks x row entries) stay small, e.g. at
  // 16^3 x 32 (256 x 1024); at 32^3 x 64 (4096 x 16384) the separate kernels win.
  // The operator's <p, A p> partial sums (complex for the generic operators:
  // two rows per rhs) come first; the fused update's |r|^2 partial sums follow.
  const bool fuse = size_t(nbrow) * size_t(blas_blocks(L)) <= (size_t(1) << 20);
  auto issue_chunk = [&]() {
    double* rr_part = L->partials + size_t(2) * nrhs * nbrow;  // read afresh: the partials may have grown
    for (int it = 0; it < chunk; ++it) {
      apply_lp(ip, Ap, p, DotOut{L->partials, nbrow});
      if (fuse) {
        launch_cg_update_fused(L, ip, xp, xa, r, p, Ap, st, nrhs, nh, L->partials, nbrow, rr_part, nbrow);
        launch_cg_xpay_fused(L, ip, p, r, st, nrhs, nh, rr_part, nb_upd, nbrow);
      } else {
        launch_cg_alpha(L, L->partials, nbrow, nbrow, st, nrhs);
        launch_cg_update(L, ip, xp, xa, r, p, Ap, st, nrhs, nh, L->partials, nbrow);
        launch_cg_beta(L, L->partials, nbrow, nb_upd, st, nrhs);
        launch_cg_xpay(L, ip, p, r, st, nrhs, nh);
      }
    }
  };

  CgGraph cg_graph;
  long long hops_per_chunk = 0, hops_p_chunk[3] = {0, 0, 0};
  int chunks = 0;
  int reliable = 0;
  bool all_verified = true;  // an initial guess can already be a solution
  for (int i = 0; i < nrhs; ++i) all_verified = all_verified && verified[i];
  bool out_of_iters = false;
  // termination also without progress: a system that keeps breaking down
  // never advances its iteration count, so stop after a few fruitless
  // restarts in a row, and in any case once 4 maxiter iterations were issued
  int stalled = 0, last_max_it = -1;
  const long long issue_cap = 4LL * prm.maxiter + chunk;
  while (!all_verified) {
    if (prm.use_graph && chunks > 0) {
      // a workspace buffer freed since the capture (an FP64 true residual can
      // grow the operator's buffers) leaves the graph with dead addresses
      if (cg_graph.exec && cg_graph.ws_gen != L->ws_gen) cg_graph.reset();
      if (!cg_graph.exec) {
        if (!L->capture_stream) WL_HIP(hipStreamCreateWithFlags(&L->capture_stream, hipStreamNonBlocking));
        hipStream_t keep = L->stream;
        const long long hop0 = L->n_hop;
        const long long hp0[3] = {L->n_hop_p[0], L->n_hop_p[1], L->n_hop_p[2]};
        L->stream = L->capture_stream;
        L->prof_capturing = 1;
        WL_HIP(hipStreamBeginCapture(L->stream, hipStreamCaptureModeThreadLocal));
        try {
          issue_chunk();
        } catch (...) {
          hipGraph_t g;
          (void)hipStreamEndCapture(L->stream, &g);
          L->stream = keep;
          L->prof_capturing = 0;
          throw;
        }
        WL_HIP(hipStreamEndCapture(L->stream, &cg_graph.graph));
        L->stream = keep;
        L->prof_capturing = 0;
        hops_per_chunk = L->n_hop - hop0;
        L->n_hop = hop0;  // capture executes nothing; replays are counted below
        for (int q = 0; q < 3; ++q) {
          hops_p_chunk[q] = L->n_hop_p[q] - hp0[q];
          L->n_hop_p[q] = hp0[q];
        }
        WL_HIP(hipGraphInstantiate(&cg_graph.exec, cg_graph.graph, nullptr, nullptr, 0));
        cg_graph.ws_gen = L->ws_gen;
      }
      WL_HIP(hipGraphLaunch(cg_graph.exec, L->stream));
      L->n_hop += hops_per_chunk;
      for (int q = 0; q < 3; ++q) L->n_hop_p[q] += hops_p_chunk[q];
    } else {
      issue_chunk();
    }
    ++chunks;
    pull_state();

    bool all_done = true, need_ru = false, broke = false;
    for (int i = 0; i < nrhs; ++i) {
      if (verified[i]) continue;
      if (S(CG_DONE, i) == 0.0) all_done = false;
      if (S(CG_DONE, i) != 0.0 || S(CG_RR, i) < delta * delta * S(CG_MAXRR, i)) need_ru = true;
      if (S(CG_BREAK, i) != 0.0) broke = true;
    }
    int max_it = 0;
    for (int i = 0; i < nrhs; ++i) max_it = std::max(max_it, int(S(CG_ITERS, i)));

    if ((mixed && need_ru) || (!mixed && all_done) || broke) {
      true_residual();
      if (mixed) launch_convert(L, ip, r, F64, r64, nrhs * nh);
      ++reliable;
      // BF16 storage (and any breakdown) restarts the Krylov space from the
      // fresh residual (restarted defect correction); FP32 keeps p
      bool restart = broke || ip == BF16;
      for (int i = 0; i < nrhs; ++i) {
        if (verified[i]) continue;
        const double t2 = prm.tol * prm.tol * bb[i];
        S(CG_BREAK, i) = 0.0;
        if (rr_true[i] <= t2) {
          S(CG_DONE, i) = 1.0;
          verified[i] = 1;
        } else if (mixed) {
          S(CG_DONE, i) = 0.0;
        } else if (S(CG_DONE, i) != 0.0) {
          S(CG_DONE, i) = 0.0;  // FP64: the iterated residual drifted; restart from x
          restart = true;
        }
        if (mixed || S(CG_DONE, i) == 0.0) {
          S(CG_RR, i) = rr_true[i];
          S(CG_MAXRR, i) = rr_true[i];
        }
      }
      if (restart) {
        if (!mixed) copy_dev(L, r, r64, fb64);
        copy_dev(L, p, r, fbi);
        for (int i = 0; i < nrhs; ++i)
          if (!verified[i]) S(CG_RR, i) = rr_true[i];
      }
      push_state();
    }
    all_verified = true;
    for (int i = 0; i < nrhs; ++i) all_verified = all_verified && verified[i];
    if (all_verified) break;
    if (max_it >= prm.maxiter) {
      out_of_iters = true;
      break;
    }
    stalled = (broke && max_it == last_max_it) ? stalled + 1 : 0;
    last_max_it = max_it;
    if (stalled >= 4 || (long long)chunks * chunk >= issue_cap) {
      out_of_iters = true;
      break;
    }
  }
  if (out_of_iters) true_residual();

  long long iters_total = 0;
  for (int i = 0; i < nrhs; ++i) iters_total += (long long)S(CG_ITERS, i);
  // K multiplications the solve needed (graph replays are not seen by the launch counters)
  if (jpa > 0) L->n_kmat = kmat0 + (iters_total + kmat_extra * nrhs) * jpa;
  if (L->solve_log_on)
    L->solve_log.push_back({iters_total, kmat_extra * nrhs, jpa > 0 ? jpa : 0});
  if (stats) {
    for (int i = 0; i < nrhs; ++i) {
      stats[i].iters = int(S(CG_ITERS, i));
      stats[i].reliable_updates = reliable;
      stats[i].converged = verified[i] ? 1 : 0;
      stats[i].true_rel_res = bb[i] > 0 ? std::sqrt(rr_true[i] / bb[i]) : 0.0;
    }
  }
  return all_verified ? WL_OK : WL_ENOCONV;
}

int cg_run(wl_lattice* L, void* x, const void* b, double kappa, const double* mu2, int nrhs, int op,
           const wl_cg_params& prm, wl_cg_stats* stats) {
  WL_REQUIRE(op == WL_OP_J || op == WL_OP_K, WL_EINVAL, "cg_solve needs WL_OP_J or WL_OP_K");
  WL_REQUIRE(op != WL_OP_K || nrhs == 1, WL_EUNSUPPORTED, "full-lattice CG takes one rhs");
  const Prec ip = Prec(prm.inner);
  const int nh = op == WL_OP_K ? 2 : 1;
  ApplyLowp lp = [&](Prec pr, void* out, const void* in, const DotOut& d) {
    op_apply(L, op, pr, out, in, kappa, mu2, nrhs, d);
  };
  Apply64 a64 = [&](void* out, const void* in) { op_apply(L, op, F64, out, in, kappa, mu2, nrhs); };
  const Prec ipr = (ip == F32 || ip == BF16) ? ip : F64;
  return cg_core(L, x, b, nrhs, nh, op_dot_blocks(L, op, ipr), spinor_bytes(F64, L->Vh),
                 spinor_bytes((ip == F32 || ip == BF16) ? ip : F64, L->Vh), lp, a64, prm, stats, 1);
}

int cg_run_batch(wl_lattice* L, void* x, const void* b, int nrhs, int nbrow, const ApplyLowp& lp, const Apply64& a64,
                 const wl_cg_params& prm, wl_cg_stats* stats) {
  const Prec ip = Prec(prm.inner);
  const Prec ipr = (ip == F32 || ip == BF16) ? ip : F64;
  const size_t hb64 = spinor_bytes(F64, L->Vh), hbi = spinor_bytes(ipr, L->Vh);
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs out of range");
  // the operator outputs are written at the lattices' sites only: clear the rest
  zero_dev(L, ws_get(L, "cg_Ap", hbi * nrhs), hbi * nrhs);
  zero_dev(L, ws_get(L, "cg_Ax64", hb64 * nrhs), hb64 * nrhs);
  return cg_core(L, x, b, nrhs, 1, nbrow, hb64, hbi, lp, a64, prm, stats, 0);
}

int cg_run_generic(wl_lattice* L, void* x, const void* b,
                   const std::function<void(Prec, void*, const void*)>& apply, const wl_cg_params& prm_in,
                   wl_cg_stats* stats, long long jpa) {
  wl_cg_params prm = prm_in;
  prm.use_graph = 0;  // the polynomial operators synchronise nothing but are host-sequenced; no capture
  const Prec ip = Prec(prm.inner);
  const int nb = blas_blocks(L);
  ApplyLowp lp = [&](Prec pr, void* out, const void* in, const DotOut& d) {
    apply(pr, out, in);
    // complex <in, out>: row 0 holds the real part, which CG needs
    launch_dot_partials(L, in, out, 1, d.partials, d.stride, 1, pr);
  };
  Apply64 a64 = [&](void* out, const void* in) { apply(F64, out, in); };
  return cg_core(L, x, b, 1, 1, nb, spinor_bytes(F64, L->Vh),
                 spinor_bytes((ip == F32 || ip == BF16) ? ip : F64, L->Vh), lp, a64, prm, stats, jpa);
}

// ------------------------------------------------------------------ multi-shift CG
// (J(mu2_s) ) x_s = b for nshift shifts of K-hat at once: CG on the smallest
// shift, the others from the collinear-residual recurrences (see
// ms_scalars_kernel).  FP64 throughout; every (rhs, shift) system freezes once
// its residual |zeta|^2 |r|^2 meets the tolerance, the iteration ends with the
// base system, and every solution is then checked by its FP64 true residual;
// a system that misses it is refined by an ordinary CG on its residual.
int cg_multishift_run(wl_lattice* L, void* x_out, const void* b, double kappa, const double* shifts, int nshift,
                      int nrhs, const wl_cg_params& prm, wl_cg_stats* stats) {
  static_assert(kMsRhsRows + MS_RHS_NROWS * kMaxRhs <= kScal, "multi-shift state exceeds the scalar area");
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs out of range");
  WL_REQUIRE(nshift >= 1 && nshift * nrhs <= kMaxSys, WL_EINVAL, "nshift * nrhs must be at most 64");
  WL_REQUIRE(shifts, WL_EINVAL, "null shifts");
  WL_REQUIRE(!prm.use_x0, WL_EUNSUPPORTED, "multi-shift CG shares one Krylov space and starts from x = 0");
  WL_REQUIRE(prm.tol > 0.0 && prm.maxiter > 0, WL_EINVAL, "cg: tol and maxiter must be positive");
  for (int s = 0; s < nshift; ++s) WL_REQUIRE(shifts[s] >= 0.0, WL_EINVAL, "shifts must be non-negative");
  const int chunk = prm.chunk > 0 ? prm.chunk : 8;
  const size_t fb = spinor_bytes(F64, L->Vh);
  const int nsys = nshift * nrhs;
  // internal order: ascending shifts, the smallest is the base system
  std::vector<int> order(nshift);
  for (int s = 0; s < nshift; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return shifts[i] < shifts[j]; });
  const double s0 = shifts[order[0]];

  char* r = static_cast<char*>(ws_get(L, "ms_r", fb * nrhs));
  char* Ap = static_cast<char*>(ws_get(L, "ms_Ap", fb * nrhs));
  char* p = static_cast<char*>(ws_get(L, "ms_p", fb * nsys));
  char* x = static_cast<char*>(ws_get(L, "ms_x", fb * nsys));
  char* r64 = static_cast<char*>(ws_get(L, "ms_r64", fb * nrhs));
  const int nbrow = op_dot_blocks(L, WL_OP_J, F64);
  WL_REQUIRE(blas_blocks(L) <= nbrow, WL_EINVAL, "cg: reduction row too narrow");
  ensure_partials(L, size_t(nrhs) * nbrow * 2 + 64);
  double* st = L->dscal + kCgState;
  double* ms = L->dscal + kMsState;
  double* mr = L->dscal + kMsRhsRows;

  std::vector<double> bb(nrhs);
  norm2_host(L, b, nrhs, bb.data());
  for (int i = 0; i < nrhs; ++i) WL_REQUIRE(std::isfinite(bb[i]), WL_EINVAL, "cg: non-finite right-hand side");
  zero_dev(L, x, fb * nsys);
  copy_dev(L, r, b, fb * nrhs);
  for (int s = 0; s < nshift; ++s) copy_dev(L, p + size_t(s) * nrhs * fb, b, fb * nrhs);

  // host mirrors of the three state blocks
  std::vector<double> hs(CG_NROWS * kMaxRhs, 0.0), hm(MS_NROWS * kMaxSys, 0.0), hr(MS_RHS_NROWS * kMaxRhs, 0.0);
  auto S = [&](int row, int i) -> double& { return hs[row * kMaxRhs + i]; };
  auto M = [&](int row, int q) -> double& { return hm[row * kMaxSys + q]; };
  for (int i = 0; i < nrhs; ++i) {
    S(CG_RR, i) = bb[i];
    S(CG_BB, i) = bb[i];
    S(CG_TOL2, i) = prm.tol * prm.tol;
    S(CG_MAXRR, i) = bb[i];
    if (bb[i] == 0.0) S(CG_DONE, i) = 1.0;
    hr[MS_APREV * kMaxRhs + i] = 1.0;
  }
  for (int s = 0; s < nshift; ++s)
    for (int i = 0; i < nrhs; ++i) {
      const int q = s * nrhs + i;
      M(MS_ZPREV, q) = M(MS_ZCUR, q) = M(MS_ZNEXT, q) = 1.0;
      M(MS_DELTA, q) = shifts[order[s]] - s0;
      if (bb[i] == 0.0) M(MS_DONE, q) = 1.0;
    }
  std::memcpy(L->hscal + kCgState, hs.data(), sizeof(double) * hs.size());
  std::memcpy(L->hscal + kMsState, hm.data(), sizeof(double) * hm.size());
  std::memcpy(L->hscal + kMsRhsRows, hr.data(), sizeof(double) * hr.size());
  WL_HIP(hipMemcpyAsync(st, L->hscal + kCgState, sizeof(double) * (kMsRhsRows + hr.size() - kCgState),
                        hipMemcpyHostToDevice, L->stream));

  std::vector<double> mu_base(nrhs, s0);
  const long long kmat0 = L->n_kmat;
  while (true) {
    for (int it = 0; it < chunk; ++it) {
      op_j(L, F64, Ap, p, kappa, mu_base.data(), nrhs, DotOut{L->partials, nbrow});
      launch_cg_alpha(L, L->partials, nbrow, nbrow, st, nrhs);
      launch_ms_scalars(L, st, ms, mr, nrhs, nshift);
      launch_ms_update(L, r, Ap, p, x, st, ms, nrhs, nshift, L->partials, nbrow);
      launch_cg_beta(L, L->partials, nbrow, blas_blocks(L), st, nrhs);
      launch_ms_xpay(L, p, r, st, ms, nrhs, nshift);
    }
    WL_HIP(hipMemcpyAsync(L->hscal + kCgState, st, sizeof(double) * (kMsRhsRows + hr.size() - kCgState),
                          hipMemcpyDeviceToHost, L->stream));
    WL_HIP(hipStreamSynchronize(L->stream));
    std::memcpy(hs.data(), L->hscal + kCgState, sizeof(double) * hs.size());
    std::memcpy(hm.data(), L->hscal + kMsState, sizeof(double) * hm.size());
    bool all = true;
    int max_it = 0;
    for (int i = 0; i < nrhs; ++i) {
      all = all && (S(CG_DONE, i) != 0.0 || S(CG_BREAK, i) != 0.0);
      max_it = std::max(max_it, int(S(CG_ITERS, i)));
    }
    if (all || max_it >= prm.maxiter) break;
  }
  long long base_iters = 0;
  for (int i = 0; i < nrhs; ++i) base_iters += (long long)S(CG_ITERS, i);
  L->n_kmat = kmat0 + base_iters;

  // true residuals per shift (batched over rhs), refinement of any miss
  std::vector<double> rr(nsys), rr1(nrhs);
  std::vector<int> refined_iters(nsys, 0);
  const double one[2] = {1.0, 0.0};
  auto residual = [&](int s) {
    std::vector<double> mu(nrhs, shifts[order[s]]);
    op_j(L, F64, r64, x + size_t(s) * nrhs * fb, kappa, mu.data(), nrhs);
    L->n_kmat += nrhs;
    double ca[2 * kMaxRhs], cb[2 * kMaxRhs];
    for (int i = 0; i < nrhs; ++i) {
      ca[2 * i] = 1.0, ca[2 * i + 1] = 0.0;
      cb[2 * i] = -1.0, cb[2 * i + 1] = 0.0;
    }
    launch_caxpby(L, r64, ca, b, cb, r64, 0, nrhs);
    norm2_host(L, r64, nrhs, rr1.data());
  };
  bool all_ok = true;  // decided by the final true residuals (a base run cut by maxiter is refined)
  for (int s = 0; s < nshift; ++s) {
    residual(s);
    for (int i = 0; i < nrhs; ++i) {
      const int q = s * nrhs + i;
      rr[q] = rr1[i];
      if (bb[i] == 0.0 || rr1[i] <= prm.tol * prm.tol * bb[i]) continue;
      // refine: x_s += J_s^-1 (b - J_s x_s), to the tolerance relative to |b|
      // (with a margin, so that the recomputed residual of x + e meets it too,
      // and its own iteration limit: maxiter bounds the base iteration)
      wl_cg_params rp = prm;
      rp.tol = std::min(0.5, 0.5 * prm.tol * std::sqrt(bb[i] / rr1[i]));
      rp.maxiter = std::max(prm.maxiter, 10000);
      rp.use_graph = 0;
      rp.use_x0 = 0;
      char* e = static_cast<char*>(ws_get(L, "ms_e", fb));
      const double mu = shifts[order[s]];
      wl_cg_stats est{};
      const int rc = cg_run(L, e, r64 + size_t(i) * fb, kappa, &mu, 1, WL_OP_J, rp, &est);
      refined_iters[q] = est.iters;
      char* xs = x + size_t(q) * fb;
      launch_caxpby(L, xs, one, xs, one, e, 0, 1);
      if (rc != WL_OK) all_ok = false;
    }
    bool any_refined = false;
    for (int i = 0; i < nrhs; ++i) any_refined = any_refined || refined_iters[s * nrhs + i] > 0;
    if (any_refined) {
      residual(s);
      for (int i = 0; i < nrhs; ++i) rr[s * nrhs + i] = rr1[i];
    }
  }
  // results in the caller's shift order
  for (int s = 0; s < nshift; ++s)
    copy_dev(L, static_cast<char*>(x_out) + size_t(order[s]) * nrhs * fb, x + size_t(s) * nrhs * fb, fb * nrhs);
  for (int s = 0; s < nshift; ++s)
    for (int i = 0; i < nrhs; ++i) {
      const int q = s * nrhs + i;
      const bool ok = bb[i] == 0.0 || rr[q] <= prm.tol * prm.tol * bb[i] * (1.0 + 1e-12);
      all_ok = all_ok && ok;
      if (stats) {
        wl_cg_stats& o = stats[order[s] * nrhs + i];
        o.iters = (M(MS_DONE, q) != 0.0 ? int(M(MS_ITERS, q)) : int(S(CG_ITERS, i))) + refined_iters[q];
        o.reliable_updates = refined_iters[q] > 0 ? 1 : 0;
        o.converged = ok ? 1 : 0;
        o.true_rel_res = bb[i] > 0 ? std::sqrt(rr[q] / bb[i]) : 0.0;
      }
    }
  return all_ok ? WL_OK : WL_ENOCONV;
}

}  // namespace wl
