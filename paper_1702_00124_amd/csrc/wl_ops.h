// Operators built from the hop kernel, and the host orchestration layers
// (solver, polynomial filter, action terms, HMC) that call them.
#pragma once
#include <functional>

#include "wl_internal.h"

namespace wl {

struct DotOut {
  double* partials = nullptr;  // Re<in, out> partials; nullptr = no reduction
  int stride = 0;
};

// intermediates of the operators supplied by the caller instead of the
// workspace: odd = the D_oe result (J, M-hat; nrhs fields) or, for the
// full-lattice K, the full M in (two halves); even = J's g5 M-hat in
struct OpScratch {
  void* odd = nullptr;
  void* even = nullptr;
};
// bytes of caller-supplied intermediates op needs (odd followed by even)
size_t op_scratch_bytes(const wl_lattice* L, int op, Prec prec, int nrhs);

// even sites: out = M-hat in (dagger: M-hat^dag), nrhs fields of precision prec
void op_mhat(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, int dagger, int nrhs,
             const OpScratch* scr = nullptr);
// one step of the Chebyshev recurrence fused into J's last hop (one rhs):
// tprev <- ct in + cw J in - tprev, eprev <- ce e + 2 in - eprev
struct ChebStep {
  void* tprev;
  const void* e;
  void* eprev;
  double ct, cw, ce;
};
// even sites: out = K-hat in + mu2[r] in; optional partials of Re<in, out>
// (one row per rhs, hop_tiles(L, prec) blocks); with cheb, out is not written
// and the Chebyshev step consumes J in (every rhs); with lin, out = lin[0] J in
// + lin[1] in, from the same last-hop epilogue
void op_j(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, const double* mu2, int nrhs,
          const DotOut& dot = DotOut(), const ChebStep* cheb = nullptr, const double* lin = nullptr,
          const OpScratch* scr = nullptr);
// full lattice (F64 halves back to back, nrhs = 1): M, M^dag, K = M^dag M
void op_m_full(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, int dagger);
void op_k_full(wl_lattice* L, Prec prec, void* out, const void* in, double kappa, const DotOut& dot = DotOut(),
               const OpScratch* scr = nullptr);
// generic dispatch used by the solver; dot rows hold 2 * blocks for the full lattice
void op_apply(wl_lattice* L, int op, Prec prec, void* out, const void* in, double kappa, const double* mu2,
              int nrhs, const DotOut& dot = DotOut(), const OpScratch* scr = nullptr);
inline int op_dot_blocks(const wl_lattice* L, int op, Prec prec) {
  return (op == WL_OP_K ? 2 : 1) * hop_tiles(L, prec);
}
inline size_t op_field_bytes(const wl_lattice* L, int op, Prec prec, int nrhs) {
  return (op == WL_OP_K ? 2 : 1) * spinor_bytes(prec, L->Vh) * size_t(nrhs);
}

// host-visible reductions over F64 fields (synchronise the stream)
void norm2_host(wl_lattice* L, const void* x, int nrhs, double* out, int nhalves = 1);
void cdot_host(wl_lattice* L, const void* x, const void* y, int nrhs, double* out /*2*nrhs*/, int nhalves = 1);

// CG (solver.cpp) on J (even sites) or the full-lattice K
int cg_run(wl_lattice* L, void* x, const void* b, double kappa, const double* mu2, int nrhs, int op,
           const wl_cg_params& prm, wl_cg_stats* stats);
// multi-shift CG on J(mu2 = shifts[s]) for nshift shifts and nrhs sources (FP64);
// x: [nshift][nrhs] fields in the order of shifts; stats [nshift * nrhs]
int cg_multishift_run(wl_lattice* L, void* x, const void* b, double kappa, const double* shifts, int nshift,
                      int nrhs, const wl_cg_params& prm, wl_cg_stats* stats);
// CG on a general HPD operator on even-site fields (one rhs, x and b F64):
// apply(prec, out, in) must leave out = A in with fields of storage precision
// prec (prm.inner for the iteration, F64 for true residuals).  Used for P(J)
// and P(J) J; jpa = the K multiplications of one application (cost count).
int cg_run_generic(wl_lattice* L, void* x, const void* b,
                   const std::function<void(Prec, void*, const void*)>& apply, const wl_cg_params& prm,
                   wl_cg_stats* stats, long long jpa);
// the solver core's operators: the inner-precision one with fused Re<in, out>
// partial sums (a row of DotOut.stride entries per rhs), and the FP64 one
using ApplyLowp = std::function<void(Prec, void*, const void*, const DotOut&)>;
using Apply64 = std::function<void(void*, const void*)>;
// CG over nrhs even-site fields of lattice L's size with the given operators
// (the mixed-volume batch): the operators must leave zero wherever they write
// nothing, and nbrow partial sums per rhs row
int cg_run_batch(wl_lattice* L, void* x, const void* b, int nrhs, int nbrow, const ApplyLowp& lp, const Apply64& a64,
                 const wl_cg_params& prm, wl_cg_stats* stats);

// mixed-volume batches (batch.cpp): slots of the largest lattice's field size
wl_batch* batch_create(wl_lattice* const* lats, int nlat);
void batch_destroy(wl_batch* B);
size_t batch_slot_bytes(const wl_batch* B, Prec prec);
int batch_count(const wl_batch* B);
wl_lattice* batch_big(const wl_batch* B);
// allocate the batch's intermediates of one precision and pack every lattice's links
void batch_prepare(wl_batch* B, Prec prec);
void batch_hop(wl_batch* B, Prec prec, void* out, const void* in, int out_parity, int dagger);
void batch_j(wl_batch* B, Prec prec, void* out, const void* in, const double* kappa, const double* mu2,
             const DotOut& dot);
int batch_cg(wl_batch* B, void* x, const void* b, const double* kappa, const double* mu2, const wl_cg_params& prm,
             wl_cg_stats* stats);

// polynomial filter (poly.cpp): nrhs fields of storage precision pr, one shift mu2
struct PolyDesc {
  int n;
  double a, b;
  int ndiv = 0;  // > 0: the quotient P_n / P_ndiv
};
void poly_apply(wl_lattice* L, int mode, void* out, const void* in, double kappa, double mu2, const PolyDesc& pd,
                Prec pr = F64, int nrhs = 1);
double poly_lead(const PolyDesc& pd);
// K multiplications (J applications) of one poly_apply per rhs: P_n n; a
// quotient P_n / P_m 2 q (Q^dag Q, q root factors); P J one more; Q, Q^dag q
long long poly_j_count(int mode, const PolyDesc& pd);
void check_poly(const PolyDesc& pd);
void poly_q_roots(const PolyDesc& pd, std::vector<double>& re, std::vector<double>& im);

// action terms (action.cpp)
void term_heatbath(wl_lattice* L, const wl_term& t, void* phi, const void* chi);
double term_action(wl_lattice* L, const wl_term& t, const void* phi, long long* cg_iters);
// chronological initial guess of one term's force solves: the last `depth`
// solutions of the term, and scratch for the minimal-residual extrapolation
// over their span (three blocks of depth F64 fields, both halves for KINV_FULL)
struct ChronoSlot {
  char* ring = nullptr;    // previous solutions; ring[next] is overwritten next
  char* basis = nullptr;   // orthonormal basis of their span
  char* abasis = nullptr;  // the solve's operator applied to the basis
  size_t fb = 0;           // bytes of one field
  int nh = 1;              // halves per field
  int depth = 0, count = 0, next = 0;
};
void term_force(wl_lattice* L, const wl_term& t, double* F, const void* phi, double coeff, long long* cg_iters,
                ChronoSlot* chrono = nullptr);

// field copies on the context stream
void copy_dev(wl_lattice* L, void* dst, const void* src, size_t bytes);
void zero_dev(wl_lattice* L, void* dst, size_t bytes);

}  // namespace wl
