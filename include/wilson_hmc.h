/* wilson_hmc.h -- C ABI of the MI355X (gfx950) two-flavour Wilson-fermion HMC hot path.
 *
 * Method: Haar, Kamleh, Zanotti, Nakamura, "Improving Polynomial-filtered
 * Hybrid Monte Carlo With Hasenbusch" (arXiv:1702.00124).  Sec. 2 defines the
 * HMC (heatbath, momenta, H = sum tr P^2 + S, the time step T[eps] and space
 * step S[eps], Metropolis), the two-flavour action phi^dag (M^dag M)^-1 phi
 * and its force, mass preconditioning and polynomial filtering; Sec. 3.1 fixes
 * Wilson fermions, hopping parameter kappa and even-odd preconditioning;
 * Sec. 3.2 the generalised multi-time-scale integrator; Sec. 4.1 the PF-MP
 * action.  Readings where the paper prints no formula:
 *
 *   M = 1 - kappa D,  (D psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
 *                                       + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
 *   (time-boundary phase t_bc on hops that wrap in t), chiral Hermitian gammas
 *   with g5 = diag(1,1,-1,-1); M-hat = 1 - kappa^2 D_eo D_oe on even sites;
 *   K-hat = M-hat^dag M-hat; J = K-hat + mu^2 (Hasenbusch shift, mu^2 form);
 *   Chebyshev filter 1 - x P_n(x) = T_{n+1}(y(x)) / T_{n+1}(y(0)),
 *   y(x) = (b + a - 2x)/(b - a);  su(3) coefficients p^a of P = sum p^a T^a,
 *   T^a = lambda^a / 2.
 *
 * Conventions of every buffer:
 *   * all field pointers are DEVICE pointers on the context's device;
 *   * canonical spinor: complex128 [nrhs][n][4 spin][3 colour], n = V (full
 *     lattice, site s = x + Lx*(y + Ly*(z + Lz*t))) or n = V/2 (the sites of
 *     one parity in lexicographic order);
 *   * canonical links: complex128 [4 mu][V][3][3];
 *   * canonical su(3) field (momenta, forces): float64 [4 mu][V][8];
 *   * internal half-lattice spinor: precision-dependent structure-of-arrays,
 *     wl_field_bytes() bytes; an internal FULL field is the even half
 *     followed by the odd half (two half fields back to back);
 *   * internal su(3) field: float64 [2 parity][4 mu][8][V/2], 256*V bytes.
 * The caller owns every field buffer; the library owns the context (packed
 * links, workspace).  Calls are ordered on the context's HIP stream; calls
 * that return host values synchronise it.
 *
 * Errors: every function returns WL_OK (0) or a negative code; nothing throws
 * or aborts across the ABI.  wl_last_error() gives the calling thread's
 * message for the last failure.  All lattice extents must be even.
 *
 * Threads: a context (and a batch, with the lattices it holds) is used by one
 * host thread at a time: calls share its workspace and device-resident solver
 * state.  Different contexts may be driven from different threads.
 */
#ifndef WILSON_HMC_H
#define WILSON_HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { WL_OK = 0, WL_EINVAL = -1, WL_EUNSUPPORTED = -2, WL_ENOMEM = -3, WL_EHIP = -4, WL_ENOCONV = -5 };

typedef enum { WL_F64 = 0, WL_F32 = 1, WL_BF16 = 2 } wl_prec;

typedef struct wl_lattice wl_lattice;

/* Thread-local message of the last failing call ("" if none). */
const char* wl_last_error(void);

/* Create a context for an Lx x Ly x Lz x Lt lattice (all even, 2 .. 32768,
 * volume at most 2^30) with
 * fermion time boundary phase t_bc (+1 periodic, -1 antiperiodic, Sec. 3.1
 * workload).  hip_stream: a hipStream_t (NULL = default stream). */
int wl_create(wl_lattice** out, const int32_t L[4], int32_t t_bc, void* hip_stream);
int wl_destroy(wl_lattice* lat);
int wl_set_stream(wl_lattice* lat, void* hip_stream);

/* Gauge links U (Sec. 2): copy canonical complex128 [4][V][3][3] in / out.
 * on_device = 1: U_canon is a device array on the context's device (stream
 * ordered); on_device = 0: a host array, staged through a workspace buffer of
 * the context (64 V bytes, kept), and the call synchronises the stream before
 * it returns, so the host array may be reused at once.  The caller keeps
 * ownership of U_canon.  WL_EINVAL for a null array or another flag value. */
int wl_set_links(wl_lattice* lat, const void* U_canon, int on_device);
int wl_get_links(wl_lattice* lat, void* U_canon, int on_device);

/* Bytes of one internal half-lattice spinor field of nrhs right-hand sides. */
int wl_field_bytes(const wl_lattice* lat, wl_prec prec, int nrhs, size_t* bytes);

/* Canonical half-lattice spinors (complex128 [nrhs][V/2][4][3]) <-> internal. */
int wl_import_spinor(wl_lattice* lat, void* dst_internal, const void* src_canon, wl_prec prec, int nrhs);
int wl_export_spinor(wl_lattice* lat, void* dst_canon, const void* src_internal, wl_prec prec, int nrhs);
/* Canonical full spinor (complex128 [V][4][3]) <-> internal F64 full field. */
int wl_import_full(wl_lattice* lat, void* dst_internal_full, const void* src_canon);
int wl_export_full(wl_lattice* lat, void* dst_canon, const void* src_internal_full);
/* Canonical su(3) field float64 [4][V][8] <-> internal float64 [2][4][8][V/2]. */
int wl_import_su3(wl_lattice* lat, double* dst_internal, const double* src_canon);
int wl_export_su3(wl_lattice* lat, double* dst_canon, const double* src_internal);

/* Wilson hopping operator, one even-odd block (Sec. 3.1; formula above):
 * out (parity out_parity) = D_{p,1-p} in, or the same block of D^dag when
 * dagger != 0.  in/out: internal half fields, nrhs right-hand sides, in the
 * storage precision prec (F64 computes in FP64, F32/BF16 in FP32). */
int wilson_dslash(wl_lattice* lat, void* out, const void* in, int out_parity, int dagger,
                  wl_prec prec, int nrhs);

/* Operators built from the hop (Sec. 2 and 3.1). */
typedef enum {
  WL_OP_M = 0,        /* full lattice M = 1 - kappa D; FULL internal fields, nrhs = 1 */
  WL_OP_MDAG = 1,     /* full lattice M^dag */
  WL_OP_K = 2,        /* full lattice K = M^dag M */
  WL_OP_MHAT = 3,     /* even sites: M-hat = 1 - kappa^2 D_eo D_oe */
  WL_OP_MHAT_DAG = 4, /* even sites: M-hat^dag */
  WL_OP_J = 5         /* even sites: J = K-hat + mu2[r] (K-hat when mu2 = 0) */
} wl_op;

/* out = op(in).  kappa: hopping parameter.  mu2: host array of nrhs shifts
 * (only WL_OP_J reads it; may be NULL = all zero).  Precision as wilson_dslash. */
int apply_K(wl_lattice* lat, void* out, const void* in, double kappa, const double* mu2, int nrhs,
            wl_op op, wl_prec prec);

/* apply_K without device allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operators, kernels and results as apply_K, with the
 * operator's intermediates in a fixed 256 MiB device scratch array that the
 * library holds on every device it runs on until the process ends (set up
 * when a context is created on that device).  Scratch needed: WL_OP_J two
 * internal half fields of nrhs rhs, WL_OP_MHAT / WL_OP_MHAT_DAG one,
 * WL_OP_K one full field, WL_OP_M / WL_OP_MDAG none.  WL_EINVAL (and
 * nothing launched) when that exceeds 256 MiB.  Every call on one device
 * shares that device's scratch: calls that overlap on one device (other
 * streams or threads) race.  Hop timing samples (wl_profile) are not taken. */
int apply_K_noalloc(wl_lattice* lat, void* out, const void* in, double kappa, const double* mu2, int nrhs,
                    wl_op op, wl_prec prec);

/* Conjugate gradient (Sec. 2: inversion of K by CG) on op = WL_OP_J (even
 * sites, nrhs right-hand sides, shifts mu2[r]) or WL_OP_K (full lattice,
 * nrhs = 1).  x0 = 0, or the contents of x when use_x0 = 1 (then r = b - A x0
 * in FP64; a rhs whose x0 already meets tol takes 0 iterations; x of a zero
 * source is set to 0); stops when the FP64 true residual |b - A x| <= tol |b|
 * for every rhs.  inner = WL_F64 runs plain FP64 CG; WL_F32 / WL_BF16 run the
 * inner iteration with that storage (FP32 arithmetic, FP64 dot products, the
 * steps accumulated in an FP32 copy of x that is added to the FP64 x before
 * each update) and FP64 reliable updates r = b - A x whenever the iterated
 * residual fell by delta since the last update.  x and b: internal F64 fields.  stats: host
 * array of nrhs entries (may be NULL).  Returns WL_ENOCONV, with x the last
 * iterate and stats filled, if some rhs misses tol within maxiter, or keeps
 * breaking down (a non-positive <p, A p>: an operator that is not positive
 * definite) through several restarts; WL_EINVAL for a non-finite |b|^2 (NaN or
 * Inf in b). */
typedef struct {
  double tol;      /* relative true-residual target, e.g. 1e-10 */
  int maxiter;     /* per rhs */
  wl_prec inner;   /* precision of the inner iteration */
  double delta;    /* reliable-update threshold (0 -> 0.1) */
  int chunk;       /* iterations between host convergence checks (0 -> 8) */
  int use_graph;   /* capture each chunk as a hipGraph and replay it */
  int use_x0;      /* 1: x holds the initial guess on entry (else x0 = 0) */
} wl_cg_params;

typedef struct {
  int iters;
  int reliable_updates;
  int converged;
  double true_rel_res;
} wl_cg_stats;

int cg_solve(wl_lattice* lat, void* x, const void* b, double kappa, const double* mu2, int nrhs,
             wl_op op, const wl_cg_params* params, wl_cg_stats* stats);

/* Multi-shift CG: x_s = J(mu2[s])^-1 b for nshift Hasenbusch shifts of
 * K-hat(kappa) at once (the shifted systems share the Krylov space of the
 * smallest shift; Sec. 2 Hasenbusch mass preconditioning in its mu2 form).
 * b: nrhs even-site F64 fields; x: nshift * nrhs fields, x[s * nrhs + r]
 * solves shift s for source r.  FP64 arithmetic; each system stops at
 * |zeta|^2 |r|^2 <= tol^2 |b|^2 and is then checked by its FP64 true residual,
 * a miss refined by an ordinary CG (params.inner) on its residual.
 * params: tol, maxiter (base iterations; a refinement may take up to
 * max(maxiter, 10000)), chunk; inner only for the refinement; use_graph
 * ignored; use_x0 must be 0 (WL_EUNSUPPORTED otherwise).  stats: host array [nshift * nrhs], same
 * order as x (iters = base iterations until the system froze, plus any
 * refinement iterations; reliable_updates = 1 if refined).  WL_EINVAL for
 * nrhs outside 1..16, nshift * nrhs > 64, negative shifts; WL_ENOCONV if a
 * system misses tol (outputs valid). */
int cg_multishift(wl_lattice* lat, void* x, const void* b, double kappa, const double* mu2, int nshift, int nrhs,
                  const wl_cg_params* params, wl_cg_stats* stats);

/* Chebyshev filter polynomial (Sec. 2, polynomial filtering): order degree on
 * [a, b] approximating 1/x, 1 - x P(x) = T_{degree+1}(y(x)) / T_{degree+1}(y(0)),
 * y(x) = (b + a - 2x)/(b - a), or its quotient by a lower order (degree_div);
 * applied to J = K-hat(kappa) + mu2 (one shift for every rhs) on even sites.
 * P = Q^dag Q with Q built from P's roots of negative imaginary part (degree
 * and degree_div even for the Q modes).  in / out: internal half fields of
 * nrhs rhs in storage precision prec (F64 computes in FP64, F32 / BF16 in
 * FP32 with that storage between the steps), distinct buffers.  P runs the
 * real three-term recurrence (degree J applications, each step fused into the
 * epilogue of its J's last hop); P J one more J; Q and Q^dag the root factors.
 * WL_EINVAL for a degree outside 1..512, an interval without 0 < a < b, a
 * divisor order that does not divide, nrhs outside 1..16 or an unknown
 * precision. */
typedef struct {
  int degree;
  double a, b;
  int degree_div; /* 0: P = P_degree; else the quotient P_degree / P_degree_div of the
                     two-filter actions (Sec. 3.3 Q(K) = P_2 / P_1, Sec. 4.2 Q(J)): its
                     roots are those of P_degree that are not roots of P_degree_div,
                     which needs (degree_div + 1) | (degree + 1) and both even */
} wl_poly;

typedef enum { WL_POLY_P = 0, WL_POLY_PJ = 1, WL_POLY_Q = 2, WL_POLY_QDAG = 3 } wl_poly_mode;

int poly_filter_apply(wl_lattice* lat, void* out, const void* in, double kappa, double mu2,
                      const wl_poly* poly, wl_poly_mode mode, int nrhs, wl_prec prec);

/* Pseudofermion action terms (Sec. 2, 3.3, 4.1, 4.2).  Every term has its
 * operator J = K-hat(kappa) + mu2 on the even sites: the paper's Hasenbusch
 * matrix J = K(kappa') is kappa = kappa', mu2 = 0; mu2 > 0 is the shifted
 * form.  W = M-hat(kappa) + i sqrt(mu2) g5, so W^dag W = J.
 *   WL_TERM_KINV_FULL  phi^dag K^-1 phi, full lattice (two-flavour action, Sec. 2)
 *   WL_TERM_KINV       phi^dag J^-1 phi
 *   WL_TERM_RATIO      phi^dag W_n J^-1 W_n^dag phi: the Hermitian form of a
 *                      correction term J_n J^-1 (Sec. 2 J K^-1; Sec. 3.3
 *                      J_1 J_2^-1, J_2 K^-1), numerator W_n = M-hat(kappa_num)
 *                      + i sqrt(mu2_num) g5 (kappa_num = 0: kappa)
 *   WL_TERM_POLY       phi^dag P(J) phi  (P = P_n, or the quotient filter
 *                      P_n / P_n_div when poly.degree_div > 0)
 *   WL_TERM_POLYK_INV  phi^dag [P(J) J]^-1 phi
 * phi / chi: internal F64 fields (FULL for KINV_FULL, even half otherwise).
 * WL_EINVAL for negative shifts or kappas, WL_EUNSUPPORTED for a shifted
 * full-lattice term. */
typedef enum {
  WL_TERM_KINV_FULL = 0,
  WL_TERM_KINV = 1,
  WL_TERM_RATIO = 2,
  WL_TERM_POLY = 3,
  WL_TERM_POLYK_INV = 4
} wl_term_kind;

typedef struct {
  wl_term_kind kind;
  double kappa;
  double mu2;
  wl_poly poly;
  wl_cg_params cg;
  double kappa_num; /* RATIO numerator (0: kappa) */
  double mu2_num;   /* RATIO numerator shift */
} wl_term;

/* phi drawn from Gaussian chi so that S(phi) = chi^dag chi (Sec. 2 heatbath). */
int wl_heatbath(wl_lattice* lat, void* phi, const wl_term* term, const void* chi);
/* S_term(phi) to host *S. */
int wl_action(wl_lattice* lat, const wl_term* term, const void* phi, double* S);

/* Fermion force (Sec. 2: dS_F/dU): F += coeff * grad^a S_term, the Lie
 * derivatives d/de S(exp(i e T^a) U_mu(x)) at e = 0.  F: internal su(3)
 * field, accumulated.  S_out: optional host action value (NULL to skip).
 * The POLY and POLYK_INV forces run over the m root factors of Q and keep
 * 3m device fields of workspace while those fit in 16 GiB (the environment
 * variable WL_CHAIN_KEEP_BYTES, a byte count, replaces the bound), else they
 * recompute them (three more hops per factor, the same result). */
int fermion_force(wl_lattice* lat, double* F, const wl_term* term, const void* phi, double coeff,
                  double* S_out);
/* The link-derivative primitive: F += coeff * grad^a Re(A^dag D C) for full
 * internal F64 fields A and C. */
int wl_force_bilinear(wl_lattice* lat, double* F, const void* A_full, const void* C_full, double coeff);

/* Wilson plaquette gauge action S_G = beta sum (1 - Re tr U_p / 3) (the
 * gauge action of the HMC workload): F += coeff * grad^a S_G. */
int wl_gauge_force(wl_lattice* lat, double* F, double beta, double coeff);
/* Mean plaquette (1/6V) sum_{x,mu<nu} Re tr U_munu / 3 to host. */
int wl_plaquette(wl_lattice* lat, double* plaq);
/* T[eps] (Sec. 2): U -> exp(i eps P) U, FP64, then SU(3) reunitarisation. */
int wl_link_update(wl_lattice* lat, const double* P, double eps);

/* One HMC trajectory (Sec. 2) with the generalised multi-scale integrator
 * (Sec. 3.2): every term i has its own leapfrog or Omelyan scheme with
 * nsteps[i] steps on [0, tau]; the gauge action is scale nterms
 * (nsteps[nterms]); updates are overlaid by time.  P: internal su(3) momenta,
 * read at the start and left at the end point.  chi: nterms internal F64
 * fields back to back (each a FULL field for KINV_FULL, else a half field).
 * u_metropolis: caller's uniform in [0,1); accept iff u < exp(-dH).  On
 * rejection the links are restored.  flags: WL_HMC_NO_METROPOLIS always keeps
 * the end point; WL_HMC_PHI_GIVEN takes chi as the pseudofermions themselves
 * and skips the heatbath (both for reversibility tests); WL_HMC_CHRONO starts
 * every force solve of a term from the chronological guess over that term's
 * last chrono_depth force solutions in the trajectory: the vector of their
 * span with the least A-norm error (minimal-residual extrapolation; chrono_depth
 * extra operator applications per solve).  Fewer iterations; the solutions
 * still meet the solver tolerance, so the trajectory is reversible to that
 * tolerance (the reverse run sees other guesses) rather than exactly. */
enum { WL_HMC_NO_METROPOLIS = 1, WL_HMC_PHI_GIVEN = 2, WL_HMC_CHRONO = 4 };
enum { WL_INT_LEAPFROG = 0, WL_INT_OMELYAN = 1 };

typedef struct {
  double beta;
  double tau;
  double omelyan_lambda; /* 0 -> 0.1931833275037836 */
  int integrator;        /* WL_INT_LEAPFROG or WL_INT_OMELYAN */
  int nterms;            /* <= 8 */
  wl_term terms[8];
  int nsteps[9];         /* per term, then the gauge action */
  int flags;
  int chrono_depth;      /* WL_HMC_CHRONO: solutions kept per term, 1..8 (0 -> 4) */
} wl_hmc_params;

typedef struct {
  double dH, H0, H1;
  double S0[9], S1[9];   /* per term, then gauge */
  double plaquette;      /* of the links the call leaves */
  int accepted;
  long long n_kmat;      /* K multiplications (the cost numerator N_mat of Sec. 3.1; rule at wl_counters) */
  long long cg_iters;
} wl_hmc_result;

int hmc_trajectory(wl_lattice* lat, const wl_hmc_params* params, double* P, const void* chi,
                   double u_metropolis, wl_hmc_result* result);

/* Mixed-volume batches: several lattices (different extents, links and kappa;
 * one device and one stream) whose hops run as ONE persistent launch, with the
 * even-odd J and a CG over the batch on top (the multi-rhs CG of Sec. 2 with
 * one system per lattice).  The batch keeps pointers to the lattices: destroy
 * it before them.  A batch field is nlat slots of wl_batch_slot_bytes each;
 * slot l holds lattice l's internal even-site field (as wl_import_spinor
 * writes it) followed by zeros: allocate batch fields zeroed, the library only
 * writes the lattices' own sites.  Calls run on the lattices' stream, use the
 * largest lattice's workspace and CG state, and synchronise like their
 * single-lattice counterparts; batch hops are not counted by wl_hop_counts.
 * WL_EINVAL for nlat outside 1..8 or lattices on other devices or streams. */
typedef struct wl_batch wl_batch;
int wl_batch_create(wl_batch** out, wl_lattice* const* lats, int nlat);
int wl_batch_destroy(wl_batch* batch);
int wl_batch_slot_bytes(const wl_batch* batch, wl_prec prec, size_t* bytes);
/* slot l of out = D_{p,1-p} (dagger: its adjoint) of slot l of in, every
 * lattice in one launch (p = out_parity) */
int wl_batch_dslash(wl_batch* batch, void* out, const void* in, int out_parity, int dagger, wl_prec prec);
/* slot l of out = (K-hat(kappa[l]) + mu2[l]) slot l of in (mu2 may be NULL) */
int wl_batch_apply_J(wl_batch* batch, void* out, const void* in, const double* kappa, const double* mu2,
                     wl_prec prec);
/* CG on every slot's J as in cg_solve (params.inner, reliable updates, graph
 * chunks, use_x0 = 0 only): stats[nlat]; WL_ENOCONV if some lattice misses tol. */
int wl_batch_cg_solve(wl_batch* batch, void* x, const void* b, const double* kappa, const double* mu2,
                      const wl_cg_params* params, wl_cg_stats* stats);

/* The overlaid schedule used by hmc_trajectory (Sec. 3.2), host only, no
 * device needed: nscales schemes with nsteps[i] steps; event k is
 * kinds[k] = 0 (S update of scale terms[k], step weights[k] tau) or 1 (T step
 * of weights[k] tau, terms[k] = -1).  Host arrays of max_events entries (any
 * may be NULL); *n_events gets the count (WL_EINVAL if it exceeds max_events). */
int wl_integrator_schedule(const int* nsteps, int nscales, int scheme, double lambda, int* kinds, int* terms,
                           double* weights, int max_events, int* n_events);

/* Counters since create.  n_hop: hop launches in single-rhs units (graph
 * replays included).  n_kmat: the cost count of Sec. 3.1, fermion-matrix K
 * multiplications, one per rhs for each application of a term's K-type
 * operator J = K-hat(kappa) + mu2 or the full-lattice K:
 *   * apply_K with WL_OP_J / WL_OP_K: 1;  WL_OP_M, MDAG, MHAT, MHAT_DAG and
 *     wilson_dslash: 0 (parts of a multiplication);
 *   * a CG on J or K: 1 per iteration of each rhs until that rhs converges,
 *     plus 1 per rhs for each FP64 residual b - A x (reliable updates, the
 *     final check, the start from a given x0); iterations a chunk issues
 *     past a rhs's convergence are not counted;
 *   * a polynomial: P_n(J) n, a quotient P_n / P_m 2q (q = its root factors
 *     of Q), P(J) J one more, Q(J) and Q(J)^dag q; a CG on P(J) or P(J) J
 *     counts its operator applications as above times these;
 *   * a J assembled inside a force chain from fields already multiplied by
 *     M-hat: 1.
 * The multi-shift CG counts one per base iteration (the shifted systems
 * share its J) and one per rhs for each residual; mixed-volume batch J: 1 per
 * lattice per launch. */
int wl_counters(const wl_lattice* lat, long long* n_hop, long long* n_kmat);
/* Tracing of the cost count: wl_solve_log(lat, 1) clears and starts a log of
 * every CG the context runs (cg_solve, the solves inside heatbaths, actions,
 * forces and trajectories; not the multi-shift or batch solvers);
 * wl_solve_log(lat, 0) stops and clears.  wl_solve_log_read copies, per
 * solve in order, the iterations summed over its rhs, its FP64 residual
 * applications (summed over rhs) and the K multiplications per operator
 * application (1 for J / K, the polynomial's count for P(J) and P(J) J)
 * into host arrays of max entries (any may be NULL); *n = the number of
 * solves (WL_EINVAL if above max). */
int wl_solve_log(wl_lattice* lat, int enable);
int wl_solve_log_read(const wl_lattice* lat, int max, int* n, long long* iters, long long* residuals,
                      long long* jpa);
/* Hop launch configuration, kept per storage precision and per rhs-count
 * class (kind 0: one rhs; 1: 2-4 rhs; 2: 5-16 rhs):
 *   variant  0 = one thread per output site (all 8 directions);
 *            1 = direction-parallel (8 wavefronts, one per direction, over 64
 *                sites, combined through LDS);
 *            2 = one thread per output site with the links shared: a
 *                workgroup takes one 64-site tile for four rhs (one
 *                wavefront each), reads the tile's 8 x 64 links once into
 *                LDS and gives variant 0's results bit for bit (from 4 rhs
 *                on; with fewer, variant 0 runs);
 *   npass    direction-parallel: up to npass (1, 2, 4) passes of 1 (FP64) or
 *            2 (FP32, BF16, even rhs counts) rhs reuse each link held in
 *            registers; site: 2 = two rhs per thread (FP32, BF16, even rhs
 *            counts), else one;
 *   use_xcd  the workgroup order: 1 = renumbered so that each of the 8 XCDs
 *            walks a contiguous range of sites; 0 = the hardware's round-robin
 *            order (several rhs groups of one tile on one XCD); 2 = z-blocked
 *            round-robin: 8 z planes at a time through every t, so that a
 *            site's t neighbours are read within a few hundred workgroups of
 *            each other, each XCD keeping its own 64-site columns of the z
 *            planes (valid where a z plane holds a multiple of 8 tiles of 64
 *            sites and Lz is a multiple of 8 above 8);
 *   stream   1 = non-temporal loads of links and epilogue operands and
 *            non-temporal output stores (pays on volumes beyond the caches),
 *            0 = ordinary cached access.
 * Results are identical for every npass and use_xcd, and for variants 0 and
 * 2; stream and variant 1 against the others change them by rounding only
 * (stream: the compiler's contraction of products into FMAs may differ;
 * variant 1: the summation order of the 8 directions).
 * wl_set_hop_config sets one class (kind = -1: all three); WL_EINVAL for
 * values outside these sets.  wl_get_hop_config reads one class (outputs may
 * be NULL).
 * wl_autotune times on this lattice, for every precision, class 0 at 1 rhs
 * over {site, direction-parallel}, classes 1 and 2 at 4 and 8 rhs over
 * {site npass 1, 2; site with shared links; direction-parallel npass 1, 2,
 * 4}, each candidate with
 * (stream, use_xcd) = (0, 1), (0, 0), (0, 2), (1, 1), (1, 0), (1, 2), as
 * bursts in which each launch reads the previous launch's output (best of 3
 * bursts of 20), and keeps the fastest of every class.  stream = 1 is a
 * candidate only where the hop's working set (links and two fields of that
 * class) exceeds the 256 MiB last-level cache, use_xcd = 2 only where valid.
 * us_out: optional host array of 3 x 84 microseconds per launch (0 for
 * candidates not timed), per precision (F64, F32, BF16): 12 for class 0 (site,
 * dp per (stream, use_xcd) in that order), then 36 for class 1 and 36 for
 * class 2 (site 1, site 2, shared, dp 1, dp 2, dp 4 per (stream, use_xcd)). */
int wl_set_hop_config(wl_lattice* lat, wl_prec prec, int kind, int variant, int npass, int use_xcd, int stream);
int wl_get_hop_config(const wl_lattice* lat, wl_prec prec, int kind, int* variant, int* npass, int* use_xcd,
                      int* stream);
int wl_autotune(wl_lattice* lat, double* us_out);
/* Tracing: average duration in microseconds of back-to-back hop launches
 * (current configuration for nrhs right-hand sides, two scratch fields owned
 * by the library, each launch reading the previous one's output), timed with
 * HIP events on the context stream: 100 warm-up launches, then the median
 * over 5 sub-bursts of nlaunch/5.  Not counted in the hop counters. */
int wl_time_hop(wl_lattice* lat, wl_prec prec, int nrhs, int nlaunch, double* avg_us);
/* Tracing: the practical HBM ceiling: a plain copy of bytes (multiple of 16,
 * at most 16 GiB) between two library buffers, reps times, alternating the
 * direction so that each copy reads the previous one's output; *gbs = bytes
 * read plus written per second (GB/s). */
int wl_stream_copy(wl_lattice* lat, size_t bytes, int reps, double* gbs);

/* Hop applications since create per storage precision (counts[wl_prec], single rhs units). */
int wl_hop_counts(const wl_lattice* lat, long long* counts);

/* Tracing: wl_profile(lat, 1) clears and starts HIP-event timing of sampled
 * single-rhs hop launches (at most 4096 per storage precision, none inside a
 * graph capture); wl_profile_read() synchronises and returns the average
 * launch duration in microseconds and the sample count per precision
 * (index = wl_prec).  wl_profile(lat, 0) stops and clears. */
int wl_profile(wl_lattice* lat, int enable);
int wl_profile_read(wl_lattice* lat, double* avg_us, long long* samples);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_HMC_H */
