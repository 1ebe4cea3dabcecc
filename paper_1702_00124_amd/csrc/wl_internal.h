// Host-side internals of libwilson_hmc: the lattice context, workspace,
// error reporting and the kernel launchers shared between translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/wilson_hmc.h"
#include "wl_device.h"

namespace wl {

constexpr int kMaxRhs = 16;
constexpr int kTuneRhs[3] = {1, 4, 8};  // rhs counts the autotuner times each hop class at
constexpr size_t kLastLevelCache = size_t(256) << 20;  // MI355X Infinity Cache
constexpr int kBlock = 256;  // threads per workgroup of the site kernels
constexpr int kScal = 2048;  // device scalar slots; the CG state starts at kCgState
constexpr int kCgState = 1024;
constexpr int kProfPairs = 4096;  // sampled hop launches timed per precision
enum HopVariant { kHopSite = 0, kHopDirParallel = 1, kHopSiteShared = 2 };
// how a hop is launched: kernel variant; npass = direction-parallel: most rhs
// passes per link held in registers (1, 2, 4), site: rhs per thread (1, 2);
// use_xcd = workgroup order: 1 XCD-contiguous ranges, 0 the hardware's
// round-robin, 2 z-blocked round-robin (kZBlock z planes at a time through
// every t, so a tile's t neighbours follow it within a few hundred
// workgroups; valid where zblock_ok);
// stream = non-temporal link and epilogue loads and output stores
struct HopConfig {
  int variant, npass, use_xcd, stream;
};
constexpr int kZBlock = 8;
// the z-blocked order needs whole 64-site tiles per z plane, a multiple of 8
// of them (so a tile's z and t neighbours share its XCD) and Lz a multiple of
// kZBlock above it
inline bool zblock_ok(const Geo& g) {
  const long long plane = (long long)g.Lxh * g.L[1];
  return plane % 64 == 0 && (plane / 64) % 8 == 0 && g.L[2] % kZBlock == 0 && g.L[2] > kZBlock;
}
// rhs-count classes with their own configuration: 1, 2-4, 5-16
constexpr int kHopKinds = 3;
inline int hop_kind(int nrhs) { return nrhs <= 1 ? 0 : (nrhs <= 4 ? 1 : 2); }

enum Prec { F64 = WL_F64, F32 = WL_F32, BF16 = WL_BF16 };

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define WL_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::wl::Error(WL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define WL_REQUIRE(cond, code, msg)         \
  do {                                      \
    if (!(cond)) throw ::wl::Error(code, msg); \
  } while (0)

// bytes of one half-lattice spinor field (padded to whole 64-site tiles)
// Bytes of one rhs of an even-odd spinor field: the tiled sites, rounded up to
// 4 KiB, plus a stagger so that the rhs of a batch (and the halves of a full
// field) do not start at addresses congruent modulo the L2 set span: a stride
// that is a multiple of a large power of two maps the same site of every rhs
// to one L2 set and one memory channel.
constexpr size_t kFieldStagger = size_t(37) << 12;  // 148 KiB: odd multiple of 4 KiB
inline size_t spinor_bytes(Prec p, int Vh) {
  const size_t raw = size_t(p == F64 ? 192 : (p == F32 ? 96 : 48)) * size_t(padded_sites(Vh));
  return ((raw + 4095) & ~size_t(4095)) + kFieldStagger;
}
// bytes of the two-row hop links of one precision: 2 parities x 4 directions
inline size_t links_bytes(Prec p, int Vh) {
  return size_t(8) * size_t(p == F64 ? 96 : (p == F32 ? 48 : 24)) * size_t(padded_sites(Vh));
}
// bytes of the full FP64 links (3 rows)
inline size_t full_links_bytes(int Vh) { return size_t(8) * 144 * size_t(padded_sites(Vh)); }
inline size_t link_bytes(Prec p) { return p == F64 ? 96 : (p == F32 ? 48 : 24); }

}  // namespace wl

// Opaque context of the C-ABI.  Owns packed links (FP64 and derived low
// precision copies), momentum backup, reduction partials and a workspace of
// named device buffers.
struct wl_lattice {
  wl::Geo geo;
  int L[4];
  int V, Vh;
  hipStream_t stream;
  int device;
  void* Ufull = nullptr;                     // FP64 links, all 3 rows (forces, gauge, updates)
  void* U[3] = {nullptr, nullptr, nullptr};  // hop links F64 / F32 / BF16, first two rows
  bool lowp_valid = false;                   // U[*] match Ufull
  double* partials = nullptr;                // reduction partials
  size_t partials_len = 0;
  double* dscal = nullptr;                   // device scalars [kScal]: results, then CG state
  double* hscal = nullptr;                   // pinned host mirror
  hipStream_t capture_stream = nullptr;      // side stream for hipGraph capture
  std::map<std::string, std::pair<void*, size_t>> ws;
  // bumped whenever a workspace buffer or the partials are freed (grown): a
  // captured graph that holds their old addresses must be captured again
  long long ws_gen = 0;
  long long n_hop = 0;                       // hop applications (single rhs units)
  long long n_hop_p[3] = {0, 0, 0};          // ... per storage precision
  long long n_kmat = 0;                      // K-hat / K applications (single rhs units)
  // hop launch configuration per storage precision and rhs-count class
  wl::HopConfig hop_cfg[3][wl::kHopKinds] = {
      {{wl::kHopDirParallel, 1, 1, 0}, {wl::kHopDirParallel, 4, 1, 0}, {wl::kHopDirParallel, 4, 1, 0}},
      {{wl::kHopDirParallel, 1, 1, 0}, {wl::kHopDirParallel, 4, 1, 0}, {wl::kHopDirParallel, 4, 1, 0}},
      {{wl::kHopSite, 1, 1, 0}, {wl::kHopSite, 1, 1, 0}, {wl::kHopSite, 1, 1, 0}}};
  // optional event timing of sampled hop launches, per storage precision
  int prof_on = 0;
  int prof_capturing = 0;
  int prof_suspended = 0;               // set by entry points that must not create events
  // optional log of the solves (wl_solve_log): iterations summed over rhs,
  // FP64 residual applications, K multiplications per operator application
  int solve_log_on = 0;
  std::vector<std::array<long long, 3>> solve_log;
  std::vector<hipEvent_t> prof_ev[3];   // start/stop pairs
  double prof_ms[3] = {0, 0, 0};
  long long prof_n[3] = {0, 0, 0};
};

namespace wl {

// workspace: named device buffer of at least `bytes`, kept for the lifetime of
// the context (grown on demand)
void* ws_get(wl_lattice* L, const std::string& name, size_t bytes);
void ensure_partials(wl_lattice* L, size_t n);
void ensure_lowp_links(wl_lattice* L);
inline int site_blocks(int n) { return (n + kBlock - 1) / kBlock; }

// ------------------------------------------------------------------ hop
struct HopEpi {
  const void* x = nullptr;  // same-parity field (precision of the hop)
  double cx = 1.0;
  double a = 1.0;           // coefficient of the hop
  int g5 = 0;               // gamma_5 applied to (cx x + a hop)
  const void* y = nullptr;  // + by[r] y
  double by[kMaxRhs] = {0};
  int dot = 0;              // 0 none, 1 Re<dotv, out>, 2 |out|^2 into partials
  const void* dotv = nullptr;
  double* partials = nullptr;
  int part_stride = 0;      // per-rhs stride of partials
  int part_off = 0;         // block offset inside a rhs row
  // fused Chebyshev step (forward hop, no dot; out is not written): for
  // every rhs, with w the result above, cheb_tprev <- ct t + cw w - cheb_tprev
  // and cheb_eprev <- ce e + 2 t - cheb_eprev (t = cheb_t, e = cheb_e; fields
  // of nrhs rhs laid out as the hop's)
  const void* cheb_t = nullptr;
  void* cheb_tprev = nullptr;
  const void* cheb_e = nullptr;
  void* cheb_eprev = nullptr;
  double cheb_ct = 0.0, cheb_cw = 0.0, cheb_ce = 0.0;
};
// workgroups (and reduction partials per rhs) of one hop launch in precision prec
int hop_tiles(const wl_lattice* L, Prec prec);

// mixed-volume batch: one hop per lattice (one rhs each) in a single launch;
// with e.dot = 1, e.partials is the lattice's row of part_len partial sums
// (entries past its tiles are cleared).  Only x, cx, a, g5, y, by[0], dot,
// dotv and partials of the epilogue apply.  Not counted in the hop counters.
constexpr int kMaxBatch = 8;
struct BatchHop {
  wl_lattice* L;
  void* out;
  const void* in;
  HopEpi e;
};
void launch_hop_batch(hipStream_t st, Prec prec, int out_parity, int dagger, const BatchHop* hops, int nlat,
                      int part_len);
// out (parity p, nrhs fields) = epilogue(D_{p,1-p} in) or its dagger
void launch_hop(wl_lattice* L, Prec prec, void* out, const void* in, int out_parity, int dagger,
                int nrhs, const HopEpi& e);

// ------------------------------------------------------------------ BLAS-1 (blas.hip)
int blas_blocks(const wl_lattice* L);
// x += alpha[r] p ; r -= alpha[r] Ap ; partial |r|^2   (p, r, Ap in prec; x in
// xprec: F64, or F32 when prec is F32 or BF16); alpha and the done flags are
// read from the device CG state st (nh = 2 when every rhs is a full-lattice
// field of two halves)
void launch_cg_update(wl_lattice* L, Prec prec, Prec xprec, void* x, void* r, const void* p, const void* Ap,
                      const double* st, int nrhs, int nh, double* partials, int stride);
// x64 += x32, x32 = 0 (nf fields; x64 F64, x32 F32)
void launch_cg_fold(wl_lattice* L, void* x64, void* x32, int nf);
// p = r + beta[r] p
void launch_cg_xpay(wl_lattice* L, Prec prec, void* p, const void* r, const double* st, int nrhs, int nh);
// the CG iteration's two vector kernels with alpha and beta derived inside
// (the operator's <p, A p> partial sums: rows of pstride, nb_dot entries; the
// |r|^2 partial sums go to rr_partials, rows of pstride, nh * blas blocks entries)
void launch_cg_update_fused(wl_lattice* L, Prec prec, Prec xprec, void* x, void* r, const void* p, const void* Ap,
                            double* st, int nrhs, int nh, const double* dot_partials, int nb_dot,
                            double* rr_partials, int pstride);
void launch_cg_xpay_fused(wl_lattice* L, Prec prec, void* p, const void* r, double* st, int nrhs, int nh,
                          const double* rr_partials, int nb_rr, int pstride);
// dst = convert(src), both nrhs half fields
void launch_convert(wl_lattice* L, Prec dprec, void* dst, Prec sprec, const void* src, int nrhs);
// out = a[r] x + b[r] (g5 ? gamma5 y : y), complex coefficients; x or y may be null
void launch_caxpby(wl_lattice* L, void* out, const double* a /*2*nrhs host*/, const void* x,
                   const double* b /*2*nrhs host*/, const void* y, int g5y, int nrhs, Prec prec = F64);
// partials of <x, y> (complex, 2 values per block) or |x|^2 over nrhs fields (FP64 sums)
void launch_dot_partials(wl_lattice* L, const void* x, const void* y, int nrhs, double* partials,
                         int stride, int complex_dot, Prec prec = F64);
// sum partials: out[r * ncomp + c] = sum_b partials[(r * ncomp + c) * stride + b], b < nb
void launch_finish_sum(wl_lattice* L, const double* partials, int stride, int nb, int nrows,
                       double* out_dev);
// plain device copy of bytes (multiple of 16) from a to b
void launch_stream_copy(wl_lattice* L, const void* a, void* b, size_t bytes);
// Chebyshev recurrence start (t0 = in, e0 = 0, e1 = in) and end (out = s (ce e + 2 t - eprev)), nrhs fields
void launch_cheb_init(wl_lattice* L, const void* in, void* t0, void* e0, void* e1, Prec prec, int nrhs = 1);
void launch_cheb_last(wl_lattice* L, const void* t, const void* e, const void* eprev, void* out, double ce, double s,
                      Prec prec, int nrhs = 1);
// CG scalar steps on the device state (see solver.cpp for the layout)
void launch_cg_alpha(wl_lattice* L, const double* partials, int stride, int nb, double* st, int nrhs);
void launch_cg_beta(wl_lattice* L, const double* partials, int stride, int nb, double* st, int nrhs);
// multi-shift CG steps (FP64 fields [nshift][nrhs]; state layout in wl_solver_state.h)
void launch_ms_scalars(wl_lattice* L, double* st, double* ms, double* mr, int nrhs, int nshift);
void launch_ms_update(wl_lattice* L, void* r, const void* Ap, const void* p, void* x, const double* st,
                      const double* ms, int nrhs, int nshift, double* partials, int pstride);
void launch_ms_xpay(wl_lattice* L, void* p, const void* r, const double* st, const double* ms, int nrhs, int nshift);

// ------------------------------------------------------------------ pack (pack.hip)
void launch_pack_links(wl_lattice* L, const void* canon);
void launch_unpack_links(wl_lattice* L, void* canon);
void launch_lowp_links(wl_lattice* L);
void launch_import_spinor(wl_lattice* L, Prec prec, void* dst, const void* canon, int nrhs);
void launch_export_spinor(wl_lattice* L, Prec prec, void* canon, const void* src, int nrhs);
void launch_split_full(wl_lattice* L, void* even, void* odd, const void* canon_full, int to_canon);
void launch_su3_io(wl_lattice* L, double* internal, const double* canon, int to_canon);

// ------------------------------------------------------------------ force / gauge (force.hip)
// F (or P) [parity][mu][8][Vh] += coeff * grad Re(A^dag D C), A and C full fields given as halves
void launch_bilinear(wl_lattice* L, double* F, const void* Ae, const void* Ao, const void* Ce,
                     const void* Co, double coeff);
void launch_gauge_force(wl_lattice* L, double* F, double coeff);  // F += coeff * grad S_G / beta
void launch_link_update(wl_lattice* L, const double* P, double eps);
void launch_plaquette_partials(wl_lattice* L, double* partials);  // per block, nb = 2 * site_blocks(Vh)
void launch_su3_sumsq_partials(wl_lattice* L, const double* P, double* partials);
void launch_unitarity_partials(wl_lattice* L, double* partials);  // max |U U^dag - 1|

}  // namespace wl
