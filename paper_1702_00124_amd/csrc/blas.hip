// Level-1 vector kernels of the solvers and of the polynomial filter, with
// dot products accumulated in FP64 at every storage precision, and the
// device-side scalar steps of conjugate gradient (alpha, beta, convergence
// flag), so that a CG iteration needs no host round trip.
//
// Reductions are deterministic: each workgroup writes one partial per rhs
// (wavefront shuffles, then LDS), and a single workgroup per rhs sums the
// partials in a fixed order.
#include "wl_internal.h"
#include "wl_solver_state.h"

namespace wl {

int blas_blocks(const wl_lattice* L) { return site_blocks(L->Vh); }

// block of an elementwise site kernel in the same XCD-contiguous order, so
// that each XCD touches the site range it handles in the hop kernels; the
// per-block partial sums are indexed by it too (same order, same sums)
__device__ __forceinline__ int site_block() { return xcd_block(blockIdx.x, gridDim.x); }

// ------------------------------------------------------------------ CG update
// fields are indexed f = rhs * nh + half (nh = 2 for full-lattice fields)
// (the iterate x is held in XP: FP64, or FP32 between a mixed CG's reliable updates)
template <typename P, typename XP>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(Geo g, char* xacc, char* r, const char* p,
                                                          const char* Ap, const double* st, size_t stride,
                                                          size_t stridex, double* partials, int pstride, int nh) {
  using R = typename P::real;
  __shared__ double lds[kBlock / 64];
  const int f = blockIdx.y;
  const int rhs = f / nh;
  const int h = site_block() * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  const double alpha = st[CG_ALPHA * kMaxRhs + rhs];
  const bool done = st[CG_DONE * kMaxRhs + rhs] != 0.0;
  double part = 0.0;
  if (h < Vh && !done) {
    const size_t off = f * stride;
    Spinor<R> pv = SpinorIO<P>::load(p + off, h, Vh);
    Spinor<R> av = SpinorIO<P>::load(Ap + off, h, Vh);
    Spinor<R> rv = SpinorIO<P>::load(r + off, h, Vh);
    using XR = typename XP::real;
    char* xb = xacc + f * stridex;
    Spinor<XR> xv = SpinorIO<XP>::load(xb, h, Vh);
    const R ar = R(alpha);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xv.c[k].r = XR(double(xv.c[k].r) + alpha * double(pv.c[k].r));
      xv.c[k].i = XR(double(xv.c[k].i) + alpha * double(pv.c[k].i));
      rv.c[k] = rv.c[k] - ar * av.c[k];
    }
    SpinorIO<XP>::store(xb, h, Vh, xv);
    SpinorIO<P>::store(r + off, h, Vh, rv);
#pragma unroll
    for (int k = 0; k < 12; ++k) part += double(rv.c[k].r) * double(rv.c[k].r) + double(rv.c[k].i) * double(rv.c[k].i);
  }
  const double s = block_sum(part, lds);
  if (threadIdx.x == 0) partials[rhs * pstride + (f % nh) * gridDim.x + site_block()] = s;
}

// ------------------------------------------------------------------ fused CG scalars
// One CG iteration after the operator is two kernels instead of four: every
// block sums the partial-sum row it needs itself (the same entries in the same
// order, so every block gets the same value) and derives alpha or beta; one
// block records the scalars.  Within a kernel the state is only written where
// no other block reads it, or as flags that go from 0 to 1 under a condition
// every block evaluates the same way.
__device__ __forceinline__ double row_sum_all(const double* row, int nb, double* lds) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += row[b];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) lds[0] = s;
  __syncthreads();
  const double v = lds[0];
  __syncthreads();
  return v;
}

// alpha = |r|^2 / <p, A p> from the operator's partial sums (row rhs of pstride,
// nb_dot entries), then x += alpha p, r -= alpha A p and the |r|^2 partial sums
// into rr_partials (row rhs of pstride)
template <typename P, typename XP>
__global__ __launch_bounds__(kBlock) void cg_update_fused_kernel(Geo g, char* xacc, char* r, const char* p,
                                                                const char* Ap, double* st, size_t stride,
                                                                size_t stridex, const double* dot_partials,
                                                                int nb_dot, double* rr_partials, int pstride,
                                                                int nh) {
  using R = typename P::real;
  __shared__ double lds[kBlock / 64];
  const int f = blockIdx.y;
  const int rhs = f / nh;
  const int blk = site_block();
  const int h = blk * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  const double pAp = row_sum_all(dot_partials + size_t(rhs) * pstride, nb_dot, lds);
  const bool done = st[CG_DONE * kMaxRhs + rhs] != 0.0;
  const bool ok = pAp > 0.0 && pAp < 1e300;  // A is HPD: <p, A p> positive and finite
  const bool brk = st[CG_BREAK * kMaxRhs + rhs] != 0.0 || (!done && !ok);
  const double rr = st[CG_RR * kMaxRhs + rhs];
  const double alpha = (done || brk) ? 0.0 : rr / pAp;
  if (blk == 0 && f % nh == 0 && threadIdx.x == 0) {
    st[CG_PAP * kMaxRhs + rhs] = pAp;
    st[CG_ALPHA * kMaxRhs + rhs] = alpha;
    st[CG_RROLD * kMaxRhs + rhs] = rr;
    if (brk) st[CG_BREAK * kMaxRhs + rhs] = 1.0;
  }
  double part = 0.0;
  if (h < Vh && !done && !brk) {
    const size_t off = f * stride;
    Spinor<R> pv = SpinorIO<P>::load(p + off, h, Vh);
    Spinor<R> av = SpinorIO<P>::load(Ap + off, h, Vh);
    Spinor<R> rv = SpinorIO<P>::load(r + off, h, Vh);
    using XR = typename XP::real;
    char* xb = xacc + f * stridex;
    Spinor<XR> xv = SpinorIO<XP>::load(xb, h, Vh);
    const R ar = R(alpha);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xv.c[k].r = XR(double(xv.c[k].r) + alpha * double(pv.c[k].r));
      xv.c[k].i = XR(double(xv.c[k].i) + alpha * double(pv.c[k].i));
      rv.c[k] = rv.c[k] - ar * av.c[k];
    }
    SpinorIO<XP>::store(xb, h, Vh, xv);
    SpinorIO<P>::store(r + off, h, Vh, rv);
#pragma unroll
    for (int k = 0; k < 12; ++k) part += double(rv.c[k].r) * double(rv.c[k].r) + double(rv.c[k].i) * double(rv.c[k].i);
  } else if (h < Vh && !done) {
    // broken down: r is left alone; its |r|^2 still goes to the partial sums
    const Spinor<R> rv = SpinorIO<P>::load(r + f * stride, h, Vh);
#pragma unroll
    for (int k = 0; k < 12; ++k) part += double(rv.c[k].r) * double(rv.c[k].r) + double(rv.c[k].i) * double(rv.c[k].i);
  }
  const double s = block_sum(part, lds);
  if (threadIdx.x == 0) rr_partials[rhs * pstride + (f % nh) * gridDim.x + blk] = s;
}

// beta = |r_new|^2 / |r_old|^2 from the update's partial sums (nb_rr entries),
// the convergence and breakdown flags, then p = r + beta p
template <typename P>
__global__ __launch_bounds__(kBlock) void cg_xpay_fused_kernel(Geo g, char* p, const char* r, double* st,
                                                              size_t stride, const double* rr_partials, int nb_rr,
                                                              int pstride, int nh) {
  using R = typename P::real;
  __shared__ double lds[kBlock / 64];
  const int f = blockIdx.y;
  const int rhs = f / nh;
  const int blk = site_block();
  const int h = blk * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  const double rr_new = row_sum_all(rr_partials + size_t(rhs) * pstride, nb_rr, lds);
  const bool done_old = st[CG_DONE * kMaxRhs + rhs] != 0.0;
  const bool brk = st[CG_BREAK * kMaxRhs + rhs] != 0.0 || !(rr_new < 1e300);  // also catches NaN
  const bool conv = !brk && rr_new <= st[CG_TOL2 * kMaxRhs + rhs] * st[CG_BB * kMaxRhs + rhs];
  const bool done = done_old || conv;
  const double beta = (brk || done_old) ? 0.0 : rr_new / st[CG_RROLD * kMaxRhs + rhs];
  if (blk == 0 && f % nh == 0 && threadIdx.x == 0) {
    if (brk) st[CG_BREAK * kMaxRhs + rhs] = 1.0;
    st[CG_BETA * kMaxRhs + rhs] = beta;  // frozen at 0 once broken down, until the host restarts it
    if (!brk && !done_old) {
      st[CG_RR * kMaxRhs + rhs] = rr_new;
      st[CG_ITERS * kMaxRhs + rhs] += 1.0;
      if (rr_new > st[CG_MAXRR * kMaxRhs + rhs]) st[CG_MAXRR * kMaxRhs + rhs] = rr_new;
      if (conv) st[CG_DONE * kMaxRhs + rhs] = 1.0;
    }
  }
  if (h >= Vh || done) return;
  const R rb = R(beta);
  const size_t off = f * stride;
  Spinor<R> pv = SpinorIO<P>::load(p + off, h, Vh);
  const Spinor<R> rv = SpinorIO<P>::load(r + off, h, Vh);
#pragma unroll
  for (int k = 0; k < 12; ++k) pv.c[k] = rv.c[k] + rb * pv.c[k];
  SpinorIO<P>::store(p + off, h, Vh, pv);
}

template <typename P>
__global__ __launch_bounds__(kBlock) void cg_xpay_kernel(Geo g, char* p, const char* r, const double* st,
                                                        size_t stride, int nh) {
  using R = typename P::real;
  const int f = blockIdx.y;
  const int rhs = f / nh;
  const int h = site_block() * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  if (h >= Vh || st[CG_DONE * kMaxRhs + rhs] != 0.0) return;
  const R beta = R(st[CG_BETA * kMaxRhs + rhs]);
  const size_t off = f * stride;
  Spinor<R> pv = SpinorIO<P>::load(p + off, h, Vh);
  const Spinor<R> rv = SpinorIO<P>::load(r + off, h, Vh);
#pragma unroll
  for (int k = 0; k < 12; ++k) pv.c[k] = rv.c[k] + beta * pv.c[k];
  SpinorIO<P>::store(p + off, h, Vh, pv);
}

template <typename PD, typename PS>
__global__ __launch_bounds__(kBlock) void convert_kernel(Geo g, char* dst, size_t dstride, const char* src,
                                                        size_t sstride) {
  const int rhs = blockIdx.y;
  const int h = site_block() * kBlock + threadIdx.x;
  if (h >= g.Vh) return;
  const auto s = SpinorIO<PS>::load(src + rhs * sstride, h, g.Vh);
  Spinor<typename PD::real> d;
#pragma unroll
  for (int k = 0; k < 12; ++k) d.c[k] = {typename PD::real(s.c[k].r), typename PD::real(s.c[k].i)};
  SpinorIO<PD>::store(dst + rhs * dstride, h, g.Vh, d);
}

struct CaxpbyArgs {
  double a[2 * kMaxRhs];
  double b[2 * kMaxRhs];
};

template <typename P>
__global__ __launch_bounds__(kBlock) void caxpby_kernel(Geo g, char* out, const char* x, const char* y, int g5y,
                                                       size_t stride, CaxpbyArgs c) {
  using R = typename P::real;
  const int rhs = blockIdx.y;
  const int h = site_block() * kBlock + threadIdx.x;
  if (h >= g.Vh) return;
  const size_t off = rhs * stride;
  const cplx<R> ca = {R(c.a[2 * rhs]), R(c.a[2 * rhs + 1])};
  const cplx<R> cb = {R(c.b[2 * rhs]), R(c.b[2 * rhs + 1])};
  Spinor<R> o;
#pragma unroll
  for (int k = 0; k < 12; ++k) o.c[k] = zero<R>();
  if (x) {
    const Spinor<R> xv = SpinorIO<P>::load(x + off, h, g.Vh);
#pragma unroll
    for (int k = 0; k < 12; ++k) o.c[k] = ca * xv.c[k];
  }
  if (y) {
    const Spinor<R> yv = SpinorIO<P>::load(y + off, h, g.Vh);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cplx<R> t = cb * yv.c[k];
      o.c[k] = (g5y && k >= 6) ? o.c[k] - t : o.c[k] + t;
    }
  }
  SpinorIO<P>::store(out + off, h, g.Vh, o);
}

// complex <x, y> = sum conj(x) y (two rows per rhs) or |x|^2 (one row per rhs), FP64 accumulation
template <typename P>
__global__ __launch_bounds__(kBlock) void dot_kernel(Geo g, const char* x, const char* y, size_t stride,
                                                    double* partials, int pstride, int cdot) {
  using R = typename P::real;
  __shared__ double lds[kBlock / 64];
  const int rhs = blockIdx.y;
  const int h = site_block() * kBlock + threadIdx.x;
  const size_t off = rhs * stride;
  double re = 0.0, im = 0.0;
  if (h < g.Vh) {
    const Spinor<R> xv = SpinorIO<P>::load(x + off, h, g.Vh);
    if (cdot) {
      const Spinor<R> yv = SpinorIO<P>::load(y + off, h, g.Vh);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        re += double(xv.c[k].r) * double(yv.c[k].r) + double(xv.c[k].i) * double(yv.c[k].i);
        im += double(xv.c[k].r) * double(yv.c[k].i) - double(xv.c[k].i) * double(yv.c[k].r);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) re += double(xv.c[k].r) * double(xv.c[k].r) + double(xv.c[k].i) * double(xv.c[k].i);
    }
  }
  const double sr = block_sum(re, lds);
  if (cdot) {
    const double si = block_sum(im, lds);
    if (threadIdx.x == 0) {
      partials[(2 * rhs) * pstride + site_block()] = sr;
      partials[(2 * rhs + 1) * pstride + site_block()] = si;
    }
  } else if (threadIdx.x == 0) {
    partials[rhs * pstride + site_block()] = sr;
  }
}

// one workgroup per row
// threads of the alpha kernel, whose row holds one partial sum per hop tile
// (16384 at 32^3 x 64); the |r|^2 rows are four times shorter and keep kBlock
constexpr int kRowThreads = 1024;

__device__ __forceinline__ double row_sum(const double* partials, int stride, int nb, int row, double* lds) {
  // eight accumulators per thread, so that its loads are in flight together
  // rather than one after another (rows reach 16384 entries at 32^3 x 64);
  // the order is fixed, so every call sums a row alike
  const double* p = partials + size_t(row) * size_t(stride);
  const int nt = blockDim.x;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 7 * nt < nb; b += 8 * nt) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += p[b + k * nt];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k)  // fewer than 8 left
    if (b + k * nt < nb) a[k] += p[b + k * nt];
  const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum(s, lds);
}

__global__ __launch_bounds__(kBlock) void finish_sum_kernel(const double* partials, int stride, int nb,
                                                           double* out) {
  __shared__ double lds[kBlock / 64];
  const double s = row_sum(partials, stride, nb, blockIdx.x, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRowThreads) void cg_alpha_kernel(const double* partials, int stride, int nb, double* st) {
  __shared__ double lds[kRowThreads / 64];
  const int r = blockIdx.x;
  const double pAp = row_sum(partials, stride, nb, r, lds);
  if (threadIdx.x == 0) {
    st[CG_PAP * kMaxRhs + r] = pAp;
    const bool done = st[CG_DONE * kMaxRhs + r] != 0.0;
    // breakdown guard: A is HPD, so <p, A p> must be positive and finite
    const bool ok = pAp > 0.0 && pAp < 1e300;
    if (!done && !ok) st[CG_BREAK * kMaxRhs + r] = 1.0;
    st[CG_ALPHA * kMaxRhs + r] = (done || !ok || st[CG_BREAK * kMaxRhs + r] != 0.0) ? 0.0 : st[CG_RR * kMaxRhs + r] / pAp;
  }
}

__global__ __launch_bounds__(kBlock) void cg_beta_kernel(const double* partials, int stride, int nb, double* st) {
  __shared__ double lds[kBlock / 64];
  const int r = blockIdx.x;
  const double rr_new = row_sum(partials, stride, nb, r, lds);
  if (threadIdx.x == 0) {
    if (!(rr_new < 1e300)) st[CG_BREAK * kMaxRhs + r] = 1.0;  // also catches NaN
    if (st[CG_BREAK * kMaxRhs + r] != 0.0) {
      st[CG_BETA * kMaxRhs + r] = 0.0;  // frozen until the host restarts it
    } else if (st[CG_DONE * kMaxRhs + r] == 0.0) {
      const double rr = st[CG_RR * kMaxRhs + r];
      st[CG_BETA * kMaxRhs + r] = rr_new / rr;
      st[CG_RR * kMaxRhs + r] = rr_new;
      st[CG_ITERS * kMaxRhs + r] += 1.0;
      if (rr_new > st[CG_MAXRR * kMaxRhs + r]) st[CG_MAXRR * kMaxRhs + r] = rr_new;
      if (rr_new <= st[CG_TOL2 * kMaxRhs + r] * st[CG_BB * kMaxRhs + r]) st[CG_DONE * kMaxRhs + r] = 1.0;
    } else {
      st[CG_BETA * kMaxRhs + r] = 0.0;
    }
  }
}


// ------------------------------------------------------------------ multi-shift CG
// State pointers: st = CG rows of the base system (kMaxRhs columns), ms = the
// multi-shift rows (kMaxSys columns), mr = per-rhs multi-shift rows.
// Shifted-system scalars for iteration i, after the base alpha_i is known:
// rotate zeta, freeze converged systems, then
//   zeta_{i+1} = zeta_i zeta_{i-1} alpha_{i-1}
//                / (alpha_i beta_{i-1} (zeta_{i-1} - zeta_i) + zeta_{i-1} alpha_{i-1} (1 + d alpha_i)),
//   alpha_s = alpha_i zeta_{i+1} / zeta_i.
__global__ __launch_bounds__(kMaxSys) void ms_scalars_kernel(double* st, double* ms, double* mr, int nrhs, int nsys) {
  const int q = threadIdx.x;
  double alpha_keep = 0.0;
  const bool active = q < nsys;
  const int r = active ? q % nrhs : 0;
  if (active) {
    double* row = ms + q;
    const double zprev = row[MS_ZCUR * kMaxSys];
    const double zcur = row[MS_ZNEXT * kMaxSys];
    row[MS_ZPREV * kMaxSys] = zprev;
    row[MS_ZCUR * kMaxSys] = zcur;
    const double alpha = st[CG_ALPHA * kMaxRhs + r];
    alpha_keep = alpha;
    const bool base_stop = st[CG_DONE * kMaxRhs + r] != 0.0 || st[CG_BREAK * kMaxRhs + r] != 0.0;
    bool done = row[MS_DONE * kMaxSys] != 0.0;
    if (!done && zcur * zcur * st[CG_RR * kMaxRhs + r] <= st[CG_TOL2 * kMaxRhs + r] * st[CG_BB * kMaxRhs + r]) {
      done = true;
      row[MS_DONE * kMaxSys] = 1.0;
      row[MS_ITERS * kMaxSys] = st[CG_ITERS * kMaxRhs + r];
    }
    if (done || base_stop || alpha == 0.0) {
      row[MS_ASHIFT * kMaxSys] = 0.0;
      row[MS_ZNEXT * kMaxSys] = zcur;
    } else {
      const double aprev = mr[MS_APREV * kMaxRhs + r];
      const double bprev = st[CG_BETA * kMaxRhs + r];
      const double d = row[MS_DELTA * kMaxSys];
      const double den = alpha * bprev * (zprev - zcur) + zprev * aprev * (1.0 + d * alpha);
      const double znext = zcur * zprev * aprev / den;
      row[MS_ZNEXT * kMaxSys] = znext;
      row[MS_ASHIFT * kMaxSys] = alpha * znext / zcur;
    }
  }
  __syncthreads();  // every system has read alpha_{i-1}
  if (active && q < nrhs && alpha_keep != 0.0) mr[MS_APREV * kMaxRhs + r] = alpha_keep;
}

// r -= alpha Ap (base, with |r|^2 partials); x_s += alpha_s p_s for every shift.
// Fields [nshift][nrhs] of stride bytes, FP64.
__global__ __launch_bounds__(kBlock) void ms_update_kernel(Geo g, char* r, const char* Ap, const char* p, char* x,
                                                          const double* st, const double* ms, size_t stride,
                                                          int nrhs, int nshift, double* partials, int pstride) {
  __shared__ double lds[kBlock / 64];
  const int rhs = blockIdx.y;
  const int h = site_block() * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  const double alpha = st[CG_ALPHA * kMaxRhs + rhs];
  double part = 0.0;
  if (h < Vh) {
    Spinor<double> rv = SpinorIO<PrecF64>::load(r + rhs * stride, h, Vh);
    if (alpha != 0.0) {
      const Spinor<double> av = SpinorIO<PrecF64>::load(Ap + rhs * stride, h, Vh);
#pragma unroll
      for (int k = 0; k < 12; ++k) rv.c[k] = rv.c[k] - alpha * av.c[k];
      SpinorIO<PrecF64>::store(r + rhs * stride, h, Vh, rv);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) part += rv.c[k].r * rv.c[k].r + rv.c[k].i * rv.c[k].i;
    for (int s = 0; s < nshift; ++s) {
      const double as = ms[MS_ASHIFT * kMaxSys + s * nrhs + rhs];
      if (as == 0.0) continue;
      const size_t off = (size_t(s) * nrhs + rhs) * stride;
      const Spinor<double> pv = SpinorIO<PrecF64>::load(p + off, h, Vh);
      Spinor<double> xv = SpinorIO<PrecF64>::load(x + off, h, Vh);
#pragma unroll
      for (int k = 0; k < 12; ++k) xv.c[k] = xv.c[k] + as * pv.c[k];
      SpinorIO<PrecF64>::store(x + off, h, Vh, xv);
    }
  }
  const double sum = block_sum(part, lds);
  if (threadIdx.x == 0) partials[rhs * pstride + site_block()] = sum;
}

// p_s = zeta_{i+1} r + beta_i (zeta_{i+1} / zeta_i)^2 p_s for every unfrozen system
__global__ __launch_bounds__(kBlock) void ms_xpay_kernel(Geo g, char* p, const char* r, const double* st,
                                                        const double* ms, size_t stride, int nrhs) {
  const int q = blockIdx.y;
  const int rhs = q % nrhs;
  const int h = site_block() * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  if (h >= Vh || ms[MS_ASHIFT * kMaxSys + q] == 0.0) return;
  const double zn = ms[MS_ZNEXT * kMaxSys + q], zc = ms[MS_ZCUR * kMaxSys + q];
  const double ratio = zn / zc;
  const double bs = st[CG_BETA * kMaxRhs + rhs] * ratio * ratio;
  const size_t off = size_t(q) * stride;
  Spinor<double> pv = SpinorIO<PrecF64>::load(p + off, h, Vh);
  const Spinor<double> rv = SpinorIO<PrecF64>::load(r + rhs * stride, h, Vh);
#pragma unroll
  for (int k = 0; k < 12; ++k) pv.c[k] = zn * rv.c[k] + bs * pv.c[k];
  SpinorIO<PrecF64>::store(p + off, h, Vh, pv);
}

// Start and end of the Chebyshev filter recurrence (the steps in between are
// fused into the hop kernels' epilogue):
//   start: t_0 = in, e_0 = 0, e_1 = in          (one read, three writes)
//   end:   out = s e_{n+1} = s (ce e_n + 2 t_n - e_{n-1}),  ce = 2 y0
// (nrhs fields, rhs = blockIdx.y, stride bytes apart)
template <typename P>
__global__ __launch_bounds__(kBlock) void cheb_init_kernel(Geo g, const char* in, char* t0, char* e0, char* e1,
                                                          size_t stride) {
  using R = typename P::real;
  const int h = site_block() * kBlock + threadIdx.x;
  if (h >= g.Vh) return;
  const size_t off = blockIdx.y * stride;
  in += off;
  t0 += off;
  e0 += off;
  e1 += off;
  const Spinor<R> v = SpinorIO<P>::load(in, h, g.Vh);
  Spinor<R> z;
#pragma unroll
  for (int k = 0; k < 12; ++k) z.c[k] = zero<R>();
  SpinorIO<P>::store(t0, h, g.Vh, v);
  SpinorIO<P>::store(e0, h, g.Vh, z);
  SpinorIO<P>::store(e1, h, g.Vh, v);
}

template <typename P>
__global__ __launch_bounds__(kBlock) void cheb_last_kernel(Geo g, const char* t, const char* e, const char* eprev,
                                                          char* out, double ce, double s, size_t stride) {
  using R = typename P::real;
  const int h = site_block() * kBlock + threadIdx.x;
  if (h >= g.Vh) return;
  const size_t off = blockIdx.y * stride;
  t += off;
  e += off;
  eprev += off;
  out += off;
  const Spinor<R> tv = SpinorIO<P>::load(t, h, g.Vh);
  const Spinor<R> ev = SpinorIO<P>::load(e, h, g.Vh);
  const Spinor<R> pv = SpinorIO<P>::load(eprev, h, g.Vh);
  const R re = R(ce), two = R(2), rs = R(s);
  Spinor<R> o;
#pragma unroll
  for (int k = 0; k < 12; ++k) o.c[k] = rs * (re * ev.c[k] + two * tv.c[k] - pv.c[k]);
  SpinorIO<P>::store(out, h, g.Vh, o);
}

// STREAM-style copy (the practical bandwidth ceiling): every thread moves four
// 16-byte vectors, loads issued before stores
__global__ __launch_bounds__(kBlock) void stream_copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                            size_t n) {
  const size_t base = (size_t(blockIdx.x) * kBlock * 4) + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const size_t i = base + size_t(k) * kBlock;
    if (i < n) v[k] = a[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const size_t i = base + size_t(k) * kBlock;
    if (i < n) b[i] = v[k];
  }
}

// ------------------------------------------------------------------ launchers
template <typename F>
static void by_prec(Prec p, F&& f) {
  switch (p) {
    case F64: f(PrecF64{}); break;
    case F32: f(PrecF32{}); break;
    case BF16: f(PrecBF16{}); break;
  }
}

static void check_xprec(Prec prec, Prec xprec) {
  WL_REQUIRE(xprec == F64 || (xprec == F32 && prec != F64), WL_EINVAL,
             "cg: the iterate is FP64, or FP32 under lower-precision storage");
}

void launch_cg_update(wl_lattice* L, Prec prec, Prec xprec, void* x, void* r, const void* p, const void* Ap,
                      const double* st, int nrhs, int nh, double* partials, int stride) {
  check_xprec(prec, xprec);
  dim3 grid(blas_blocks(L), nrhs * nh);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    auto go = [&](auto X) {
      using XT = decltype(X);
      hipLaunchKernelGGL((cg_update_kernel<PT, XT>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)x, (char*)r,
                         (const char*)p, (const char*)Ap, st, spinor_bytes(prec, L->Vh), spinor_bytes(xprec, L->Vh),
                         partials, stride, nh);
    };
    if (xprec == F64) go(PrecF64{});
    else go(PrecF32{});
  });
  WL_HIP(hipGetLastError());
}

void launch_cg_update_fused(wl_lattice* L, Prec prec, Prec xprec, void* x, void* r, const void* p, const void* Ap,
                            double* st, int nrhs, int nh, const double* dot_partials, int nb_dot,
                            double* rr_partials, int pstride) {
  check_xprec(prec, xprec);
  dim3 grid(blas_blocks(L), nrhs * nh);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    auto go = [&](auto X) {
      using XT = decltype(X);
      hipLaunchKernelGGL((cg_update_fused_kernel<PT, XT>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)x,
                         (char*)r, (const char*)p, (const char*)Ap, st, spinor_bytes(prec, L->Vh),
                         spinor_bytes(xprec, L->Vh), dot_partials, nb_dot, rr_partials, pstride, nh);
    };
    if (xprec == F64) go(PrecF64{});
    else go(PrecF32{});
  });
  WL_HIP(hipGetLastError());
}

// x64 += x32 and x32 = 0 over nf fields: a mixed CG's FP32 iterate folded into
// the FP64 solution before each FP64 true residual
__global__ __launch_bounds__(kBlock) void cg_fold_kernel(Geo g, char* x64, char* x32, size_t s64, size_t s32) {
  const int f = blockIdx.y;
  const int h = site_block() * kBlock + threadIdx.x;
  const int Vh = g.Vh;
  if (h >= Vh) return;
  char* xb = x64 + f * s64;
  char* yb = x32 + f * s32;
  Spinor<double> xv = SpinorIO<PrecF64>::load(xb, h, Vh);
  const Spinor<float> yv = SpinorIO<PrecF32>::load(yb, h, Vh);
  Spinor<float> z;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    xv.c[k].r += double(yv.c[k].r);
    xv.c[k].i += double(yv.c[k].i);
    z.c[k].r = 0.0f;
    z.c[k].i = 0.0f;
  }
  SpinorIO<PrecF64>::store(xb, h, Vh, xv);
  SpinorIO<PrecF32>::store(yb, h, Vh, z);
}

void launch_cg_fold(wl_lattice* L, void* x64, void* x32, int nf) {
  dim3 grid(blas_blocks(L), nf);
  hipLaunchKernelGGL(cg_fold_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, (char*)x64, (char*)x32,
                     spinor_bytes(F64, L->Vh), spinor_bytes(F32, L->Vh));
  WL_HIP(hipGetLastError());
}

void launch_cg_xpay_fused(wl_lattice* L, Prec prec, void* p, const void* r, double* st, int nrhs, int nh,
                          const double* rr_partials, int nb_rr, int pstride) {
  dim3 grid(blas_blocks(L), nrhs * nh);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((cg_xpay_fused_kernel<PT>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)p,
                       (const char*)r, st, spinor_bytes(prec, L->Vh), rr_partials, nb_rr, pstride, nh);
  });
  WL_HIP(hipGetLastError());
}

void launch_cg_xpay(wl_lattice* L, Prec prec, void* p, const void* r, const double* st, int nrhs, int nh) {
  dim3 grid(blas_blocks(L), nrhs * nh);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((cg_xpay_kernel<PT>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)p, (const char*)r,
                       st, spinor_bytes(prec, L->Vh), nh);
  });
  WL_HIP(hipGetLastError());
}

void launch_convert(wl_lattice* L, Prec dprec, void* dst, Prec sprec, const void* src, int nrhs) {
  dim3 grid(blas_blocks(L), nrhs);
  by_prec(dprec, [&](auto PD) {
    by_prec(sprec, [&](auto PS) {
      using D = decltype(PD);
      using S = decltype(PS);
      hipLaunchKernelGGL((convert_kernel<D, S>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)dst,
                         spinor_bytes(dprec, L->Vh), (const char*)src, spinor_bytes(sprec, L->Vh));
    });
  });
  WL_HIP(hipGetLastError());
}

void launch_caxpby(wl_lattice* L, void* out, const double* a, const void* x, const double* b, const void* y,
                   int g5y, int nrhs, Prec prec) {
  CaxpbyArgs c{};
  for (int r = 0; r < 2 * nrhs; ++r) {
    c.a[r] = a ? a[r] : 0.0;
    c.b[r] = b ? b[r] : 0.0;
  }
  dim3 grid(blas_blocks(L), nrhs);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((caxpby_kernel<PT>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)out, (const char*)x,
                       (const char*)y, g5y, spinor_bytes(prec, L->Vh), c);
  });
  WL_HIP(hipGetLastError());
}

void launch_dot_partials(wl_lattice* L, const void* x, const void* y, int nrhs, double* partials, int stride,
                         int complex_dot, Prec prec) {
  dim3 grid(blas_blocks(L), nrhs);
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((dot_kernel<PT>), grid, dim3(kBlock), 0, L->stream, L->geo, (const char*)x, (const char*)y,
                       spinor_bytes(prec, L->Vh), partials, stride, complex_dot);
  });
  WL_HIP(hipGetLastError());
}

void launch_finish_sum(wl_lattice* L, const double* partials, int stride, int nb, int nrows, double* out) {
  hipLaunchKernelGGL(finish_sum_kernel, dim3(nrows), dim3(kBlock), 0, L->stream, partials, stride, nb, out);
  WL_HIP(hipGetLastError());
}

void launch_cg_alpha(wl_lattice* L, const double* partials, int stride, int nb, double* st, int nrhs) {
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(nrhs), dim3(kRowThreads), 0, L->stream, partials, stride, nb, st);
  WL_HIP(hipGetLastError());
}

void launch_cg_beta(wl_lattice* L, const double* partials, int stride, int nb, double* st, int nrhs) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(nrhs), dim3(kBlock), 0, L->stream, partials, stride, nb, st);
  WL_HIP(hipGetLastError());
}

void launch_ms_scalars(wl_lattice* L, double* st, double* ms, double* mr, int nrhs, int nshift) {
  hipLaunchKernelGGL(ms_scalars_kernel, dim3(1), dim3(kMaxSys), 0, L->stream, st, ms, mr, nrhs, nrhs * nshift);
  WL_HIP(hipGetLastError());
}

void launch_ms_update(wl_lattice* L, void* r, const void* Ap, const void* p, void* x, const double* st,
                      const double* ms, int nrhs, int nshift, double* partials, int pstride) {
  hipLaunchKernelGGL(ms_update_kernel, dim3(blas_blocks(L), nrhs), dim3(kBlock), 0, L->stream, L->geo, (char*)r,
                     (const char*)Ap, (const char*)p, (char*)x, st, ms, spinor_bytes(F64, L->Vh), nrhs, nshift,
                     partials, pstride);
  WL_HIP(hipGetLastError());
}

void launch_ms_xpay(wl_lattice* L, void* p, const void* r, const double* st, const double* ms, int nrhs,
                    int nshift) {
  hipLaunchKernelGGL(ms_xpay_kernel, dim3(blas_blocks(L), nrhs * nshift), dim3(kBlock), 0, L->stream, L->geo,
                     (char*)p, (const char*)r, st, ms, spinor_bytes(F64, L->Vh), nrhs);
  WL_HIP(hipGetLastError());
}

void launch_cheb_init(wl_lattice* L, const void* in, void* t0, void* e0, void* e1, Prec prec, int nrhs) {
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((cheb_init_kernel<PT>), dim3(blas_blocks(L), nrhs), dim3(kBlock), 0, L->stream, L->geo,
                       (const char*)in, (char*)t0, (char*)e0, (char*)e1, spinor_bytes(prec, L->Vh));
  });
  WL_HIP(hipGetLastError());
}

void launch_cheb_last(wl_lattice* L, const void* t, const void* e, const void* eprev, void* out, double ce, double s,
                      Prec prec, int nrhs) {
  by_prec(prec, [&](auto P) {
    using PT = decltype(P);
    hipLaunchKernelGGL((cheb_last_kernel<PT>), dim3(blas_blocks(L), nrhs), dim3(kBlock), 0, L->stream, L->geo,
                       (const char*)t, (const char*)e, (const char*)eprev, (char*)out, ce, s,
                       spinor_bytes(prec, L->Vh));
  });
  WL_HIP(hipGetLastError());
}

void launch_stream_copy(wl_lattice* L, const void* a, void* b, size_t bytes) {
  const size_t n = bytes / 16;
  const size_t nb = (n + 4 * kBlock - 1) / (4 * kBlock);
  hipLaunchKernelGGL(stream_copy_kernel, dim3(unsigned(nb)), dim3(kBlock), 0, L->stream, (const float4*)a, (float4*)b, n);
  WL_HIP(hipGetLastError());
}

}  // namespace wl
