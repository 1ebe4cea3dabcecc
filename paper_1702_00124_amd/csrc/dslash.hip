// Wilson hop kernel, one even-odd block per launch (Sec. 3.1 Wilson fermions
// with even-odd preconditioning; formula in include/wilson_hmc.h):
//
//   out(x) = epilogue( sum_mu (1 - s g_mu) U_mu(x) in(x+mu)
//                           + (1 + s g_mu) U_mu(x-mu)^dag in(x-mu) ),
//   s = +1 for D, -1 for D^dag,
//
// for every site x of the output parity.  One thread per output site and
// NR right-hand sides: each link is loaded once and used for all NR spinors.
// Neighbour spinors are projected to half spinors (2 x 3) before the SU(3)
// product and rebuilt after it.  The stencil is HBM-bound (about 0.9 flop per
// byte in FP64), so the kernel is written for coalesced 16-byte loads and an
// L2-friendly, XCD-aware tile order; no MFMA.
#include "wl_internal.h"

namespace wl {

struct HopArgs {
  Geo g;
  int parity;  // output parity
  const char* in;
  char* out;
  const char* links;  // packed links of this precision, [2][4][...][Vh]
  size_t rhs_stride;  // bytes between rhs fields
  const char* x;
  double cx;
  double a;
  int g5;
  const char* y;
  double by[kMaxRhs];
  int dot;
  const char* dotv;
  double* partials;
  int part_stride;
  int part_off;
  int use_xcd;
};

template <typename P, int MU, int DAG, int NR>
__device__ __forceinline__ void hop_dir(const HopArgs& a, const Coord& c, int h, int r0,
                                        Spinor<typename P::real>* acc) {
  using R = typename P::real;
  constexpr int SF = DAG ? +1 : -1;  // projector sign of the forward term
  constexpr int SB = -SF;
  const int Vh = a.g.Vh;
  const size_t lb = LinkIO<P>::bytes * size_t(Vh);
  bool wrap;
  // forward: U_mu(x) in(x + mu)
  {
    const int hf = neighbour<MU>(a.g, c, +1, &wrap);
    const SU3<R> U = LinkIO<P>::load(a.links + (a.parity * 4 + MU) * lb, h, Vh);
    const R ph = wrap ? R(a.g.tbc) : R(1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const Spinor<R> s = SpinorIO<P>::load(a.in + (r0 + r) * a.rhs_stride, hf, Vh);
      Half<R> hp = project<MU, SF>(s);
      Half<R> w;
      su3_mul(U, hp.c, w.c);
      su3_mul(U, hp.c + 3, w.c + 3);
#pragma unroll
      for (int k = 0; k < 6; ++k) w.c[k] = ph * w.c[k];
      reconstruct_add<MU, SF>(acc[r], w);
    }
  }
  // backward: U_mu(x - mu)^dag in(x - mu)
  {
    const int hb = neighbour<MU>(a.g, c, -1, &wrap);
    const SU3<R> U = LinkIO<P>::load(a.links + ((1 - a.parity) * 4 + MU) * lb, hb, Vh);
    const R ph = wrap ? R(a.g.tbc) : R(1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const Spinor<R> s = SpinorIO<P>::load(a.in + (r0 + r) * a.rhs_stride, hb, Vh);
      Half<R> hp = project<MU, SB>(s);
      Half<R> w;
      su3_dag_mul(U, hp.c, w.c);
      su3_dag_mul(U, hp.c + 3, w.c + 3);
#pragma unroll
      for (int k = 0; k < 6; ++k) w.c[k] = ph * w.c[k];
      reconstruct_add<MU, SB>(acc[r], w);
    }
  }
}

template <typename P, int DAG, int NR>
__global__ __launch_bounds__(kBlock) void hop_kernel(HopArgs a) {
  using R = typename P::real;
  __shared__ double lds[kBlock / 64];
  const int b = a.use_xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int h = b * kBlock + threadIdx.x;
  const int Vh = a.g.Vh;
  const int r0 = blockIdx.y * NR;
  double part[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) part[r] = 0.0;

  if (h < Vh) {
    const Coord c = site_coords(a.g, h, a.parity);
    Spinor<R> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r].c[k] = zero<R>();
    hop_dir<P, 0, DAG, NR>(a, c, h, r0, acc);
    hop_dir<P, 1, DAG, NR>(a, c, h, r0, acc);
    hop_dir<P, 2, DAG, NR>(a, c, h, r0, acc);
    hop_dir<P, 3, DAG, NR>(a, c, h, r0, acc);

#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t off = (r0 + r) * a.rhs_stride;
      Spinor<R> o;
      const R ca = R(a.a);
#pragma unroll
      for (int k = 0; k < 12; ++k) o.c[k] = ca * acc[r].c[k];
      if (a.x) {
        const Spinor<R> xv = SpinorIO<P>::load(a.x + off, h, Vh);
        const R cx = R(a.cx);
#pragma unroll
        for (int k = 0; k < 12; ++k) o.c[k] = o.c[k] + cx * xv.c[k];
      }
      if (a.g5) {
#pragma unroll
        for (int k = 6; k < 12; ++k) o.c[k] = R(-1) * o.c[k];
      }
      if (a.y) {
        const Spinor<R> yv = SpinorIO<P>::load(a.y + off, h, Vh);
        const R cy = R(a.by[r0 + r]);
#pragma unroll
        for (int k = 0; k < 12; ++k) o.c[k] = o.c[k] + cy * yv.c[k];
      }
      SpinorIO<P>::store(a.out + off, h, Vh, o);
      if (a.dot == 1) {
        const Spinor<R> dv = SpinorIO<P>::load(a.dotv + off, h, Vh);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) s += double(dv.c[k].r) * double(o.c[k].r) + double(dv.c[k].i) * double(o.c[k].i);
        part[r] = s;
      } else if (a.dot == 2) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) s += double(o.c[k].r) * double(o.c[k].r) + double(o.c[k].i) * double(o.c[k].i);
        part[r] = s;
      }
    }
  }
  if (a.dot) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double s = block_sum(part[r], lds);
      if (threadIdx.x == 0) a.partials[(r0 + r) * a.part_stride + a.part_off + b] = s;
    }
  }
}

int hop_grid_blocks(const wl_lattice* L) { return site_blocks(L->Vh); }

template <typename P, int DAG>
static void dispatch_nr(const HopArgs& a, int nrhs, hipStream_t st, int nb) {
  // rhs per thread: FP64 keeps one (the register budget of a double spinor
  // accumulator plus hoisted loads); FP32/BF16 share each link over two
  int nr = 1;
  if (sizeof(typename P::real) == 4 && nrhs % 2 == 0) nr = 2;
  dim3 grid(nb, nrhs / nr);
  switch (nr) {
    case 2: hipLaunchKernelGGL((hop_kernel<P, DAG, 2>), grid, dim3(kBlock), 0, st, a); break;
    default: hipLaunchKernelGGL((hop_kernel<P, DAG, 1>), grid, dim3(kBlock), 0, st, a); break;
  }
}

template <typename P>
static void dispatch(const HopArgs& a, int dagger, int nrhs, hipStream_t st, int nb) {
  if (dagger) dispatch_nr<P, 1>(a, nrhs, st, nb);
  else dispatch_nr<P, 0>(a, nrhs, st, nb);
}

void launch_hop(wl_lattice* L, Prec prec, void* out, const void* in, int out_parity, int dagger,
                int nrhs, const HopEpi& e) {
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs out of range");
  WL_REQUIRE(out != in, WL_EINVAL, "hop output must not alias its input");
  if (prec != F64) ensure_lowp_links(L);
  HopArgs a;
  a.g = L->geo;
  a.parity = out_parity;
  a.in = static_cast<const char*>(in);
  a.out = static_cast<char*>(out);
  a.links = static_cast<const char*>(L->U[prec]);
  a.rhs_stride = spinor_bytes(prec, L->Vh);
  a.x = static_cast<const char*>(e.x);
  a.cx = e.cx;
  a.a = e.a;
  a.g5 = e.g5;
  a.y = static_cast<const char*>(e.y);
  for (int r = 0; r < kMaxRhs; ++r) a.by[r] = e.by[r];
  a.dot = e.dot;
  a.dotv = static_cast<const char*>(e.dotv);
  a.partials = e.partials;
  a.part_stride = e.part_stride;
  a.part_off = e.part_off;
  a.use_xcd = L->use_xcd;
  const int nb = hop_grid_blocks(L);
  // sampled event timing (never inside a graph capture)
  const bool timed = L->prof_on && !L->prof_capturing && nrhs == 1 && L->prof_ev[prec].size() < 2 * kProfPairs;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    WL_HIP(hipEventRecord(e0, L->stream));
  }
  switch (prec) {
    case F64: dispatch<PrecF64>(a, dagger, nrhs, L->stream, nb); break;
    case F32: dispatch<PrecF32>(a, dagger, nrhs, L->stream, nb); break;
    case BF16: dispatch<PrecBF16>(a, dagger, nrhs, L->stream, nb); break;
  }
  WL_HIP(hipGetLastError());
  if (timed) {
    WL_HIP(hipEventRecord(e1, L->stream));
    L->prof_ev[prec].push_back(e0);
    L->prof_ev[prec].push_back(e1);
  }
  L->n_hop += nrhs;
  L->n_hop_p[prec] += nrhs;
}

}  // namespace wl
