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
#include <algorithm>
#include <atomic>
#include <type_traits>

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
  int rows;  // rhs groups per tile
  int nrhs;  // rhs of the launch
  // fused Chebyshev step (every rhs): with w the epilogue's result,
  //   tprev <- ct t + cw w - tprev,  eprev <- ce e + 2 t - eprev,  w not stored
  const char* ch_t;
  char* ch_tprev;
  const char* ch_e;
  char* ch_eprev;
  double ch_ct, ch_cw, ch_ce;
};

// Flattened grid: block b -> (tile, rhs group).  The XCD-aware renumbering
// gives each XCD a contiguous block range, and the rhs groups of one tile are
// adjacent inside it, so a tile's links are fetched once into that XCD's L2
// and reused by every group.  In the hardware's round-robin deal (orders 0
// and 2) the groups of a tile are kept on one XCD instead: blocks b, b + 8,
// b + 16, ... take the groups of the tile that b alone would take with one
// group (the grid is padded to whole groups of 8 tiles, hop_grid).  The
// z-blocked order walks kZBlock z planes through every t before the next
// planes: a tile's t neighbours are then kZBlock planes of tiles away instead
// of a whole time slice (what the L2 has to hold between the two reads), and
// with a multiple of 8 tiles per plane its z and t neighbours are dealt to its
// own XCD.  False for the padding blocks.
template <int SITES>  // sites per workgroup
__device__ __forceinline__ bool hop_block_seq(const HopArgs& a, int* seq, int* row) {
  if (a.use_xcd == 1) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    *seq = b / a.rows;
    *row = b - *seq * a.rows;
    return true;
  }
  const int b = blockIdx.x;
  const int g8 = b / (8 * a.rows);
  const int rem = b - g8 * 8 * a.rows;
  *row = rem >> 3;
  *seq = g8 * 8 + (rem & 7);
  return *seq < (a.g.Vh + SITES - 1) / SITES;
}

// direction-parallel kernel: the workgroup's 64-site tile
template <int SITES>
__device__ __forceinline__ bool hop_block_coords(const HopArgs& a, int* tile, int* row) {
  int seq;
  if (!hop_block_seq<SITES>(a, &seq, row)) return false;
  if (a.use_xcd != 2) {
    *tile = seq;
    return true;
  }
  const int tz = a.g.Lxh * a.g.L[1] / SITES;  // workgroup tiles per z plane
  const int j = seq % tz;
  int r = seq / tz;
  const int zi = r % kZBlock;
  r /= kZBlock;
  const int t = r % a.g.L[3];
  const int zb = r / a.g.L[3];
  *tile = (t * a.g.L[2] + zb * kZBlock + zi) * tz + j;
  return true;
}

// thread-per-site kernel: the 64-site tile of the calling wavefront.  Its
// workgroup's 4 wavefronts take 4 consecutive tiles, or in the z-blocked order
// one 64-site column of 4 consecutive z planes, workgroups walking the columns
// of a plane fastest: with a multiple of 8 columns per plane every XCD keeps
// its own columns through all z and t, so a site's z and t neighbours come from
// its own L2 as the direction-parallel kernel's do.
__device__ __forceinline__ bool site_tile(const HopArgs& a, int* tile64, int* row) {
  constexpr int W = kBlock / 64;  // wavefronts per workgroup
  int seq;
  if (!hop_block_seq<kBlock>(a, &seq, row)) return false;
  const int w = threadIdx.x >> 6;
  if (a.use_xcd != 2) {
    *tile64 = seq * W + w;
    return true;
  }
  const int tz = a.g.Lxh * a.g.L[1] / 64;  // columns per z plane
  const int j = seq % tz;
  int r = seq / tz;
  const int zq = r % (kZBlock / W);
  r /= kZBlock / W;
  const int t = r % a.g.L[3];
  const int zb = r / a.g.L[3];
  *tile64 = (t * a.g.L[2] + zb * kZBlock + zq * W + w) * tz + j;
  return true;
}

// blocks of a hop launch over tiles of SITES sites and a.rows rhs groups
template <int SITES>
static int hop_grid(const HopArgs& a) {
  const int nt = (a.g.Vh + SITES - 1) / SITES;
  return a.use_xcd == 1 ? nt * a.rows : (nt + 7) / 8 * 8 * a.rows;
}

// ------------------------------------------------------------------ BF16 products from packed storage
// A stored BF16 complex number is a pair (re in the low half, im in the high
// half): the operand format of the bf16 dot product with FP32 accumulation,
// d = a.lo b.lo + a.hi b.hi + c, whose products are exact in FP32.  With a
// spinor component p = (pr, pi) as stored, Re(u p) = (ur, -ui).p and
// Im(u p) = (ui, ur).p; for the adjoint product conj(u) p the pairs are
// (ur, ui) and (-ui, ur).  The spin projection (1 + S g_mu) p = p_top + c p_bot,
// c one of +1, -1, +i, -i, is folded into the products: u (-p) is (A, B) on
// -p, u (i p) is (B, A) on (-p, p) and u (-i p) (B, A) on (p, -p), with -p the
// stored pairs with both sign bits flipped, so the projected half spinor is
// never formed: no unpacking of the input and no rounding of the projection.
// The link's third row is rebuilt from the two stored rows by the same dot
// products (FP32 sums of exact products) and rounded to BF16 like them.
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c,
                                         false);
}
// a.b with a zero accumulator (the compiler's own choice of encoding: a
// dot product written as inline assembly is invisible to its hazard checks)
__device__ __forceinline__ float dot2_first(uint32_t a, uint32_t b) { return dot2(a, b, 0.0f); }
__device__ __forceinline__ uint32_t swap16(uint32_t u) { return __builtin_amdgcn_alignbit(u, u, 16); }

// the product matrix's entries (a, b) as the pairs A (real part) and B
// (imaginary part of the product)
struct Bf16Link {
  uint32_t A[9], B[9];
};

// links of one direction; the forward product takes U, the backward one U^dag
template <int FWD>
__device__ __forceinline__ void bf16_link(const char* base, int h, Bf16Link* L, bool stream) {
  const uint2* b = reinterpret_cast<const uint2*>(base);
  uint32_t m[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const uint2 v = stream ? ld_stream(b + fidx(j, h, 3)) : b[fidx(j, h, 3)];
    m[2 * j] = v.x;
    m[2 * j + 1] = v.y;
  }
  // third row m[6 + j] = conj(m[k] m[3 + l] - m[l] m[3 + k]), (j, k, l) cyclic,
  // from the pairs: Re(a b) = a.conj(b), Im(a b) = a.swap(b)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = (j + 1) % 3, l = (j + 2) % 3;
    const uint32_t a = m[k], b = m[3 + l], c = m[l], d = m[3 + k];
    const float re = dot2(c, d ^ 0x00008000u, dot2_first(a, b ^ 0x80000000u));  // Re(a b) - Re(c d)
    const float im = dot2(c, swap16(d), dot2_first(a, swap16(b) ^ 0x80008000u));  // -(Im(a b) - Im(c d))
    m[6 + j] = pack_bf16x2(re, im);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const int e = 3 * a + bb;
      const uint32_t w = FWD ? m[3 * a + bb] : m[3 * bb + a];  // U_ab, or conj(U_ba) for U^dag
      const uint32_t sw = swap16(w);
      if (FWD) {
        L->A[e] = w ^ 0x80000000u;   // (ur, -ui)
        L->B[e] = sw;                // (ui, ur)
      } else {
        L->A[e] = w;                 // (ur, ui)
        L->B[e] = sw ^ 0x00008000u;  // (-ui, ur)
      }
    }
}

// (product matrix) (p_top + c p_bot) for one half spinor: 3 complex results,
// 36 dot products; CC: 0 -> c = +1, 1 -> -1, 2 -> +i, 3 -> -i
template <int CC>
__device__ __forceinline__ void bf16_half(const Bf16Link& L, const uint32_t* pt, const uint32_t* pb, cplx<float>* w) {
  uint32_t nb[3];  // -p_bot
#pragma unroll
  for (int bb = 0; bb < 3; ++bb) nb[bb] = pb[bb] ^ 0x80008000u;
  // the operands of p_bot's products for the real and the imaginary part
  const uint32_t* pr = (CC == 0 || CC == 3) ? pb : nb;
  const uint32_t* pi = (CC == 0 || CC == 2) ? pb : nb;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float re = dot2_first(L.A[3 * a], pt[0]), im = dot2_first(L.B[3 * a], pt[0]);
#pragma unroll
    for (int bb = 1; bb < 3; ++bb) {
      const int e = 3 * a + bb;
      re = dot2(L.A[e], pt[bb], re);
      im = dot2(L.B[e], pt[bb], im);
    }
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const int e = 3 * a + bb;
      if (CC <= 1) {  // c = +-1: Re = A.(c p), Im = B.(c p)
        re = dot2(L.A[e], pr[bb], re);
        im = dot2(L.B[e], pi[bb], im);
      } else {        // c = +-i: Re = B.(-+p), Im = A.(+-p)
        re = dot2(L.B[e], pr[bb], re);
        im = dot2(L.A[e], pi[bb], im);
      }
    }
    w[a] = {re, im};
  }
}

// the two projected halves of (1 + S g_MU) p, multiplied: p as 12 stored pairs
// (component 3 spin + colour); h0 = p0 + c0 p_b0, h1 = p1 + c1 p_b1 as in project()
template <int MU, int S>
__device__ __forceinline__ void bf16_project_mul(const Bf16Link& L, const uint32_t* p, cplx<float>* w) {
  constexpr int mi = S > 0 ? 3 : 2, pi = S > 0 ? 2 : 3;  // c = -S i, c = +S i
  constexpr int m1 = S > 0 ? 1 : 0, p1 = S > 0 ? 0 : 1;  // c = -S,   c = +S
  if (MU == 0) {         // h0 = p0 - S i p3, h1 = p1 - S i p2
    bf16_half<mi>(L, p + 0, p + 9, w);
    bf16_half<mi>(L, p + 3, p + 6, w + 3);
  } else if (MU == 1) {  // h0 = p0 - S p3, h1 = p1 + S p2
    bf16_half<m1>(L, p + 0, p + 9, w);
    bf16_half<p1>(L, p + 3, p + 6, w + 3);
  } else if (MU == 2) {  // h0 = p0 - S i p2, h1 = p1 + S i p3
    bf16_half<mi>(L, p + 0, p + 6, w);
    bf16_half<pi>(L, p + 3, p + 9, w + 3);
  } else {               // h0 = p0 + S p2, h1 = p1 + S p3
    bf16_half<p1>(L, p + 0, p + 6, w);
    bf16_half<p1>(L, p + 3, p + 9, w + 3);
  }
}

// ------------------------------------------------------------------ links shared through LDS
// The shared-link variant of the thread-per-site kernel gives a workgroup one
// 64-site tile and four rhs, one per wavefront.  Wavefront w reads the tile's
// two links of direction w (forward at the site, backward at its neighbour)
// once and puts them in LDS; after one barrier every wavefront takes all 8
// from there.  BF16 keeps the product pairs (18 words per link: the pair forms
// and the third row are built once per tile instead of once per rhs); FP32 and
// FP64 keep the two stored rows (12 and 24 words) and rebuild the third row per
// rhs in the same expression as the thread-per-site kernel.  The arithmetic is
// that kernel's, bit for bit.
template <typename P>
constexpr int shl_words() {
  return std::is_same<P, PrecBF16>::value ? 18 : (std::is_same<P, PrecF32>::value ? 12 : 24);
}
__device__ __forceinline__ void shl_put(uint32_t* S, int d, const Bf16Link& U, int lane) {
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    S[(d * 18 + e) * 64 + lane] = U.A[e];
    S[(d * 18 + 9 + e) * 64 + lane] = U.B[e];
  }
}
__device__ __forceinline__ void shl_get(const uint32_t* S, int d, Bf16Link* U, int lane) {
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    U->A[e] = S[(d * 18 + e) * 64 + lane];
    U->B[e] = S[(d * 18 + 9 + e) * 64 + lane];
  }
}
__device__ __forceinline__ void shl_put(uint32_t* S, int d, const SU3<float>& U, int lane) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    S[(d * 12 + 2 * k) * 64 + lane] = __builtin_bit_cast(uint32_t, U.m[k].r);
    S[(d * 12 + 2 * k + 1) * 64 + lane] = __builtin_bit_cast(uint32_t, U.m[k].i);
  }
}
__device__ __forceinline__ void shl_get(const uint32_t* S, int d, SU3<float>* U, int lane) {
#pragma unroll
  for (int k = 0; k < 6; ++k)
    U->m[k] = {__builtin_bit_cast(float, S[(d * 12 + 2 * k) * 64 + lane]),
               __builtin_bit_cast(float, S[(d * 12 + 2 * k + 1) * 64 + lane])};
  third_row(*U);
}
__device__ __forceinline__ void shl_put(uint32_t* S, int d, const SU3<double>& U, int lane) {
  uint2* S2 = reinterpret_cast<uint2*>(S);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    S2[(d * 12 + 2 * k) * 64 + lane] = __builtin_bit_cast(uint2, U.m[k].r);
    S2[(d * 12 + 2 * k + 1) * 64 + lane] = __builtin_bit_cast(uint2, U.m[k].i);
  }
}
__device__ __forceinline__ void shl_get(const uint32_t* S, int d, SU3<double>* U, int lane) {
  const uint2* S2 = reinterpret_cast<const uint2*>(S);
#pragma unroll
  for (int k = 0; k < 6; ++k)
    U->m[k] = {__builtin_bit_cast(double, S2[(d * 12 + 2 * k) * 64 + lane]),
               __builtin_bit_cast(double, S2[(d * 12 + 2 * k + 1) * 64 + lane])};
  third_row(*U);
}
// the two links of direction MU into LDS (directions 2 MU forward, 2 MU + 1 backward)
template <typename P, int MU, bool ST>
__device__ __forceinline__ void shl_build(const HopArgs& a, const Coord& c, int h, uint32_t* S, int lane) {
  const size_t lb = LinkIO<P>::bytes * size_t(a.g.Vhp);
  const char* fwd = a.links + (a.parity * 4 + MU) * lb;
  const char* bwd = a.links + ((1 - a.parity) * 4 + MU) * lb;
  bool wrap;
  const int hb = neighbour<MU>(a.g, c, -1, &wrap);
  if constexpr (std::is_same<P, PrecBF16>::value) {
    Bf16Link U;
    bf16_link<1>(fwd, h, &U, ST);
    shl_put(S, 2 * MU, U, lane);
    bf16_link<0>(bwd, hb, &U, ST);
    shl_put(S, 2 * MU + 1, U, lane);
  } else {
    shl_put(S, 2 * MU, LinkIO<P>::template load<ST>(fwd, h, a.g.Vh), lane);
    shl_put(S, 2 * MU + 1, LinkIO<P>::template load<ST>(bwd, hb, a.g.Vh), lane);
  }
}

// SHL: the links from the tile's copy S in LDS (the shared-link variant)
template <typename P, int MU, int DAG, int NR, bool ST, bool SHL = false>
__device__ __forceinline__ void hop_dir(const HopArgs& a, const Coord& c, int h, int r0,
                                        Spinor<typename P::real>* acc, const uint32_t* S = nullptr) {
  using R = typename P::real;
  constexpr int SF = DAG ? +1 : -1;  // projector sign of the forward term
  constexpr int SB = -SF;
  const int Vh = a.g.Vh;
  const size_t lb = LinkIO<P>::bytes * size_t(a.g.Vhp);
  bool wrap;
  if constexpr (std::is_same<P, PrecBF16>::value) {  // products from the stored pairs
#pragma unroll
    for (int fwd = 1; fwd >= 0; --fwd) {
      const int hn = neighbour<MU>(a.g, c, fwd ? +1 : -1, &wrap);
      Bf16Link U;
      if constexpr (SHL) shl_get(S, 2 * MU + (fwd ? 0 : 1), &U, (threadIdx.x & 63));
      else if (fwd) bf16_link<1>(a.links + (a.parity * 4 + MU) * lb, h, &U, ST);
      else bf16_link<0>(a.links + ((1 - a.parity) * 4 + MU) * lb, hn, &U, ST);
      const R ph = wrap ? R(a.g.tbc) : R(1);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint4* b = reinterpret_cast<const uint4*>(a.in + (r0 + r) * a.rhs_stride);
        uint32_t p[12];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const uint4 v = b[fidx(j, hn, 3)];
          p[4 * j] = v.x;
          p[4 * j + 1] = v.y;
          p[4 * j + 2] = v.z;
          p[4 * j + 3] = v.w;
        }
        Half<R> w;
        if (fwd) bf16_project_mul<MU, SF>(U, p, w.c);
        else bf16_project_mul<MU, SB>(U, p, w.c);
        if (MU == 3) {
#pragma unroll
          for (int k = 0; k < 6; ++k) w.c[k] = ph * w.c[k];
        }
        if (fwd) reconstruct_add<MU, SF>(acc[r], w);
        else reconstruct_add<MU, SB>(acc[r], w);
      }
    }
    return;
  }
  // forward: U_mu(x) in(x + mu)
  {
    const int hf = neighbour<MU>(a.g, c, +1, &wrap);
    SU3<R> U;
    if constexpr (SHL) shl_get(S, 2 * MU, &U, (threadIdx.x & 63));
    else U = LinkIO<P>::template load<ST>(a.links + (a.parity * 4 + MU) * lb, h, Vh);
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
    SU3<R> U;
    if constexpr (SHL) shl_get(S, 2 * MU + 1, &U, (threadIdx.x & 63));
    else U = LinkIO<P>::template load<ST>(a.links + ((1 - a.parity) * 4 + MU) * lb, hb, Vh);
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

// epilogue field access, streaming or cached
template <typename P, bool ST>
__device__ __forceinline__ Spinor<typename P::real> epi_load(const char* base, int h, int Vh) {
  if constexpr (ST) return SpinorIO<P>::load_nt(base, h, Vh);
  else return SpinorIO<P>::load(base, h, Vh);
}
template <typename P, bool ST>
__device__ __forceinline__ void epi_store(char* base, int h, int Vh, const Spinor<typename P::real>& v) {
  if constexpr (ST) SpinorIO<P>::store_nt(base, h, Vh, v);
  else SpinorIO<P>::store(base, h, Vh, v);
}
template <typename P, bool ST>
__device__ __forceinline__ void epi_load_unit(const char* base, int u, int h, int Vh, cplx<typename P::real>* c) {
  if constexpr (ST) UnitIO<P>::load_nt(base, u, h, Vh, c);
  else UnitIO<P>::load(base, u, h, Vh, c);
}
template <typename P, bool ST>
__device__ __forceinline__ void epi_store_unit(char* base, int u, int h, int Vh, const cplx<typename P::real>* c) {
  if constexpr (ST) UnitIO<P>::store_nt(base, u, h, Vh, c);
  else UnitIO<P>::store(base, u, h, Vh, c);
}

// the fused Chebyshev step on one 16-byte unit u of site h of the rhs at byte
// offset off, w = the unit's result
template <typename P, bool ST>
__device__ __forceinline__ void cheb_unit(const HopArgs& a, size_t off, int u, int h, int Vh,
                                          const cplx<typename P::real>* w) {
  using R = typename P::real;
  using UIO = UnitIO<P>;
  cplx<R> t[UIO::CPU], tp[UIO::CPU], e[UIO::CPU], ep[UIO::CPU];
  epi_load_unit<P, ST>(a.ch_t + off, u, h, Vh, t);
  epi_load_unit<P, ST>(a.ch_tprev + off, u, h, Vh, tp);
  epi_load_unit<P, ST>(a.ch_e + off, u, h, Vh, e);
  epi_load_unit<P, ST>(a.ch_eprev + off, u, h, Vh, ep);
  const R rt = R(a.ch_ct), rw = R(a.ch_cw), re = R(a.ch_ce), two = R(2);
#pragma unroll
  for (int q = 0; q < UIO::CPU; ++q) {
    tp[q] = rt * t[q] + rw * w[q] - tp[q];
    ep[q] = re * e[q] + two * t[q] - ep[q];
  }
  epi_store_unit<P, ST>(a.ch_tprev + off, u, h, Vh, tp);
  epi_store_unit<P, ST>(a.ch_eprev + off, u, h, Vh, ep);
}

template <int WORDS>
__device__ __forceinline__ uint32_t* shl_lds() {
  __shared__ __align__(16) uint32_t S[8 * WORDS * 64];  // FP64 reads it as 8-byte words
  return S;
}

// SHL: the shared-link variant (one 64-site tile for four rhs per workgroup, NR = 1)
template <typename P, int DAG, int NR, bool ST, bool CHEB = false, bool SHL = false>
__global__ __launch_bounds__(kBlock) void hop_kernel(HopArgs a) {
  using R = typename P::real;
  static_assert(!SHL || (NR == 1 && !CHEB && kBlock == 4 * 64), "shared links: 4 x 1 rhs");
  int tile, row;
  if constexpr (SHL) {
    if (!hop_block_coords<kSiteTile>(a, &tile, &row)) return;
  } else {
    if (!site_tile(a, &tile, &row)) return;
  }
  const int h = tile * 64 + (threadIdx.x & 63);
  const int Vh = a.g.Vh;
  const int r0 = SHL ? row * 4 + (threadIdx.x >> 6) : row * NR;
  double part[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) part[r] = 0.0;
  const uint32_t* S = nullptr;
  if constexpr (SHL) {
    uint32_t* St = shl_lds<shl_words<P>()>();
    if (h < Vh) {
      const Coord c = site_coords(a.g, h, a.parity);
      const int lane = threadIdx.x & 63;
      switch (threadIdx.x >> 6) {
        case 0: shl_build<P, 0, ST>(a, c, h, St, lane); break;
        case 1: shl_build<P, 1, ST>(a, c, h, St, lane); break;
        case 2: shl_build<P, 2, ST>(a, c, h, St, lane); break;
        default: shl_build<P, 3, ST>(a, c, h, St, lane); break;
      }
    }
    __syncthreads();
    if (r0 >= a.nrhs) return;  // the whole wavefront: no rhs left for it
    S = St;
  }

  if (h < Vh) {
    const Coord c = site_coords(a.g, h, a.parity);
    Spinor<R> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r].c[k] = zero<R>();
    hop_dir<P, 0, DAG, NR, ST, SHL>(a, c, h, r0, acc, S);
    hop_dir<P, 1, DAG, NR, ST, SHL>(a, c, h, r0, acc, S);
    hop_dir<P, 2, DAG, NR, ST, SHL>(a, c, h, r0, acc, S);
    hop_dir<P, 3, DAG, NR, ST, SHL>(a, c, h, r0, acc, S);

#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t off = (r0 + r) * a.rhs_stride;
      Spinor<R> o;
      const R ca = R(a.a);
#pragma unroll
      for (int k = 0; k < 12; ++k) o.c[k] = ca * acc[r].c[k];
      if (a.x) {
        const Spinor<R> xv = epi_load<P, ST>(a.x + off, h, Vh);
        const R cx = R(a.cx);
#pragma unroll
        for (int k = 0; k < 12; ++k) o.c[k] = o.c[k] + cx * xv.c[k];
      }
      if (a.g5) {
#pragma unroll
        for (int k = 6; k < 12; ++k) o.c[k] = R(-1) * o.c[k];
      }
      if (a.y) {
        const Spinor<R> yv = epi_load<P, ST>(a.y + off, h, Vh);
        const R cy = R(a.by[r0 + r]);
#pragma unroll
        for (int k = 0; k < 12; ++k) o.c[k] = o.c[k] + cy * yv.c[k];
      }
      if constexpr (CHEB) {
        using UIO = UnitIO<P>;
#pragma unroll
        for (int u = 0; u < UIO::NU; ++u) cheb_unit<P, ST>(a, off, u, h, Vh, o.c + u * UIO::CPU);
        continue;
      }
      epi_store<P, ST>(a.out + off, h, Vh, o);
      if (a.dot == 1) {
        const Spinor<R> dv = epi_load<P, ST>(a.dotv + off, h, Vh);
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
  // one partial per wavefront of 64 sites, as in the direction-parallel variant
  const int slot = tile;
  if (a.dot && slot * 64 < Vh) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double s = wave_sum(part[r]);
      if ((threadIdx.x & 63) == 0) a.partials[(r0 + r) * a.part_stride + a.part_off + slot] = s;
    }
  }
}

// ------------------------------------------------------------------ direction-parallel variant
// One workgroup = 8 wavefronts over the same 64 consecutive output sites;
// wavefront d = 2 mu + (0 forward, 1 backward) loads its direction's link
// once, projects, multiplies and writes the half-spinor result of every rhs
// to LDS; after one barrier the wavefronts rebuild and sum the 8 directions
// per 16-byte storage unit and run the epilogue.  Eight times the wavefronts
// of the site kernel at the same coalescing (every load is 64 consecutive
// sites), which hides memory latency on small lattices.
constexpr int kDpSites = 64;
constexpr int kDpThreads = 8 * kDpSites;

// the link a direction-parallel wavefront holds: unpacked SU(3) in FP32 / FP64,
// the dot-product pairs for BF16
template <typename P>
struct DpLink {
  using type = SU3<typename P::real>;
};
template <>
struct DpLink<PrecBF16> {
  using type = Bf16Link;
};

// the wavefront's direction: its neighbour, time-boundary phase and link
template <typename P, int MU, int FWD, bool ST>
__device__ __forceinline__ void dp_link(const HopArgs& a, const Coord& c, int h, typename DpLink<P>::type* U,
                                        int* hn, typename P::real* ph) {
  using R = typename P::real;
  const int Vh = a.g.Vh;
  const size_t lb = LinkIO<P>::bytes * size_t(a.g.Vhp);
  bool wrap;
  *hn = neighbour<MU>(a.g, c, FWD ? +1 : -1, &wrap);
  const char* base = FWD ? a.links + (a.parity * 4 + MU) * lb : a.links + ((1 - a.parity) * 4 + MU) * lb;
  if constexpr (std::is_same<P, PrecBF16>::value) {
    bf16_link<FWD>(base, FWD ? h : *hn, U, ST);
  } else {
    *U = LinkIO<P>::template load<ST>(base, FWD ? h : *hn, Vh);
  }
  *ph = wrap ? R(a.g.tbc) : R(1);
}

// project, multiply and store to LDS the half-spinor results of NRP rhs
template <typename P, int MU, int FWD, int DAG, int NRP>
__device__ __forceinline__ void dp_spin(const HopArgs& a, const typename DpLink<P>::type& U, int hn,
                                        typename P::real ph, int r0, cplx<typename P::real>* W, int lane) {
  using R = typename P::real;
  constexpr int S = FWD ? (DAG ? +1 : -1) : (DAG ? -1 : +1);  // projector sign (1 + S g_mu)
  constexpr int D = 2 * MU + (FWD ? 0 : 1);
  if constexpr (std::is_same<P, PrecBF16>::value) {
#pragma unroll
    for (int r = 0; r < NRP; ++r) {
      const uint4* b = reinterpret_cast<const uint4*>(a.in + (r0 + r) * a.rhs_stride);
      uint32_t p[12];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const uint4 v = b[fidx(j, hn, 3)];
        p[4 * j] = v.x;
        p[4 * j + 1] = v.y;
        p[4 * j + 2] = v.z;
        p[4 * j + 3] = v.w;
      }
      cplx<float> w[6];
      bf16_project_mul<MU, S>(U, p, w);
#pragma unroll
      for (int k = 0; k < 6; ++k) W[((r * 8 + D) * 6 + k) * kDpSites + lane] = MU == 3 ? ph * w[k] : w[k];
    }
  } else {
#pragma unroll
    for (int r = 0; r < NRP; ++r) {
      const Spinor<R> s = SpinorIO<P>::load(a.in + (r0 + r) * a.rhs_stride, hn, a.g.Vh);
      const Half<R> hp = project<MU, S>(s);
      Half<R> w;
      if (FWD) {
        su3_mul(U, hp.c, w.c);
        su3_mul(U, hp.c + 3, w.c + 3);
      } else {
        su3_dag_mul(U, hp.c, w.c);
        su3_dag_mul(U, hp.c + 3, w.c + 3);
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) W[((r * 8 + D) * 6 + k) * kDpSites + lane] = MU == 3 ? ph * w.c[k] : w.c[k];
    }
  }
}

// sum over the 8 directions of the rebuilt spinor component (spin s, colour col)
// from the half-spinor results W[d][3 k + col]; the lower spin rows carry the
// projector's phases, which flip sign between forward and backward terms
template <int DAG, typename R>
__device__ __forceinline__ cplx<R> dp_recon(const cplx<R>* W, int s, int col, int lane) {
  auto w = [&](int d, int k) { return W[(d * 6 + 3 * k + col) * kDpSites + lane]; };
  if (s < 2) {
    cplx<R> acc = w(0, s);
#pragma unroll
    for (int d = 1; d < 8; ++d) acc = acc + w(d, s);
    return acc;
  }
  const R sf = DAG ? R(1) : R(-1);  // forward projector sign
  auto df = [&](int mu, int k) { return w(2 * mu, k) - w(2 * mu + 1, k); };
  cplx<R> acc;
  if (s == 2)  // x: +i h1, y: +h1, z: +i h0, t: +h0
    acc = times_i(df(0, 1)) + df(1, 1) + times_i(df(2, 0)) + df(3, 0);
  else         // x: +i h0, y: -h0, z: -i h1, t: +h1
    acc = times_i(df(0, 0)) - df(1, 0) - times_i(df(2, 1)) + df(3, 1);
  return sf * acc;
}

// NRP rhs share one LDS pass; NPASS passes reuse the link held in registers,
// so each link is read once for NRP * NPASS rhs
template <typename P, int DAG, int NRP, int NPASS, bool ST, bool CHEB = false>
__global__ __launch_bounds__(kDpThreads) void hop_dp_kernel(HopArgs a) {
  using R = typename P::real;
  using UIO = UnitIO<P>;
  constexpr int NR = NRP * NPASS;
  __shared__ cplx<R> W[NRP * 8 * 6 * kDpSites];
  __shared__ double red[kDpThreads / 64];
  int tile, row;
  if (!hop_block_coords<kDpSites>(a, &tile, &row)) return;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int Vh = a.g.Vh;
  const int h = tile * kDpSites + lane;
  const bool active = h < Vh;
  const int r0 = row * NR;
  typename DpLink<P>::type U;
  int hn = 0;
  R ph = R(1);
  if (active) {
    const Coord c = site_coords(a.g, h, a.parity);
    switch (wv) {
      case 0: dp_link<P, 0, 1, ST>(a, c, h, &U, &hn, &ph); break;
      case 1: dp_link<P, 0, 0, ST>(a, c, h, &U, &hn, &ph); break;
      case 2: dp_link<P, 1, 1, ST>(a, c, h, &U, &hn, &ph); break;
      case 3: dp_link<P, 1, 0, ST>(a, c, h, &U, &hn, &ph); break;
      case 4: dp_link<P, 2, 1, ST>(a, c, h, &U, &hn, &ph); break;
      case 5: dp_link<P, 2, 0, ST>(a, c, h, &U, &hn, &ph); break;
      case 6: dp_link<P, 3, 1, ST>(a, c, h, &U, &hn, &ph); break;
      default: dp_link<P, 3, 0, ST>(a, c, h, &U, &hn, &ph); break;
    }
  }
  double part[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) part[r] = 0.0;
  const R ca = R(a.a), cx = R(a.cx);
#pragma unroll
  for (int pass = 0; pass < NPASS; ++pass) {
    const int rp = r0 + pass * NRP;
    if (active) {
      switch (wv) {
        case 0: dp_spin<P, 0, 1, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 1: dp_spin<P, 0, 0, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 2: dp_spin<P, 1, 1, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 3: dp_spin<P, 1, 0, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 4: dp_spin<P, 2, 1, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 5: dp_spin<P, 2, 0, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        case 6: dp_spin<P, 3, 1, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
        default: dp_spin<P, 3, 0, DAG, NRP>(a, U, hn, ph, rp, W, lane); break;
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int r = 0; r < NRP; ++r) {
        const size_t off = (rp + r) * a.rhs_stride;
        const R cy = R(a.by[rp + r]);
        for (int u = wv; u < UIO::NU; u += 8) {
          cplx<R> o[UIO::CPU], xv[UIO::CPU], yv[UIO::CPU];
          if (a.x) epi_load_unit<P, ST>(a.x + off, u, h, Vh, xv);
          if (a.y) epi_load_unit<P, ST>(a.y + off, u, h, Vh, yv);
#pragma unroll
          for (int q = 0; q < UIO::CPU; ++q) {
            const int comp = u * UIO::CPU + q;
            const int s = comp / 3;
            o[q] = ca * dp_recon<DAG>(W + r * 8 * 6 * kDpSites, s, comp - 3 * s, lane);
            if (a.x) o[q] = o[q] + cx * xv[q];
            if (a.g5 && s >= 2) o[q] = R(-1) * o[q];
            if (a.y) o[q] = o[q] + cy * yv[q];
          }
          if constexpr (CHEB) {
            cheb_unit<P, ST>(a, off, u, h, Vh, o);
            continue;
          }
          epi_store_unit<P, ST>(a.out + off, u, h, Vh, o);
          if (a.dot == 1) {
            cplx<R> dv[UIO::CPU];
            epi_load_unit<P, ST>(a.dotv + off, u, h, Vh, dv);
#pragma unroll
            for (int q = 0; q < UIO::CPU; ++q)
              part[pass * NRP + r] += double(dv[q].r) * double(o[q].r) + double(dv[q].i) * double(o[q].i);
          } else if (a.dot == 2) {
#pragma unroll
            for (int q = 0; q < UIO::CPU; ++q)
              part[pass * NRP + r] += double(o[q].r) * double(o[q].r) + double(o[q].i) * double(o[q].i);
          }
        }
      }
    }
    if (pass + 1 < NPASS) __syncthreads();  // W is rewritten by the next pass
  }
  if (a.dot) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double sum = block_sum(part[r], red);
      if (threadIdx.x == 0) a.partials[(r0 + r) * a.part_stride + a.part_off + tile] = sum;
    }
  }
}

int hop_tiles(const wl_lattice* L, Prec) { return (L->Vh + kDpSites - 1) / kDpSites; }

template <typename P, int DAG, int NRP, bool ST>
static void dispatch_dp(HopArgs a, int nrhs, hipStream_t st, int max_pass) {
  // passes per block: the largest of 4, 2, 1 within max_pass dividing the rhs groups
  const int groups = nrhs / NRP;
  const int npass = (max_pass >= 4 && groups % 4 == 0) ? 4 : ((max_pass >= 2 && groups % 2 == 0) ? 2 : 1);
  a.rows = groups / npass;
  const dim3 grid(hop_grid<kDpSites>(a));
  switch (npass) {
    case 4: hipLaunchKernelGGL((hop_dp_kernel<P, DAG, NRP, 4, ST>), grid, dim3(kDpThreads), 0, st, a); break;
    case 2: hipLaunchKernelGGL((hop_dp_kernel<P, DAG, NRP, 2, ST>), grid, dim3(kDpThreads), 0, st, a); break;
    default: hipLaunchKernelGGL((hop_dp_kernel<P, DAG, NRP, 1, ST>), grid, dim3(kDpThreads), 0, st, a); break;
  }
}

template <typename P, int DAG, bool ST>
static void dispatch_nr(HopArgs a, int nrhs, hipStream_t st, const HopConfig& c) {
  if constexpr (DAG == 0) {
    if (a.ch_t) {  // fused Chebyshev step: forward hop, one rhs per pass / thread
      a.rows = nrhs;
      if (c.variant == kHopDirParallel)
        hipLaunchKernelGGL((hop_dp_kernel<P, 0, 1, 1, ST, true>), dim3(hop_grid<kDpSites>(a)), dim3(kDpThreads), 0,
                           st, a);
      else
        hipLaunchKernelGGL((hop_kernel<P, 0, 1, ST, true>), dim3(hop_grid<kBlock>(a)), dim3(kBlock), 0, st, a);
      return;
    }
  }
  // rhs per LDS pass (direction-parallel) or per thread (site): two for FP32
  // and BF16 with an even rhs count when the configuration allows, else one
  constexpr bool narrow = sizeof(typename P::real) == 4;
  // shared links from four rhs on; below that the plain thread-per-site kernel
  if (c.variant == kHopSiteShared && nrhs >= 4) {
    a.rows = (nrhs + 3) / 4;
    hipLaunchKernelGGL((hop_kernel<P, DAG, 1, ST, false, true>), dim3(hop_grid<kSiteTile>(a)), dim3(kBlock), 0, st,
                       a);
    return;
  }
  const bool two = narrow && nrhs % 2 == 0 && (c.variant == kHopDirParallel || c.npass >= 2);
  if (c.variant == kHopDirParallel) {
    if constexpr (narrow) {
      if (two) {
        dispatch_dp<P, DAG, 2, ST>(a, nrhs, st, c.npass);
        return;
      }
    }
    dispatch_dp<P, DAG, 1, ST>(a, nrhs, st, c.npass);
    return;
  }
  if constexpr (narrow) {
    if (two) {
      a.rows = nrhs / 2;
      hipLaunchKernelGGL((hop_kernel<P, DAG, 2, ST>), dim3(hop_grid<kBlock>(a)), dim3(kBlock), 0, st, a);
      return;
    }
  }
  a.rows = nrhs;
  hipLaunchKernelGGL((hop_kernel<P, DAG, 1, ST>), dim3(hop_grid<kBlock>(a)), dim3(kBlock), 0, st, a);
}

template <typename P>
static void dispatch(const HopArgs& a, int dagger, int nrhs, hipStream_t st, const HopConfig& c) {
  if (c.stream) {
    if (dagger) dispatch_nr<P, 1, true>(a, nrhs, st, c);
    else dispatch_nr<P, 0, true>(a, nrhs, st, c);
  } else {
    if (dagger) dispatch_nr<P, 1, false>(a, nrhs, st, c);
    else dispatch_nr<P, 0, false>(a, nrhs, st, c);
  }
}

// ------------------------------------------------------------------ mixed-volume batch
// One launch over the hops of several lattices of different volumes (one rhs
// each; its own geometry, links, fields and epilogue).  Lattice l owns tiles
// [tile0[l], tile0[l + 1]) of the batch's tile range.  Fields are tiled by 64
// sites, so a site's address does not depend on the lattice's extent and each
// lattice's fields can sit in equal slots sized for the largest lattice.
// Persistent: the grid holds at most the workgroups resident at once, each
// walking the tile range with stride gridDim.x.
struct BatchDesc {
  Geo g;
  int parity;
  const char* links;
  const char* in;
  char* out;
  const char* x;  // epilogue: out = g5^g5 (cx x + a hop) + by y
  const char* y;
  double cx, a, by;
  int g5;
  int dot;  // 1: Re<dotv, out> partial sums into partials[tile], zero up to part_len
  const char* dotv;
  double* partials;
};
struct BatchArgs {
  BatchDesc d[kMaxBatch];
  int tile0[kMaxBatch + 1];
  int nlat;
  int part_len;
};

// one wavefront's direction of a batch tile: link, neighbour, projected product into LDS
template <typename P, int MU, int FWD, int DAG>
__device__ __forceinline__ void dp_dir(const HopArgs& a, const Coord& c, int h, cplx<typename P::real>* W, int lane) {
  typename DpLink<P>::type U;
  int hn = 0;
  typename P::real ph;
  dp_link<P, MU, FWD, false>(a, c, h, &U, &hn, &ph);
  dp_spin<P, MU, FWD, DAG, 1>(a, U, hn, ph, 0, W, lane);
}

template <typename P, int DAG>
__global__ __launch_bounds__(kDpThreads) void hop_dp_batch_kernel(BatchArgs ba) {
  using R = typename P::real;
  using UIO = UnitIO<P>;
  __shared__ cplx<R> W[8 * 6 * kDpSites];
  __shared__ double red[kDpThreads / 64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  // each row of partial sums is summed whole: clear what the lattice's tiles leave
  for (int l = blockIdx.x; l < ba.nlat; l += gridDim.x)
    if (ba.d[l].dot)
      for (int i = ba.tile0[l + 1] - ba.tile0[l] + int(threadIdx.x); i < ba.part_len; i += kDpThreads)
        ba.d[l].partials[i] = 0.0;
  // XCD-aware: with the grid a multiple of 8, the workgroups the hardware puts
  // on one XCD walk one contiguous eighth of the concatenated tiles, so a
  // tile's neighbours are mostly read through that XCD's own L2
  const int total = ba.tile0[ba.nlat];
  int t0 = blockIdx.x, t1 = total, step = gridDim.x;
  if ((gridDim.x & 7) == 0) {
    const int per = (total + 7) >> 3;
    step = gridDim.x >> 3;
    t0 = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    t1 = min(total, ((blockIdx.x & 7) + 1) * per);
  }
  for (int t = t0; t < t1; t += step) {
    int l = 0;
    while (l + 1 < ba.nlat && t >= ba.tile0[l + 1]) ++l;
    const BatchDesc& d = ba.d[l];
    HopArgs a;  // the fields the direction helpers read
    a.g = d.g;
    a.parity = d.parity;
    a.links = d.links;
    a.in = d.in;
    a.rhs_stride = 0;
    const int tile = t - ba.tile0[l];
    const int h = tile * kDpSites + lane;
    const int Vh = d.g.Vh;
    const bool active = h < Vh;
    if (active) {
      const Coord c = site_coords(a.g, h, a.parity);
      switch (wv) {
        case 0: dp_dir<P, 0, 1, DAG>(a, c, h, W, lane); break;
        case 1: dp_dir<P, 0, 0, DAG>(a, c, h, W, lane); break;
        case 2: dp_dir<P, 1, 1, DAG>(a, c, h, W, lane); break;
        case 3: dp_dir<P, 1, 0, DAG>(a, c, h, W, lane); break;
        case 4: dp_dir<P, 2, 1, DAG>(a, c, h, W, lane); break;
        case 5: dp_dir<P, 2, 0, DAG>(a, c, h, W, lane); break;
        case 6: dp_dir<P, 3, 1, DAG>(a, c, h, W, lane); break;
        default: dp_dir<P, 3, 0, DAG>(a, c, h, W, lane); break;
      }
    }
    __syncthreads();
    double part = 0.0;
    if (active) {
      const R ca = R(d.a), cx = R(d.cx), cy = R(d.by);
      for (int u = wv; u < UIO::NU; u += 8) {
        cplx<R> o[UIO::CPU], xv[UIO::CPU], yv[UIO::CPU];
        if (d.x) UIO::load(d.x, u, h, Vh, xv);
        if (d.y) UIO::load(d.y, u, h, Vh, yv);
#pragma unroll
        for (int q = 0; q < UIO::CPU; ++q) {
          const int comp = u * UIO::CPU + q;
          const int sp = comp / 3;
          o[q] = ca * dp_recon<DAG>(W, sp, comp - 3 * sp, lane);
          if (d.x) o[q] = o[q] + cx * xv[q];
          if (d.g5 && sp >= 2) o[q] = R(-1) * o[q];
          if (d.y) o[q] = o[q] + cy * yv[q];
        }
        UIO::store(d.out, u, h, Vh, o);
        if (d.dot) {
          cplx<R> dv[UIO::CPU];
          UIO::load(d.dotv, u, h, Vh, dv);
#pragma unroll
          for (int q = 0; q < UIO::CPU; ++q) part += double(dv[q].r) * double(o[q].r) + double(dv[q].i) * double(o[q].i);
        }
      }
    }
    if (d.dot) {
      const double sum = block_sum(part, red);
      if (threadIdx.x == 0) d.partials[tile] = sum;
    }
    __syncthreads();  // W and red are rewritten by the next tile
  }
}

template <typename P, int DAG>
static int batch_grid(int total) {
  // workgroups resident at once on the current device (cached per instantiation and device)
  constexpr int kMaxDevices = 64;
  static std::atomic<int> resident[kMaxDevices];
  int dev = 0;
  WL_HIP(hipGetDevice(&dev));
  WL_REQUIRE(dev >= 0 && dev < kMaxDevices, WL_EUNSUPPORTED, "batch: device index out of range");
  int n = resident[dev].load();
  if (!n) {
    int cus = 0, per_cu = 0;
    WL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    WL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hop_dp_batch_kernel<P, DAG>, kDpThreads, 0));
    n = std::max(1, cus * per_cu);
    resident[dev].store(n);
  }
  // a multiple of 8 for the kernel's XCD-aware tile ranges (some workgroups
  // may find no tile)
  return (std::min(total, n) + 7) & ~7;
}

void launch_hop_batch(hipStream_t st, Prec prec, int out_parity, int dagger, const BatchHop* hops, int nlat,
                      int part_len) {
  WL_REQUIRE(nlat >= 1 && nlat <= kMaxBatch, WL_EINVAL, "batch: 1 to 8 lattices");
  BatchArgs ba{};
  ba.nlat = nlat;
  ba.part_len = part_len;
  ba.tile0[0] = 0;
  for (int l = 0; l < nlat; ++l) {
    const BatchHop& b = hops[l];
    wl_lattice* L = b.L;
    WL_REQUIRE(b.out != b.in, WL_EINVAL, "hop output must not alias its input");
    WL_REQUIRE(!b.e.dot || (b.e.dot == 1 && b.e.partials && hop_tiles(L, prec) <= part_len), WL_EINVAL,
               "batch: dot partials need a row of at least the lattice's tiles");
    ensure_lowp_links(L);
    BatchDesc& d = ba.d[l];
    d.g = L->geo;
    d.parity = out_parity;
    d.links = static_cast<const char*>(L->U[prec]);
    d.in = static_cast<const char*>(b.in);
    d.out = static_cast<char*>(b.out);
    d.x = static_cast<const char*>(b.e.x);
    d.y = static_cast<const char*>(b.e.y);
    d.cx = b.e.cx;
    d.a = b.e.a;
    d.by = b.e.by[0];
    d.g5 = b.e.g5;
    d.dot = b.e.dot;
    d.dotv = static_cast<const char*>(b.e.dotv);
    d.partials = b.e.partials;
    ba.tile0[l + 1] = ba.tile0[l] + hop_tiles(L, prec);
  }
  const int total = ba.tile0[nlat];
  auto go = [&](auto P) {
    using PT = decltype(P);
    if (dagger)
      hipLaunchKernelGGL((hop_dp_batch_kernel<PT, 1>), dim3(batch_grid<PT, 1>(total)), dim3(kDpThreads), 0, st, ba);
    else
      hipLaunchKernelGGL((hop_dp_batch_kernel<PT, 0>), dim3(batch_grid<PT, 0>(total)), dim3(kDpThreads), 0, st, ba);
  };
  switch (prec) {
    case F64: go(PrecF64{}); break;
    case F32: go(PrecF32{}); break;
    case BF16: go(PrecBF16{}); break;
  }
  WL_HIP(hipGetLastError());
}

void launch_hop(wl_lattice* L, Prec prec, void* out, const void* in, int out_parity, int dagger,
                int nrhs, const HopEpi& e) {
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs out of range");
  WL_REQUIRE(out != in, WL_EINVAL, "hop output must not alias its input");
  WL_REQUIRE(!e.cheb_t || (!dagger && !e.dot), WL_EINVAL, "fused Chebyshev step: forward hop, no dot");
  ensure_lowp_links(L);
  HopArgs a;
  a.g = L->geo;
  a.parity = out_parity;
  a.in = static_cast<const char*>(in);
  a.out = static_cast<char*>(out);
  a.links = static_cast<const char*>(L->U[prec]);
  a.rhs_stride = spinor_bytes(prec, L->Vh);
  a.nrhs = nrhs;
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
  a.ch_t = static_cast<const char*>(e.cheb_t);
  a.ch_tprev = static_cast<char*>(e.cheb_tprev);
  a.ch_e = static_cast<const char*>(e.cheb_e);
  a.ch_eprev = static_cast<char*>(e.cheb_eprev);
  a.ch_ct = e.cheb_ct;
  a.ch_cw = e.cheb_cw;
  a.ch_ce = e.cheb_ce;
  const HopConfig& cfg = L->hop_cfg[prec][hop_kind(nrhs)];
  a.use_xcd = cfg.use_xcd;
  // sampled event timing (never inside a graph capture)
  const bool timed = L->prof_on && !L->prof_capturing && !L->prof_suspended && nrhs == 1 &&
                     L->prof_ev[prec].size() < 2 * kProfPairs;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    WL_HIP(hipEventRecord(e0, L->stream));
  }
  switch (prec) {
    case F64: dispatch<PrecF64>(a, dagger, nrhs, L->stream, cfg); break;
    case F32: dispatch<PrecF32>(a, dagger, nrhs, L->stream, cfg); break;
    case BF16: dispatch<PrecBF16>(a, dagger, nrhs, L->stream, cfg); break;
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
