// Device-side building blocks for the Wilson-fermion kernels on gfx950.
//
// Conventions (the paper fixes none; see include/wilson_hmc.h):
//   * half-lattice site h of parity p: xh = h % (Lx/2), then y, z, t from
//     h / (Lx/2); x = 2*xh + ((y + z + t + p) & 1).  The i-th site of a parity
//     in lexicographic order s = x + Lx*(y + Ly*(z + Lz*t)) has h = i.
//   * spinor component c = 3*spin + colour; chiral gamma basis with
//     gamma_5 = diag(1, 1, -1, -1).
//   * storage is structure-of-arrays within tiles of 64 sites, so that a
//     wavefront reads 64 consecutive sites per load instruction (16 bytes per
//     lane) and all components of a tile lie in one contiguous block:
//     element (component u of NU, site h) sits at ((h/64) NU + u) 64 + h%64,
//     and a field spans Vh rounded up to a multiple of 64 sites:
//       F64  spinor: double2, NU = 12   link: double2, NU = 6  (two rows)
//       F32  spinor: float4,  NU = 6    link: float4,  NU = 3  (two rows)
//       BF16 spinor: uint4,   NU = 3    link: uint2,   NU = 3  (two rows)
//     with the third link row rebuilt as conj(row0 x row1) (SU(3)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wl {

// ------------------------------------------------------------------ tiled field index
constexpr int kSiteTile = 64;
__host__ __device__ constexpr int padded_sites(int n) { return (n + kSiteTile - 1) / kSiteTile * kSiteTile; }
__device__ __forceinline__ int fidx(int u, int h, int NU) { return ((h >> 6) * NU + u) * kSiteTile + (h & 63); }

// ------------------------------------------------------------------ complex
template <typename T>
struct cplx {
  T r, i;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.r, s * a.i}; }
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.r, -a.i}; }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
// i * a
template <typename T>
__device__ __forceinline__ cplx<T> times_i(cplx<T> a) { return {-a.i, a.r}; }
template <typename T>
__device__ __forceinline__ cplx<T> zero() { return {T(0), T(0)}; }

// ------------------------------------------------------------------ bf16
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
// two FP32 values rounded to nearest even into one word (lo, hi): one
// v_cvt_pk_bf16_f32 on gfx950
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

// ------------------------------------------------------------------ storage precisions
struct PrecF64 {
  using real = double;
  static constexpr int spinor_bytes = 192;  // per site per rhs
};
struct PrecF32 {
  using real = float;
  static constexpr int spinor_bytes = 96;
};
struct PrecBF16 {
  using real = float;  // compute type
  static constexpr int spinor_bytes = 48;
};

template <typename T>
struct Spinor {
  cplx<T> c[12];  // 3*spin + colour
};
template <typename T>
struct Half {
  cplx<T> c[6];  // 3*k + colour, k = 0, 1
};
template <typename T>
struct SU3 {
  cplx<T> m[9];  // row-major
};

// ------------------------------------------------------------------ streaming access
// Non-temporal loads and stores for data a hop touches exactly once (links:
// each link serves one output site forward and one backward; the epilogue's
// operands; the output), so that on volumes beyond the caches they do not push
// the neighbour spinors, which are read 8 times, out of L2.  On volumes that
// fit the caches the next kernel's input is this one's output, and streaming
// stores lose that reuse: the hop takes them as a per-launch option.
typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef unsigned v2u_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const v2d_t v = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const v4f_t v = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_stream(const uint2* p) {
  const v2u_t v = __builtin_nontemporal_load(reinterpret_cast<const v2u_t*>(p));
  return make_uint2(v.x, v.y);
}
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
  const v4u_t v = __builtin_nontemporal_load(reinterpret_cast<const v4u_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
// non-temporal stores for hop outputs: the hop never reads them back
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  __builtin_nontemporal_store(v2d_t{v.x, v.y}, reinterpret_cast<v2d_t*>(p));
}
__device__ __forceinline__ void st_stream(float4* p, float4 v) {
  __builtin_nontemporal_store(v4f_t{v.x, v.y, v.z, v.w}, reinterpret_cast<v4f_t*>(p));
}
__device__ __forceinline__ void st_stream(uint4* p, uint4 v) {
  __builtin_nontemporal_store(v4u_t{v.x, v.y, v.z, v.w}, reinterpret_cast<v4u_t*>(p));
}

// spinor load/store: base points at one rhs of one parity
template <typename P>
struct SpinorIO;

template <>
struct SpinorIO<PrecF64> {
  static __device__ __forceinline__ Spinor<double> load(const void* base, int h, int Vh) {
    const double2* b = reinterpret_cast<const double2*>(base);
    Spinor<double> s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double2 v = b[fidx(c, h, 12)];
      s.c[c] = {v.x, v.y};
    }
    return s;
  }
  static __device__ __forceinline__ void store(void* base, int h, int Vh, const Spinor<double>& s) {
    double2* b = reinterpret_cast<double2*>(base);
#pragma unroll
    for (int c = 0; c < 12; ++c) b[fidx(c, h, 12)] = make_double2(s.c[c].r, s.c[c].i);
  }
  static __device__ __forceinline__ Spinor<double> load_nt(const void* base, int h, int Vh) {
    const double2* b = reinterpret_cast<const double2*>(base);
    Spinor<double> s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 v = ld_stream(b + fidx(c, h, 12));
      s.c[c] = {v.x, v.y};
    }
    return s;
  }
  static __device__ __forceinline__ void store_nt(void* base, int h, int Vh, const Spinor<double>& s) {
    double2* b = reinterpret_cast<double2*>(base);
#pragma unroll
    for (int c = 0; c < 12; ++c) st_stream(b + fidx(c, h, 12), make_double2(s.c[c].r, s.c[c].i));
  }
};

template <>
struct SpinorIO<PrecF32> {
  static __device__ __forceinline__ Spinor<float> load(const void* base, int h, int Vh) {
    const float4* b = reinterpret_cast<const float4*>(base);
    Spinor<float> s;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 v = b[fidx(j, h, 6)];
      s.c[2 * j] = {v.x, v.y};
      s.c[2 * j + 1] = {v.z, v.w};
    }
    return s;
  }
  static __device__ __forceinline__ void store(void* base, int h, int Vh, const Spinor<float>& s) {
    float4* b = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int j = 0; j < 6; ++j)
      b[fidx(j, h, 6)] = make_float4(s.c[2 * j].r, s.c[2 * j].i, s.c[2 * j + 1].r, s.c[2 * j + 1].i);
  }
  static __device__ __forceinline__ Spinor<float> load_nt(const void* base, int h, int Vh) {
    const float4* b = reinterpret_cast<const float4*>(base);
    Spinor<float> s;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float4 v = ld_stream(b + fidx(j, h, 6));
      s.c[2 * j] = {v.x, v.y};
      s.c[2 * j + 1] = {v.z, v.w};
    }
    return s;
  }
  static __device__ __forceinline__ void store_nt(void* base, int h, int Vh, const Spinor<float>& s) {
    float4* b = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int j = 0; j < 6; ++j)
      st_stream(b + fidx(j, h, 6), make_float4(s.c[2 * j].r, s.c[2 * j].i, s.c[2 * j + 1].r, s.c[2 * j + 1].i));
  }
};

template <>
struct SpinorIO<PrecBF16> {
  static __device__ __forceinline__ Spinor<float> load(const void* base, int h, int Vh) {
    const uint4* b = reinterpret_cast<const uint4*>(base);
    Spinor<float> s;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uint4 v = b[fidx(j, h, 3)];
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) s.c[4 * j + q] = {bf16_to_f32(w[q] & 0xFFFFu), bf16_to_f32(w[q] >> 16)};
    }
    return s;
  }
  static __device__ __forceinline__ void store(void* base, int h, int Vh, const Spinor<float>& s) {
    uint4* b = reinterpret_cast<uint4*>(base);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uint4 v;
      v.x = pack_bf16x2(s.c[4 * j + 0].r, s.c[4 * j + 0].i);
      v.y = pack_bf16x2(s.c[4 * j + 1].r, s.c[4 * j + 1].i);
      v.z = pack_bf16x2(s.c[4 * j + 2].r, s.c[4 * j + 2].i);
      v.w = pack_bf16x2(s.c[4 * j + 3].r, s.c[4 * j + 3].i);
      b[fidx(j, h, 3)] = v;
    }
  }
  static __device__ __forceinline__ Spinor<float> load_nt(const void* base, int h, int Vh) {
    const uint4* b = reinterpret_cast<const uint4*>(base);
    Spinor<float> s;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint4 v = ld_stream(b + fidx(j, h, 3));
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) s.c[4 * j + q] = {bf16_to_f32(w[q] & 0xFFFFu), bf16_to_f32(w[q] >> 16)};
    }
    return s;
  }
  static __device__ __forceinline__ void store_nt(void* base, int h, int Vh, const Spinor<float>& s) {
    uint4* b = reinterpret_cast<uint4*>(base);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uint4 v;
      v.x = pack_bf16x2(s.c[4 * j + 0].r, s.c[4 * j + 0].i);
      v.y = pack_bf16x2(s.c[4 * j + 1].r, s.c[4 * j + 1].i);
      v.z = pack_bf16x2(s.c[4 * j + 2].r, s.c[4 * j + 2].i);
      v.w = pack_bf16x2(s.c[4 * j + 3].r, s.c[4 * j + 3].i);
      st_stream(b + fidx(j, h, 3), v);
    }
  }
};

// storage units of a spinor: 16-byte vectors (F64: 1 complex, F32: 2, BF16: 4)
template <typename P>
struct UnitIO;

template <>
struct UnitIO<PrecF64> {
  static constexpr int NU = 12, CPU = 1;
  static __device__ __forceinline__ void load(const void* base, int u, int h, int Vh, cplx<double>* c) {
    const double2 v = reinterpret_cast<const double2*>(base)[fidx(u, h, 12)];
    c[0] = {v.x, v.y};
  }
  static __device__ __forceinline__ void store(void* base, int u, int h, int Vh, const cplx<double>* c) {
    reinterpret_cast<double2*>(base)[fidx(u, h, 12)] = make_double2(c[0].r, c[0].i);
  }
  static __device__ __forceinline__ void load_nt(const void* base, int u, int h, int Vh, cplx<double>* c) {
    const double2 v = ld_stream(reinterpret_cast<const double2*>(base) + fidx(u, h, 12));
    c[0] = {v.x, v.y};
  }
  static __device__ __forceinline__ void store_nt(void* base, int u, int h, int Vh, const cplx<double>* c) {
    st_stream(reinterpret_cast<double2*>(base) + fidx(u, h, 12), make_double2(c[0].r, c[0].i));
  }
};

template <>
struct UnitIO<PrecF32> {
  static constexpr int NU = 6, CPU = 2;
  static __device__ __forceinline__ void load(const void* base, int u, int h, int Vh, cplx<float>* c) {
    const float4 v = reinterpret_cast<const float4*>(base)[fidx(u, h, 6)];
    c[0] = {v.x, v.y};
    c[1] = {v.z, v.w};
  }
  static __device__ __forceinline__ void store(void* base, int u, int h, int Vh, const cplx<float>* c) {
    reinterpret_cast<float4*>(base)[fidx(u, h, 6)] = make_float4(c[0].r, c[0].i, c[1].r, c[1].i);
  }
  static __device__ __forceinline__ void load_nt(const void* base, int u, int h, int Vh, cplx<float>* c) {
    const float4 v = ld_stream(reinterpret_cast<const float4*>(base) + fidx(u, h, 6));
    c[0] = {v.x, v.y};
    c[1] = {v.z, v.w};
  }
  static __device__ __forceinline__ void store_nt(void* base, int u, int h, int Vh, const cplx<float>* c) {
    st_stream(reinterpret_cast<float4*>(base) + fidx(u, h, 6), make_float4(c[0].r, c[0].i, c[1].r, c[1].i));
  }
};

template <>
struct UnitIO<PrecBF16> {
  static constexpr int NU = 3, CPU = 4;
  static __device__ __forceinline__ void load(const void* base, int u, int h, int Vh, cplx<float>* c) {
    const uint4 v = reinterpret_cast<const uint4*>(base)[fidx(u, h, 3)];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = {bf16_to_f32(w[q] & 0xFFFFu), bf16_to_f32(w[q] >> 16)};
  }
  static __device__ __forceinline__ void store(void* base, int u, int h, int Vh, const cplx<float>* c) {
    uint4 v;
    v.x = pack_bf16x2(c[0].r, c[0].i);
    v.y = pack_bf16x2(c[1].r, c[1].i);
    v.z = pack_bf16x2(c[2].r, c[2].i);
    v.w = pack_bf16x2(c[3].r, c[3].i);
    reinterpret_cast<uint4*>(base)[fidx(u, h, 3)] = v;
  }
  static __device__ __forceinline__ void load_nt(const void* base, int u, int h, int Vh, cplx<float>* c) {
    const uint4 v = ld_stream(reinterpret_cast<const uint4*>(base) + fidx(u, h, 3));
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = {bf16_to_f32(w[q] & 0xFFFFu), bf16_to_f32(w[q] >> 16)};
  }
  static __device__ __forceinline__ void store_nt(void* base, int u, int h, int Vh, const cplx<float>* c) {
    uint4 v;
    v.x = pack_bf16x2(c[0].r, c[0].i);
    v.y = pack_bf16x2(c[1].r, c[1].i);
    v.z = pack_bf16x2(c[2].r, c[2].i);
    v.w = pack_bf16x2(c[3].r, c[3].i);
    st_stream(reinterpret_cast<uint4*>(base) + fidx(u, h, 3), v);
  }
};

// link load: base points at [mu] block of one parity
template <typename T>
__device__ __forceinline__ void third_row(SU3<T>& u) {
  u.m[6] = conj(u.m[1] * u.m[5] - u.m[2] * u.m[4]);
  u.m[7] = conj(u.m[2] * u.m[3] - u.m[0] * u.m[5]);
  u.m[8] = conj(u.m[0] * u.m[4] - u.m[1] * u.m[3]);
}

template <typename P>
struct LinkIO;

template <>
struct LinkIO<PrecF64> {
  static constexpr int bytes = 96;  // per link: two rows of double2
  template <bool ST = false>
  static __device__ __forceinline__ SU3<double> load(const void* base, int h, int Vh) {
    const double2* b = reinterpret_cast<const double2*>(base);
    SU3<double> u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2 v = ST ? ld_stream(b + fidx(k, h, 6)) : b[fidx(k, h, 6)];
      u.m[k] = {v.x, v.y};
    }
    third_row(u);
    return u;
  }
};

template <>
struct LinkIO<PrecF32> {
  static constexpr int bytes = 48;
  template <bool ST = false>
  static __device__ __forceinline__ SU3<float> load(const void* base, int h, int Vh) {
    const float4* b = reinterpret_cast<const float4*>(base);
    SU3<float> u;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float4 v = ST ? ld_stream(b + fidx(j, h, 3)) : b[fidx(j, h, 3)];
      u.m[2 * j] = {v.x, v.y};
      u.m[2 * j + 1] = {v.z, v.w};
    }
    third_row(u);
    return u;
  }
};

template <>
struct LinkIO<PrecBF16> {
  static constexpr int bytes = 24;
  template <bool ST = false>
  static __device__ __forceinline__ SU3<float> load(const void* base, int h, int Vh) {
    const uint2* b = reinterpret_cast<const uint2*>(base);
    SU3<float> u;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint2 v = ST ? ld_stream(b + fidx(j, h, 3)) : b[fidx(j, h, 3)];
      u.m[2 * j] = {bf16_to_f32(v.x & 0xFFFFu), bf16_to_f32(v.x >> 16)};
      u.m[2 * j + 1] = {bf16_to_f32(v.y & 0xFFFFu), bf16_to_f32(v.y >> 16)};
    }
    third_row(u);
    return u;
  }
};

// ------------------------------------------------------------------ SU(3) x colour vector
template <typename T>
__device__ __forceinline__ void su3_mul(const SU3<T>& u, const cplx<T>* v, cplx<T>* w) {
#pragma unroll
  for (int a = 0; a < 3; ++a) w[a] = u.m[3 * a] * v[0] + u.m[3 * a + 1] * v[1] + u.m[3 * a + 2] * v[2];
}
template <typename T>
__device__ __forceinline__ void su3_dag_mul(const SU3<T>& u, const cplx<T>* v, cplx<T>* w) {
#pragma unroll
  for (int a = 0; a < 3; ++a) w[a] = cmul(u.m[a], v[0]) + cmul(u.m[3 + a], v[1]) + cmul(u.m[6 + a], v[2]);
}

// ------------------------------------------------------------------ spin projection
// (1 + s gamma_MU) psi, s = +-1, has two independent spin rows h0, h1 (chiral
// basis); the lower rows are phases times h0 / h1.  MU = 0..3 is x, y, z, t.
template <int MU, typename T>
__device__ __forceinline__ Half<T> project_s(const Spinor<T>& p, T s) {
  Half<T> h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> p0 = p.c[a], p1 = p.c[3 + a], p2 = p.c[6 + a], p3 = p.c[9 + a];
    if (MU == 0) {         // h0 = p0 - s i p3, h1 = p1 - s i p2
      h.c[a] = p0 - s * times_i(p3);
      h.c[3 + a] = p1 - s * times_i(p2);
    } else if (MU == 1) {  // h0 = p0 - s p3, h1 = p1 + s p2
      h.c[a] = p0 - s * p3;
      h.c[3 + a] = p1 + s * p2;
    } else if (MU == 2) {  // h0 = p0 - s i p2, h1 = p1 + s i p3
      h.c[a] = p0 - s * times_i(p2);
      h.c[3 + a] = p1 + s * times_i(p3);
    } else {               // h0 = p0 + s p2, h1 = p1 + s p3
      h.c[a] = p0 + s * p2;
      h.c[3 + a] = p1 + s * p3;
    }
  }
  return h;
}
template <int MU, int S, typename T>
__device__ __forceinline__ Half<T> project(const Spinor<T>& p) {
  return project_s<MU>(p, T(S));
}

// acc += (1 + S gamma_MU)-reconstruction of the half spinor w
template <int MU, int S, typename T>
__device__ __forceinline__ void reconstruct_add(Spinor<T>& acc, const Half<T>& w) {
  const T s = T(S);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> h0 = w.c[a], h1 = w.c[3 + a];
    acc.c[a] = acc.c[a] + h0;
    acc.c[3 + a] = acc.c[3 + a] + h1;
    if (MU == 0) {         // r2 = s i h1, r3 = s i h0
      acc.c[6 + a] = acc.c[6 + a] + s * times_i(h1);
      acc.c[9 + a] = acc.c[9 + a] + s * times_i(h0);
    } else if (MU == 1) {  // r2 = s h1, r3 = -s h0
      acc.c[6 + a] = acc.c[6 + a] + s * h1;
      acc.c[9 + a] = acc.c[9 + a] - s * h0;
    } else if (MU == 2) {  // r2 = s i h0, r3 = -s i h1
      acc.c[6 + a] = acc.c[6 + a] + s * times_i(h0);
      acc.c[9 + a] = acc.c[9 + a] - s * times_i(h1);
    } else {               // r2 = s h0, r3 = s h1
      acc.c[6 + a] = acc.c[6 + a] + s * h0;
      acc.c[9 + a] = acc.c[9 + a] + s * h1;
    }
  }
}

// ------------------------------------------------------------------ geometry
struct Geo {
  int L[4];
  int Lxh;   // Lx / 2
  int Vh;    // V / 2
  int Vhp;   // Vh rounded up to whole 64-site tiles (field extent)
  int tbc;   // +1 periodic, -1 antiperiodic in time (fermions only)
  // reciprocals of Lxh, Ly, Lz for the site-coordinate divisions (geo_init)
  double rcp[3];
};

// fill the derived fields of a geometry whose L, Lxh, Vh, Vhp, tbc are set
inline void geo_init(Geo& g) {
  g.rcp[0] = 1.0 / g.Lxh;
  g.rcp[1] = 1.0 / g.L[1];
  g.rcp[2] = 1.0 / g.L[2];
}

// floor(n / d) for 0 <= n < 2^30 and 1 <= d <= 2^15, r = 1 / d rounded to
// nearest: (n + 1/2) r in FP64 is within 2^-22 of (n + 1/2) / d, whose
// distance to the nearest integer is at least 1 / (2 d) >= 2^-16, so the
// truncation is exact (three instructions instead of an integer division)
__device__ __forceinline__ int div_rcp(int n, double r) {
  return int(__builtin_fma(double(n), r, 0.5 * r));
}

struct Coord {
  int x, y, z, t;
};

__device__ __forceinline__ Coord site_coords(const Geo& g, int h, int parity) {
  Coord c;
  int r = div_rcp(h, g.rcp[0]);
  const int xh = h - r * g.Lxh;
  int q = div_rcp(r, g.rcp[1]);
  c.y = r - q * g.L[1];
  c.t = div_rcp(q, g.rcp[2]);
  c.z = q - c.t * g.L[2];
  c.x = 2 * xh + ((c.y + c.z + c.t + parity) & 1);
  return c;
}

__device__ __forceinline__ int half_index(const Geo& g, int x, int y, int z, int t) {
  return (x >> 1) + g.Lxh * (y + g.L[1] * (z + g.L[2] * t));
}

// half index of x + dir * mu_hat (periodic wrap); *wrapped = crossed the time edge
template <int MU>
__device__ __forceinline__ int neighbour(const Geo& g, Coord c, int dir, bool* wrapped) {
  int x = c.x, y = c.y, z = c.z, t = c.t;
  *wrapped = false;
  if (MU == 0) {
    x += dir;
    x = (x < 0) ? x + g.L[0] : (x >= g.L[0] ? x - g.L[0] : x);
  } else if (MU == 1) {
    y += dir;
    y = (y < 0) ? y + g.L[1] : (y >= g.L[1] ? y - g.L[1] : y);
  } else if (MU == 2) {
    z += dir;
    z = (z < 0) ? z + g.L[2] : (z >= g.L[2] ? z - g.L[2] : z);
  } else {
    t += dir;
    if (t < 0) {
      t += g.L[3];
      *wrapped = true;
    } else if (t >= g.L[3]) {
      t -= g.L[3];
      *wrapped = true;
    }
  }
  return half_index(g, x, y, z, t);
}

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin
// over the 8 XCDs (each with its own L2); renumber so that each XCD walks a
// contiguous range of sites and finds its neighbours' data in its own L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ------------------------------------------------------------------ wavefront reduction
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum (blockDim.x a multiple of 64, at most 1024); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) s += lds[k];
  }
  __syncthreads();
  return s;
}

}  // namespace wl
