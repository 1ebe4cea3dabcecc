// Layout conversion at the library boundary: canonical lexicographic arrays
// (complex128 [V][4][3] spinors, [4][V][3][3] links, float64 [4][V][8]
// su(3) coefficients) <-> the internal even-odd structure-of-arrays layouts of
// wl_device.h, and the FP32 / BF16 two-row copies of the links.
#include "wl_internal.h"

namespace wl {

// parity and half index of the flat site s (all extents even)
__device__ __forceinline__ void site_parity(const Geo& g, int s, int* p, int* h) {
  int x = s % g.L[0];
  int r = s / g.L[0];
  int y = r % g.L[1];
  r /= g.L[1];
  int z = r % g.L[2];
  int t = r / g.L[2];
  *p = (x + y + z + t) & 1;
  *h = s >> 1;
}

__global__ void pack_links_kernel(Geo g, const double2* canon, double2* U) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  const int V = 2 * g.Vh;
  if (s >= V) return;
  int p, h;
  site_parity(g, s, &p, &h);
  const double2* src = canon + (size_t(mu) * V + s) * 9;
  double2* dst = U + size_t(p * 4 + mu) * 9 * g.Vhp;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[fidx(k, h, 9)] = src[k];
}

__global__ void unpack_links_kernel(Geo g, double2* canon, const double2* U) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  const int V = 2 * g.Vh;
  if (s >= V) return;
  int p, h;
  site_parity(g, s, &p, &h);
  double2* dst = canon + (size_t(mu) * V + s) * 9;
  const double2* src = U + size_t(p * 4 + mu) * 9 * g.Vhp;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k] = src[fidx(k, h, 9)];
}

// hop copies of the links (FP64, FP32, BF16) keep the first two rows only
__global__ void lowp_links_kernel(Geo g, const double2* U, double2* U64, float4* U32, uint2* U16) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int pm = blockIdx.y;  // parity * 4 + mu
  if (h >= g.Vh) return;
  const double2* src = U + size_t(pm) * 9 * g.Vhp;
  double2 m[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) m[k] = src[fidx(k, h, 9)];
#pragma unroll
  for (int k = 0; k < 6; ++k) U64[size_t(pm) * 6 * g.Vhp + fidx(k, h, 6)] = m[k];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double2 a = m[2 * j], b = m[2 * j + 1];
    U32[size_t(pm) * 3 * g.Vhp + fidx(j, h, 3)] = make_float4(float(a.x), float(a.y), float(b.x), float(b.y));
    uint2 v;
    v.x = pack_bf16x2(float(a.x), float(a.y));
    v.y = pack_bf16x2(float(b.x), float(b.y));
    U16[size_t(pm) * 3 * g.Vhp + fidx(j, h, 3)] = v;
  }
}

template <typename P>
__global__ void import_spinor_kernel(Geo g, char* dst, size_t stride, const double2* canon) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (h >= g.Vh) return;
  const double2* src = canon + (size_t(r) * g.Vh + h) * 12;
  Spinor<typename P::real> s;
#pragma unroll
  for (int k = 0; k < 12; ++k) s.c[k] = {typename P::real(src[k].x), typename P::real(src[k].y)};
  SpinorIO<P>::store(dst + r * stride, h, g.Vh, s);
}

template <typename P>
__global__ void export_spinor_kernel(Geo g, double2* canon, const char* src, size_t stride) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (h >= g.Vh) return;
  const auto s = SpinorIO<P>::load(src + r * stride, h, g.Vh);
  double2* dst = canon + (size_t(r) * g.Vh + h) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2(double(s.c[k].r), double(s.c[k].i));
}

// canonical full field <-> (even half, odd half) of F64 internal fields
__global__ void split_full_kernel(Geo g, char* even, char* odd, double2* canon, int to_canon) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= 2 * g.Vh) return;
  int p, h;
  site_parity(g, s, &p, &h);
  char* half = p ? odd : even;
  double2* c = canon + size_t(s) * 12;
  if (to_canon) {
    const Spinor<double> v = SpinorIO<PrecF64>::load(half, h, g.Vh);
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = make_double2(v.c[k].r, v.c[k].i);
  } else {
    Spinor<double> v;
#pragma unroll
    for (int k = 0; k < 12; ++k) v.c[k] = {c[k].x, c[k].y};
    SpinorIO<PrecF64>::store(half, h, g.Vh, v);
  }
}

__global__ void su3_io_kernel(Geo g, double* internal, double* canon, int to_canon) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  const int V = 2 * g.Vh;
  if (s >= V) return;
  int p, h;
  site_parity(g, s, &p, &h);
  double* c = canon + (size_t(mu) * V + s) * 8;
  double* in = internal + size_t(p * 4 + mu) * 8 * g.Vh;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (to_canon) c[a] = in[a * g.Vh + h];
    else in[a * g.Vh + h] = c[a];
  }
}

// ------------------------------------------------------------------ launchers
void launch_pack_links(wl_lattice* L, const void* canon) {
  dim3 grid(site_blocks(L->V), 4);
  hipLaunchKernelGGL(pack_links_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, (const double2*)canon,
                     (double2*)L->Ufull);
  WL_HIP(hipGetLastError());
  L->lowp_valid = false;
}

void launch_unpack_links(wl_lattice* L, void* canon) {
  dim3 grid(site_blocks(L->V), 4);
  hipLaunchKernelGGL(unpack_links_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, (double2*)canon,
                     (const double2*)L->Ufull);
  WL_HIP(hipGetLastError());
}

void launch_lowp_links(wl_lattice* L) {
  dim3 grid(site_blocks(L->Vh), 8);
  hipLaunchKernelGGL(lowp_links_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, (const double2*)L->Ufull,
                     (double2*)L->U[F64], (float4*)L->U[F32], (uint2*)L->U[BF16]);
  WL_HIP(hipGetLastError());
  L->lowp_valid = true;
}

void launch_import_spinor(wl_lattice* L, Prec prec, void* dst, const void* canon, int nrhs) {
  dim3 grid(site_blocks(L->Vh), nrhs);
  const size_t st = spinor_bytes(prec, L->Vh);
  switch (prec) {
    case F64: hipLaunchKernelGGL((import_spinor_kernel<PrecF64>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)dst, st, (const double2*)canon); break;
    case F32: hipLaunchKernelGGL((import_spinor_kernel<PrecF32>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)dst, st, (const double2*)canon); break;
    case BF16: hipLaunchKernelGGL((import_spinor_kernel<PrecBF16>), grid, dim3(kBlock), 0, L->stream, L->geo, (char*)dst, st, (const double2*)canon); break;
  }
  WL_HIP(hipGetLastError());
}

void launch_export_spinor(wl_lattice* L, Prec prec, void* canon, const void* src, int nrhs) {
  dim3 grid(site_blocks(L->Vh), nrhs);
  const size_t st = spinor_bytes(prec, L->Vh);
  switch (prec) {
    case F64: hipLaunchKernelGGL((export_spinor_kernel<PrecF64>), grid, dim3(kBlock), 0, L->stream, L->geo, (double2*)canon, (const char*)src, st); break;
    case F32: hipLaunchKernelGGL((export_spinor_kernel<PrecF32>), grid, dim3(kBlock), 0, L->stream, L->geo, (double2*)canon, (const char*)src, st); break;
    case BF16: hipLaunchKernelGGL((export_spinor_kernel<PrecBF16>), grid, dim3(kBlock), 0, L->stream, L->geo, (double2*)canon, (const char*)src, st); break;
  }
  WL_HIP(hipGetLastError());
}

void launch_split_full(wl_lattice* L, void* even, void* odd, const void* canon_full, int to_canon) {
  hipLaunchKernelGGL(split_full_kernel, dim3(site_blocks(L->V)), dim3(kBlock), 0, L->stream, L->geo, (char*)even,
                     (char*)odd, (double2*)canon_full, to_canon);
  WL_HIP(hipGetLastError());
}

void launch_su3_io(wl_lattice* L, double* internal, const double* canon, int to_canon) {
  dim3 grid(site_blocks(L->V), 4);
  hipLaunchKernelGGL(su3_io_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, internal, (double*)canon, to_canon);
  WL_HIP(hipGetLastError());
}

}  // namespace wl
