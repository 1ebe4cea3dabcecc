// Link-space kernels of the HMC (Sec. 2): the fermion-force bilinear, the
// plaquette gauge force, the time step U -> exp(i eps P) U with SU(3)
// reunitarisation, and the FP64 reductions of the Hamiltonian.
//
// su(3) fields are float64 [parity][mu][8][Vh] (coefficients of
// P = sum_a p^a T^a, T^a = lambda^a / 2).  The Lie derivative of a linear form
// Re tr(i T^a G) is taken from the 3x3 matrix G by su3_grad below.
#include "wl_internal.h"

namespace wl {

using cd = cplx<double>;

__device__ __forceinline__ void mat_mul(const cd* a, const cd* b, cd* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
// c = a * b^dag
__device__ __forceinline__ void mat_mul_dag(const cd* a, const cd* b, cd* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * conj(b[3 * j]) + a[3 * i + 1] * conj(b[3 * j + 1]) + a[3 * i + 2] * conj(b[3 * j + 2]);
}
// c = a^dag * b
__device__ __forceinline__ void mat_dag_mul(const cd* a, const cd* b, cd* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c[3 * i + j] = cmul(a[i], b[j]) + cmul(a[3 + i], b[3 + j]) + cmul(a[6 + i], b[6 + j]);
}

// g^a = Re(i tr(T^a G)) = -Im tr(T^a G)
__device__ __forceinline__ void su3_grad(const cd* W, double* g) {
  g[0] = -0.5 * (W[1].i + W[3].i);
  g[1] = -0.5 * (W[1].r - W[3].r);
  g[2] = -0.5 * (W[0].i - W[4].i);
  g[3] = -0.5 * (W[2].i + W[6].i);
  g[4] = -0.5 * (W[2].r - W[6].r);
  g[5] = -0.5 * (W[5].i + W[7].i);
  g[6] = -0.5 * (W[5].r - W[7].r);
  g[7] = -(W[0].i + W[4].i - 2.0 * W[8].i) * 0.28867513459481288225;  // 1 / (2 sqrt 3)
}

// P = sum_a p^a T^a
__device__ __forceinline__ void su3_from_coeffs(const double* p, cd* H) {
  const double s3 = 0.57735026918962576451;  // 1 / sqrt 3
  H[0] = {0.5 * (p[2] + p[7] * s3), 0.0};
  H[4] = {0.5 * (-p[2] + p[7] * s3), 0.0};
  H[8] = {-p[7] * s3, 0.0};
  H[1] = {0.5 * p[0], -0.5 * p[1]};
  H[3] = {0.5 * p[0], 0.5 * p[1]};
  H[2] = {0.5 * p[3], -0.5 * p[4]};
  H[6] = {0.5 * p[3], 0.5 * p[4]};
  H[5] = {0.5 * p[5], -0.5 * p[6]};
  H[7] = {0.5 * p[5], 0.5 * p[6]};
}

// F64 links in the tiled layout of wl_device.h: block (parity, mu) of 9 x Vhp
__device__ __forceinline__ const double2* link_ptr(const void* U, int p, int mu, int Vhp) {
  return reinterpret_cast<const double2*>(U) + size_t(p * 4 + mu) * 9 * Vhp;
}

__device__ __forceinline__ void load_link(const void* U, int p, int mu, int h, int Vhp, cd* m) {
  const double2* b = link_ptr(U, p, mu, Vhp);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 v = b[fidx(k, h, 9)];
    m[k] = {v.x, v.y};
  }
}

__device__ __forceinline__ Coord step(const Geo& g, Coord c, int nu, int d) {
  int* v = nu == 0 ? &c.x : (nu == 1 ? &c.y : (nu == 2 ? &c.z : &c.t));
  *v += d;
  if (*v < 0) *v += g.L[nu];
  if (*v >= g.L[nu]) *v -= g.L[nu];
  return c;
}

__device__ __forceinline__ void load_link_at(const void* U, const Geo& g, Coord c, int mu, cd* m) {
  const int p = (c.x + c.y + c.z + c.t) & 1;
  load_link(U, p, mu, half_index(g, c.x, c.y, c.z, c.t), g.Vhp, m);
}

// ------------------------------------------------------------------ fermion bilinear
// For link (x, mu), y = x + mu:  W = U Xi - Theta U^dag with
//   Xi    = sum_k hC_k (x) hA_k^dag,  h = upper rows of (1 - g_mu) C(y), (1 - g_mu) A(x)
//   Theta = sum_k gC_k (x) gA_k^dag,  g = upper rows of (1 + g_mu) C(x), (1 + g_mu) A(y)
// (the lower spin rows of a projected spinor are unit phases times the upper
// rows, so the four-spin sums reduce to the two upper rows).  Xi and Theta
// have rank two, so W is formed without them and without any 3x3 product:
//   W_ij = sum_k (U hC_k)_i conj(hA_k)_j - gC_k,i conj(U gA_k)_j,
// four SU(3) x vector products and, of W, only the entries the su(3)
// coefficients read (imaginary diagonal, the six off-diagonal entries).  The
// link comes from the two-row FP64 copy, its third row rebuilt.
template <int MU>
__device__ __forceinline__ void bilinear_dir(const Geo& g, const Coord& c, int p, int h, const char* Ah[2],
                                             const char* Ch[2], const char* U2, double* F, double coeff) {
  bool wrap;
  const int hy = neighbour<MU>(g, c, +1, &wrap);
  const char* Ub = U2 + size_t(p * 4 + MU) * LinkIO<PrecF64>::bytes * g.Vhp;
  const double ph = wrap ? double(g.tbc) : 1.0;
  // W accumulated in two stages (U hC (x) hA^dag, then - gC (x) (U gA)^dag), the
  // scheduler kept from hoisting the second stage's loads into the first: four
  // spinors in flight at once held every wavefront to two per SIMD
  cd w01, w10, w02, w20, w12, w21;
  double d0, d1, d2;
  {
    const Half<double> hC = project<MU, -1>(SpinorIO<PrecF64>::load(Ch[1 - p], hy, g.Vh));
    const Half<double> hA = project<MU, -1>(SpinorIO<PrecF64>::load(Ah[p], h, g.Vh));
    const SU3<double> U = LinkIO<PrecF64>::load(Ub, h, g.Vh);
    cd u[6];  // ph U hC_k
    su3_mul(U, hC.c, u);
    su3_mul(U, hC.c + 3, u + 3);
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = ph * u[k];
    auto P = [&](int i, int j) { return u[i] * conj(hA.c[j]) + u[3 + i] * conj(hA.c[3 + j]); };
    w01 = P(0, 1), w10 = P(1, 0), w02 = P(0, 2), w20 = P(2, 0), w12 = P(1, 2), w21 = P(2, 1);
    d0 = P(0, 0).i, d1 = P(1, 1).i, d2 = P(2, 2).i;
  }
  __builtin_amdgcn_sched_barrier(0);
  {
    const Half<double> gA = project<MU, +1>(SpinorIO<PrecF64>::load(Ah[1 - p], hy, g.Vh));
    const Half<double> gC = project<MU, +1>(SpinorIO<PrecF64>::load(Ch[p], h, g.Vh));
    const SU3<double> U = LinkIO<PrecF64>::load(Ub, h, g.Vh);  // again, from the cache
    cd v[6];  // ph U gA_k
    su3_mul(U, gA.c, v);
    su3_mul(U, gA.c + 3, v + 3);
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = ph * v[k];
    auto Q = [&](int i, int j) { return gC.c[i] * conj(v[j]) + gC.c[3 + i] * conj(v[3 + j]); };
    w01 = w01 - Q(0, 1), w10 = w10 - Q(1, 0), w02 = w02 - Q(0, 2), w20 = w20 - Q(2, 0);
    w12 = w12 - Q(1, 2), w21 = w21 - Q(2, 1);
    d0 -= Q(0, 0).i, d1 -= Q(1, 1).i, d2 -= Q(2, 2).i;
  }
  // g^a = Re(i tr(T^a W)) = -Im tr(T^a W), T^a = lambda^a / 2
  double gr[8];
  gr[0] = -0.5 * (w01.i + w10.i);
  gr[1] = -0.5 * (w01.r - w10.r);
  gr[2] = -0.5 * (d0 - d1);
  gr[3] = -0.5 * (w02.i + w20.i);
  gr[4] = -0.5 * (w02.r - w20.r);
  gr[5] = -0.5 * (w12.i + w21.i);
  gr[6] = -0.5 * (w12.r - w21.r);
  gr[7] = -(d0 + d1 - 2.0 * d2) * 0.28867513459481288225;  // 1 / (2 sqrt 3)
  double* f = F + size_t(p * 4 + MU) * 8 * g.Vh;
#pragma unroll
  for (int a = 0; a < 8; ++a) f[a * g.Vh + h] += coeff * gr[a];
}

// one thread per link (x, mu): four times the threads of a thread per site,
// which the latency of the neighbour gathers needs.  A workgroup holds 64
// sites, one wavefront per direction, so the site's own spinors, read by all
// four wavefronts, come from the CU's cache after the first.
constexpr int kBilSites = 64;
__global__ __launch_bounds__(4 * kBilSites) void bilinear_kernel(Geo g, double* F, const char* Ae, const char* Ao,
                                                                const char* Ce, const char* Co, const char* U2,
                                                                double coeff) {
  const int h = blockIdx.x * kBilSites + (threadIdx.x & (kBilSites - 1));
  const int p = blockIdx.y;
  const int mu = threadIdx.x / kBilSites;  // uniform in the wavefront
  if (h >= g.Vh) return;
  const char* Ah[2] = {Ae, Ao};
  const char* Ch[2] = {Ce, Co};
  const Coord c = site_coords(g, h, p);
  switch (mu) {
    case 0: bilinear_dir<0>(g, c, p, h, Ah, Ch, U2, F, coeff); break;
    case 1: bilinear_dir<1>(g, c, p, h, Ah, Ch, U2, F, coeff); break;
    case 2: bilinear_dir<2>(g, c, p, h, Ah, Ch, U2, F, coeff); break;
    default: bilinear_dir<3>(g, c, p, h, Ah, Ch, U2, F, coeff); break;
  }
}

// ------------------------------------------------------------------ gauge force
// G = U_mu(x) A_mu(x), A the six staples; F += coeff * Re(i tr(T^a G))
__global__ __launch_bounds__(kBlock) void gauge_force_kernel(Geo g, double* F, const void* U, double coeff) {
  const int h = blockIdx.x * kBlock + threadIdx.x;
  const int p = blockIdx.y >> 2;
  const int mu = blockIdx.y & 3;
  if (h >= g.Vh) return;
  const Coord x = site_coords(g, h, p);
  cd A[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) A[k] = zero<double>();
  const Coord xm = step(g, x, mu, +1);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    cd a[9], b[9], c[9], t[9], s[9];
    // upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    load_link_at(U, g, xm, nu, a);
    load_link_at(U, g, step(g, x, nu, +1), mu, b);
    load_link_at(U, g, x, nu, c);
    mat_mul_dag(a, b, t);
    mat_mul_dag(t, c, s);
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = A[k] + s[k];
    // lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    const Coord xn = step(g, x, nu, -1);
    load_link_at(U, g, step(g, xm, nu, -1), nu, a);
    load_link_at(U, g, xn, mu, b);
    load_link_at(U, g, xn, nu, c);
    cd ba[9];
    mat_mul(b, a, ba);       // U_mu(x-nu) U_nu(x+mu-nu)
    mat_dag_mul(ba, c, s);   // (U_mu U_nu)^dag U_nu(x-nu)
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = A[k] + s[k];
  }
  cd Um[9], G[9];
  load_link(U, p, mu, h, g.Vhp, Um);
  mat_mul(Um, A, G);
  double gr[8];
  su3_grad(G, gr);
  double* f = F + size_t(p * 4 + mu) * 8 * g.Vh;
#pragma unroll
  for (int a = 0; a < 8; ++a) f[a * g.Vh + h] += coeff * gr[a];
}

// ------------------------------------------------------------------ time step
// exp(X) for X = i eps P by a degree-12 Taylor series after scaling by 2^-s
// (|X / 2^s| <= 1/4, truncation below 1e-17), then s squarings; FP64.
__device__ void su3_expi(const double* p, double eps, cd* E) {
  cd H[9];
  su3_from_coeffs(p, H);
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) n2 += H[k].r * H[k].r + H[k].i * H[k].i;
  double nrm = fabs(eps) * sqrt(n2);
  int s = 0;
  while (nrm > 0.25 && s < 30) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = eps * ldexp(1.0, -s);
  cd X[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = {-sc * H[k].i, sc * H[k].r};  // i sc H
  // Horner: E = 1 + X(1 + X/2(1 + X/3(...)))
  cd T[9], Tn[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) T[k] = zero<double>();
  T[0] = T[4] = T[8] = {1.0, 0.0};
  for (int n = 12; n >= 1; --n) {
    mat_mul(X, T, Tn);
    const double inv = 1.0 / n;
#pragma unroll
    for (int k = 0; k < 9; ++k) T[k] = inv * Tn[k];
    T[0].r += 1.0;
    T[4].r += 1.0;
    T[8].r += 1.0;
  }
  for (int q = 0; q < s; ++q) {
    mat_mul(T, T, Tn);
#pragma unroll
    for (int k = 0; k < 9; ++k) T[k] = Tn[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) E[k] = T[k];
}

__device__ __forceinline__ void reunitarize(cd* u) {
  double n0 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n0 += u[k].r * u[k].r + u[k].i * u[k].i;
  n0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = n0 * u[k];
  cd d = cmul(u[0], u[3]) + cmul(u[1], u[4]) + cmul(u[2], u[5]);  // <r0, r1>
#pragma unroll
  for (int k = 0; k < 3; ++k) u[3 + k] = u[3 + k] - d * u[k];
  double n1 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n1 += u[3 + k].r * u[3 + k].r + u[3 + k].i * u[3 + k].i;
  n1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int k = 0; k < 3; ++k) u[3 + k] = n1 * u[3 + k];
  SU3<double> m;
#pragma unroll
  for (int k = 0; k < 6; ++k) m.m[k] = u[k];
  third_row(m);
  u[6] = m.m[6];
  u[7] = m.m[7];
  u[8] = m.m[8];
}

__global__ __launch_bounds__(kBlock) void link_update_kernel(Geo g, void* U, const double* P, double eps) {
  const int h = blockIdx.x * kBlock + threadIdx.x;
  const int pm = blockIdx.y;
  if (h >= g.Vh) return;
  double pc[8];
  const double* pp = P + size_t(pm) * 8 * g.Vh;
#pragma unroll
  for (int a = 0; a < 8; ++a) pc[a] = pp[a * g.Vh + h];
  cd E[9], Um[9], Un[9];
  su3_expi(pc, eps, E);
  double2* b = reinterpret_cast<double2*>(U) + size_t(pm) * 9 * g.Vhp;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 v = b[fidx(k, h, 9)];
    Um[k] = {v.x, v.y};
  }
  mat_mul(E, Um, Un);
  reunitarize(Un);
#pragma unroll
  for (int k = 0; k < 9; ++k) b[fidx(k, h, 9)] = make_double2(Un[k].r, Un[k].i);
}

// ------------------------------------------------------------------ reductions
__global__ __launch_bounds__(kBlock) void plaquette_kernel(Geo g, const void* U, double* partials) {
  __shared__ double lds[kBlock / 64];
  const int h = blockIdx.x * kBlock + threadIdx.x;
  const int p = blockIdx.y;
  double s = 0.0;
  if (h < g.Vh) {
    const Coord x = site_coords(g, h, p);
    for (int mu = 0; mu < 4; ++mu) {
      for (int nu = mu + 1; nu < 4; ++nu) {
        cd a[9], b[9], c[9], d[9], t1[9], t2[9];
        load_link(U, p, mu, h, g.Vhp, a);
        load_link_at(U, g, step(g, x, mu, +1), nu, b);
        load_link_at(U, g, step(g, x, nu, +1), mu, c);
        load_link(U, p, nu, h, g.Vhp, d);
        mat_mul(a, b, t1);  // U_mu(x) U_nu(x+mu)
        mat_mul(d, c, t2);  // U_nu(x) U_mu(x+nu)
        // Re tr(t1 t2^dag)
#pragma unroll
        for (int k = 0; k < 9; ++k) s += t1[k].r * t2[k].r + t1[k].i * t2[k].i;
      }
    }
    s *= (1.0 / 3.0);
  }
  const double r = block_sum(s, lds);
  if (threadIdx.x == 0) partials[p * gridDim.x + blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void sumsq_kernel(const double* P, size_t n, double* partials) {
  __shared__ double lds[kBlock / 64];
  double s = 0.0;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) s += P[i] * P[i];
  const double r = block_sum(s, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// ------------------------------------------------------------------ launchers
void launch_bilinear(wl_lattice* L, double* F, const void* Ae, const void* Ao, const void* Ce, const void* Co,
                     double coeff) {
  ensure_lowp_links(L);  // the two-row FP64 link copy
  dim3 grid((L->Vh + kBilSites - 1) / kBilSites, 2);  // (64-site tile, parity)
  hipLaunchKernelGGL(bilinear_kernel, grid, dim3(4 * kBilSites), 0, L->stream, L->geo, F, (const char*)Ae,
                     (const char*)Ao, (const char*)Ce, (const char*)Co, (const char*)L->U[F64], coeff);
  WL_HIP(hipGetLastError());
}

void launch_gauge_force(wl_lattice* L, double* F, double coeff) {
  dim3 grid(site_blocks(L->Vh), 8);
  hipLaunchKernelGGL(gauge_force_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, F, L->Ufull, coeff);
  WL_HIP(hipGetLastError());
}

void launch_link_update(wl_lattice* L, const double* P, double eps) {
  dim3 grid(site_blocks(L->Vh), 8);
  hipLaunchKernelGGL(link_update_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, L->Ufull, P, eps);
  WL_HIP(hipGetLastError());
  L->lowp_valid = false;
}

void launch_plaquette_partials(wl_lattice* L, double* partials) {
  dim3 grid(site_blocks(L->Vh), 2);
  hipLaunchKernelGGL(plaquette_kernel, grid, dim3(kBlock), 0, L->stream, L->geo, L->Ufull, partials);
  WL_HIP(hipGetLastError());
}

void launch_su3_sumsq_partials(wl_lattice* L, const double* P, double* partials) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(site_blocks(L->Vh)), dim3(kBlock), 0, L->stream, P,
                     size_t(64) * L->Vh, partials);
  WL_HIP(hipGetLastError());
}

}  // namespace wl
