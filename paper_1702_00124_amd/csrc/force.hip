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
// rows, so the four-spin sums reduce to the two upper rows).  Both halves have
// one form, X_s = sum_k (U v_k) (x) w_k^dag with v from site y, w from site x:
//   s = 0:  v = (1 - g_mu) C(y), w = (1 - g_mu) A(x),   W = X_0 - X_1^dag,
//   s = 1:  v = (1 + g_mu) A(y), w = (1 + g_mu) C(x),
// and since Re(i tr(T^a M^dag)) = -Re(i tr(T^a M)) for Hermitian T^a, the link's
// eight su(3) coefficients are g(X_0) + g(X_1).  A lane computes one X_s (of X
// only the entries the coefficients read), the two lanes of a link swap halves
// of their eight coefficients, and each updates four of the link's F entries.
constexpr int kBilSites = 32;

template <int MU>
__device__ __forceinline__ void bilinear_finish(int s, const Spinor<double>& vs, const double2* own,
                                                const double2* lrow, double* f, const double* fo, double cf,
                                                int vh) {
  const double sg = s ? 1.0 : -1.0;
  const Half<double> v = project_s<MU>(vs, sg);
  Spinor<double> ws;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 e = own[k * kBilSites];
    ws.c[k] = {e.x, e.y};
  }
  const Half<double> w = project_s<MU>(ws, sg);
  SU3<double> U;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double2 e = lrow[k * kBilSites];
    U.m[k] = {e.x, e.y};
  }
  third_row(U);
  cd u[6];  // U v_k
  su3_mul(U, v.c, u);
  su3_mul(U, v.c + 3, u + 3);
  auto X = [&](int i, int j) { return u[i] * conj(w.c[j]) + u[3 + i] * conj(w.c[3 + j]); };
  const cd x01 = X(0, 1), x10 = X(1, 0), x02 = X(0, 2), x20 = X(2, 0), x12 = X(1, 2), x21 = X(2, 1);
  const double d0 = X(0, 0).i, d1 = X(1, 1).i, d2 = X(2, 2).i;
  // g^a = Re(i tr(T^a X)) = -Im tr(T^a X), T^a = lambda^a / 2
  double gr[8];
  gr[0] = -0.5 * (x01.i + x10.i);
  gr[1] = -0.5 * (x01.r - x10.r);
  gr[2] = -0.5 * (d0 - d1);
  gr[3] = -0.5 * (x02.i + x20.i);
  gr[4] = -0.5 * (x02.r - x20.r);
  gr[5] = -0.5 * (x12.i + x21.i);
  gr[6] = -0.5 * (x12.r - x21.r);
  gr[7] = -(d0 + d1 - 2.0 * d2) * 0.28867513459481288225;  // 1 / (2 sqrt 3)
  // lane s keeps coefficients 4s .. 4s+3 and sends the other four to its partner
  // (lane ^ 32, the same link)
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double mine = s ? gr[4 + a] : gr[a];
    const double other = __shfl_xor(s ? gr[a] : gr[4 + a], 32, 64);
    f[size_t(a) * vh] = fo[a] + cf * (mine + other);
  }
}

// A workgroup holds 32 sites of one parity, one wavefront per direction, the
// two halves of a wavefront the two terms of the same 32 links.  The sites' own
// spinors (A and C, used by all four directions) and the links' two stored rows
// (one loaded by each half) pass through LDS, so each is read from memory once
// per workgroup; the neighbour spinors are read by the lanes that use them.
// Work items alternate parity (32 sites of parity 0, the same 32 of parity 1,
// ...), so the neighbour spinors one parity gathers are the other parity's
// own.  On large lattices the hardware's round-robin deal of workgroups over
// the 8 XCDs is regrouped into runs of kBilChunk consecutive work items per
// XCD: the x, y, z neighbours of a run are mostly in it and come from that
// XCD's L2, while the chip as a whole still sweeps the lattice in order, so the
// t neighbours, read again one t slice later, come from the Infinity Cache
// (at 32^3 x 64: 572 us per bilinear, against 592 us in round-robin order and
// 707 us with each XCD sweeping its own contiguous eighth of the lattice).
constexpr int kBilChunk = 64;
__global__ __launch_bounds__(256) void bilinear_kernel(Geo g, int nwork, int chunked, double* F, const char* Ae,
                                                       const char* Ao, const char* Ce, const char* Co,
                                                       const char* U2, double coeff) {
  __shared__ double2 own[2 * 12 * kBilSites];  // [A, C][unit][site]
  __shared__ double2 lrow[4 * 6 * kBilSites];  // [mu][unit of the two rows][site]
  const int b = blockIdx.x;
  const int wk = chunked ? (b & ~(8 * kBilChunk - 1)) | ((b & 7) * kBilChunk) | ((b >> 3) & (kBilChunk - 1)) : b;
  if (wk >= nwork) return;  // whole workgroups
  const int p = wk & 1;
  const int h0 = (wk >> 1) * kBilSites;
  const int t = threadIdx.x, lane = t & 63, s = lane >> 5, j = lane & 31, mu = t >> 6;
  const int h = h0 + j;
  const bool act = h < g.Vh;
  const char* Ap = p ? Ao : Ae;  // own parity
  const char* Cp = p ? Co : Ce;
  const char* An = p ? Ae : Ao;  // the neighbours' parity
  const char* Cn = p ? Ce : Co;
  double fo[4] = {0.0, 0.0, 0.0, 0.0};
  double* f = F + size_t(p * 4 + mu) * 8 * g.Vh + size_t(4 * s) * g.Vh + h;
  Spinor<double> vs;
  double cf = coeff;
  if (act) {
    const Coord c = site_coords(g, h, p);
    bool wrap = false;
    int hy;
    switch (mu) {
      case 0: hy = neighbour<0>(g, c, +1, &wrap); break;
      case 1: hy = neighbour<1>(g, c, +1, &wrap); break;
      case 2: hy = neighbour<2>(g, c, +1, &wrap); break;
      default: hy = neighbour<3>(g, c, +1, &wrap); break;
    }
    if (wrap) cf *= double(g.tbc);  // the link's fermion phase, common to both terms
    vs = SpinorIO<PrecF64>::load(s ? An : Cn, hy, g.Vh);
#pragma unroll
    for (int a = 0; a < 4; ++a) fo[a] = f[size_t(a) * g.Vh];
    const double2* ub = reinterpret_cast<const double2*>(U2 + size_t(p * 4 + mu) * LinkIO<PrecF64>::bytes * g.Vhp);
#pragma unroll
    for (int k = 0; k < 3; ++k) lrow[(mu * 6 + 3 * s + k) * kBilSites + j] = ub[fidx(3 * s + k, h, 6)];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // 2 fields x 12 units x 32 sites, three per thread
    const int idx = t + 256 * i, fld = idx / (12 * kBilSites), rem = idx - fld * 12 * kBilSites;
    const int hs = h0 + (rem & (kBilSites - 1));
    if (hs < g.Vh)
      own[idx] = reinterpret_cast<const double2*>(fld ? Cp : Ap)[fidx(rem / kBilSites, hs, 12)];
  }
  __syncthreads();
  if (!act) return;  // both lanes of a link leave together
  const double2* ow = own + (s ? 12 * kBilSites : 0) + j;
  const double2* lr = lrow + mu * 6 * kBilSites + j;
  switch (mu) {  // uniform in the wavefront
    case 0: bilinear_finish<0>(s, vs, ow, lr, f, fo, cf, g.Vh); break;
    case 1: bilinear_finish<1>(s, vs, ow, lr, f, fo, cf, g.Vh); break;
    case 2: bilinear_finish<2>(s, vs, ow, lr, f, fo, cf, g.Vh); break;
    default: bilinear_finish<3>(s, vs, ow, lr, f, fo, cf, g.Vh); break;
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
  const int nwork = 2 * ((L->Vh + kBilSites - 1) / kBilSites);  // (32 sites, parity)
  const int run = 8 * kBilChunk;                                 // one run per XCD
  const int chunked = nwork >= 8 * run;
  dim3 grid(chunked ? (nwork + run - 1) / run * run : nwork);
  hipLaunchKernelGGL(bilinear_kernel, grid, dim3(256), 0, L->stream, L->geo, nwork, chunked, F, (const char*)Ae,
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
