// Mixed-volume batches: lattices of different extents (each with its own links
// and kappa) whose hops run as one launch, with the even-odd operators and a CG
// over the batch built on it (the multi-rhs solves of Sec. 2 with one system per
// lattice instead of one per right-hand side).
//
// A batch field is nlat equal slots, slot l holding lattice l's even-site field
// in its own tiled layout (a site's address does not depend on the lattice's
// extent) and zeros past its sites.  Slots are sized for the largest lattice,
// whose stream, CG state and workspace the batch uses, so the solver's
// elementwise kernels and reductions run over all slots as over the rhs of one
// lattice: the zero sites add nothing and stay zero.
#include <algorithm>

#include "wl_ops.h"

struct wl_batch {
  std::vector<wl_lattice*> lat;
  wl_lattice* big = nullptr;          // the lattice with the most sites
  void* tmp[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // per precision: odd, even
};

namespace wl {

size_t batch_slot_bytes(const wl_batch* B, Prec prec) { return spinor_bytes(prec, B->big->Vh); }

int batch_count(const wl_batch* B) { return int(B->lat.size()); }

wl_lattice* batch_big(const wl_batch* B) { return B->big; }

wl_batch* batch_create(wl_lattice* const* lats, int nlat) {
  WL_REQUIRE(lats && nlat >= 1 && nlat <= kMaxBatch, WL_EINVAL, "batch: 1 to 8 lattices");
  auto* B = new wl_batch;
  for (int l = 0; l < nlat; ++l) {
    if (!lats[l] || lats[l]->device != lats[0]->device || lats[l]->stream != lats[0]->stream) {
      delete B;
      throw Error(WL_EINVAL, "batch: lattices must be non-null and share one device and stream");
    }
    B->lat.push_back(lats[l]);
    if (!B->big || lats[l]->Vh > B->big->Vh) B->big = lats[l];
  }
  return B;
}

void batch_destroy(wl_batch* B) {
  if (!B) return;
  (void)hipSetDevice(B->big->device);
  (void)hipStreamSynchronize(B->big->stream);
  for (auto& t : B->tmp)
    for (void* p : t)
      if (p) (void)hipFree(p);
  delete B;
}

// the odd and even intermediates of the batch operators, zero where no lattice
// has a site (the hops write only their lattices' sites)
static void* batch_tmp(wl_batch* B, Prec prec, int which) {
  void*& p = B->tmp[prec][which];
  if (!p) {
    const size_t bytes = batch_slot_bytes(B, prec) * B->lat.size();
    WL_HIP(hipMalloc(&p, bytes));
    WL_HIP(hipMemsetAsync(p, 0, bytes, B->big->stream));
  }
  return p;
}

void batch_prepare(wl_batch* B, Prec prec) {
  batch_tmp(B, prec, 0);
  batch_tmp(B, prec, 1);
  for (wl_lattice* L : B->lat) ensure_lowp_links(L);
}

void batch_hop(wl_batch* B, Prec prec, void* out, const void* in, int out_parity, int dagger) {
  const int n = batch_count(B);
  const size_t sb = batch_slot_bytes(B, prec);
  std::vector<BatchHop> hops(n);
  for (int l = 0; l < n; ++l)
    hops[l] = BatchHop{B->lat[l], static_cast<char*>(out) + l * sb, static_cast<const char*>(in) + l * sb, HopEpi()};
  launch_hop_batch(B->big->stream, prec, out_parity, dagger, hops.data(), n, 0);
}

// out_l = J_l in_l = g5 M-hat g5 M-hat in_l + mu2[l] in_l with the lattice's
// own kappa[l] (as op_j); with dot.partials, Re<in_l, out_l> partial sums in
// row l of dot.stride entries
void batch_j(wl_batch* B, Prec prec, void* out, const void* in, const double* kappa, const double* mu2,
             const DotOut& dot) {
  const int n = batch_count(B);
  const size_t sb = batch_slot_bytes(B, prec);
  char* odd = static_cast<char*>(batch_tmp(B, prec, 0));
  char* even = static_cast<char*>(batch_tmp(B, prec, 1));
  auto slot = [&](const void* base, int l) { return static_cast<char*>(const_cast<void*>(base)) + l * sb; };
  std::vector<BatchHop> h(n);
  hipStream_t st = B->big->stream;
  for (int l = 0; l < n; ++l) h[l] = BatchHop{B->lat[l], slot(odd, l), slot(in, l), HopEpi()};
  launch_hop_batch(st, prec, 1, 0, h.data(), n, 0);  // D_oe in
  for (int l = 0; l < n; ++l) {
    HopEpi e;
    e.x = slot(in, l);
    e.a = -kappa[l] * kappa[l];
    e.g5 = 1;
    h[l] = BatchHop{B->lat[l], slot(even, l), slot(odd, l), e};
  }
  launch_hop_batch(st, prec, 0, 0, h.data(), n, 0);  // g5 M-hat in
  for (int l = 0; l < n; ++l) h[l] = BatchHop{B->lat[l], slot(odd, l), slot(even, l), HopEpi()};
  launch_hop_batch(st, prec, 1, 0, h.data(), n, 0);
  for (int l = 0; l < n; ++l) {
    HopEpi e;
    e.x = slot(even, l);
    e.a = -kappa[l] * kappa[l];
    e.g5 = 1;
    if (mu2 && mu2[l] != 0.0) {
      e.y = slot(in, l);
      e.by[0] = mu2[l];
    }
    if (dot.partials) {
      e.dot = 1;
      e.dotv = slot(in, l);
      e.partials = dot.partials + size_t(l) * dot.stride;
    }
    h[l] = BatchHop{B->lat[l], slot(out, l), slot(odd, l), e};
  }
  launch_hop_batch(st, prec, 0, 0, h.data(), n, dot.partials ? dot.stride : 0);
  for (wl_lattice* L : B->lat) L->n_kmat += 1;
}

int batch_cg(wl_batch* B, void* x, const void* b, const double* kappa, const double* mu2, const wl_cg_params& prm,
             wl_cg_stats* stats) {
  WL_REQUIRE(kappa, WL_EINVAL, "batch CG needs one kappa per lattice");
  const Prec ip = Prec(prm.inner);
  const Prec ipr = (ip == F32 || ip == BF16) ? ip : F64;
  batch_prepare(B, ipr);
  batch_prepare(B, F64);
  wl_lattice* big = B->big;
  const int nbrow = std::max(hop_tiles(big, ipr), blas_blocks(big));
  ApplyLowp lp = [&](Prec pr, void* out, const void* in, const DotOut& d) { batch_j(B, pr, out, in, kappa, mu2, d); };
  Apply64 a64 = [&](void* out, const void* in) { batch_j(B, F64, out, in, kappa, mu2, DotOut()); };
  return cg_run_batch(big, x, b, batch_count(B), nbrow, lp, a64, prm, stats);
}

}  // namespace wl
