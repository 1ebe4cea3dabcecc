// extern "C" entry points of libwilson_hmc (declared in include/wilson_hmc.h).
// Every call validates its arguments, runs inside a guard that turns internal
// errors into return codes, and records the message for wl_last_error().
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "wl_ops.h"

namespace wl {
void scratch_register(int device);
void* scratch_ptr(int device);
size_t scratch_limit();
int hmc_run(wl_lattice* L, const wl_hmc_params& prm, double* P, const void* chi, double u, wl_hmc_result* res);
double plaquette_host(wl_lattice* L);
struct Event {
  int kind;
  int term;
  double w;
};
std::vector<Event> merge_schedule(const std::vector<int>& nsteps, int scheme, double lam);
}  // namespace wl

using namespace wl;

namespace {

thread_local std::string g_err;

template <typename F>
int guard(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return WL_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return WL_EINVAL;
  } catch (...) {
    g_err = "unknown error";
    return WL_EINVAL;
  }
}

void check_lat(const wl_lattice* L) { WL_REQUIRE(L != nullptr, WL_EINVAL, "null lattice"); }

void set_device(const wl_lattice* L) { WL_HIP(hipSetDevice(L->device)); }

void device_alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) throw Error(WL_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  WL_HIP(e);
}

}  // namespace

namespace wl {

void* ws_get(wl_lattice* L, const std::string& name, size_t bytes) {
  auto it = L->ws.find(name);
  if (it != L->ws.end() && it->second.second >= bytes) return it->second.first;
  if (it != L->ws.end()) {
    WL_HIP(hipStreamSynchronize(L->stream));
    WL_HIP(hipFree(it->second.first));
    L->ws.erase(it);
    ++L->ws_gen;
  }
  void* p = nullptr;
  device_alloc(&p, bytes);
  L->ws[name] = {p, bytes};
  return p;
}

void ensure_partials(wl_lattice* L, size_t n) {
  if (L->partials_len >= n) return;
  if (L->partials) {
    WL_HIP(hipStreamSynchronize(L->stream));
    WL_HIP(hipFree(L->partials));
    L->partials = nullptr;
    ++L->ws_gen;
  }
  device_alloc(reinterpret_cast<void**>(&L->partials), n * sizeof(double));
  L->partials_len = n;
}

void ensure_lowp_links(wl_lattice* L) {
  if (!L->lowp_valid) launch_lowp_links(L);
}

}  // namespace wl

extern "C" {

const char* wl_last_error(void) { return g_err.c_str(); }

int wl_create(wl_lattice** out, const int32_t Ls[4], int32_t t_bc, void* hip_stream) {
  return guard([&]() {
    WL_REQUIRE(out && Ls, WL_EINVAL, "null argument");
    *out = nullptr;
    for (int m = 0; m < 4; ++m)
      WL_REQUIRE(Ls[m] >= 2 && Ls[m] <= 32768 && Ls[m] % 2 == 0, WL_EINVAL,
                 "lattice extents must be even, >= 2 and <= 32768");
    WL_REQUIRE(t_bc == 1 || t_bc == -1, WL_EINVAL, "t_bc must be +1 or -1");
    const long long V = (long long)Ls[0] * Ls[1] * Ls[2] * Ls[3];
    WL_REQUIRE(V <= (1LL << 30), WL_EUNSUPPORTED, "volume too large");
    wl_lattice* L = new wl_lattice();
    try {
      WL_HIP(hipGetDevice(&L->device));
      scratch_register(L->device);
      for (int m = 0; m < 4; ++m) {
        L->L[m] = Ls[m];
        L->geo.L[m] = Ls[m];
      }
      L->V = int(V);
      L->Vh = int(V / 2);
      L->geo.Lxh = Ls[0] / 2;
      L->geo.Vh = L->Vh;
      L->geo.Vhp = padded_sites(L->Vh);
      L->geo.tbc = t_bc;
      geo_init(L->geo);
      L->stream = static_cast<hipStream_t>(hip_stream);
      device_alloc(&L->Ufull, full_links_bytes(L->Vh));
      for (int p = 0; p < 3; ++p) device_alloc(&L->U[p], links_bytes(Prec(p), L->Vh));
      device_alloc(reinterpret_cast<void**>(&L->dscal), kScal * sizeof(double));
      WL_HIP(hipHostMalloc(reinterpret_cast<void**>(&L->hscal), kScal * sizeof(double), hipHostMallocDefault));
      WL_HIP(hipMemsetAsync(L->Ufull, 0, full_links_bytes(L->Vh), L->stream));
      WL_HIP(hipMemsetAsync(L->dscal, 0, kScal * sizeof(double), L->stream));
      ensure_partials(L, size_t(4) * kMaxRhs * site_blocks(L->Vh) + 64);
      WL_HIP(hipStreamSynchronize(L->stream));
    } catch (...) {
      wl_destroy(L);
      throw;
    }
    *out = L;
    return WL_OK;
  });
}

int wl_destroy(wl_lattice* L) {
  if (!L) return WL_OK;
  (void)hipSetDevice(L->device);
  (void)hipStreamSynchronize(L->stream);
  for (auto& kv : L->ws) (void)hipFree(kv.second.first);
  for (int p = 0; p < 3; ++p)
    if (L->U[p]) (void)hipFree(L->U[p]);
  if (L->Ufull) (void)hipFree(L->Ufull);
  if (L->partials) (void)hipFree(L->partials);
  if (L->dscal) (void)hipFree(L->dscal);
  if (L->hscal) (void)hipHostFree(L->hscal);
  if (L->capture_stream) (void)hipStreamDestroy(L->capture_stream);
  for (int p = 0; p < 3; ++p)
    for (hipEvent_t e : L->prof_ev[p]) (void)hipEventDestroy(e);
  delete L;
  return WL_OK;
}

int wl_set_stream(wl_lattice* L, void* s) {
  return guard([&]() {
    check_lat(L);
    WL_HIP(hipStreamSynchronize(L->stream));
    L->stream = static_cast<hipStream_t>(s);
    return WL_OK;
  });
}

int wl_set_links(wl_lattice* L, const void* U, int on_device) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(U, WL_EINVAL, "null links");
    WL_REQUIRE(on_device == 0 || on_device == 1, WL_EINVAL, "on_device must be 0 or 1");
    set_device(L);
    if (!on_device) {  // stage the host array in the workspace, then pack on the device
      const size_t bytes = size_t(4) * L->V * 9 * 16;
      void* stage = ws_get(L, "links_stage", bytes);
      WL_HIP(hipMemcpyAsync(stage, U, bytes, hipMemcpyHostToDevice, L->stream));
      launch_pack_links(L, stage);
      WL_HIP(hipStreamSynchronize(L->stream));  // the host array may be reused on return
      return WL_OK;
    }
    launch_pack_links(L, U);
    return WL_OK;
  });
}

int wl_get_links(wl_lattice* L, void* U, int on_device) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(U, WL_EINVAL, "null links");
    WL_REQUIRE(on_device == 0 || on_device == 1, WL_EINVAL, "on_device must be 0 or 1");
    set_device(L);
    if (!on_device) {
      const size_t bytes = size_t(4) * L->V * 9 * 16;
      void* stage = ws_get(L, "links_stage", bytes);
      launch_unpack_links(L, stage);
      WL_HIP(hipMemcpyAsync(U, stage, bytes, hipMemcpyDeviceToHost, L->stream));
      WL_HIP(hipStreamSynchronize(L->stream));
      return WL_OK;
    }
    launch_unpack_links(L, U);
    return WL_OK;
  });
}

int wl_field_bytes(const wl_lattice* L, wl_prec prec, int nrhs, size_t* bytes) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(bytes && nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "bad arguments");
    WL_REQUIRE(prec == WL_F64 || prec == WL_F32 || prec == WL_BF16, WL_EINVAL, "unknown precision");
    *bytes = spinor_bytes(Prec(prec), L->Vh) * nrhs;
    return WL_OK;
  });
}

static void check_prec_rhs(wl_prec prec, int nrhs) {
  WL_REQUIRE(prec == WL_F64 || prec == WL_F32 || prec == WL_BF16, WL_EINVAL, "unknown precision");
  WL_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, WL_EINVAL, "nrhs must be 1..16");
}

int wl_import_spinor(wl_lattice* L, void* dst, const void* src, wl_prec prec, int nrhs) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    launch_import_spinor(L, Prec(prec), dst, src, nrhs);
    return WL_OK;
  });
}

int wl_export_spinor(wl_lattice* L, void* dst, const void* src, wl_prec prec, int nrhs) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    launch_export_spinor(L, Prec(prec), dst, src, nrhs);
    return WL_OK;
  });
}

int wl_import_full(wl_lattice* L, void* dst, const void* src) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    char* d = static_cast<char*>(dst);
    launch_split_full(L, d, d + spinor_bytes(F64, L->Vh), src, 0);
    return WL_OK;
  });
}

int wl_export_full(wl_lattice* L, void* dst, const void* src) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    char* s = const_cast<char*>(static_cast<const char*>(src));
    launch_split_full(L, s, s + spinor_bytes(F64, L->Vh), dst, 1);
    return WL_OK;
  });
}

int wl_import_su3(wl_lattice* L, double* dst, const double* src) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    launch_su3_io(L, dst, src, 0);
    return WL_OK;
  });
}

int wl_export_su3(wl_lattice* L, double* dst, const double* src) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(dst && src, WL_EINVAL, "null field");
    set_device(L);
    launch_su3_io(L, const_cast<double*>(src), dst, 1);
    return WL_OK;
  });
}

int wilson_dslash(wl_lattice* L, void* out, const void* in, int out_parity, int dagger, wl_prec prec, int nrhs) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(out && in, WL_EINVAL, "null field");
    WL_REQUIRE(out_parity == 0 || out_parity == 1, WL_EINVAL, "parity must be 0 or 1");
    set_device(L);
    HopEpi e;
    launch_hop(L, Prec(prec), out, in, out_parity, dagger ? 1 : 0, nrhs, e);
    return WL_OK;
  });
}

int apply_K(wl_lattice* L, void* out, const void* in, double kappa, const double* mu2, int nrhs, wl_op op,
            wl_prec prec) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(out && in && out != in, WL_EINVAL, "null or aliased field");
    set_device(L);
    op_apply(L, op, Prec(prec), out, in, kappa, mu2, nrhs);
    return WL_OK;
  });
}

int apply_K_noalloc(wl_lattice* L, void* out, const void* in, double kappa, const double* mu2, int nrhs, wl_op op,
                    wl_prec prec) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(out && in && out != in, WL_EINVAL, "null or aliased field");
    WL_REQUIRE(op >= WL_OP_M && op <= WL_OP_J, WL_EINVAL, "unknown operator");
    WL_REQUIRE(nrhs == 1 || op == WL_OP_J || op == WL_OP_MHAT || op == WL_OP_MHAT_DAG, WL_EUNSUPPORTED,
               "full-lattice operators take one rhs");
    const size_t need = op_scratch_bytes(L, op, Prec(prec), nrhs);
    WL_REQUIRE(need <= scratch_limit(), WL_EINVAL,
               "apply_K_noalloc: this operator needs " + std::to_string(need) + " bytes of scratch, above the "
               "fixed " + std::to_string(scratch_limit()) + "-byte limit (use apply_K)");
    set_device(L);
    char* base = static_cast<char*>(scratch_ptr(L->device));
    OpScratch scr;
    scr.odd = base;
    scr.even = base + op_scratch_bytes(L, WL_OP_MHAT, Prec(prec), nrhs);  // J: after the odd fields
    L->prof_suspended = 1;  // no timing events from this call
    try {
      op_apply(L, op, Prec(prec), out, in, kappa, mu2, nrhs, DotOut(), &scr);
    } catch (...) {
      L->prof_suspended = 0;
      throw;
    }
    L->prof_suspended = 0;
    return WL_OK;
  });
}

int cg_solve(wl_lattice* L, void* x, const void* b, double kappa, const double* mu2, int nrhs, wl_op op,
             const wl_cg_params* params, wl_cg_stats* stats) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(x && b && params && x != b, WL_EINVAL, "null or aliased argument");
    set_device(L);
    return cg_run(L, x, b, kappa, mu2, nrhs, op, *params, stats);
  });
}

int cg_multishift(wl_lattice* L, void* x, const void* b, double kappa, const double* mu2, int nshift, int nrhs,
                  const wl_cg_params* params, wl_cg_stats* stats) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(x && b && params && mu2 && x != b, WL_EINVAL, "null or aliased argument");
    set_device(L);
    return cg_multishift_run(L, x, b, kappa, mu2, nshift, nrhs, *params, stats);
  });
}

int poly_filter_apply(wl_lattice* L, void* out, const void* in, double kappa, double mu2, const wl_poly* poly,
                      wl_poly_mode mode, int nrhs, wl_prec prec) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(out && in && poly && out != in, WL_EINVAL, "null or aliased argument");
    set_device(L);
    poly_apply(L, mode, out, in, kappa, mu2, PolyDesc{poly->degree, poly->a, poly->b, poly->degree_div}, Prec(prec),
               nrhs);
    return WL_OK;
  });
}

int wl_heatbath(wl_lattice* L, void* phi, const wl_term* term, const void* chi) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(phi && term && chi && phi != chi, WL_EINVAL, "null or aliased argument");
    set_device(L);
    term_heatbath(L, *term, phi, chi);
    return WL_OK;
  });
}

int wl_action(wl_lattice* L, const wl_term* term, const void* phi, double* S) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(term && phi && S, WL_EINVAL, "null argument");
    set_device(L);
    *S = term_action(L, *term, phi, nullptr);
    return WL_OK;
  });
}

int fermion_force(wl_lattice* L, double* F, const wl_term* term, const void* phi, double coeff, double* S_out) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(F && term && phi, WL_EINVAL, "null argument");
    set_device(L);
    term_force(L, *term, F, phi, coeff, nullptr);
    if (S_out) *S_out = term_action(L, *term, phi, nullptr);
    return WL_OK;
  });
}

int wl_force_bilinear(wl_lattice* L, double* F, const void* A, const void* C, double coeff) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(F && A && C, WL_EINVAL, "null argument");
    set_device(L);
    const size_t hb = spinor_bytes(F64, L->Vh);
    const char* a = static_cast<const char*>(A);
    const char* c = static_cast<const char*>(C);
    launch_bilinear(L, F, a, a + hb, c, c + hb, coeff);
    return WL_OK;
  });
}

int wl_gauge_force(wl_lattice* L, double* F, double beta, double coeff) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(F, WL_EINVAL, "null argument");
    set_device(L);
    launch_gauge_force(L, F, -coeff * beta / 3.0);
    return WL_OK;
  });
}

int wl_plaquette(wl_lattice* L, double* plaq) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(plaq, WL_EINVAL, "null argument");
    set_device(L);
    *plaq = plaquette_host(L);
    return WL_OK;
  });
}

int wl_link_update(wl_lattice* L, const double* P, double eps) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(P, WL_EINVAL, "null argument");
    set_device(L);
    launch_link_update(L, P, eps);
    return WL_OK;
  });
}

int hmc_trajectory(wl_lattice* L, const wl_hmc_params* params, double* P, const void* chi, double u,
                   wl_hmc_result* result) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(params && P && (chi || params->nterms == 0), WL_EINVAL, "null argument");
    set_device(L);
    return hmc_run(L, *params, P, chi, u, result);
  });
}

int wl_profile(wl_lattice* L, int enable) {
  return guard([&]() {
    check_lat(L);
    WL_HIP(hipStreamSynchronize(L->stream));
    for (int p = 0; p < 3; ++p) {
      for (hipEvent_t e : L->prof_ev[p]) WL_HIP(hipEventDestroy(e));
      L->prof_ev[p].clear();
      L->prof_ms[p] = 0.0;
      L->prof_n[p] = 0;
    }
    L->prof_on = enable ? 1 : 0;
    return WL_OK;
  });
}

int wl_profile_read(wl_lattice* L, double* avg_us /*[3]*/, long long* samples /*[3]*/) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(avg_us && samples, WL_EINVAL, "null argument");
    WL_HIP(hipStreamSynchronize(L->stream));
    for (int p = 0; p < 3; ++p) {
      auto& ev = L->prof_ev[p];
      for (size_t k = 0; k + 1 < ev.size(); k += 2) {
        float ms = 0.f;
        WL_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
        L->prof_ms[p] += ms;
        L->prof_n[p] += 1;
        WL_HIP(hipEventDestroy(ev[k]));
        WL_HIP(hipEventDestroy(ev[k + 1]));
      }
      ev.clear();
      samples[p] = L->prof_n[p];
      avg_us[p] = L->prof_n[p] ? 1e3 * L->prof_ms[p] / L->prof_n[p] : 0.0;
    }
    return WL_OK;
  });
}

int wl_hop_counts(const wl_lattice* L, long long* counts) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(counts, WL_EINVAL, "null argument");
    for (int p = 0; p < 3; ++p) counts[p] = L->n_hop_p[p];
    return WL_OK;
  });
}

int wl_set_hop_config(wl_lattice* L, wl_prec prec, int kind, int variant, int npass, int use_xcd, int stream) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, 1);
    WL_REQUIRE(kind >= -1 && kind < kHopKinds, WL_EINVAL, "hop class must be -1, 0, 1 or 2");
    WL_REQUIRE(variant == kHopSite || variant == kHopDirParallel || variant == kHopSiteShared, WL_EINVAL,
               "unknown hop variant");
    WL_REQUIRE(npass == 1 || npass == 2 || npass == 4, WL_EINVAL, "npass must be 1, 2 or 4");
    WL_REQUIRE(use_xcd == 0 || use_xcd == 1 ||
                   (use_xcd == 2 && zblock_ok(L->geo)),
               WL_EINVAL, "use_xcd must be 0, 1, or 2 where the lattice allows the z-blocked order");
    WL_REQUIRE(stream == 0 || stream == 1, WL_EINVAL, "stream must be 0 or 1");
    WL_HIP(hipStreamSynchronize(L->stream));
    for (int k = 0; k < kHopKinds; ++k)
      if (kind == -1 || kind == k) L->hop_cfg[prec][k] = HopConfig{variant, npass, use_xcd, stream};
    return WL_OK;
  });
}

int wl_get_hop_config(const wl_lattice* L, wl_prec prec, int kind, int* variant, int* npass, int* use_xcd,
                      int* stream) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, 1);
    WL_REQUIRE(kind >= 0 && kind < kHopKinds, WL_EINVAL, "hop class must be 0, 1 or 2");
    const HopConfig& c = L->hop_cfg[prec][kind];
    if (variant) *variant = c.variant;
    if (npass) *npass = c.npass;
    if (use_xcd) *use_xcd = c.use_xcd;
    if (stream) *stream = c.stream;
    return WL_OK;
  });
}

int wl_time_hop(wl_lattice* L, wl_prec prec, int nrhs, int nlaunch, double* avg_us) {
  return guard([&]() {
    check_lat(L);
    check_prec_rhs(prec, nrhs);
    WL_REQUIRE(avg_us && nlaunch >= 1 && nlaunch <= 100000, WL_EINVAL, "bad arguments");
    set_device(L);
    const size_t fb = spinor_bytes(F64, L->Vh) * nrhs;  // large enough for every precision
    void* a = ws_get(L, "tune_a", fb);
    void* b = ws_get(L, "tune_b", fb);
    WL_HIP(hipMemsetAsync(a, 0, fb, L->stream));
    WL_HIP(hipMemsetAsync(b, 0, fb, L->stream));
    hipEvent_t e0, e1;
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    HopEpi e;
    // warm-up long enough for the clocks to leave any idle state, then the
    // median of 5 sub-bursts; launches alternate between the two fields, so
    // each reads the previous one's output, as in a solver
    const int warm = 100, nsub = 5, per = std::max(1, nlaunch / nsub);
    auto hop = [&](int i) { launch_hop(L, Prec(prec), i & 1 ? a : b, i & 1 ? b : a, i & 1, 0, nrhs, e); };
    for (int i = 0; i < warm; ++i) hop(i);
    std::vector<double> sub;
    for (int k = 0; k < nsub; ++k) {
      WL_HIP(hipEventRecord(e0, L->stream));
      for (int i = 0; i < per; ++i) hop(i);
      WL_HIP(hipEventRecord(e1, L->stream));
      WL_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      WL_HIP(hipEventElapsedTime(&ms, e0, e1));
      sub.push_back(1e3 * ms / per);
    }
    std::sort(sub.begin(), sub.end());
    *avg_us = sub[nsub / 2];
    L->n_hop -= (long long)(warm + nsub * per) * nrhs;
    L->n_hop_p[prec] -= (long long)(warm + nsub * per) * nrhs;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return WL_OK;
  });
}

int wl_stream_copy(wl_lattice* L, size_t bytes, int reps, double* gbs) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(gbs && reps >= 1 && bytes >= 16 && bytes % 16 == 0 && bytes <= (size_t(1) << 34), WL_EINVAL,
               "bad arguments");
    set_device(L);
    void* a = ws_get(L, "stream_a", bytes);
    void* b = ws_get(L, "stream_b", bytes);
    WL_HIP(hipMemsetAsync(a, 0, bytes, L->stream));
    hipEvent_t e0, e1;
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    // alternate the direction, so that every copy reads what the previous one
    // wrote (as a solver's kernels do), not a cache-resident constant source
    launch_stream_copy(L, a, b, bytes);
    WL_HIP(hipEventRecord(e0, L->stream));
    for (int i = 0; i < reps; ++i) launch_stream_copy(L, i & 1 ? a : b, i & 1 ? b : a, bytes);
    WL_HIP(hipEventRecord(e1, L->stream));
    WL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    WL_HIP(hipEventElapsedTime(&ms, e0, e1));
    *gbs = 2.0 * double(bytes) * reps / (1e-3 * ms) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // release the two buffers (they can be large)
    for (const char* n : {"stream_a", "stream_b"}) {
      auto it = L->ws.find(n);
      WL_HIP(hipStreamSynchronize(L->stream));
      WL_HIP(hipFree(it->second.first));
      L->ws.erase(it);
    }
    return WL_OK;
  });
}

// best of 3 bursts of 20 hop launches (after 5 warm-ups), microseconds per
// launch, on scratch fields; not counted in the hop counters
static double tune_burst(wl_lattice* L, Prec p, void* fa, void* fb, int nrhs, hipEvent_t e0, hipEvent_t e1) {
  HopEpi e;
  // ping-pong: each launch reads the previous one's output, as in a solver
  for (int i = 0; i < 5; ++i) launch_hop(L, p, i & 1 ? fa : fb, i & 1 ? fb : fa, i & 1, 0, nrhs, e);
  double us = 1e30;
  for (int rep = 0; rep < 3; ++rep) {
    WL_HIP(hipEventRecord(e0, L->stream));
    for (int i = 0; i < 20; ++i) launch_hop(L, p, i & 1 ? fa : fb, i & 1 ? fb : fa, i & 1, 0, nrhs, e);
    WL_HIP(hipEventRecord(e1, L->stream));
    WL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    WL_HIP(hipEventElapsedTime(&ms, e0, e1));
    us = std::min(us, 1e3 * ms / 20);
  }
  L->n_hop -= 65LL * nrhs;
  L->n_hop_p[p] -= 65LL * nrhs;
  return us;
}

int wl_autotune(wl_lattice* L, double* us_out) {
  return guard([&]() {
    check_lat(L);
    set_device(L);
    hipEvent_t e0, e1;
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    const size_t fb = spinor_bytes(F64, L->Vh) * kTuneRhs[kHopKinds - 1];
    void* a = ws_get(L, "tune_a", fb);
    void* b = ws_get(L, "tune_b", fb);
    WL_HIP(hipMemsetAsync(a, 0, fb, L->stream));
    WL_HIP(hipMemsetAsync(b, 0, fb, L->stream));
    int slot = 0;
    for (int p = 0; p < 3; ++p) {
      for (int k = 0; k < kHopKinds; ++k) {
        // one rhs: site and direction-parallel; several: site with 1 or 2 rhs
        // per thread, site with the links shared in LDS and
        // direction-parallel with 1, 2 or 4 passes; each in every workgroup
        // order, cached then streaming
        // streaming access only where the hop's working set (links and two
        // fields) exceeds the last-level cache: below it the next kernel reads
        // this hop's output from the cache, which a burst of hops cannot show
        const size_t wset = links_bytes(Prec(p), L->Vh) + 2 * spinor_bytes(Prec(p), L->Vh) * kTuneRhs[k];
        const int max_stream = wset > kLastLevelCache ? 1 : 0;
        std::vector<HopConfig> cand;
        for (int stm = 0; stm <= 1; ++stm)
          for (int xcd : {1, 0, 2}) {
            if (k == 0) {
              cand.push_back({kHopSite, 1, xcd, stm});
              cand.push_back({kHopDirParallel, 1, xcd, stm});
            } else {
              for (int np : {1, 2}) cand.push_back({kHopSite, np, xcd, stm});
              cand.push_back({kHopSiteShared, 1, xcd, stm});
              for (int np : {1, 2, 4}) cand.push_back({kHopDirParallel, np, xcd, stm});
            }
          }
        double best = 1e30;
        HopConfig keep = L->hop_cfg[p][k];
        for (const HopConfig& c : cand) {
          if (c.stream > max_stream || (c.use_xcd == 2 && !zblock_ok(L->geo))) {  // not here
            if (us_out) us_out[slot] = 0.0;
            ++slot;
            continue;
          }
          L->hop_cfg[p][k] = c;
          const double us = tune_burst(L, Prec(p), b, a, kTuneRhs[k], e0, e1);
          if (us_out) us_out[slot] = us;
          ++slot;
          if (us < best) {
            best = us;
            keep = c;
          }
        }
        L->hop_cfg[p][k] = keep;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return WL_OK;
  });
}

int wl_integrator_schedule(const int* nsteps, int nscales, int scheme, double lambda, int* kinds, int* terms,
                           double* weights, int max_events, int* n_events) {
  return guard([&]() {
    WL_REQUIRE(nsteps && n_events && nscales >= 1 && nscales <= 9, WL_EINVAL, "bad arguments");
    WL_REQUIRE(scheme == WL_INT_LEAPFROG || scheme == WL_INT_OMELYAN, WL_EINVAL, "unknown integrator");
    std::vector<int> ns(nsteps, nsteps + nscales);
    for (int n : ns) WL_REQUIRE(n >= 1 && n <= 100000, WL_EINVAL, "nsteps out of range");
    const auto ev = merge_schedule(ns, scheme, lambda > 0.0 ? lambda : 0.1931833275037836);
    *n_events = int(ev.size());
    WL_REQUIRE(int(ev.size()) <= max_events, WL_EINVAL, "event buffer too small");
    for (size_t i = 0; i < ev.size(); ++i) {
      if (kinds) kinds[i] = ev[i].kind;
      if (terms) terms[i] = ev[i].term;
      if (weights) weights[i] = ev[i].w;
    }
    return WL_OK;
  });
}

int wl_batch_create(wl_batch** out, wl_lattice* const* lats, int nlat) {
  return guard([&]() {
    WL_REQUIRE(out, WL_EINVAL, "null argument");
    *out = nullptr;
    *out = batch_create(lats, nlat);
    return WL_OK;
  });
}

int wl_batch_destroy(wl_batch* B) {
  batch_destroy(B);
  return WL_OK;
}

int wl_batch_slot_bytes(const wl_batch* B, wl_prec prec, size_t* bytes) {
  return guard([&]() {
    WL_REQUIRE(B && bytes, WL_EINVAL, "null argument");
    WL_REQUIRE(prec >= WL_F64 && prec <= WL_BF16, WL_EINVAL, "unknown precision");
    *bytes = batch_slot_bytes(B, Prec(prec));
    return WL_OK;
  });
}

int wl_batch_dslash(wl_batch* B, void* out, const void* in, int out_parity, int dagger, wl_prec prec) {
  return guard([&]() {
    WL_REQUIRE(B && out && in && out != in, WL_EINVAL, "null or aliased argument");
    WL_REQUIRE(out_parity == 0 || out_parity == 1, WL_EINVAL, "parity must be 0 or 1");
    WL_REQUIRE(prec >= WL_F64 && prec <= WL_BF16, WL_EINVAL, "unknown precision");
    set_device(batch_big(B));
    batch_hop(B, Prec(prec), out, in, out_parity, dagger ? 1 : 0);
    return WL_OK;
  });
}

int wl_batch_apply_J(wl_batch* B, void* out, const void* in, const double* kappa, const double* mu2, wl_prec prec) {
  return guard([&]() {
    WL_REQUIRE(B && out && in && kappa && out != in, WL_EINVAL, "null or aliased argument");
    WL_REQUIRE(prec >= WL_F64 && prec <= WL_BF16, WL_EINVAL, "unknown precision");
    set_device(batch_big(B));
    batch_prepare(B, Prec(prec));
    batch_j(B, Prec(prec), out, in, kappa, mu2, DotOut());
    return WL_OK;
  });
}

int wl_batch_cg_solve(wl_batch* B, void* x, const void* b, const double* kappa, const double* mu2,
                      const wl_cg_params* params, wl_cg_stats* stats) {
  return guard([&]() {
    WL_REQUIRE(B && x && b && kappa && params && x != b, WL_EINVAL, "null or aliased argument");
    WL_REQUIRE(!params->use_x0, WL_EUNSUPPORTED, "batch CG starts from x = 0");
    set_device(batch_big(B));
    return batch_cg(B, x, b, kappa, mu2, *params, stats);
  });
}

int wl_solve_log(wl_lattice* L, int enable) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(enable == 0 || enable == 1, WL_EINVAL, "enable must be 0 or 1");
    L->solve_log.clear();
    L->solve_log_on = enable;
    return WL_OK;
  });
}

int wl_solve_log_read(const wl_lattice* L, int max, int* n, long long* iters, long long* residuals, long long* jpa) {
  return guard([&]() {
    check_lat(L);
    WL_REQUIRE(n && max >= 0, WL_EINVAL, "bad arguments");
    *n = int(L->solve_log.size());
    WL_REQUIRE(*n <= max, WL_EINVAL, "solve log longer than the buffers");
    for (int i = 0; i < *n; ++i) {
      if (iters) iters[i] = L->solve_log[i][0];
      if (residuals) residuals[i] = L->solve_log[i][1];
      if (jpa) jpa[i] = L->solve_log[i][2];
    }
    return WL_OK;
  });
}

int wl_counters(const wl_lattice* L, long long* n_hop, long long* n_kmat) {
  return guard([&]() {
    check_lat(L);
    if (n_hop) *n_hop = L->n_hop;
    if (n_kmat) *n_kmat = L->n_kmat;
    return WL_OK;
  });
}

}  // extern "C"
