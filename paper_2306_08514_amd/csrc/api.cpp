// C ABI of the SRP-map library; see include/srp.h for the contract.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/srp.h"
#include "device.hpp"
#include "plan.hpp"

struct srp_plan_s {
  srp::HostPlan hp;
  srp::DevicePlan dp;
  srp_opts opts;
  bool has_device = false;
  double plan_seconds = 0;
};

namespace {

thread_local std::string g_err;

srp_status fail(int code, const std::string& msg) {
  g_err = msg;
  return static_cast<srp_status>(code);
}

// Makes the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (dev < 0) return;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) {
      if (hipSetDevice(dev) != hipSuccess) throw srp::Error{SRP_E_HIP, "hipSetDevice failed"};
      changed = true;
    }
  }
  ~DeviceGuard() {
    if (changed && prev >= 0) (void)hipSetDevice(prev);
  }
};

int plan_threads() {
  unsigned n = std::thread::hardware_concurrency();
  if (n == 0) n = 4;
  return static_cast<int>(std::min(n, 16u));
}

bool dtype_ok(srp_variant v, srp_dtype d) {
  switch (d) {
    case SRP_F32:
    case SRP_BF16:
    case SRP_F16:
    case SRP_FP8_E4M3: return true;
    case SRP_F64: return v == SRP_FD;
  }
  return false;
}

#define SRP_GUARD(...)                                                    \
  try {                                                                   \
    __VA_ARGS__                                                           \
  } catch (const srp::Error& e) {                                         \
    return fail(e.code, e.msg);                                           \
  } catch (const std::bad_alloc&) {                                       \
    return fail(SRP_E_NOMEM, "host allocation failed");                   \
  } catch (const std::exception& e) {                                     \
    return fail(SRP_E_INVALID, e.what());                                 \
  } catch (...) {                                                         \
    return fail(SRP_E_HIP, "unexpected failure");                         \
  }

}  // namespace

extern "C" {

void srp_default_opts(srp_opts* o) {
  if (!o) return;
  o->c = 343.0;
  o->n_aux = 2;
  o->dtype = SRP_F32;
  o->device = 0;
  o->frame_tile = 1024;
  o->hbm_budget = 0;
  o->sampling = 0;
  o->fd_steering = 0;
  o->far_field = 0;
  o->global_fit = 0;
}

const char* srp_last_error(void) { return g_err.c_str(); }

srp_status srp_plan(const double* mics, int M, const double* grid, int64_t J, double fs, int N,
                    srp_variant variant, int rank_or_q, const srp_opts* opts, srp_plan_t* out) {
  if (!out) return fail(SRP_E_INVALID, "out must not be NULL");
  *out = nullptr;
  srp_opts o;
  srp_default_opts(&o);
  if (opts) o = *opts;
  if (variant < SRP_FD || variant > SRP_LR) return fail(SRP_E_INVALID, "unknown variant");
  const bool fixed = variant == SRP_FD || variant == SRP_SI || variant == SRP_TD;  // rank_or_q ignored
  if (o.dtype < SRP_F32 || o.dtype > SRP_F64) return fail(SRP_E_INVALID, "unknown dtype");
  if (!dtype_ok(variant, o.dtype)) return fail(SRP_E_UNSUPPORTED, "dtype not offered for this variant");
  if (!fixed && rank_or_q < 1) return fail(SRP_E_INVALID, "rank_or_q must be >= 1");
  if (o.frame_tile < 1) return fail(SRP_E_INVALID, "frame_tile must be >= 1");
  if (o.sampling < 0 || o.sampling > 2) return fail(SRP_E_INVALID, "sampling must be 0, 1 or 2");
  if (o.fd_steering < 0 || o.fd_steering > 2) return fail(SRP_E_INVALID, "fd_steering must be 0, 1 or 2");
  if (o.global_fit < 0 || o.global_fit > 2) return fail(SRP_E_INVALID, "global_fit must be 0, 1 or 2");
  if (o.global_fit && variant != SRP_SLRI && variant != SRP_SSPI)
    return fail(SRP_E_INVALID, "global_fit applies to SLRI and SSPI only");
  if (o.global_fit == 2 && variant != SRP_SLRI)
    return fail(SRP_E_INVALID, "global_fit 2 (randomized fit) applies to SLRI only");
  if (variant == SRP_SLRI && !o.global_fit && rank_or_q > 32)
    return fail(SRP_E_UNSUPPORTED, "SLRI rank per pair above 32 is not built");
  if (variant == SRP_SSPI && rank_or_q > 16) return fail(SRP_E_UNSUPPORTED, "SSPI with Q above 16 is not built");
  if (variant == SRP_LR && rank_or_q > 1024) return fail(SRP_E_UNSUPPORTED, "LR-SRP with R_H above 1024 is not built");
  if (variant == SRP_LR && o.device < 0)
    return fail(SRP_E_UNSUPPORTED, "LR-SRP fits on the device; host-only plans are not offered");
  SRP_GUARD({
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<srp_plan_s> plan(new srp_plan_s());
    plan->opts = o;
    srp::HostPlan& hp = plan->hp;
    hp.form = variant;
    hp.variant = variant == SRP_SI ? SRP_SLRI : (variant == SRP_TD ? SRP_SSPI : variant);
    hp.dtype = o.dtype;
    hp.requested = rank_or_q;
    srp::build_geometry(hp, mics, M, grid, J, fs, N, o.c, o.n_aux, o.far_field != 0);
    srp::choose_sampling(hp, o.sampling);
    hp.device_fit = o.device >= 0;
    hp.fd_steering = o.fd_steering;
    hp.global_fit = o.global_fit != 0;
    hp.global_rand = o.global_fit == 2;
    if (variant == SRP_SLRI && hp.global_fit) srp::build_slri_global(hp, rank_or_q, plan_threads());
    if (variant == SRP_SLRI && !hp.global_fit) srp::build_slri(hp, rank_or_q, plan_threads());
    if (variant == SRP_SI) srp::build_slri(hp, 2 * hp.max_np + 1, plan_threads());
    if (variant == SRP_SSPI && hp.global_fit) srp::build_sspi_global(hp, rank_or_q, plan_threads());
    if (variant == SRP_SSPI && !hp.global_fit) srp::build_sspi(hp, rank_or_q, plan_threads());
    if (variant == SRP_TD) srp::build_sspi(hp, 1, plan_threads());
    if (variant == SRP_LR) {
      const int64_t n = static_cast<int64_t>(hp.P) * (hp.K - 1);
      if (rank_or_q > std::min<int64_t>(hp.J, n)) throw srp::Error{SRP_E_INVALID, "R_H exceeds min(J, P (K - 1))"};
      hp.RH = rank_or_q;
    }
    srp::count_macs(hp);
    if (o.device >= 0) {
      DeviceGuard g(o.device);
      try {
        srp::device_build(hp, plan->dp, o.frame_tile, o.hbm_budget);
      } catch (...) {
        srp::device_free(plan->dp);
        throw;
      }
      plan->has_device = true;
      // the device holds everything compute needs; drop the host copies of
      // the TDOAs and fits (srp_plan_export serves host-only plans)
      std::vector<double>().swap(hp.x);
      std::vector<double>().swap(hp.U);
      std::vector<double>().swap(hp.w);
      std::vector<int32_t>().swap(hp.start);
    }
    plan->plan_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = plan.release();
    return SRP_OK;
  })
}

srp_status srp_workspace_size(srp_plan_t plan, int64_t L, size_t* bytes) {
  if (!plan || !bytes) return fail(SRP_E_INVALID, "NULL argument");
  if (L < 0) return fail(SRP_E_INVALID, "L must be >= 0");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan");
  SRP_GUARD({
    *bytes = L == 0 ? 0 : srp::workspace_bytes(plan->hp, plan->dp, L, plan->opts.frame_tile);
    return SRP_OK;
  })
}

srp_status srp_compute(srp_plan_t plan, const void* frames, int64_t L, void* maps, int64_t ld_maps,
                       void* workspace, size_t ws_bytes, void* stream) {
  if (!plan) return fail(SRP_E_INVALID, "NULL plan");
  if (L < 0) return fail(SRP_E_INVALID, "L must be >= 0");
  if (ld_maps == 0) ld_maps = plan->hp.J;
  if (ld_maps < plan->hp.J) return fail(SRP_E_INVALID, "ld_maps must be 0 or >= J");
  if (L == 0) return SRP_OK;
  if (!frames || !maps) return fail(SRP_E_INVALID, "frames and maps must be device pointers");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan cannot compute");
  SRP_GUARD({
    DeviceGuard g(plan->dp.device);
    srp::device_compute(plan->hp, plan->dp, frames, L, maps, ld_maps, workspace, ws_bytes,
                        plan->opts.frame_tile, static_cast<hipStream_t>(stream));
    return SRP_OK;
  })
}

srp_status srp_compute_static(srp_plan_t plan, const void* frames, int64_t L, void* maps, int64_t ld_maps,
                              void* stream) {
  if (!plan) return fail(SRP_E_INVALID, "NULL plan");
  if (L < 0) return fail(SRP_E_INVALID, "L must be >= 0");
  if (ld_maps == 0) ld_maps = plan->hp.J;
  if (ld_maps < plan->hp.J) return fail(SRP_E_INVALID, "ld_maps must be 0 or >= J");
  if (L == 0) return SRP_OK;
  if (!frames || !maps) return fail(SRP_E_INVALID, "frames and maps must be device pointers");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan cannot compute");
  SRP_GUARD({
    DeviceGuard g(plan->dp.device);
    srp::device_compute_static(plan->hp, plan->dp, frames, L, maps, ld_maps, plan->opts.frame_tile,
                               static_cast<hipStream_t>(stream));
    return SRP_OK;
  })
}

srp_status srp_argmax(const void* maps, srp_dtype dtype, int64_t L, int64_t J, int64_t ld_maps,
                      int64_t* idx, double* val, void* stream) {
  if (L < 0 || J < 1) return fail(SRP_E_INVALID, "need L >= 0 and J >= 1");
  if (ld_maps < J) return fail(SRP_E_INVALID, "ld_maps must be >= J");
  if (dtype != SRP_F32 && dtype != SRP_F64) return fail(SRP_E_INVALID, "maps must be float32 or float64");
  if (L == 0) return SRP_OK;
  if (!maps || !idx || !val) return fail(SRP_E_INVALID, "maps, idx and val must be device pointers");
  SRP_GUARD({
    srp::device_argmax(maps, dtype == SRP_F64, L, J, ld_maps, idx, val, static_cast<hipStream_t>(stream));
    return SRP_OK;
  })
}

srp_status srp_crossspec(srp_plan_t plan, const void* frames, int64_t L, void* psi, void* stream) {
  if (!plan) return fail(SRP_E_INVALID, "NULL plan");
  if (L < 0) return fail(SRP_E_INVALID, "L must be >= 0");
  if (L == 0) return SRP_OK;
  if (!frames || !psi) return fail(SRP_E_INVALID, "frames and psi must be device pointers");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan cannot compute");
  SRP_GUARD({
    DeviceGuard g(plan->dp.device);
    srp::device_crossspec(plan->hp, plan->dp, frames, L, psi, static_cast<hipStream_t>(stream));
    return SRP_OK;
  })
}

srp_status srp_gcc_samples(srp_plan_t plan, const void* frames, int64_t L, float* xi, void* stream) {
  if (!plan) return fail(SRP_E_INVALID, "NULL plan");
  if (L < 0) return fail(SRP_E_INVALID, "L must be >= 0");
  if (L == 0) return SRP_OK;
  if (!frames || !xi) return fail(SRP_E_INVALID, "frames and xi must be device pointers");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan cannot compute");
  if (plan->hp.variant == SRP_FD) return fail(SRP_E_INVALID, "FD plans have no sampling stage");
  SRP_GUARD({
    DeviceGuard g(plan->dp.device);
    srp::device_gcc_samples(plan->hp, plan->dp, frames, L, xi, nullptr, 0, plan->opts.frame_tile,
                            static_cast<hipStream_t>(stream));
    return SRP_OK;
  })
}

srp_status srp_plan_info_get(srp_plan_t plan, srp_plan_info* info) {
  if (!plan || !info) return fail(SRP_E_INVALID, "NULL argument");
  const srp::HostPlan& hp = plan->hp;
  std::memset(info, 0, sizeof(*info));
  info->M = hp.M;
  info->P = hp.P;
  info->K = hp.K;
  info->J = hp.J;
  info->PN = hp.PN;
  info->max_np = hp.max_np;
  info->rank_or_q = hp.variant == SRP_SLRI ? hp.R : (hp.variant == SRP_SSPI ? hp.Q : (hp.variant == SRP_LR ? hp.RH : 0));
  info->variant = static_cast<srp_variant>(hp.form);
  info->dtype = static_cast<srp_dtype>(hp.dtype);
  info->mean_n = hp.mean_n;
  info->macs_per_map = hp.macs_per_map;
  info->device_bytes = plan->dp.resident_bytes;
  info->plan_seconds = plan->plan_seconds;
  info->map_pitch = (hp.J + 127) / 128 * 128;
  info->sampling_fft = hp.fft ? 1 : 0;
  info->fd_generated = plan->dp.fd_gen ? 1 : 0;
  if (hp.variant == SRP_SSPI) {
    const int ntiles = static_cast<int>((hp.J + 255) / 256);
    info->sspi_dense_tiles = plan->dp.sspi_dense ? plan->dp.n_dtiles : 0;
    info->sspi_band_tiles = plan->dp.sspi_band ? ntiles : 0;
    info->sspi_gather_tiles = plan->dp.sspi_dense ? plan->dp.n_gtiles : (plan->dp.sspi_band ? 0 : ntiles);
  }
  return SRP_OK;
}

srp_status srp_plan_export(srp_plan_t plan, const char* what, void* dst, size_t bytes, size_t* needed) {
  if (!plan || !what) return fail(SRP_E_INVALID, "NULL argument");
  const srp::HostPlan& hp = plan->hp;
  const void* src = nullptr;
  size_t n = 0;
  std::vector<int32_t> tmp;
  const std::string w(what);
  if (plan->has_device && (w == "tdoa" || w == "slri_u" || w == "sspi_start" || w == "sspi_w"))
    return fail(SRP_E_INVALID, "'" + w + "' is kept only by host-only plans");
  if (w == "tdoa") {
    src = hp.x.data();
    n = hp.x.size() * sizeof(double);
  } else if (w == "np") {
    src = hp.np.data();
    n = hp.np.size() * 4;
  } else if (w == "pairs") {
    tmp.resize(2 * hp.P);
    for (int p = 0; p < hp.P; ++p) {
      tmp[2 * p] = hp.pair_m[p];
      tmp[2 * p + 1] = hp.pair_mp[p];
    }
    src = tmp.data();
    n = tmp.size() * 4;
  } else if (w == "slri_u" && hp.variant == SRP_SLRI) {
    src = hp.U.data();
    n = hp.U.size() * sizeof(double);
  } else if (w == "slri_v" && hp.variant == SRP_SLRI) {
    src = hp.V.data();
    n = hp.V.size() * sizeof(double);
  } else if (w == "slri_s" && hp.variant == SRP_SLRI) {
    src = hp.sv.data();
    n = hp.sv.size() * sizeof(double);
  } else if (w == "lr_s" && hp.variant == SRP_LR) {
    src = hp.lr_s.data();
    n = hp.lr_s.size() * sizeof(double);
  } else if (w == "sspi_start" && hp.variant == SRP_SSPI) {
    src = hp.start.data();
    n = hp.start.size() * 4;
  } else if (w == "sspi_w" && hp.variant == SRP_SSPI) {
    src = hp.w.data();
    n = hp.w.size() * sizeof(double);
  } else {
    return fail(SRP_E_INVALID, "no plan data named '" + w + "' for this variant");
  }
  if (needed) *needed = n;
  if (!dst) return SRP_OK;
  if (bytes < n) return fail(SRP_E_INVALID, "destination too small");
  std::memcpy(dst, src, n);
  return SRP_OK;
}

srp_status srp_profile_enable(srp_plan_t plan, int enable) {
  if (!plan) return fail(SRP_E_INVALID, "NULL plan");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan");
  plan->dp.profiling = enable != 0;
  return SRP_OK;
}

srp_status srp_profile_collect(srp_plan_t plan, srp_kernel_time* out, int capacity, int* count) {
  if (!plan || !count || capacity < 0 || (capacity > 0 && !out)) return fail(SRP_E_INVALID, "bad argument");
  if (!plan->has_device) return fail(SRP_E_INVALID, "host-only plan");
  SRP_GUARD({
    DeviceGuard g(plan->dp.device);
    std::vector<std::pair<std::string, std::pair<double, int64_t>>> acc;
    srp::device_profile_collect(plan->dp, acc);
    *count = static_cast<int>(acc.size());
    for (int i = 0; i < capacity && i < static_cast<int>(acc.size()); ++i) {
      std::memset(out[i].name, 0, sizeof(out[i].name));
      std::strncpy(out[i].name, acc[i].first.c_str(), sizeof(out[i].name) - 1);
      out[i].total_ms = acc[i].second.first;
      out[i].launches = acc[i].second.second;
    }
    return SRP_OK;
  })
}

void srp_destroy(srp_plan_t plan) {
  if (!plan) return;
  if (plan->has_device) {
    try {
      DeviceGuard g(plan->dp.device);
      srp::device_free(plan->dp);
    } catch (...) {
    }
  }
  delete plan;
}

}  // extern "C"
