// Drives the host half of libsrp (plan construction, operator fits, window
// selection, plan exports, argument checks) through the C ABI with host-only
// plans (opts.device = -1), for a build under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Prints one line per case:
//   case <name> status <s> <export>=<sum of |values|> ...
// and exits non-zero when a status differs from the expected one or an
// exported value is not finite.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "srp.h"

namespace {

int failures = 0;

struct Geometry {
  std::string name;
  std::vector<double> mics, grid;
  int M = 0;
  int64_t J = 0;
  double fs = 16000.0;
  int N = 512;
  bool far = false;
};

Geometry circle_array(const std::string& name, int M, double radius, double z_mics) {
  Geometry g;
  g.name = name;
  g.M = M;
  for (int m = 0; m < M; ++m) {
    const double a = 2.0 * M_PI * m / M;
    g.mics.insert(g.mics.end(), {radius * std::cos(a), radius * std::sin(a), z_mics});
  }
  return g;
}

void box_grid(Geometry& g, int nx, int ny, int nz, double x0, double x1, double y0, double y1, double z0,
              double z1) {
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k < nz; ++k) {
        const double x = nx > 1 ? x0 + (x1 - x0) * i / (nx - 1) : x0;
        const double y = ny > 1 ? y0 + (y1 - y0) * j / (ny - 1) : y0;
        const double z = nz > 1 ? z0 + (z1 - z0) * k / (nz - 1) : z0;
        g.grid.insert(g.grid.end(), {x, y, z});
      }
  g.J = static_cast<int64_t>(g.grid.size() / 3);
}

void sphere_directions(Geometry& g, int n_el, int n_az) {
  for (int e = 0; e < n_el; ++e)
    for (int a = 0; a < n_az; ++a) {
      const double el = 0.5 * M_PI * e / n_el, az = 2.0 * M_PI * a / n_az;
      g.grid.insert(g.grid.end(), {std::cos(el) * std::cos(az), std::cos(el) * std::sin(az), std::sin(el)});
    }
  g.J = static_cast<int64_t>(g.grid.size() / 3);
  g.far = true;
}

// sum of |values| of one export (after checking the size query), or -1 when
// the plan has no such data
double export_sum(srp_plan_t plan, const char* what, bool is_int) {
  size_t need = 0;
  if (srp_plan_export(plan, what, nullptr, 0, &need) != SRP_OK) return -1.0;
  std::vector<unsigned char> buf(need + 8);
  size_t need2 = 0;
  if (need > 0 && srp_plan_export(plan, what, buf.data(), need - 1, &need2) == SRP_OK) {
    std::printf("  export %s accepted a short buffer\n", what);
    ++failures;
  }
  if (srp_plan_export(plan, what, buf.data(), need, &need2) != SRP_OK || need2 != need) {
    std::printf("  export %s failed: %s\n", what, srp_last_error());
    ++failures;
    return -1.0;
  }
  double s = 0.0;
  if (is_int) {
    const int32_t* v = reinterpret_cast<const int32_t*>(buf.data());
    for (size_t i = 0; i < need / 4; ++i) s += std::fabs(static_cast<double>(v[i]));
  } else {
    const double* v = reinterpret_cast<const double*>(buf.data());
    for (size_t i = 0; i < need / 8; ++i) {
      if (!std::isfinite(v[i])) {
        std::printf("  export %s: non-finite value at %zu\n", what, i);
        ++failures;
        return -1.0;
      }
      s += std::fabs(v[i]);
    }
  }
  return s;
}

struct Case {
  const Geometry* g;
  const char* label;
  srp_variant variant;
  int rq;
  int global;
  int n_aux;
  srp_dtype dtype;
  srp_status expect;
};

void run(const Case& c) {
  srp_opts o;
  srp_default_opts(&o);
  o.device = -1;
  o.global_fit = c.global;
  o.n_aux = c.n_aux;
  o.dtype = c.dtype;
  o.far_field = c.g->far ? 1 : 0;
  srp_plan_t plan = nullptr;
  const srp_status st = srp_plan(c.g->mics.data(), c.g->M, c.g->grid.data(), c.g->J, c.g->fs, c.g->N, c.variant,
                                 c.rq, &o, &plan);
  std::printf("case %s/%s status %d", c.g->name.c_str(), c.label, static_cast<int>(st));
  if (st != c.expect) {
    std::printf(" (expected %d: %s)\n", static_cast<int>(c.expect), srp_last_error());
    ++failures;
    if (plan) srp_destroy(plan);
    return;
  }
  if (st != SRP_OK) {
    std::printf("\n");
    return;
  }
  srp_plan_info info;
  if (srp_plan_info_get(plan, &info) != SRP_OK) {
    std::printf(" info failed\n");
    ++failures;
  } else {
    std::printf(" P=%d K=%d PN=%d max_np=%d rq=%d macs=%.17g", info.P, info.K, info.PN, info.max_np,
                info.rank_or_q, info.macs_per_map);
  }
  const char* dbl[] = {"tdoa", "slri_u", "slri_v", "slri_s", "sspi_w"};
  const char* ints[] = {"np", "pairs", "sspi_start"};
  for (const char* w : dbl) {
    const double s = export_sum(plan, w, false);
    if (s >= 0) std::printf(" %s=%.17g", w, s);
  }
  for (const char* w : ints) {
    const double s = export_sum(plan, w, true);
    if (s >= 0) std::printf(" %s=%.17g", w, s);
  }
  std::printf("\n");
  // a host-only plan has no device half
  size_t ws = 0;
  if (srp_workspace_size(plan, 4, &ws) != SRP_E_INVALID) {
    std::printf("  workspace_size accepted a host-only plan\n");
    ++failures;
  }
  float dummy[4] = {0, 0, 0, 0};
  if (srp_compute(plan, dummy, 1, dummy, 0, nullptr, 0, nullptr) != SRP_E_INVALID) {
    std::printf("  compute accepted a host-only plan\n");
    ++failures;
  }
  srp_destroy(plan);
}

// checks a status and releases whatever plan the call returned
void expect_status(const char* label, srp_status got, srp_status want, srp_plan_t* plan = nullptr) {
  std::printf("check %s status %d\n", label, static_cast<int>(got));
  if (got != want) {
    std::printf("  expected %d: %s\n", static_cast<int>(want), srp_last_error());
    ++failures;
  }
  if (plan && *plan) {
    if (got != SRP_OK) {
      std::printf("  a failed call returned a plan\n");
      ++failures;
    }
    srp_destroy(*plan);
    *plan = nullptr;
  }
}

}  // namespace

int main() {
  // four microphones on a 0.2 m square over a 30 x 30 plane, N = 512
  Geometry sq = circle_array("square4", 4, 0.1 * std::sqrt(2.0), 0.0);
  box_grid(sq, 30, 30, 1, -1.5, 1.5, -1.5, 1.5, 1.0, 1.0);
  // eight microphones on a 0.3 m circle over a 12 x 12 x 6 room grid, N = 1024
  Geometry uca = circle_array("uca8", 8, 0.15, 1.2);
  uca.N = 1024;
  box_grid(uca, 12, 12, 6, 0.0, 5.0, 0.0, 5.0, 0.0, 2.5);
  // the same array in the far field, a half sphere of directions
  Geometry ff = circle_array("uca8ff", 8, 0.15, 0.0);
  ff.N = 1024;
  sphere_directions(ff, 9, 24);
  // 32 microphones on a 2 m disc rim over a small box, N = 2048
  Geometry disc = circle_array("disc32", 32, 1.0, 0.0);
  disc.N = 2048;
  box_grid(disc, 8, 8, 4, -1.0, 1.0, -1.0, 1.0, 0.5, 2.0);

  const Case cases[] = {
      {&sq, "fd", SRP_FD, 0, 0, 2, SRP_F32, SRP_OK},
      {&sq, "fd_f64", SRP_FD, 0, 0, 2, SRP_F64, SRP_OK},
      {&sq, "slri1", SRP_SLRI, 1, 0, 2, SRP_F32, SRP_OK},
      {&sq, "slri8", SRP_SLRI, 8, 0, 2, SRP_BF16, SRP_OK},
      {&sq, "slri32", SRP_SLRI, 32, 0, 2, SRP_F32, SRP_OK},
      {&sq, "si", SRP_SI, 0, 0, 2, SRP_F32, SRP_OK},
      {&sq, "sspi1", SRP_SSPI, 1, 0, 2, SRP_F32, SRP_OK},
      {&sq, "sspi4", SRP_SSPI, 4, 0, 2, SRP_FP8_E4M3, SRP_OK},
      {&sq, "sspi16", SRP_SSPI, 16, 0, 2, SRP_F32, SRP_OK},
      {&sq, "td_naux0", SRP_TD, 0, 0, 0, SRP_F32, SRP_OK},
      {&sq, "slri_global20", SRP_SLRI, 20, 1, 2, SRP_F32, SRP_OK},
      {&sq, "sspi_global3", SRP_SSPI, 3, 1, 2, SRP_BF16, SRP_OK},
      {&uca, "slri8", SRP_SLRI, 8, 0, 2, SRP_BF16, SRP_OK},
      {&uca, "sspi4", SRP_SSPI, 4, 0, 2, SRP_BF16, SRP_OK},
      {&uca, "td_naux0", SRP_TD, 0, 0, 0, SRP_F32, SRP_OK},
      {&uca, "si", SRP_SI, 0, 0, 2, SRP_F32, SRP_OK},
      {&uca, "slri_global140", SRP_SLRI, 140, 1, 2, SRP_BF16, SRP_OK},
      {&uca, "sspi_global3", SRP_SSPI, 3, 1, 2, SRP_BF16, SRP_OK},
      {&ff, "slri8", SRP_SLRI, 8, 0, 2, SRP_BF16, SRP_OK},
      {&ff, "sspi4", SRP_SSPI, 4, 0, 2, SRP_BF16, SRP_OK},
      {&ff, "slri_global64", SRP_SLRI, 64, 1, 2, SRP_F32, SRP_OK},
      {&disc, "fd", SRP_FD, 0, 0, 2, SRP_BF16, SRP_OK},
      {&disc, "slri8", SRP_SLRI, 8, 0, 2, SRP_BF16, SRP_OK},
      {&disc, "sspi4", SRP_SSPI, 4, 0, 2, SRP_BF16, SRP_OK},
      {&disc, "sspi_global2", SRP_SSPI, 2, 1, 2, SRP_BF16, SRP_OK},
      {&disc, "td_naux0", SRP_TD, 0, 0, 0, SRP_F32, SRP_OK},
      // argument errors
      {&sq, "slri33", SRP_SLRI, 33, 0, 2, SRP_F32, SRP_E_UNSUPPORTED},
      {&sq, "sspi17", SRP_SSPI, 17, 0, 2, SRP_F32, SRP_E_UNSUPPORTED},
      {&sq, "sspi0", SRP_SSPI, 0, 0, 2, SRP_F32, SRP_E_INVALID},
      {&sq, "fd_global", SRP_FD, 0, 1, 2, SRP_F32, SRP_E_INVALID},
      {&sq, "lr_host", SRP_LR, 8, 0, 2, SRP_F32, SRP_E_UNSUPPORTED},
      {&sq, "slri_f64", SRP_SLRI, 8, 0, 2, SRP_F64, SRP_E_UNSUPPORTED},
      {&sq, "naux_neg", SRP_FD, 0, 0, -1, SRP_F32, SRP_E_INVALID},
  };
  for (const Case& c : cases) run(c);

  srp_plan_t plan = nullptr;
  srp_opts o;
  srp_default_opts(&o);
  o.device = -1;
  expect_status("null_out", srp_plan(sq.mics.data(), 4, sq.grid.data(), sq.J, 16000, 512, SRP_FD, 0, &o, nullptr),
                SRP_E_INVALID);
  expect_status("one_mic", srp_plan(sq.mics.data(), 1, sq.grid.data(), sq.J, 16000, 512, SRP_FD, 0, &o, &plan),
                SRP_E_INVALID, &plan);
  expect_status("odd_N", srp_plan(sq.mics.data(), 4, sq.grid.data(), sq.J, 16000, 511, SRP_FD, 0, &o, &plan),
                SRP_E_INVALID, &plan);
  expect_status("aliased_lags",
                srp_plan(disc.mics.data(), 32, disc.grid.data(), disc.J, 16000, 128, SRP_FD, 0, &o, &plan),
                SRP_E_INVALID, &plan);
  expect_status("no_candidates", srp_plan(sq.mics.data(), 4, sq.grid.data(), 0, 16000, 512, SRP_FD, 0, &o, &plan),
                SRP_E_INVALID, &plan);
  std::vector<double> bad_mics = sq.mics;
  bad_mics[4] = NAN;
  expect_status("nan_mic", srp_plan(bad_mics.data(), 4, sq.grid.data(), sq.J, 16000, 512, SRP_FD, 0, &o, &plan),
                SRP_E_INVALID, &plan);
  std::vector<double> dup_mics = sq.mics;
  for (int i = 0; i < 3; ++i) dup_mics[3 + i] = dup_mics[i];
  // two microphones at one point: that pair's TDOA is zero everywhere, which
  // the method allows (its GCC contributes a constant)
  expect_status("coincident_mics",
                srp_plan(dup_mics.data(), 4, sq.grid.data(), sq.J, 16000, 512, SRP_FD, 0, &o, &plan), SRP_OK, &plan);
  o.far_field = 1;
  expect_status("far_field_not_unit",
                srp_plan(sq.mics.data(), 4, sq.grid.data(), sq.J, 16000, 512, SRP_FD, 0, &o, &plan), SRP_E_INVALID, &plan);
  o.far_field = 0;
  o.global_fit = 1;
  expect_status("global_slri_pn_limit",
                srp_plan(disc.mics.data(), 32, disc.grid.data(), disc.J, 16000, 2048, SRP_SLRI, 64, &o, &plan),
                SRP_E_UNSUPPORTED, &plan);
  expect_status("argmax_bad_dtype", srp_argmax(nullptr, SRP_BF16, 1, 1, 0, nullptr, nullptr, nullptr),
                SRP_E_INVALID);
  srp_destroy(nullptr);
  std::printf("failures %d\n", failures);
  return failures == 0 ? 0 : 1;
}
