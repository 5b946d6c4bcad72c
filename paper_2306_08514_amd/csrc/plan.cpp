// Host-side FP64 plan construction.  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <thread>

#include "../../include/srp.h"

namespace srp {

namespace {

void fail(const std::string& msg) { throw Error{SRP_E_INVALID, msg}; }

}  // namespace

// Runs body(i) for i in [0, n) on up to `threads` threads.
void parallel_for(int n, int threads, const std::function<void(int)>& body) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; ++i) body(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  std::vector<Error> errs(threads, Error{0, ""});
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t] {
      try {
        for (int i = next++; i < n; i = next++) body(i);
      } catch (const Error& e) {
        errs[t] = e;
      } catch (...) {
        errs[t] = Error{SRP_E_NOMEM, "host allocation failed during plan build"};
      }
    });
  }
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (e.code != 0) throw e;
}


double sinc_shift(double x, int n) {
  // sin(pi (x - n)) = (-1)^(n + k0) sin(pi r) with x = k0 + r, |r| <= 1/2;
  // the reduction x - rint(x) is exact in FP64.
  const double d = x - static_cast<double>(n);
  if (d == 0.0) return 1.0;
  const double k0 = std::rint(x);
  const double r = x - k0;
  const double s = std::sin(M_PI * r);
  const long long parity = (static_cast<long long>(k0) + n) & 1LL;
  const double num = parity ? -s : s;
  return num / (M_PI * d);
}

void build_geometry(HostPlan& hp, const double* mics, int M, const double* grid,
                    int64_t J, double fs, int N, double c, int n_aux, bool far_field) {
  if (!mics || !grid) fail("mics and grid must be non-NULL host pointers");
  if (M < 2) fail("need at least 2 microphones");
  if (M > 64) fail("at most 64 microphones are supported");
  if (J < 1) fail("need at least one candidate location");
  if (!(fs > 0) || !std::isfinite(fs)) fail("fs must be positive and finite");
  if (N < 8 || (N & 1)) fail("N must be even and >= 8");
  if (N > 16384) fail("N above 16384 is not supported");
  if (!(c > 0) || !std::isfinite(c)) fail("speed of sound must be positive");
  if (n_aux < 0) fail("n_aux must be >= 0");
  for (int i = 0; i < 3 * M; ++i)
    if (!std::isfinite(mics[i])) fail("non-finite microphone coordinate");
  for (int64_t i = 0; i < 3 * J; ++i)
    if (!std::isfinite(grid[i])) fail("non-finite grid coordinate");

  hp.M = M;
  hp.J = J;
  hp.fs = fs;
  hp.N = N;
  hp.K = N / 2;
  hp.c = c;
  hp.n_aux = n_aux;
  hp.P = M * (M - 1) / 2;
  hp.mics.assign(mics, mics + 3 * M);
  hp.grid.assign(grid, grid + 3 * J);

  // pairs (m, m'), m > m', m' outer (the double sum of eq. (8))
  hp.pair_m.clear();
  hp.pair_mp.clear();
  for (int mp = 0; mp < M - 1; ++mp)
    for (int m = mp + 1; m < M; ++m) {
      hp.pair_m.push_back(m);
      hp.pair_mp.push_back(mp);
    }

  // N_p = floor(d_p fs / c) + N_aux, eq. (33)
  hp.np.resize(hp.P);
  hp.off.resize(hp.P);
  hp.PN = 0;
  hp.max_np = 0;
  for (int p = 0; p < hp.P; ++p) {
    const double* a = &mics[3 * hp.pair_m[p]];
    const double* b = &mics[3 * hp.pair_mp[p]];
    const double d = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                               (a[2] - b[2]) * (a[2] - b[2]));
    const int n_p = static_cast<int>(std::floor(d * fs / c)) + n_aux;
    if (2 * n_p + 1 > N)
      fail("frame too short: 2 N_p + 1 > N for a pair (lags would alias)");
    hp.np[p] = n_p;
    hp.off[p] = hp.PN;
    hp.PN += 2 * n_p + 1;
    hp.max_np = std::max(hp.max_np, n_p);
  }
  hp.mean_n = static_cast<double>(hp.PN) / hp.P;

  // TDOA in samples, near field, eq. (3)
  hp.far_field = far_field;
  if (far_field) {
    // far-field TDOA, the far limit of (3): x_p = -(r_m - r_m')^T u fs / c
    for (int64_t j = 0; j < J; ++j) {
      const double* u = &grid[3 * j];
      const double len = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (!(std::fabs(1.0 - len) <= 1e-6)) fail("far-field grid rows must be unit vectors");
    }
    hp.x.assign(static_cast<size_t>(hp.P) * J, 0.0);
    for (int p = 0; p < hp.P; ++p) {
      const double* rm = &mics[3 * hp.pair_m[p]];
      const double* rq = &mics[3 * hp.pair_mp[p]];
      const double d0 = rm[0] - rq[0], d1 = rm[1] - rq[1], d2 = rm[2] - rq[2];
      double* xp = &hp.x[static_cast<size_t>(p) * J];
      for (int64_t j = 0; j < J; ++j) {
        const double* u = &grid[3 * j];
        xp[j] = -(d0 * u[0] + d1 * u[1] + d2 * u[2]) * fs / c;
      }
    }
    return;
  }
  hp.x.assign(static_cast<size_t>(hp.P) * J, 0.0);
  const int chunks = static_cast<int>(std::min<int64_t>(64, std::max<int64_t>(1, J / 4096)));
  const unsigned hw = std::thread::hardware_concurrency();
  parallel_for(chunks, static_cast<int>(std::min(std::max(hw, 1u), 16u)), [&](int ch) {
    std::vector<double> dist(static_cast<size_t>(M));
    for (int64_t j = J * ch / chunks; j < J * (ch + 1) / chunks; ++j) {
      const double* q = &grid[3 * j];
      for (int m = 0; m < M; ++m) {
        const double* r = &mics[3 * m];
        dist[m] = std::sqrt((r[0] - q[0]) * (r[0] - q[0]) + (r[1] - q[1]) * (r[1] - q[1]) +
                            (r[2] - q[2]) * (r[2] - q[2]));
      }
      for (int p = 0; p < hp.P; ++p)
        hp.x[static_cast<size_t>(p) * J + j] = (dist[hp.pair_m[p]] - dist[hp.pair_mp[p]]) * fs / c;
    }
  });
}

void sym_eig(std::vector<double>& a, int n, std::vector<double>& evals,
             std::vector<double>& evecs) {
  evecs.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) evecs[static_cast<size_t>(i) * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[static_cast<size_t>(i) * n + j]; };
  auto V = [&](int i, int j) -> double& { return evecs[static_cast<size_t>(i) * n + j]; };
  double scale = 0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(A(i, i)));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    if (off <= 1e-30 * scale * scale || off == 0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        // rotation angle: t = tan(phi) solves t^2 + 2 theta t - 1 = 0 with
        // theta = (a_qq - a_pp) / (2 a_pq); the smaller root is stable
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0);
        const double sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q of A
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q of A
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = cs * vkp - sn * vkq;
          V(k, q) = sn * vkp + cs * vkq;
        }
      }
    }
  }
  // sort descending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int u, int v) { return A(u, u) > A(v, v); });
  evals.resize(n);
  std::vector<double> sorted(static_cast<size_t>(n) * n);
  for (int c = 0; c < n; ++c) {
    evals[c] = A(idx[c], idx[c]);
    for (int r = 0; r < n; ++r) sorted[static_cast<size_t>(r) * n + c] = V(r, idx[c]);
  }
  evecs.swap(sorted);
}

// Symmetric eigendecomposition by Householder reduction to tridiagonal form
// followed by the implicitly shifted QL iteration; same interface as sym_eig.
// The orthogonal factor is accumulated transposed (row i = i-th basis
// vector) so that both the reduction and the QL rotations touch contiguous
// rows.
void sym_eig_tridiag(std::vector<double>& a, int n, std::vector<double>& evals,
                     std::vector<double>& evecs) {
  auto A = [&](int i, int j) -> double& { return a[static_cast<size_t>(i) * n + j]; };
  std::vector<double> zt(static_cast<size_t>(n) * n, 0.0);  // Q^T, later Z^T
  auto Z = [&](int i, int j) -> double& { return zt[static_cast<size_t>(i) * n + j]; };
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  std::vector<double> v(n), p(n), w(n), r(n);
  // reduction: step k annihilates column k below the subdiagonal with the
  // reflector H = I - 2 v v^T, v supported on k+1..n-1; A <- H A H and
  // Q^T <- H Q^T
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += A(i, k) * A(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (A(k + 1, k) > 0) alpha = -alpha;
    std::fill(v.begin(), v.end(), 0.0);
    for (int i = k + 1; i < n; ++i) v[i] = A(i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // H A H = A - v w^T - w v^T with p = A v, w = 2 (p - (v^T p) v)
    for (int i = k; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
      p[i] = s;
    }
    double kv = 0.0;
    for (int i = k + 1; i < n; ++i) kv += v[i] * p[i];
    for (int i = k; i < n; ++i) w[i] = 2.0 * (p[i] - kv * v[i]);
    for (int i = k; i < n; ++i) {
      double* ai = &A(i, 0);
      const double vi = v[i], wi = w[i];
      for (int j = k; j < n; ++j) ai[j] -= vi * w[j] + wi * v[j];
    }
    // Q^T <- H Q^T: rows k+1.. change by -2 v (v^T Q^T)
    std::fill(r.begin(), r.end(), 0.0);
    for (int i = k + 1; i < n; ++i) {
      const double vi = v[i];
      const double* zi = &Z(i, 0);
      for (int c = 0; c < n; ++c) r[c] += vi * zi[c];
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = 2.0 * v[i];
      double* zi = &Z(i, 0);
      for (int c = 0; c < n; ++c) zi[c] -= f * r[c];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
  // implicit QL with shifts from the trailing 2 x 2 block: e[i] couples
  // d[i] and d[i + 1]; a chase from m - 1 down to l applies plane rotations
  // to rows i, i + 1 of Z^T.  An off-diagonal counts as negligible against
  // the norm of the whole tridiagonal matrix, so blocks of (near-)zero
  // eigenvalues of a rank-deficient Gram matrix deflate too; the small
  // eigenvalues are then accurate to eps |T|, the accuracy the Gram route
  // gives them anyway.
  double tst = 0.0;
  for (int i = 0; i < n; ++i) tst = std::max(tst, std::fabs(d[i]) + std::fabs(e[i]) + (i ? std::fabs(e[i - 1]) : 0.0));
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        if (std::fabs(e[m]) <= std::numeric_limits<double>::epsilon() * tst) break;
      }
      if (m == l) break;
      if (iter == 100) throw Error{SRP_E_INVALID, "eigensolver did not converge"};
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double rr = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(rr, g));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool early = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        rr = std::hypot(f, g);
        e[i + 1] = rr;
        if (rr == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / rr;
        c = g / rr;
        g = d[i + 1] - pp;
        rr = (d[i] - g) * s + 2.0 * c * b;
        pp = s * rr;
        d[i + 1] = g + pp;
        g = c * rr - b;
        double* zi = &Z(i, 0);
        double* zi1 = &Z(i + 1, 0);
        for (int k = 0; k < n; ++k) {
          const double a0 = zi[k], a1 = zi1[k];
          zi1[k] = s * a0 + c * a1;
          zi[k] = c * a0 - s * a1;
        }
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int u, int w2) { return d[u] > d[w2]; });
  evals.resize(n);
  evecs.assign(static_cast<size_t>(n) * n, 0.0);
  for (int c = 0; c < n; ++c) {
    evals[c] = d[idx[c]];
    const double* zc = &Z(idx[c], 0);
    for (int rrow = 0; rrow < n; ++rrow) evecs[static_cast<size_t>(rrow) * n + c] = zc[rrow];
  }
}

void slri_fit_pair(HostPlan& hp, int p, std::vector<double>& G) {
  const int nmax = 2 * hp.max_np + 1;
  const int n = 2 * hp.np[p] + 1;
  const int r_p = hp.rp[p];
  // eigenvectors of G are the right singular vectors of Lambda_p,
  // eigenvalues the squared singular values
  std::vector<double> ev, vec;
  if (n <= 64)
    sym_eig(G, n, ev, vec);
  else
    sym_eig_tridiag(G, n, ev, vec);
  for (int i = 0; i < n; ++i) hp.sv[static_cast<size_t>(p) * nmax + i] = std::sqrt(std::max(0.0, ev[i]));
  double* Vp = &hp.V[static_cast<size_t>(p) * nmax * hp.R];
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < r_p; ++r) Vp[static_cast<size_t>(i) * hp.R + r] = vec[static_cast<size_t>(i) * n + r];
}

void build_slri(HostPlan& hp, int R, int threads) {
  if (R < 1) fail("rank must be >= 1");
  const int nmax = 2 * hp.max_np + 1;
  hp.R = std::min(R, nmax);
  hp.rp.resize(hp.P);
  for (int p = 0; p < hp.P; ++p) hp.rp[p] = std::min(R, 2 * hp.np[p] + 1);
  hp.V.assign(static_cast<size_t>(hp.P) * nmax * hp.R, 0.0);
  hp.sv.assign(static_cast<size_t>(hp.P) * nmax, 0.0);
  const bool si = hp.form == SRP_SI;
  if (si) {
    // SI-SRP (44): U_p = Lambda_p, V_p = I (every lag kept, no fit)
    for (int p = 0; p < hp.P; ++p)
      for (int i = 0; i < 2 * hp.np[p] + 1; ++i) {
        hp.V[(static_cast<size_t>(p) * nmax + i) * hp.R + i] = 1.0;
        hp.sv[static_cast<size_t>(p) * nmax + i] = 1.0;
      }
  }
  if (hp.device_fit) return;  // Gram matrices and U come from the device
  const int64_t J = hp.J;
  hp.U.assign(static_cast<size_t>(hp.P) * J * hp.R, 0.0);
  parallel_for(hp.P, threads, [&](int p) {
    const int n_p = hp.np[p];
    const int n = 2 * n_p + 1;
    const int r_p = hp.rp[p];
    const double* x = &hp.x[static_cast<size_t>(p) * J];
    // Gram matrix G = Lambda_p^T Lambda_p accumulated row by row in FP64
    std::vector<double> G(static_cast<size_t>(n) * n, 0.0), lam(n);
    for (int64_t j = 0; j < J; ++j) {
      for (int i = 0; i < n; ++i) lam[i] = sinc_shift(x[j], i - n_p);
      for (int a = 0; a < n; ++a) {
        const double la = lam[a];
        double* g = &G[static_cast<size_t>(a) * n];
        for (int b = a; b < n; ++b) g[b] += la * lam[b];
      }
    }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < a; ++b) G[static_cast<size_t>(a) * n + b] = G[static_cast<size_t>(b) * n + a];
    if (!si) slri_fit_pair(hp, p, G);
    // U_p = Lambda_p V_p (= left singular vectors times singular values)
    const double* Vp = &hp.V[static_cast<size_t>(p) * nmax * hp.R];
    double* Up = &hp.U[static_cast<size_t>(p) * J * hp.R];
    for (int64_t j = 0; j < J; ++j) {
      for (int i = 0; i < n; ++i) lam[i] = sinc_shift(x[j], i - n_p);
      for (int r = 0; r < r_p; ++r) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += lam[i] * Vp[static_cast<size_t>(i) * hp.R + r];
        Up[static_cast<size_t>(j) * hp.R + r] = s;
      }
    }
  });
}

void slri_fit_global(HostPlan& hp, std::vector<double>& G) {
  const int n = hp.PN;
  std::vector<double> ev, vec;
  if (n <= 64)
    sym_eig(G, n, ev, vec);
  else
    sym_eig_tridiag(G, n, ev, vec);
  for (int i = 0; i < n; ++i) hp.sv[i] = std::sqrt(std::max(0.0, ev[i]));
  for (int a = 0; a < n; ++a)
    for (int r = 0; r < hp.R; ++r) hp.V[static_cast<size_t>(a) * hp.R + r] = vec[static_cast<size_t>(a) * n + r];
}

void build_slri_global(HostPlan& hp, int R, int threads) {
  if (R < 1) fail("rank must be >= 1");
  const int n = hp.PN;
  // the exact fit decomposes the PN x PN Gram matrix; wider stacks take the
  // randomized fit on the device
  if (n > 4096) hp.global_rand = true;
  if (hp.global_rand && !hp.device_fit)
    throw Error{SRP_E_UNSUPPORTED,
                "host-only plans fit the global SLRI through the Gram matrix (PN <= 4096); the randomized fit runs "
                "on the device"};
  hp.R = std::min(R, n);
  hp.rp.assign(hp.P, 0);
  hp.V.assign(static_cast<size_t>(n) * hp.R, 0.0);
  hp.sv.assign(n, 0.0);
  if (hp.device_fit) return;  // Gram matrix and U come from the device
  const int64_t J = hp.J;
  // stacked column a <-> (pair, lag)
  std::vector<int> pa(n), la(n);
  for (int p = 0; p < hp.P; ++p)
    for (int i = 0; i < 2 * hp.np[p] + 1; ++i) {
      pa[hp.off[p] + i] = p;
      la[hp.off[p] + i] = i - hp.np[p];
    }
  const int64_t CH = 512;
  std::vector<double> lam(static_cast<size_t>(CH) * n);
  auto fill = [&](int64_t j0, int64_t rows) {
    parallel_for(static_cast<int>(rows), threads, [&](int r) {
      double* row = &lam[static_cast<size_t>(r) * n];
      for (int a = 0; a < n; ++a) row[a] = sinc_shift(hp.x[static_cast<size_t>(pa[a]) * J + j0 + r], la[a]);
    });
  };
  std::vector<double> G(static_cast<size_t>(n) * n, 0.0);
  for (int64_t j0 = 0; j0 < J; j0 += CH) {
    const int64_t rows = std::min(CH, J - j0);
    fill(j0, rows);
    parallel_for(n, threads, [&](int a) {
      double* g = &G[static_cast<size_t>(a) * n];
      for (int64_t r = 0; r < rows; ++r) {
        const double* row = &lam[static_cast<size_t>(r) * n];
        const double va = row[a];
        for (int b = a; b < n; ++b) g[b] += va * row[b];
      }
    });
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < a; ++b) G[static_cast<size_t>(a) * n + b] = G[static_cast<size_t>(b) * n + a];
  slri_fit_global(hp, G);
  // U = Lambda V (left singular vectors times singular values)
  hp.U.assign(static_cast<size_t>(J) * hp.R, 0.0);
  for (int64_t j0 = 0; j0 < J; j0 += CH) {
    const int64_t rows = std::min(CH, J - j0);
    fill(j0, rows);
    parallel_for(static_cast<int>(rows), threads, [&](int r) {
      const double* row = &lam[static_cast<size_t>(r) * n];
      double* u = &hp.U[static_cast<size_t>(j0 + r) * hp.R];
      for (int a = 0; a < n; ++a) {
        const double v = row[a];
        const double* Va = &hp.V[static_cast<size_t>(a) * hp.R];
        for (int c = 0; c < hp.R; ++c) u[c] += v * Va[c];
      }
    });
  }
}

void build_sspi(HostPlan& hp, int Q, int threads) {
  if (Q < 1) fail("Q must be >= 1");
  const int nmax = 2 * hp.max_np + 1;
  hp.Q = std::min(Q, nmax);
  hp.qp.resize(hp.P);
  for (int p = 0; p < hp.P; ++p) hp.qp[p] = std::min(Q, 2 * hp.np[p] + 1);
  if (hp.device_fit) return;  // windows and weights come from the device
  const int64_t J = hp.J;
  hp.start.assign(static_cast<size_t>(J) * hp.P, 0);
  hp.w.assign(static_cast<size_t>(J) * hp.P * hp.Q, 0.0);
  const int chunks = 64;
  parallel_for(chunks, threads, [&](int ch) {
    const int64_t j0 = J * ch / chunks, j1 = J * (ch + 1) / chunks;
    for (int64_t j = j0; j < j1; ++j) {
      for (int p = 0; p < hp.P; ++p) {
        const int n_p = hp.np[p];
        const int q = hp.qp[p];
        const double x = hp.x[static_cast<size_t>(p) * J + j];
        double* w = &hp.w[(static_cast<size_t>(j) * hp.P + p) * hp.Q];
        if (hp.form == SRP_TD) {
          // conv. TD-SRP (23): the lag nearest to x (half away from zero),
          // unit weight, kept in the sampled range [-N_p, N_p]
          const double r = std::min(std::max(std::copysign(std::floor(std::fabs(x) + 0.5), x),
                                             static_cast<double>(-n_p)), static_cast<double>(n_p));
          hp.start[static_cast<size_t>(j) * hp.P + p] = static_cast<int>(r);
          w[0] = 1.0;
          continue;
        }
        // the q integers nearest to x, clamped to [-N_p, N_p]; |sinc(x - n)|
        // decreases with |x - n|, so these are the q largest entries
        double s = std::ceil(x - 0.5 * q);
        s = std::min(std::max(s, static_cast<double>(-n_p)), static_cast<double>(n_p - q + 1));
        const int si = static_cast<int>(s);
        hp.start[static_cast<size_t>(j) * hp.P + p] = si;
        for (int t = 0; t < q; ++t) w[t] = sinc_shift(x, si + t);
      }
    }
  });
}

namespace {

// Lags n in [-N, N] with |sinc(x - n)| >= tau, x = k0 + r with the reduced
// sine sr = |sin(pi r)|: |sinc(x - n)| = sr / (pi |x - n|) for n != x, so
// they are the lags within sr / (pi tau) of x, a contiguous run [lo, hi].
// At integer x only n = x (value 1) is nonzero.
inline void kept_window(double x, double sr, int N, double tau, int& lo, int& hi) {
  if (tau > 1.0) {
    lo = 0;
    hi = -1;
    return;
  }
  if (sr == 0.0) {
    lo = hi = static_cast<int>(x);
    return;
  }
  const double d = sr / (M_PI * tau);
  lo = static_cast<int>(std::max(std::ceil(x - d), static_cast<double>(-N)));
  hi = static_cast<int>(std::min(std::floor(x + d), static_cast<double>(N)));
}

}  // namespace

void build_sspi_global(HostPlan& hp, int qbar, int threads) {
  if (qbar < 1) fail("Q must be >= 1");
  const int64_t J = hp.J;
  const int P = hp.P;
  const double target = static_cast<double>(qbar) * J * P;  // Q_Lambda
  if (target > static_cast<double>(J) * hp.PN) fail("Q_Lambda = Q J P exceeds the J x PN entries of Lambda");
  // reduced sines, pair-major
  std::vector<double> sr(static_cast<size_t>(P) * J);
  const int chunks = 64;
  parallel_for(chunks, threads, [&](int ch) {
    const size_t e0 = sr.size() * ch / chunks, e1 = sr.size() * (ch + 1) / chunks;
    for (size_t e = e0; e < e1; ++e) {
      const double x = hp.x[e];
      sr[e] = std::fabs(std::sin(M_PI * (x - std::nearbyint(x))));
    }
  });
  auto count = [&](double tau) {
    std::vector<double> part(chunks, 0.0);
    parallel_for(chunks, threads, [&](int ch) {
      const size_t e0 = sr.size() * ch / chunks, e1 = sr.size() * (ch + 1) / chunks;
      double c = 0;
      for (size_t e = e0; e < e1; ++e) {
        int lo, hi;
        kept_window(hp.x[e], sr[e], hp.np[e / J], tau, lo, hi);
        c += std::max(0, hi - lo + 1);
      }
      part[ch] = c;
    });
    double c = 0;
    for (double v : part) c += v;
    return c;
  };
  // largest tau with count(tau) >= Q_Lambda, by bisection over the bit
  // patterns of positive doubles (ordered like their values)
  uint64_t lo = 1, hi;  // lo: the smallest subnormal; count(hi) < target
  const double above = std::nextafter(1.0, 2.0);
  std::memcpy(&hi, &above, 8);
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    double t;
    std::memcpy(&t, &mid, 8);
    if (count(t) >= target) lo = mid; else hi = mid;
  }
  std::memcpy(&hp.tau, &lo, 8);
  double tau_above;  // the next magnitude up: count(tau_above) < Q_Lambda
  std::memcpy(&tau_above, &hi, 8);
  // every entry strictly above tau ...
  hp.gstart.assign(static_cast<size_t>(P) * J, 0);
  hp.gcount.assign(static_cast<size_t>(P) * J, 0);
  std::vector<double> nnz(chunks, 0.0);
  parallel_for(chunks, threads, [&](int ch) {
    const size_t e0 = sr.size() * ch / chunks, e1 = sr.size() * (ch + 1) / chunks;
    for (size_t e = e0; e < e1; ++e) {
      const int N = hp.np[e / J];
      int a, b;
      kept_window(hp.x[e], sr[e], N, tau_above, a, b);
      const int c = std::max(0, b - a + 1);
      // an empty window still needs a start inside the pair's lags
      hp.gstart[e] = c > 0 ? a : std::min(std::max(static_cast<int>(std::nearbyint(hp.x[e])), -N), N);
      hp.gcount[e] = c;
      nnz[ch] += c;
    }
  });
  double kept = 0;
  for (double v : nnz) kept += v;
  // ... then entries equal to tau, in the order of the stacked matrix
  // (candidate-major, then pair and lag), until exactly Q_Lambda are kept.
  // A tie lies at the threshold distance from x, so it extends a window at
  // one of its ends and the kept lags stay contiguous.
  for (int64_t j = 0; j < J && kept < target; ++j)
    for (int p = 0; p < P && kept < target; ++p) {
      const size_t e = static_cast<size_t>(p) * J + j;
      int a, b;
      kept_window(hp.x[e], sr[e], hp.np[p], hp.tau, a, b);
      int s0 = hp.gstart[e], c0 = hp.gcount[e];
      if (b - a + 1 <= c0) continue;
      for (int n = a; n <= b && kept < target; ++n) {
        if (c0 > 0 && n >= s0 && n < s0 + c0) continue;  // already kept
        if (c0 == 0) {
          s0 = n;
        } else if (n < s0) {
          s0 = n;
        } else if (n != s0 + c0) {
          continue;  // not adjacent: cannot happen for a tie, kept contiguous
        }
        ++c0;
        kept += 1;
      }
      hp.gstart[e] = s0;
      hp.gcount[e] = c0;
    }
  hp.nnz = kept;
  hp.Q = 0;
  for (int32_t c : hp.gcount) hp.Q = std::max(hp.Q, static_cast<int>(c));
  hp.Q = std::max(hp.Q, 1);
  hp.qp.assign(P, hp.Q);
  if (hp.device_fit) return;  // the device forms the weights from the windows
  hp.start.assign(static_cast<size_t>(J) * P, 0);
  hp.w.assign(static_cast<size_t>(J) * P * hp.Q, 0.0);
  parallel_for(chunks, threads, [&](int ch) {
    const int64_t j0 = J * ch / chunks, j1 = J * (ch + 1) / chunks;
    for (int64_t j = j0; j < j1; ++j)
      for (int p = 0; p < P; ++p) {
        const size_t e = static_cast<size_t>(p) * J + j;
        hp.start[static_cast<size_t>(j) * P + p] = hp.gstart[e];
        double* w = &hp.w[(static_cast<size_t>(j) * P + p) * hp.Q];
        for (int t = 0; t < hp.gcount[e]; ++t) w[t] = sinc_shift(hp.x[e], hp.gstart[e] + t);
      }
  });
}

void choose_sampling(HostPlan& hp, int mode) {
  const bool pow2 = hp.N >= 8 && hp.N <= 4096 && (hp.N & (hp.N - 1)) == 0;
  const double direct = 2.0 * hp.PN * (hp.K - 1);
  const double ifft = 8.0 * hp.P * hp.K * std::log2(2.0 * hp.K);
  if (mode == 2 && !pow2)
    throw Error{SRP_E_UNSUPPORTED, "iFFT sampling needs N a power of two, at most 4096"};
  // the direct kernel holds the table rows of every lag in LDS: at most
  // 128 lags per pair; past that only the iFFT form runs
  const bool direct_fits = 2 * hp.max_np + 1 <= 128;
  if (mode == 1 && !direct_fits)
    throw Error{SRP_E_UNSUPPORTED, "too many lags for the direct sampling kernel; use the iFFT form"};
  hp.fft = mode == 2 || (mode == 0 && pow2 && (ifft < direct || !direct_fits));
  if (mode == 0 && !direct_fits && !pow2)
    throw Error{SRP_E_UNSUPPORTED, "too many lags for the direct sampling kernel and N is not a power of two"};
}

void count_macs(HostPlan& hp) {
  const double J = static_cast<double>(hp.J);
  // sampling by (49): the direct product or the iFFT, whichever runs
  const double samp = hp.fft ? 8.0 * hp.P * hp.K * std::log2(2.0 * hp.K) : 2.0 * hp.PN * (hp.K - 1);
  if (hp.variant == SRP_FD) {
    hp.macs_per_map = 2.0 * J * hp.P * (hp.K - 1);
  } else if (hp.variant == SRP_LR) {
    hp.macs_per_map = 2.0 * J * hp.RH + 4.0 * hp.RH * hp.P * (hp.K - 1);  // (30)
  } else if (hp.variant == SRP_SLRI && hp.global_fit) {
    hp.macs_per_map = J * hp.R + static_cast<double>(hp.R) * hp.PN + samp;  // (61)
  } else if (hp.variant == SRP_SLRI) {
    double tall = 0, fat = 0;
    for (int p = 0; p < hp.P; ++p) {
      tall += J * hp.rp[p];
      if (hp.form != SRP_SI) fat += static_cast<double>(hp.rp[p]) * (2 * hp.np[p] + 1);  // SI: V = I
    }
    hp.macs_per_map = tall + fat + samp;
  } else if (hp.global_fit) {
    hp.macs_per_map = hp.nnz + samp;  // (62) with the kept entries Q_Lambda
  } else {
    double nnz = 0;
    for (int p = 0; p < hp.P; ++p) nnz += J * hp.qp[p];
    hp.macs_per_map = nnz + samp;
  }
}

std::vector<int32_t> compact_order(const HostPlan& hp, int tile, int sub) {
  const int64_t J = hp.J;
  if (J > std::numeric_limits<int32_t>::max()) fail("too many candidates for a compact order");
  if (tile < 1 || sub < 1 || tile % sub) fail("tile must be a multiple of sub");
  // TDOA sensitivity per axis: mean over sampled candidates and all pairs of
  // |d x_p / d r_a| = |u_m - u_m'|_a fs / c (u: unit vector from the mic to
  // the candidate; far field: the TDOA is linear in the direction, the
  // gradient |r_m - r_m'|_a fs / c)
  double sens[3] = {0.0, 0.0, 0.0};
  const int64_t step = std::max<int64_t>(1, J / 4096);
  int64_t ns = 0;
  for (int64_t j = 0; j < J; j += step, ++ns) {
    const double* r = &hp.grid[3 * j];
    for (int p = 0; p < hp.P; ++p) {
      const double* a = &hp.mics[3 * hp.pair_m[p]];
      const double* b = &hp.mics[3 * hp.pair_mp[p]];
      if (hp.far_field) {
        for (int k = 0; k < 3; ++k) sens[k] += std::fabs(a[k] - b[k]);
        continue;
      }
      double da = 0.0, db = 0.0;
      for (int k = 0; k < 3; ++k) {
        da += (r[k] - a[k]) * (r[k] - a[k]);
        db += (r[k] - b[k]) * (r[k] - b[k]);
      }
      da = std::sqrt(da);
      db = std::sqrt(db);
      for (int k = 0; k < 3; ++k) {
        const double ua = da > 0 ? (r[k] - a[k]) / da : 0.0, ub = db > 0 ? (r[k] - b[k]) / db : 0.0;
        sens[k] += std::fabs(ua - ub);
      }
    }
  }
  for (double& v : sens) v = v / static_cast<double>(std::max<int64_t>(ns, 1)) + 1e-12;
  std::vector<int32_t> order(static_cast<size_t>(J));
  for (int64_t j = 0; j < J; ++j) order[j] = static_cast<int32_t>(j);
  auto coord = [&](int32_t j, int k) { return hp.grid[3 * static_cast<size_t>(j) + k]; };
  // explicit stack of ranges [a, b) to split at multiples of `size`
  struct Range {
    int64_t a, b;
    int size;
  };
  std::vector<Range> stack{{0, J, tile}};
  while (!stack.empty()) {
    const Range rg = stack.back();
    stack.pop_back();
    const int64_t n = rg.b - rg.a;
    if (n <= rg.size) {
      if (rg.size == tile && sub < tile) {
        stack.push_back({rg.a, rg.b, sub});  // split the tile into subtiles
      } else if (rg.size == sub) {
        std::sort(order.begin() + rg.a, order.begin() + rg.b);
      }
      continue;
    }
    int axis = 0;
    double best = -1.0;
    for (int k = 0; k < 3; ++k) {
      double lo = std::numeric_limits<double>::infinity(), hi = -lo;
      for (int64_t i = rg.a; i < rg.b; ++i) {
        lo = std::min(lo, coord(order[i], k));
        hi = std::max(hi, coord(order[i], k));
      }
      const double e = (hi - lo) * sens[k];
      if (e > best) {
        best = e;
        axis = k;
      }
    }
    const int64_t half = (n + 2 * rg.size - 1) / (2 * rg.size) * rg.size;  // a multiple of size, >= n / 2
    const int64_t m = rg.a + std::min(half, n - 1);
    std::nth_element(order.begin() + rg.a, order.begin() + m, order.begin() + rg.b, [&](int32_t x, int32_t y) {
      const double cx = coord(x, axis), cy = coord(y, axis);
      return cx < cy || (cx == cy && x < y);
    });
    // the right part is split first only after the left (stack order keeps
    // the output order: left then right)
    stack.push_back({m, rg.b, rg.size});
    stack.push_back({rg.a, m, rg.size});
  }
  return order;
}

}  // namespace srp

