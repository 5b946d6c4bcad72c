// Host-side FP64 plan construction for the SRP-map library.
//
// Everything here depends only on the array geometry, the candidate grid and
// the frequency resolution, so it is computed once, upfront (Sec. IV-B), in
// FP64: pair enumeration, TDOAs, lag ranges, the per-pair low-rank factors of
// the sinc interpolation matrices and the sparse interpolation windows.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace srp {

struct HostPlan {
  // geometry and sizes
  int M = 0, P = 0, K = 0, N = 0;
  int64_t J = 0;
  double fs = 0, c = 0;
  int n_aux = 0;
  int variant = 0;  // machinery: SRP_FD, SRP_SLRI (also SI) or SRP_SSPI (also TD)
  int form = 0;     // the srp_variant requested (SI and TD run on the SLRI / SSPI machinery)
  int dtype = 0;    // srp_dtype
  int requested = 0;

  std::vector<double> mics;  // [M][3]
  std::vector<double> grid;  // [J][3]
  std::vector<int32_t> pair_m, pair_mp;  // [P]
  std::vector<int32_t> np;               // N_p
  std::vector<int32_t> off;              // stacked lag offset of pair p
  int PN = 0;
  int max_np = 0;
  double mean_n = 0;

  std::vector<double> x;  // [P][J] TDOA in samples

  // SLRI (per-pair truncated SVD of Lambda_p)
  int R = 0;                 // columns per pair in U (max_p R_p)
  std::vector<int32_t> rp;   // R_p
  std::vector<double> U;     // [P][J][R], zero for r >= R_p
  std::vector<double> V;     // [P][2 max_np + 1][R], rows n + N_p, zero-padded
  std::vector<double> sv;    // [P][2 max_np + 1] singular values, descending

  // SSPI (Q largest-magnitude taps per (location, pair))
  int Q = 0;                    // taps stored per (j, p) (max_p Q_p)
  std::vector<int32_t> qp;      // Q_p
  std::vector<int32_t> start;   // [J][P] first lag s (in -N_p..N_p)
  std::vector<double> w;        // [J][P][Q], zero for q >= Q_p
  // global SSPI (55): every entry of the stacked Lambda with |Lambda| >= tau,
  // tau the Q_Lambda-th largest magnitude; per (j, p) a window of gcount
  // nearest lags from gstart (pair-major [P][J])
  double tau = 0;
  double nnz = 0;                 // entries kept
  std::vector<int32_t> gstart, gcount;

  // LR-SRP (eqs. (26)-(29)): rank R_H of the truncated SVD of H
  int RH = 0;
  std::vector<double> lr_s;  // the R_H largest singular values of H

  bool fft = false;  // GCC sampling by the iFFT of (46) instead of the direct product of (40)
  bool device_fit = false;  // SLRI Gram matrices and U, SSPI windows are computed on the device
  int fd_steering = 0;      // FD steering operand: 0 auto, 1 resident, 2 generated
  bool far_field = false;   // grid rows are unit directions (far-field TDOAs)
  bool global_fit = false;  // SLRI: one rank-R fit of the stacked Lambda (54); SSPI: global top-Q_Lambda (55)
  bool global_rand = false;  // SLRI global fit by randomized subspace iteration (device plans)

  double macs_per_map = 0;
};

// Validates the arguments and fills geometry, pairs, TDOAs and lag ranges.
// Throws srp::Error on invalid input.
void build_geometry(HostPlan& hp, const double* mics, int M, const double* grid,
                    int64_t J, double fs, int N, double c, int n_aux, bool far_field = false);

// Chooses the GCC sampling form: mode 1 = direct product (40), 2 = iFFT
// (46), 0 = the cheaper of the two operation counts of (49), 2 PN (K-1)
// against 8 P K log2(2K); the iFFT needs N a power of two up to 4096.
void choose_sampling(HostPlan& hp, int mode);

// Per-pair rank-R truncated SVD of Lambda_p (Sec. IV-A, eq. (54) per pair).
// With device_fit only the ranks and the V / sv storage are set up; the
// device builds the Gram matrices and U.
void build_slri(HostPlan& hp, int R, int threads);

// Global low-rank interpolation (Sec. IV-A, eq. (54) over the stacked
// Lambda of (43)): the rank-R truncated SVD of the J x PN matrix, through
// its PN x PN Gram matrix.  V [PN][R], sv [PN], U [J][R] (host plans).
// With device_fit only the sizes are set up.
void build_slri_global(HostPlan& hp, int R, int threads);

// V and the singular values of the global fit from G = Lambda^T Lambda
// (PN x PN row-major, destroyed).
void slri_fit_global(HostPlan& hp, std::vector<double>& G);

// V_p and the singular values of pair p from its Gram matrix
// G = Lambda_p^T Lambda_p (n x n row-major, destroyed).
void slri_fit_pair(HostPlan& hp, int p, std::vector<double>& G);

void parallel_for(int n, int threads, const std::function<void(int)>& body);

// Per-(location, pair) Q-tap windows (Sec. IV-A, eq. (55) per row and pair).
void build_sspi(HostPlan& hp, int Q, int threads);

// Global sparse interpolation (Sec. IV-A, eq. (55) over the stacked
// Lambda): keep the Q_Lambda = qbar J P largest-magnitude entries.
void build_sspi_global(HostPlan& hp, int qbar, int threads);

// Run-time MAC counts per map (eqs. (24), (61), (62); sampling by the
// direct product, 2 PN (K-1)).
void count_macs(HostPlan& hp);

// Candidate order for tiled products: consecutive runs of `tile` candidates
// (all but the last full) that are compact where the TDOAs change most,
// each split the same way into runs of `sub` (tile a multiple of sub).
// Balanced k-d splits on the grid coordinates: a range goes at a multiple
// of `tile` (then `sub`) candidates along the axis whose extent times the
// mean |dx_p / d axis| over the pairs is largest; a subtile's candidates are
// in increasing index.  Returns the candidate of each position.
std::vector<int32_t> compact_order(const HostPlan& hp, int tile, int sub);

// sinc(x - n) for integer n, accurate for large |x| (argument reduced
// exactly in FP64).
double sinc_shift(double x, int n);

// Symmetric eigendecomposition by cyclic Jacobi rotations.  a: n x n
// row-major (destroyed), evals: n (descending), evecs: n x n row-major with
// eigenvector i in column i.
void sym_eig(std::vector<double>& a, int n, std::vector<double>& evals,
             std::vector<double>& evecs);

// The same by Householder tridiagonalisation and implicit QL (large n).
void sym_eig_tridiag(std::vector<double>& a, int n, std::vector<double>& evals,
                     std::vector<double>& evecs);

struct Error {
  int code;
  std::string msg;
};

}  // namespace srp
