// Device-resident plan operands and the hot-path launch sequence.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/srp.h"
#include "plan.hpp"

namespace srp {

// One entry of a batched GEMM: element offsets of the three operands and the
// number of valid output rows of that batch.
struct GemmBatch {
  int64_t x_off, w_off, c_off;
  int nx;
  int pad;
};

struct DevicePlan {
  int device = -1;
  // common
  int Kp = 0;        // per-pair slot width of the cross-spectrum rows (elements)
  int64_t Jpad = 0;  // rows of the resident weight operands
  int32_t* d_pm = nullptr;   // pair tables
  int32_t* d_pmp = nullptr;
  int32_t* d_np = nullptr;
  int32_t* d_off = nullptr;
  // FD
  void* d_H = nullptr;       // [Jpad][P*Kp] steering (cos, -sin) in dtype
  bool fd_gen = false;       // steering generated on the fly from d_xg
  int fd_ksplit = 1;         // contraction splits of the resident FD GEMM (few candidate tiles)
  double* d_xg = nullptr;    // [P][J] TDOAs in samples (generated steering)
  // sampling (SLRI, SSPI)
  float* d_S = nullptr;       // direct sampling: iDFT table [gd_nct 32][2 gd_kb], rows 2 cos / -2 sin
  void* d_S16 = nullptr;      // its BF16 (hi, lo) halves, per 4 bins 16 B hi + 16 B lo (16-bit, FP8 plans)
  int gd_kb = 0;              // bins per table row: K - 1 rounded up to the kernel's chunk
  int gd_nct = 0;             // 32-lag column tiles of the table
  int gd_ft = 0;              // frames per block of the direct sampling kernel
  float2* d_tw = nullptr;      // iFFT sampling: exp(+2 pi i t / K), t < K/2
  float2* d_w2 = nullptr;      // iFFT sampling: exp(+i pi k / K), k < K
  int logk = 0;                // log2 K
  // SLRI
  int Kc = 0;                // columns of the tall GEMM (P*R padded)
  void* d_U = nullptr;       // [Jpad][Kc] in dtype
  float* d_V = nullptr;      // [P][2 max_np + 1][R]
  float* d_gscale = nullptr; // [P] activation scale of pair p in the fat stage
  float tall_alpha = 1.0f;   // undoes the activation scale in the tall GEMM
  std::vector<std::pair<const void*, int>> tall_slots;  // resident blocks of each streaming-kernel variant
  // LR-SRP: fat operand F [Fpad][P*Kp] FP32 (rows 2r, 2r+1 give Re, Im of
  // (H_fat psi)_r), tall operand in d_U (columns 2 Re T, -2 Im T)
  float* d_F = nullptr;
  int Fpad = 0;
  float lr_gscale = 1.0f;    // activation scale applied when g is narrowed
  // SSPI
  int32_t* d_start = nullptr;  // [P][J] absolute stacked lag index of tap 0
  void* d_w = nullptr;         // [P][J][Q] in dtype (f32, bf16, f16 or fp8)
  int2* d_win = nullptr;          // [J / 256 tiles][P] (first row, rows) lag window of a tile
  int sspi_cap = 0;               // LDS rows per staged chunk of the gather
  int sspi_q = 0;                 // taps per record read by the gather (>= the selection's Q)
  // dense-window SSPI on the matrix cores (16-bit weights): per 256-candidate
  // tile the pairs' lag windows, each rounded up to 8-lag chunks, form a contraction
  // of up to sspi_kmax columns: B [Jpad][kmax] in dtype, the chunk columns of
  // each tile in the frame-major samples (-1: zero), and the column map of
  // those samples [PNA] (stacked lag or -1 for the alignment padding).  Tiles
  // whose windows do not fit stay on the gather: the two tile lists.
  bool sspi_dense = false;
  int sspi_kmax = 0, sspi_pna = 0;
  int sspi_xw = 0;                 // width of one shifted copy of the frame-major samples (PNA + 16)
  void* d_B = nullptr;
  int32_t* d_ctab = nullptr;
  int32_t* d_colmap = nullptr;
  int32_t* d_dtiles = nullptr;     // tiles on the matrix cores
  int32_t* d_gtiles = nullptr;     // tiles left to the gather
  int n_dtiles = 0, n_gtiles = 0;
  // SSPI band product on the matrix cores (16-bit weights, Q <= 8, when the
  // dense windows do not fit), over tiles of a compact candidate order: per
  // tile and pair the band descriptor
  // [tiles][P] and the first pair of the next LDS pass [tiles][P]; the
  // records are then tile-major ([tiles][P][256] starts in d_start and
  // sspi_qw words of packed FP16 taps per record in d_w); xb is the
  // frame-major FP16 copy of the samples, sspi_xb columns wide
  bool sspi_band = false;
  void* d_bdesc = nullptr;
  uint16_t* d_bnext = nullptr;
  int32_t* d_border = nullptr;  // candidate at each position of the compact order [tiles 256]
  int sspi_qw = 0;
  int sspi_fr = 0;              // frames per block of the band product (64 or 128)
  int sspi_xb = 0;
  // per-kernel timing (see srp_profile_enable)
  struct Span {
    const char* name;
    hipEvent_t start, stop;
  };
  bool profiling = false;
  std::vector<Span> spans;
  std::vector<hipEvent_t> event_pool;
  // plan-owned workspace when the caller passes none
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t resident_bytes = 0;
};

// Allocates and fills the device operands of a plan.  Throws srp::Error.
void device_build(HostPlan& hp, DevicePlan& dp, int64_t frame_tile, size_t budget);
void device_free(DevicePlan& dp);

// per-map argmax (ties to the smallest index, NaN never wins)
void device_argmax(const void* maps, bool f64, int64_t L, int64_t J, int64_t ld, int64_t* idx, double* val,
                   hipStream_t st);

size_t workspace_bytes(const HostPlan& hp, const DevicePlan& dp, int64_t L, int64_t frame_tile);

// Enqueues the map computation for L frames on `stream`.
void device_compute(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L,
                    void* maps, int64_t ld_maps, void* ws, size_t ws_bytes, int64_t frame_tile,
                    hipStream_t stream);

// Bytes of the per-device static scratch workspace of srp_compute_static.
constexpr size_t STATIC_SCRATCH_BYTES = SRP_STATIC_SCRATCH_BYTES;

// device_compute with the static scratch as its workspace and the largest
// frame tile (at most frame_tile) whose workspace fits it; throws
// SRP_E_UNSUPPORTED when even the smallest tile does not fit.
void device_compute_static(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L,
                           void* maps, int64_t ld_maps, int64_t frame_tile, hipStream_t stream);

// Waits for the recorded spans and accumulates them per kernel name.
void device_profile_collect(DevicePlan& dp, std::vector<std::pair<std::string, std::pair<double, int64_t>>>& out);

void device_crossspec(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L,
                      void* psi, hipStream_t stream);

void device_gcc_samples(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L,
                        float* xi, void* ws, size_t ws_bytes, int64_t frame_tile,
                        hipStream_t stream);

}  // namespace srp
