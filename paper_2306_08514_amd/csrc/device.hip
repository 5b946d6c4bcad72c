// HIP kernels for gfx950 (MI355X) and the hot-path launch sequence.
//
// Hot path per frame tile (one map per STFT frame):
//   phat_kernel      PHAT-weighted cross-spectra psi_p[l, k] (FD)      eq. (2)
//   gemm_fd16        z = 2 Re[H psi] as a real MFMA GEMM (resident H)  eq. (22)
//   fd_gen16, fd_gen the same with H generated in LDS from the TDOAs    eqs. (19), (22)
//   gcc_direct       PHAT + xi_p = 2 Re[S_p psi_p]                      eqs. (2), (40)
//   gcc_fft          PHAT + xi_p by the iFFT                            eq. (46)
//   slri_fat_mfma    g_p = V_p^T xi_p (global fit: slri_fat_global_mfma) eq. (57)
//   tall_ws          z = sum_p U_p g_p                                  eq. (57)
//   sspi_gather      z = sum_p sum_q w[j,p,q] xi_p[s(j,p) + q]          eq. (58)
//                    (dense-window tiles: tall_ws; large apertures: sspi_band)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <thread>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "../../include/srp.h"
#include "device.hpp"

namespace srp {

// ------------------------------------------------------------------ types --

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// OCP FP8 E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits, max
// 448, no infinities, S.1111.111 is NaN).
struct fp8 {
  uint8_t bits;
};

__host__ __device__ inline uint8_t e4m3_encode(float x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  const float a = std::fabs(x);
  if (!(a == a)) return static_cast<uint8_t>(0x7F | sign);
  if (a >= 448.0f) return static_cast<uint8_t>(0x7E | sign);  // saturate
  if (a < 0.015625f) {
    // subnormal grid m * 2^-9; rounding to 8 lands on the smallest normal
    return static_cast<uint8_t>(static_cast<int>(std::rint(a * 512.0f)) | sign);
  }
  int e;
  const float f = std::frexp(a, &e);  // a = f 2^e, f in [1/2, 1)
  int q = static_cast<int>(std::rint((2.0f * f - 1.0f) * 8.0f));  // ties to even
  int E = e - 1 + 7;
  if (q == 8) {
    q = 0;
    E += 1;
  }
  int code = (E << 3) | q;
  if (code > 0x7E) code = 0x7E;
  return static_cast<uint8_t>(code | sign);
}

__host__ __device__ inline float e4m3_decode(uint8_t c) {
  const int E = (c >> 3) & 15, m = c & 7;
  if ((c & 0x7F) == 0x7F) return NAN;
  const float v = E ? std::ldexp(1.0f + m / 8.0f, E - 7) : std::ldexp(static_cast<float>(m), -9);
  return (c & 0x80) ? -v : v;
}

template <typename T>
__device__ inline T cvt(float v);
template <>
__device__ inline float cvt<float>(float v) { return v; }
template <>
__device__ inline __bf16 cvt<__bf16>(float v) { return static_cast<__bf16>(v); }
template <>
__device__ inline _Float16 cvt<_Float16>(float v) { return static_cast<_Float16>(v); }
template <>
__device__ inline fp8 cvt<fp8>(float v) { return fp8{e4m3_encode(v)}; }

template <typename T>
__device__ inline T cvt64(double v) { return cvt<T>(static_cast<float>(v)); }
template <>
__device__ inline double cvt64<double>(double v) { return v; }

// ------------------------------------------------------------ error check --

#define HIP_OK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw Error{e_ == hipErrorOutOfMemory ? SRP_E_NOMEM : SRP_E_HIP,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_)};                    \
  } while (0)

// Power-of-two scale of the stored SSPI weights: 2^8 for FP8 E4M3, whose
// normal range starts at 2^-6 (|w| <= 1 becomes |w| <= 256 < 448, and taps
// down to 2^-14 stay normal); 1 for the other types.  The gather multiplies
// its sums by the inverse, exactly.
template <typename TW>
__host__ __device__ constexpr float sspi_wscale() {
  return std::is_same<TW, fp8>::value ? 256.0f : 1.0f;
}

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{SRP_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

static inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
static inline size_t align256(size_t a) { return (a + 255) & ~static_cast<size_t>(255); }

static hipEvent_t take_event(DevicePlan& dp) {
  if (!dp.event_pool.empty()) {
    hipEvent_t e = dp.event_pool.back();
    dp.event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  HIP_OK(hipEventCreate(&e));
  return e;
}

// Launches `launch` and, while profiling is enabled, brackets it with a pair
// of events recorded on the same stream.
#define TRACED(dp, kname, st, launch)                     \
  do {                                                    \
    hipEvent_t a_ = nullptr;                              \
    if ((dp).profiling) {                                 \
      a_ = take_event(dp);                                \
      HIP_OK(hipEventRecord(a_, st));                     \
    }                                                     \
    launch;                                               \
    if (a_) {                                             \
      hipEvent_t b_ = take_event(dp);                     \
      HIP_OK(hipEventRecord(b_, st));                     \
      (dp).spans.push_back(DevicePlan::Span{kname, a_, b_}); \
    }                                                     \
  } while (0)

// s_waitcnt with vmcnt = N and no wait on the other counters (gfx9
// encoding: vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8])
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// s_waitcnt with vmcnt = N, lgkmcnt = 0 (this wave's LDS reads are done)
template <int N>
__device__ inline void wait_vm_lds() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Tiles of the FD GEMM (FP32, 16-bit, FP8): 256 x 256 outputs, K in 64-byte
// stages (see gemm_fd16).
constexpr int FD16_TILE = 256, FD16_SB = 64, FD16_NBUF = 5;
constexpr int FD16_STAGE = 2 * FD16_TILE * FD16_SB;  // 32 KB
constexpr int FD16_NI = FD16_STAGE / 1024 / 4;       // loads per wave per stage

// Bank swizzle of a stage row: its four 16-byte chunks, chunk c of row r at
// position c ^ fd16_swz(r mod 16).
__host__ __device__ inline int fd16_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// Byte offset of byte kb of row j in the tile-major operands of the FD GEMM
// (FP32, 16-bit, FP8): [j / 256][kb / 64][j mod 256][64 bytes], each
// 64-byte row piece swizzled by fd16_swz, so that one stage of a 256-row
// tile is 16 KB in the order the GEMM's LDS stage holds it.  rb = bytes per
// row (a multiple of 64).
__host__ __device__ inline int64_t fd16_tiled(int64_t j, int64_t kb, int64_t rb) {
  const int64_t r = j % FD16_TILE;
  return ((j / FD16_TILE * (rb / FD16_SB) + kb / FD16_SB) * FD16_TILE + r) * FD16_SB +
         16 * (((kb % FD16_SB) / 16) ^ fd16_swz(static_cast<int>(r & 15))) + kb % 16;
}

// ============================================================ PHAT kernel ==
//
// One wave per block; a thread owns one single-sided bin k = 1 + slot of one
// frame.  u_m = y_m / |y_m| is formed once per microphone and staged in LDS,
// then psi_p = u_m conj(u_m') for every pair, which equals
// y_m y_m'^* / |y_m y_m'^*| of eq. (2), and 0 where either bin is 0.
// Output layout: out[l * ld_l + p * ld_p + 2 * slot + {re, im}], or that
// row-major operand tile-major (fd16_tiled) for the FD GEMM (FP32, 16-bit,
// FP8) and the 16-bit generated-steering kernel;
// slots in [K-1, kslots) are written as zeros (row padding).

template <typename TO, typename TC>
__global__ __launch_bounds__(64) void phat_kernel(const float2* __restrict__ Y, int M, int K,
                                                  int P, const int32_t* __restrict__ pm,
                                                  const int32_t* __restrict__ pmp,
                                                  TO* __restrict__ out, int64_t ld_l,
                                                  int64_t ld_p, int kslots, bool tiled) {
  extern __shared__ __attribute__((aligned(16))) unsigned char phat_lds[];
  TC* ur = reinterpret_cast<TC*>(phat_lds);  // [M][64] real
  TC* ui = ur + M * 64;                      // [M][64] imag
  const int tid = threadIdx.x;
  const int slot = blockIdx.x * 64 + tid;
  const int64_t l = blockIdx.y;
  const bool live = slot < K - 1;
  if (live) {
    const float2* yl = Y + l * M * (K + 1) + (slot + 1);
    for (int m = 0; m < M; ++m) {
      const float2 y = yl[static_cast<int64_t>(m) * (K + 1)];
      TC a = y.x, b = y.y;
      const TC s = std::max(std::fabs(a), std::fabs(b));
      if (s > 0) {
        a /= s;
        b /= s;
        const TC r = TC(1) / std::sqrt(std::fma(a, a, b * b));
        a *= r;
        b *= r;
      } else {
        a = 0;
        b = 0;
      }
      ur[m * 64 + tid] = a;
      ui[m * 64 + tid] = b;
    }
  }
  // same wave wrote and reads its own column: no barrier needed across waves
  if (slot >= kslots) return;
  const int64_t rb = ld_l * static_cast<int64_t>(sizeof(TO));
  for (int p = 0; p < P; ++p) {
    // (re, im) share a 16-byte chunk of the tile-major layout
    const int64_t e0 = p * ld_p + 2 * static_cast<int64_t>(slot);
    TO* o = tiled ? reinterpret_cast<TO*>(reinterpret_cast<unsigned char*>(out) +
                                          fd16_tiled(l, e0 * static_cast<int64_t>(sizeof(TO)), rb))
                  : out + l * ld_l + e0;
    TC re = 0, im = 0;
    if (live) {
      const int m = pm[p], mq = pmp[p];
      const TC ar = ur[m * 64 + tid], ai = ui[m * 64 + tid];
      const TC br = ur[mq * 64 + tid], bi = ui[mq * 64 + tid];
      re = std::fma(ar, br, ai * bi);  // u_m conj(u_m')
      im = std::fma(ai, br, -(ar * bi));
    }
    o[0] = cvt64<TO>(re);
    o[1] = cvt64<TO>(im);
  }
}

// ============================================================ MFMA GEMM ====
//
// C[r][c] = alpha * sum_k X[r][k] W[c][k] with both operands row-major and
// K-contiguous.  A block of 256 threads (4 waves) computes a BX x BW tile of
// C; waves are arranged WGX (along r) x 4/WGX (along c); each wave covers
// 32 x 32 MFMA blocks.  The MFMA A-operand is X (rows of C), the B-operand
// is W (columns of C), so consecutive lanes hold consecutive columns of C
// and the stores are coalesced along c.  K is staged through LDS in BKB-byte
// slices with a one-slice register prefetch.
//
// Per-lane operand layout: for a 32 x 32 block, lane i supplies row i % 32
// and the K-half (i / 32) of each MFMA step; X and W use the same lane -> k
// assignment, so each MFMA step accumulates every k of its slice exactly
// once whatever the instruction's internal k order.

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {  // v_mfma_f32_32x32x2_f32, 4 per 32-byte step
  static constexpr int STEP = 32;
  __device__ static inline void run(const i32x4* a, const i32x4* b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[0].x), __int_as_float(b[0].x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[0].y), __int_as_float(b[0].y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[0].z), __int_as_float(b[0].z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[0].w), __int_as_float(b[0].w), c, 0, 0, 0);
  }
};

template <>
struct Mfma<__bf16> {  // v_mfma_f32_32x32x16_bf16
  static constexpr int STEP = 32;
  __device__ static inline void run(const i32x4* a, const i32x4* b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                __builtin_bit_cast(bf16x8, b[0]), c, 0, 0, 0);
  }
};

template <>
struct Mfma<_Float16> {  // v_mfma_f32_32x32x16_f16
  static constexpr int STEP = 32;
  __device__ static inline void run(const i32x4* a, const i32x4* b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[0]),
                                               __builtin_bit_cast(f16x8, b[0]), c, 0, 0, 0);
  }
};

template <>
struct Mfma<fp8> {  // v_mfma_f32_32x32x64_f8f6f4, both operands E4M3, unit scales
  static constexpr int STEP = 64;
  __device__ static inline void run(const i32x4* a, const i32x4* b, f32x16& c) {
    const i32x8 av = __builtin_shufflevector(a[0], a[1], 0, 1, 2, 3, 4, 5, 6, 7);
    const i32x8 bv = __builtin_shufflevector(b[0], b[1], 0, 1, 2, 3, 4, 5, 6, 7);
    // format 0 = E4M3 for A and B; E8M0 scale 127 = 2^0
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
  }
};

// Maps a linear block id to (W tile, X tile) so that the blocks one XCD
// receives (workgroups are dispatched round-robin over the 8 XCDs: ids x,
// x + 8, ...) walk a contiguous range of W tiles with the X tiles innermost;
// a W tile is then fetched from HBM once into that XCD's L2 and reused by
// every X tile.  The grid holds a multiple of 8 blocks.
__device__ inline bool xcd_tile(int nw_tiles, int nx_tiles, int& wt, int& xt) {
  const int b = blockIdx.x;
  const int per = static_cast<int>(gridDim.x) / 8;
  const int gidx = (b % 8) * per + b / 8;
  if (gidx >= nw_tiles * nx_tiles) return false;
  wt = gidx / nx_tiles;
  xt = gidx % nx_tiles;
  return true;
}

template <typename T, int BX, int BW, int WGX, int BKB, bool NT>
__global__ __launch_bounds__(256) void gemm_nt(const GemmBatch* __restrict__ batches,
                                               const T* __restrict__ X, int64_t ldx,
                                               const T* __restrict__ W, int64_t ldw,
                                               float* __restrict__ C, int64_t ldc, int nw,
                                               int kdim, float alpha, int nx_single,
                                               int nw_tiles, int nx_tiles, int64_t cz_rows) {
  constexpr int STEP = Mfma<T>::STEP;
  constexpr int LB = STEP / 2;   // bytes per lane per step
  constexpr int NV = LB / 16;    // 16-byte vectors per lane per step
  constexpr int ROWB = BKB + 16; // padded LDS row
  constexpr int WGW = 4 / WGX;
  constexpr int WX = BX / WGX, WW = BW / WGW;
  constexpr int NBX = WX / 32, NBW = WW / 32;
  static_assert(NBX >= 1 && NBW >= 1, "tile too small");
  static_assert(BKB % STEP == 0, "slice must hold whole steps");
  constexpr int CPR = BKB / 16;  // 16-byte chunks per row per slice
  constexpr int NCH = (BX + BW) * CPR;
  constexpr int PER = (NCH + 255) / 256;
  __shared__ __attribute__((aligned(16))) unsigned char lds[(BX + BW) * ROWB];

  // batched (one entry per blockIdx.z) or a single product with nx rows
  // whose contraction is split over blockIdx.z: split z covers elements
  // [z kdim, (z + 1) kdim) and writes rows [z cz_rows, ...) of C
  const int64_t kz = static_cast<int64_t>(blockIdx.z) * kdim;
  const GemmBatch bt = batches ? batches[blockIdx.z]
                               : GemmBatch{kz, kz, static_cast<int64_t>(blockIdx.z) * cz_rows, nx_single, 0};
  const int nx = bt.nx;
  int wt, xt;
  if (!xcd_tile(nw_tiles, nx_tiles, wt, xt)) return;  // uniform over the block
  const int x0 = xt * BX;
  const int w0 = wt * BW;
  if (x0 >= nx) return;
  const unsigned char* Xb = reinterpret_cast<const unsigned char*>(X + bt.x_off);
  const unsigned char* Wb = reinterpret_cast<const unsigned char*>(W + bt.w_off);
  C += bt.c_off * ldc;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wx = (wave / WGW) * WX, ww = (wave % WGW) * WW;
  const int r32 = lane & 31, g = lane >> 5;

  const int64_t xrow = ldx * static_cast<int64_t>(sizeof(T));
  const int64_t wrow = ldw * static_cast<int64_t>(sizeof(T));
  i32x4 pre[PER];
  auto gload = [&](int kb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * 256;
      if (NCH % 256 == 0 || c < NCH) {
        const int row = c / CPR, col = c % CPR;
        const unsigned char* src =
            row < BX ? Xb + (x0 + row) * xrow + kb + col * 16
                     : Wb + static_cast<int64_t>(w0 + row - BX) * wrow + kb + col * 16;
        pre[i] = *reinterpret_cast<const i32x4*>(src);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * 256;
      if (NCH % 256 == 0 || c < NCH) {
        const int row = c / CPR, col = c % CPR;
        *reinterpret_cast<i32x4*>(lds + row * ROWB + col * 16) = pre[i];
      }
    }
  };

  f32x16 acc[NBX][NBW];
#pragma unroll
  for (int a = 0; a < NBX; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;

  const int kbytes = kdim * static_cast<int>(sizeof(T));
  gload(0);
  for (int kb = 0; kb < kbytes; kb += BKB) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (kb + BKB < kbytes) gload(kb + BKB);
#pragma unroll
    for (int s = 0; s < BKB; s += STEP) {
      i32x4 fa[NBX][NV], fb[NBW][NV];
#pragma unroll
      for (int a = 0; a < NBX; ++a) {
        const unsigned char* p = lds + (wx + a * 32 + r32) * ROWB + s + g * LB;
#pragma unroll
        for (int v = 0; v < NV; ++v) fa[a][v] = *reinterpret_cast<const i32x4*>(p + 16 * v);
      }
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        const unsigned char* p = lds + (BX + ww + b * 32 + r32) * ROWB + s + g * LB;
#pragma unroll
        for (int v = 0; v < NV; ++v) fb[b][v] = *reinterpret_cast<const i32x4*>(p + 16 * v);
      }
#pragma unroll
      for (int a = 0; a < NBX; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) Mfma<T>::run(fa[a], fb[b], acc[a][b]);
    }
  }

  // 32 x 32 accumulator layout: register v of lane i holds row
  // 8 (v / 4) + 4 (i / 32) + v % 4 and column i % 32
#pragma unroll
  for (int a = 0; a < NBX; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      const int col = w0 + ww + b * 32 + r32;
      if (col >= nw) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = x0 + wx + a * 32 + 8 * (v / 4) + 4 * g + (v % 4);
        if (row < nx) {
          float* dst = C + static_cast<int64_t>(row) * ldc + col;
          if (NT)
            __builtin_nontemporal_store(alpha * acc[a][b][v], dst);
          else
            *dst = alpha * acc[a][b][v];
        }
      }
    }
}

// The generated-steering seeds of one (pair, candidate): bin 1, (cos,
// sin)(pi x / K), and the 16-bin advance (cos, sin)(16 pi x / K), each phase
// reduced in FP64 (t - rint t) before sincospi.  Not inlined, so that both
// generating kernels run the same instructions (inlined, the FP64 sincospi
// was contracted differently and a few seeds differed in the last bit).
struct FdSeed {
  double s1, c1, s16, c16;
};
__device__ __noinline__ FdSeed fd_gen_seed(double x, int K) {
  FdSeed r;
  const double t = x / (2.0 * K);
  sincospi(2.0 * (t - rint(t)), &r.s1, &r.c1);
  const double v = 16.0 * x / (2.0 * K);
  sincospi(2.0 * (v - rint(v)), &r.s16, &r.c16);
  return r;
}

// conv. FD-SRP with the steering operand generated on the fly (plans whose
// H would not fit in HBM): z = alpha (psi H^T) as in gemm_nt, but each
// 128-byte K slice of the BW = 256 rows of H is computed into LDS instead of
// read: slots 2 (k - 1), 2 (k - 1) + 1 of pair p hold cos theta, -sin theta,
// theta = pi k x_p(j) / K (eq. (19) with (14)).  A thread fills the BINS
// consecutive bins of its row in the slice, in groups of 16: at the first
// slice of a pair the angle of bin 1 is reduced in FP64 (t = x / 2K,
// theta = 2 pi (t - rint t)) and evaluated by sincospi; each further group
// starts from that FP64 value advanced by one rotation of 16 bins per group
// (at most K / 16 rotations, error ~1e-15), and within a group the bins
// follow by FP32 rotation by exp(+i pi x / K), a chain of 15 steps.  This
// is the sequence fd_gen16 generates, so that a frame's map is the same
// whichever of the two kernels its batch size selects.
//
// With blockIdx.y the contraction is split at pair boundaries (plans with
// few candidate tiles), each split writing its partial product.
//
// FLUSH (FP32 operands): each pair's products are summed in accumulators of
// their own and added to the running total at the next pair.  One FP32
// accumulator over the whole contraction (2 P (K - 1) terms, 1.0e6 on the
// 2 m disc) drifts by about eps sqrt(n / 2) relative (4.6e-5 measured); per
// pair the drift is that of 2 (K - 1) terms plus a P-term outer sum.
template <typename T, int BX, int WGX, bool FLUSH = false>
__global__ __launch_bounds__(256) void fd_gen(const T* __restrict__ X, int64_t ldx,
                                              const double* __restrict__ xg, int64_t J, int K, int Kp,
                                              float* __restrict__ C, int64_t ldc, int nx, int kdim, float alpha,
                                              int nw_tiles, int nx_tiles, int pps, int64_t cz_rows) {
  constexpr int BW = 256, BKB = 128;  // 256 candidates: one generated row per thread (189 -> 168 ms on the 2 m disc)
  constexpr int STEP = Mfma<T>::STEP;
  constexpr int LB = STEP / 2;
  constexpr int NV = LB / 16;
  constexpr int ROWB = BKB + 16;
  constexpr int WGW = 4 / WGX;
  constexpr int WX = BX / WGX, WW = BW / WGW;
  constexpr int NBX = WX / 32, NBW = WW / 32;
  static_assert(NBX >= 1 && NBW >= 1, "tile too small");
  constexpr int CPR = BKB / 16;                         // 16-byte chunks per row per slice
  constexpr int XCH = BX * CPR;                         // X chunks per slice
  constexpr int PER = (XCH + 255) / 256;
  constexpr int EPS = BKB / static_cast<int>(sizeof(T));  // elements per row per slice
  constexpr int BPS = EPS / 2;                          // bins per row per slice
  constexpr int TPR = 256 / BW;                         // threads per row (2)
  constexpr int BINS = BPS / TPR;                       // bins per thread
  __shared__ __attribute__((aligned(16))) unsigned char lds[(BX + BW) * ROWB];

  int wt, xt;
  if (!xcd_tile(nw_tiles, nx_tiles, wt, xt)) return;
  const int x0 = xt * BX;
  const int w0 = wt * BW;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wx = (wave / WGW) * WX, ww = (wave % WGW) * WW;
  const int r32 = lane & 31, g = lane >> 5;
  const unsigned char* Xb = reinterpret_cast<const unsigned char*>(X);
  const int64_t xrow = ldx * static_cast<int64_t>(sizeof(T));

  // generator: row gr of the tile, bins gb0 .. gb0 + BINS - 1 of the slice
  const int gr = tid / TPR, gpart = tid % TPR;
  const int64_t gj = w0 + gr;
  const bool glive = gj < J;

  i32x4 pre[PER];
  auto gload = [&](int kb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * 256;
      if (XCH % 256 == 0 || c < XCH) {
        const int row = c / CPR, col = c % CPR;
        pre[i] = i32x4{0, 0, 0, 0};
        if (x0 + row < nx) pre[i] = *reinterpret_cast<const i32x4*>(Xb + (x0 + row) * xrow + kb + col * 16);
      }
    }
  };

  f32x16 acc[NBX][NBW], tot[FLUSH ? NBX : 1][FLUSH ? NBW : 1];
#pragma unroll
  for (int a = 0; a < NBX; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  if constexpr (FLUSH) {
#pragma unroll
    for (int a = 0; a < NBX; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) tot[a][b][v] = 0.0f;
  }

  // split blockIdx.y of the contraction: pairs [y pps, (y + 1) pps), its
  // partial product to rows [y cz_rows, ...) of C
  const int kb0 = static_cast<int>(blockIdx.y) * pps * Kp * static_cast<int>(sizeof(T));
  const int kbytes = min(kdim, (static_cast<int>(blockIdx.y) + 1) * pps * Kp) * static_cast<int>(sizeof(T));
  C += static_cast<int64_t>(blockIdx.y) * cz_rows * ldc;
  double gx = 0.0, gs_c = 1.0, gs_s = 0.0, gadv_c = 1.0, gadv_s = 0.0;  // generator state
  float gstep_c = 1.0f, gstep_s = 0.0f;
  gload(kb0);
  for (int kb = kb0; kb < kbytes; kb += BKB) {
    if constexpr (FLUSH) {
      if (kb > kb0 && (kb / static_cast<int>(sizeof(T))) % Kp == 0) {  // a new pair: uniform over the block
#pragma unroll
        for (int a = 0; a < NBX; ++a)
#pragma unroll
          for (int b = 0; b < NBW; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              tot[a][b][v] += acc[a][b][v];
              acc[a][b][v] = 0.0f;
            }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * 256;
      if (XCH % 256 == 0 || c < XCH) {
        const int row = c / CPR, col = c % CPR;
        *reinterpret_cast<i32x4*>(lds + row * ROWB + col * 16) = pre[i];
      }
    }
    // generate this slice's BW rows of H: the thread's first angle of the
    // slice comes from an FP64 seed, exact at the first slice of each pair
    // and advanced by one FP64 rotation per further slice; its BINS bins by
    // FP32 rotation; 64 bytes per thread go to LDS as four 16-byte stores
    {
      const int e0 = kb / static_cast<int>(sizeof(T));  // first element of the slice in the row
      const int p = e0 / Kp;
      const int kfirst = (e0 % Kp) / 2 + 1 + gpart * BINS;  // first bin of this thread
      static_assert(BINS % 16 == 0 && TPR == 1, "16-bin seed groups, one row per thread");
      if (glive && e0 % Kp == 0) {
        // the pair's first slice (kfirst = 1): seed bin 1, the one-bin FP32
        // step and the 16-bin FP64 advance, as fd_gen16 takes them
        gx = xg[static_cast<int64_t>(p) * J + gj];
        const FdSeed sd = fd_gen_seed(gx, K);
        gs_s = sd.s1;
        gs_c = sd.c1;
        gadv_s = sd.s16;
        gadv_c = sd.c16;
        gstep_c = static_cast<float>(gs_c);
        gstep_s = static_cast<float>(gs_s);
      }
      T vals[2 * BINS];
#pragma unroll
      for (int q = 0; q < BINS / 16; ++q) {
        // each 16 bins start from the FP64 seed, which then advances by 16
        // bins (explicit fma, so that fd_gen16 reproduces every value)
        float c = static_cast<float>(gs_c), sn = static_cast<float>(gs_s);
        const double cn = __builtin_fma(gs_c, gadv_c, -(gs_s * gadv_s));
        gs_s = __builtin_fma(gs_c, gadv_s, gs_s * gadv_c);
        gs_c = cn;
#pragma unroll
        for (int b = 16 * q; b < 16 * q + 16; ++b) {
          const bool ok = glive && kfirst + b <= K - 1;
          vals[2 * b] = cvt<T>(ok ? c : 0.0f);
          vals[2 * b + 1] = cvt<T>(ok ? -sn : 0.0f);
          // (c + i s) <- (c + i s)(step_c + i step_s)
          const float cf = __builtin_fmaf(c, gstep_c, -(sn * gstep_s));
          sn = __builtin_fmaf(c, gstep_s, sn * gstep_c);
          c = cf;
        }
      }
      unsigned char* dst = lds + (BX + gr) * ROWB + gpart * (BKB / TPR);
#pragma unroll
      for (int i = 0; i < BKB / TPR / 16; ++i) {
        i32x4 w4;
        __builtin_memcpy(&w4, reinterpret_cast<const unsigned char*>(vals) + 16 * i, 16);
        *reinterpret_cast<i32x4*>(dst + 16 * i) = w4;
      }
    }
    __syncthreads();
    if (kb + BKB < kbytes) gload(kb + BKB);
#pragma unroll
    for (int s = 0; s < BKB; s += STEP) {
      i32x4 fa[NBX][NV], fb[NBW][NV];
#pragma unroll
      for (int a = 0; a < NBX; ++a) {
        const unsigned char* q = lds + (wx + a * 32 + r32) * ROWB + s + g * LB;
#pragma unroll
        for (int v = 0; v < NV; ++v) fa[a][v] = *reinterpret_cast<const i32x4*>(q + 16 * v);
      }
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        const unsigned char* q = lds + (BX + ww + b * 32 + r32) * ROWB + s + g * LB;
#pragma unroll
        for (int v = 0; v < NV; ++v) fb[b][v] = *reinterpret_cast<const i32x4*>(q + 16 * v);
      }
#pragma unroll
      for (int a = 0; a < NBX; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) Mfma<T>::run(fa[a], fb[b], acc[a][b]);
    }
  }
  if constexpr (FLUSH) {
#pragma unroll
    for (int a = 0; a < NBX; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][v] += tot[a][b][v];
  }
  // 32 x 32 accumulator layout: register v of lane i holds row
  // 8 (v / 4) + 4 (i / 32) + v % 4 and column i % 32
#pragma unroll
  for (int a = 0; a < NBX; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      const int64_t col = w0 + ww + b * 32 + r32;
      if (col >= J) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = x0 + wx + a * 32 + 8 * (v / 4) + 4 * g + (v % 4);
        if (row < nx) C[static_cast<int64_t>(row) * ldc + col] = alpha * acc[a][b][v];
      }
    }
}

// 16-bit conv. FD-SRP with generated steering: the tiles (BXF = 256 frames
// for batches of more than 128, 64 frames for smaller ones, either way 256
// candidates and the same generation code, so a frame's map does not depend
// on its batch), LDS stages, bank swizzle and software pipeline of gemm_fd16,
// with the
// cross-spectra (tile-major, fd16_tiled) streamed through a ring of FG_NBX
// stages and the steering stage generated into one of FG_NBH LDS buffers
// two stages before the MFMAs read it, half a stage per MFMA step, so that
// the generation's vector work issues between the matrix instructions.
// Thread r generates row r (candidate w0 + r): at a pair's first stage its
// first angle (bin 1) comes from the FP64 sincospi of the reduced phase;
// each stage's first bin is that FP64 value advanced by a 16-bin FP64
// rotation per stage, and the stage's 16 bins follow by FP32 rotation by
// exp(+i pi x / K) (a chain of 15 steps); bins k > K - 1 are zero.
// blockIdx.y splits the contraction at pair boundaries as in fd_gen.
constexpr int FG_NBX = 6, FG_NBH = 3;
constexpr int FG_XST = FD16_TILE * FD16_SB;  // 16 KB: one operand's stage

template <typename T, int BXF>
__global__ __launch_bounds__(256) void fd_gen16(const T* __restrict__ X, int64_t ldx,
                                                const double* __restrict__ xg, int64_t J, int K, int Kp,
                                                float* __restrict__ C, int64_t ldc, int nx, int P, float alpha,
                                                int nw_tiles, int nx_tiles, int pps, int64_t cz_rows) {
  static_assert(sizeof(T) == 2, "16-bit operands");
  static_assert(BXF == 256 || BXF == 64, "256- or 64-frame tiles");
  constexpr int STEP = Mfma<T>::STEP;
  // waves: 2 x 2 of 128 x 128 (256-frame tiles) or 1 x 4 of 64 x 64
  constexpr int WGY = BXF == 256 ? 2 : 1, WGX = 4 / WGY;
  constexpr int NA = BXF / WGY / 32, NB = FD16_TILE / WGX / 32;  // 32 x 32 blocks per wave
  constexpr int XST = BXF * FD16_SB;     // a cross-spectra stage
  constexpr int NL = XST / 1024 / 4;     // its loads per wave
  static_assert((FG_NBX - 1) * NL < 64, "vmcnt holds at most 63 loads");
  static_assert(FG_NBX * XST + FG_NBH * FG_XST <= 160 * 1024, "LDS");
  __shared__ __attribute__((aligned(16))) unsigned char lds[FG_NBX * XST + FG_NBH * FG_XST];
  unsigned char* const hb = lds + FG_NBX * XST;

  int wt, xt;
  if (!xcd_tile(nw_tiles, nx_tiles, wt, xt)) return;  // uniform over the block
  const int x0 = xt * BXF, w0 = wt * FD16_TILE;
  if (x0 >= nx) return;
  const int p0 = static_cast<int>(blockIdx.y) * pps, p1 = min(P, p0 + pps);
  if (p0 >= p1) return;
  const int spp = Kp * 2 / FD16_SB;  // stages per pair (even)
  const int ns = (p1 - p0) * spp;
  C += static_cast<int64_t>(blockIdx.y) * cz_rows * ldc;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // cross-spectra loads: psi is tile-major in 256-row tiles (fd16_tiled), so
  // a 64-frame tile is a contiguous quarter of each 16 KB stage; wave w
  // fills rows 16 NL w .. 16 NL (w + 1) - 1 of the tile's stage
  const int64_t nstg = ldx * 2 / FD16_SB;
  const unsigned char* src =
      reinterpret_cast<const unsigned char*>(X) +
      ((static_cast<int64_t>(x0 / FD16_TILE) * nstg + static_cast<int64_t>(p0) * spp) * FD16_TILE + x0 % FD16_TILE +
       16 * NL * wave) *
          FD16_SB +
      16 * lane;
  auto issue = [&](int s) {
    unsigned char* dst = lds + (s % FG_NBX) * XST + wave * NL * 1024;
    const unsigned char* sp = src + static_cast<int64_t>(min(s, ns - 1)) * FG_XST;
#pragma unroll
    for (int i = 0; i < NL; ++i)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(sp + 1024 * i),
                                       (__attribute__((address_space(3))) void*)(dst + 1024 * i), 16, 0, 0);
  };

  // generator of row tid
  const int64_t gj = w0 + tid;
  const bool glive = gj < J;
  const int gsw = fd16_swz(tid & 15);
  double sc = 1.0, ss = 0.0, ac = 1.0, as = 0.0;  // FP64 seed (next stage's first bin) and 16-bin advance
  float fc = 1.0f, fs = 0.0f, cc = 1.0f, cs = 0.0f;  // FP32 one-bin step and running value
  int kfirst = 1;
  auto seed_pair = [&](int p) {
    const double x = glive ? xg[static_cast<int64_t>(p) * J + gj] : 0.0;
    const FdSeed sd = fd_gen_seed(x, K);  // bin 1 (theta = pi x / K) and the 16-bin advance
    ss = sd.s1;
    sc = sd.c1;
    as = sd.s16;
    ac = sd.c16;
    fc = static_cast<float>(sc);
    fs = static_cast<float>(ss);
  };
  auto gen_begin = [&](int g) {
    cc = static_cast<float>(sc);
    cs = static_cast<float>(ss);
    kfirst = (g % spp) * 16 + 1;
    // explicit fma: fd_gen reproduces the same seeds
    const double cn = __builtin_fma(sc, ac, -(ss * as));
    ss = __builtin_fma(sc, as, ss * ac);
    sc = cn;
  };
  // bins 8 h .. 8 h + 7 of stage g: chunks 2 h, 2 h + 1 of row tid
  auto gen_half = [&](int g, int h) {
    unsigned char* row = hb + (g % FG_NBH) * FG_XST + tid * FD16_SB;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = 2 * h + q;
      uint32_t w4[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool ok = glive && kfirst + 4 * c + b <= K - 1;
        const T re = cvt<T>(ok ? cc : 0.0f), im = cvt<T>(ok ? -cs : 0.0f);
        uint16_t ur, ui;
        __builtin_memcpy(&ur, &re, 2);
        __builtin_memcpy(&ui, &im, 2);
        w4[b] = static_cast<uint32_t>(ur) | (static_cast<uint32_t>(ui) << 16);
        const float cn = __builtin_fmaf(cc, fc, -(cs * fs));
        cs = __builtin_fmaf(cc, fs, cs * fc);
        cc = cn;
      }
      *reinterpret_cast<i32x4*>(row + 16 * (c ^ gsw)) =
          i32x4{static_cast<int>(w4[0]), static_cast<int>(w4[1]), static_cast<int>(w4[2]), static_cast<int>(w4[3])};
    }
  };

  const int r32 = lane & 31, g = lane >> 5;
  const int wy = wave / WGX, wx = wave % WGX;
  f32x16 acc[NA][NB];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  const int sw = fd16_swz(r32 & 15);
  const int xrow = (wy * 32 * NA + r32) * FD16_SB, wrow = (wx * 32 * NB + r32) * FD16_SB;
  auto frags = [&](int s, auto tc, i32x4 (&fa)[NA], i32x4 (&fb)[NB]) {
    constexpr int t = decltype(tc)::value;
    const unsigned char* bx = lds + (s % FG_NBX) * XST;
    const unsigned char* bw = hb + (s % FG_NBH) * FG_XST;
    const int pos = 16 * (((t * STEP) / 16 + g) ^ sw);
#pragma unroll
    for (int a = 0; a < NA; ++a) fa[a] = *reinterpret_cast<const i32x4*>(bx + xrow + pos + a * 32 * FD16_SB);
#pragma unroll
    for (int b = 0; b < NB; ++b) fb[b] = *reinterpret_cast<const i32x4*>(bw + wrow + pos + b * 32 * FD16_SB);
  };
  auto mfmas = [&](const i32x4 (&fa)[NA], const i32x4 (&fb)[NB]) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) Mfma<T>::run(&fa[a], &fb[b], acc[a][b]);
  };
  // MFMA step t of consumption stage s (fragments in ca, cb) while half h = t
  // of generation stage s + 2 is written; at t = 1 the barrier publishes
  // stage s + 1 (its cross-spectra landed: NBX - 2 later stages may stay in
  // flight; its steering was written during stage s - 1) and the ring slot
  // of stage s takes stage s + NBX.
  auto step = [&](int s, auto tc, i32x4 (&ca)[NA], i32x4 (&cb)[NB], i32x4 (&na)[NA], i32x4 (&nb)[NB]) {
    constexpr int t = decltype(tc)::value;
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));  // this step's fragments (read one step ago)
    if constexpr (t == 0) {
      frags(s, std::integral_constant<int, 1>{}, na, nb);
      gen_begin(s + 2);
      gen_half(s + 2, 0);
    } else {
      wait_vm_lds<(FG_NBX - 2) * NL>();
      asm volatile("s_barrier" ::: "memory");
      issue(s + FG_NBX);
      frags(s + 1, std::integral_constant<int, 0>{}, na, nb);
      gen_half(s + 2, 1);  // buffer (s + 2) mod NBH is free since the barrier of stage s
    }
    mfmas(ca, cb);
    // interleave: each MFMA followed by a few vector instructions of the
    // generation, the fragment reads and (t = 1) the loads
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 80 / (NA * NB), 0);  // VALU
      if (i < NA + NB) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
      if (t == 1 && i < NL) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  for (int s = 0; s < FG_NBX; ++s) issue(s);
  seed_pair(p0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    gen_begin(s);
    gen_half(s, 0);
    gen_half(s, 1);
  }
  wait_vm_lds<(FG_NBX - 1) * NL>();  // stage 0 has landed
  asm volatile("s_barrier" ::: "memory");
  i32x4 fa0[NA], fb0[NB], fa1[NA], fb1[NB];
  frags(0, std::integral_constant<int, 0>{}, fa0, fb0);
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  for (int s = 0; s < ns; s += 2) {
    // the generation stages s + 2, s + 3 start a pair together (spp even)
    if (s + 2 < ns && (s + 2) % spp == 0) seed_pair(p0 + (s + 2) / spp);
    step(s, I0{}, fa0, fb0, fa1, fb1);
    step(s, I1{}, fa1, fb1, fa0, fb0);
    step(s + 1, I0{}, fa0, fb0, fa1, fb1);
    step(s + 1, I1{}, fa1, fb1, fa0, fb0);
  }
  wait_vm_lds<0>();  // the reloads past the last stage

  const int rbase = x0 + wy * 32 * NA + 4 * g;
  const int64_t cbase = static_cast<int64_t>(w0) + wx * 32 * NB + r32;
  float* cp = C + static_cast<int64_t>(rbase) * ldc + cbase;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ro = a * 32 + 8 * (v / 4) + (v % 4);
      if (rbase + ro >= nx) continue;
      float* rp = cp + ro * ldc;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (cbase + b * 32 < J) rp[b * 32] = alpha * acc[a][b][v];
    }
}

// FP64 variant on v_mfma_f64_16x16x4_f64: 64 x 64 tile, 4 waves of 32 x 32,
// each 2 x 2 blocks of 16 x 16.  Lane i supplies row i % 16 and k slot i / 16
// of each 4-deep step; accumulator register v of lane i holds row
// 4 v + i / 16, column i % 16 (the FP64 accumulator interleaves rows across
// lane groups, unlike the FP32 32 x 32 layout).
__global__ __launch_bounds__(256) void gemm_nt_f64(const double* __restrict__ X, int64_t ldx,
                                                   const double* __restrict__ W, int64_t ldw,
                                                   double* __restrict__ C, int64_t ldc, int nx,
                                                   int nw, int kdim, double alpha) {
  constexpr int BX = 64, BW = 64, BK = 16, ROW = BK + 1;
  __shared__ double xs[BX * ROW];
  __shared__ double ws[BW * ROW];
  const int x0 = blockIdx.y * BX, w0 = blockIdx.x * BW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wx = (wave >> 1) * 32, ww = (wave & 1) * 32;
  const int r16 = lane & 15, g = lane >> 4;
  f64x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  for (int k0 = 0; k0 < kdim; k0 += BK) {
    __syncthreads();
    for (int e = tid; e < (BX + BW) * BK; e += 256) {
      const int row = e / BK, col = e % BK;
      if (row < BX)
        xs[row * ROW + col] = X[static_cast<int64_t>(x0 + row) * ldx + k0 + col];
      else
        ws[(row - BX) * ROW + col] = W[static_cast<int64_t>(w0 + row - BX) * ldw + k0 + col];
    }
    __syncthreads();
    for (int s = 0; s < BK; s += 4) {
      double fa[2], fb[2];
      for (int a = 0; a < 2; ++a) fa[a] = xs[(wx + a * 16 + r16) * ROW + s + g];
      for (int b = 0; b < 2; ++b) fb[b] = ws[(ww + b * 16 + r16) * ROW + s + g];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int col = w0 + ww + b * 16 + r16;
      if (col >= nw) continue;
      for (int v = 0; v < 4; ++v) {
        const int row = x0 + wx + a * 16 + 4 * v + g;
        if (row < nx) C[static_cast<int64_t>(row) * ldc + col] = alpha * acc[a][b][v];
      }
    }
}

// =============================================== sampling front end ======
//
// PHAT cross-spectra (eq. (2)) and GCC sampling (eq. (40)), straight from
// the frames: the direct product in gcc_direct (below), the iFFT of (46)
// in gcc_fft.

// y / |y| (0 for y = 0) with the hardware reciprocal square root; squared
// magnitudes outside [2^-100, 2^100] are rescaled first so that neither
// underflow nor overflow can occur.
// Every contraction is spelled out with fmaf: left to the compiler, a * a +
// b * b is contracted one way in some unrolled copies and the other way in
// others, and a frame's result would then depend on its slot in the tile.
__device__ inline float2 unit_phase(float2 y) {
  float a = y.x, b = y.y;
  float n2 = __builtin_fmaf(a, a, b * b);
  if (!(n2 >= 0x1p-100f && n2 <= 0x1p100f)) {
    const float s = std::max(std::fabs(a), std::fabs(b));
    if (!(s > 0.0f)) return make_float2(0.0f, 0.0f);
    a /= s;
    b /= s;
    n2 = __builtin_fmaf(a, a, b * b);
  }
  const float r = __builtin_amdgcn_rsqf(n2);
  return make_float2(a * r, b * r);
}

// iFFT sampling (46): xi_p[n] for n = -N_p..N_p as samples of the unscaled
// length-2K inverse DFT of the Hermitian spectrum psi_p (zero at DC and
// Nyquist).  A block owns one (frame, pair): psi = u_m conj(u_m') with
// u = y/|y| is formed in LDS, the real length-2K transform is folded into one
// complex length-K transform (z[i] = x[2i] + j x[2i+1] is the inverse DFT of
// E[k] + j O[k], E[k] = psi[k] + conj psi[K-k], O[k] = (psi[k] - conj
// psi[K-k]) exp(i pi k / K)), which runs as a radix-2 Stockham transform in
// LDS.  The 2 N_p + 1 wanted samples go to xi [L][PN] (frame-major, written
// contiguously); transpose_lp then forms xi^T.  Every block runs the same
// instruction sequence, so a frame's samples do not depend on its batch.
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

template <int LOGK>
__global__ __launch_bounds__(256) void gcc_fft(const float2* __restrict__ Y, int M, int P,
                                               const int32_t* __restrict__ pm, const int32_t* __restrict__ pmp,
                                               const int32_t* __restrict__ np, const int32_t* __restrict__ off,
                                               const float2* __restrict__ tw, const float2* __restrict__ w2,
                                               float* __restrict__ xi, int64_t ldx) {
  constexpr int K = 1 << LOGK;
  __shared__ float2 bufA[K], bufB[K];
  const int tid = threadIdx.x;
  const int64_t l = blockIdx.x / P;
  const int p = blockIdx.x % P;
  const float2* ym = Y + (l * M + pm[p]) * (K + 1);
  const float2* yq = Y + (l * M + pmp[p]) * (K + 1);
  for (int k = tid; k < K; k += 256) {
    float2 v = make_float2(0.0f, 0.0f);
    if (k >= 1) {
      const float2 a = unit_phase(ym[k]), b = unit_phase(yq[k]);
      v = make_float2(__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.y, b.x, -(a.x * b.y)));
    }
    bufA[k] = v;
  }
  __syncthreads();
  for (int k = tid; k < K; k += 256) {
    const float2 a = bufA[k];
    const float2 c = k == 0 ? make_float2(0.0f, 0.0f) : bufA[K - k];
    const float2 e = make_float2(a.x + c.x, a.y - c.y);
    const float2 o = cmul(make_float2(a.x - c.x, a.y + c.y), w2[k]);
    bufB[k] = make_float2(e.x - o.y, e.y + o.x);
  }
  __syncthreads();
  float2* src = bufB;
  float2* dst = bufA;
#pragma unroll
  for (int s = 0; s < LOGK; ++s) {
    const int mm = 1 << s, half = (K >> (s + 1)) << s;  // butterfly span l * m = K / 2
    for (int b = tid; b < K / 2; b += 256) {
      const int j = b >> s, k = b & (mm - 1);
      const float2 c0 = src[k + j * mm], c1 = src[k + j * mm + half];
      dst[k + 2 * j * mm] = make_float2(c0.x + c1.x, c0.y + c1.y);
      dst[k + 2 * j * mm + mm] = cmul(tw[j * mm], make_float2(c0.x - c1.x, c0.y - c1.y));
    }
    __syncthreads();
    float2* t = src;
    src = dst;
    dst = t;
  }
  const int npp = np[p];
  float* out = xi + l * ldx + off[p];
  for (int i = tid; i < 2 * npp + 1; i += 256) {
    const int t = (i - npp + 2 * K) & (2 * K - 1);
    const float2 z = src[t >> 1];
    out[i] = (t & 1) ? z.y : z.x;
  }
}

// xi [L][ldx] -> xi^T [PN][ldt] through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void transpose_lp(const float* __restrict__ xi, int64_t ldx, int L, int PN,
                                                    float* __restrict__ xiT, int64_t ldt) {
  __shared__ float t[32][33];
  const int n0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int l = l0 + r, n = n0 + tx;
    t[r][tx] = (l < L && n < PN) ? xi[static_cast<int64_t>(l) * ldx + n] : 0.0f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int n = n0 + r, l = l0 + tx;
    if (n < PN && l < L) xiT[static_cast<int64_t>(n) * ldt + l] = t[tx][r];
  }
}

// ========================================================= direct sampling ===
//
// xi_p[l][n] = sum_{k=1}^{K-1} S[n][k] . psi_p[l, k] (eq. (40)) with the
// real pairing S . psi = S_re Re psi + S_im Im psi, S[n][k] = (2 cos,
// -2 sin)(pi k n / K), as one product whose rows are the (frame, pair)
// combinations and whose columns are the lags -max_np..max_np of the table
// S that every pair shares (each pair keeps its own 2 N_p + 1 lags).
// A block owns `ft` frames (ft P rows, in tiles of 32) and up to GD_TILES
// (row tile, 32-lag column tile) products.  Per chunk of GD_CB bins it
// stages u = y / |y| of its frames' microphones (each (frame, mic, bin)
// normalised once) and the chunk's table columns in LDS; its sixteen waves
// multiply the four products, each over one quarter of the chunk's bins, on
// v_mfma_f32_32x32x2_f32 (k slot 0 walks the even bin pairs, slot 1 the odd
// ones, Re then Im), each lane forming psi_p = u_m conj(u_m') of its row,
// and the quarters are added in LDS.  Four waves per product hide the LDS
// latency that one wave per SIMD left exposed (measured: 44 us against 49
// with two waves per product and 55 with four loader waves feeding eight
// multiplying ones, room workload, 125,000 candidates).  SPLIT (plans with
// 16-bit or FP8 operands, whose later stages round far coarser): the
// products run on v_mfma_f32_32x32x16_bf16 with psi and the table split
// into BF16 (hi, lo) halves (the table's halves precomputed: per 4 bins 16
// bytes of hi then 16 of lo, the byte layout of the FP32 table), three
// products per step in place of 16 FP32 ones per 8 bins (37 -> 29 us).
// The frames and the table are read once per block (the table is shared
// by every pair), and the next chunk is loaded into registers while the
// current one is multiplied (two chunks ahead was slower: 35 us).  Every
// frame runs the same instruction sequence, so its samples do not depend
// on the batch.
constexpr int GD_CB = 64;                 // bins per chunk
constexpr int GD_ROWB = GD_CB * 8 + 16;   // bytes per LDS row (a (frame, mic) or a table row)
constexpr int GD_FM = 64;                 // max frames x microphones per block
constexpr int GD_TILES = 4;               // products per block (each split over four waves)
constexpr int GD_NCT = 4;                 // max 32-lag column tiles (2 max_np + 1 <= 128)

template <int NCT, bool SPLIT>
__global__ __launch_bounds__(1024) void gcc_direct(const float2* __restrict__ Y, int M, int K, int L, int P,
                                                  const int32_t* __restrict__ pm, const int32_t* __restrict__ pmp,
                                                  const int32_t* __restrict__ np, const int32_t* __restrict__ off,
                                                  int max_np, const float* __restrict__ S, int Kb, int ft, int nrt,
                                                  int nct, float* __restrict__ xiT, int64_t ldxi) {
  extern __shared__ __attribute__((aligned(16))) unsigned char gd_lds[];
  unsigned char* u_lds = gd_lds;                                 // [ft M + 1 zero row][GD_ROWB]
  unsigned char* s_lds = gd_lds + (GD_FM + 1) * GD_ROWB;        // [NCT 32][GD_ROWB]
  constexpr int NT = 1024;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r32 = lane & 31, kq = lane >> 5;
  const int64_t fbase = static_cast<int64_t>(blockIdx.x) * ft;
  const int fm_rows = ft * M;
  const int ntiles = nrt * nct;
  // wave w: product (tile) w % 4 of the block's group, bins of quarter w / 4
  // of every chunk; the quarters' partial tiles are added in LDS at the end
  const int t = blockIdx.y * GD_TILES + (wave & 3);
  const int half = wave >> 2;  // quarter of the chunk's bins (0..3)
  const bool tlive = t < ntiles;  // uniform over the wave
  int ta, tb, tcol;
  {
    const int rt = tlive ? t / nct : 0, ct = tlive ? t % nct : 0;
    const int rho = rt * 32 + r32;
    const int fl = rho / P, p = rho % P;
    const bool ok = tlive && rho < ft * P && fbase + fl < L;
    // this lane's row: LDS offsets of u_m and u_m' (the zero row for padding
    // rows and frames past L) and of its lag's table row
    ta = (ok ? fl * M + pm[p] : fm_rows) * GD_ROWB + half * (GD_CB / 4) * 8;
    tb = (ok ? fl * M + pmp[p] : fm_rows) * GD_ROWB + half * (GD_CB / 4) * 8;
    tcol = (ct * 32 + r32) * GD_ROWB + half * (GD_CB / 4) * 8;
  }
  for (int e = tid; e < GD_ROWB / 16; e += NT)
    *reinterpret_cast<f32x4*>(u_lds + fm_rows * GD_ROWB + 16 * e) = f32x4{0.f, 0.f, 0.f, 0.f};

  constexpr int UPT = GD_FM * (GD_CB / 2) / NT;     // bin pairs of u per thread
  constexpr int SPT = NCT * 32 * (GD_CB / 2) / NT;  // 16-byte table pieces per thread
  f32x4 uy[UPT], sv[SPT];
  const int uitems = fm_rows * (GD_CB / 2);
  constexpr int sitems = NCT * 32 * (GD_CB / 2);  // rows past nct 32 are zero in the table
  const int nchunks = Kb / GD_CB;

  auto gload = [&](int c, f32x4 (&uy)[UPT], f32x4 (&sv)[SPT]) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int e = tid + NT * i;
      uy[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (e < uitems) {
        const int row = e / (GD_CB / 2), b2 = e % (GD_CB / 2);
        const int fl = row / M, m = row % M;
        const int k = c * GD_CB + 2 * b2 + 1;  // bins k, k + 1
        const int64_t f = fbase + fl;
        if (f < L) {
          const float2* yr = Y + (f * M + m) * (K + 1);
          if (k + 1 <= K - 1) {
            const float2 a0 = yr[k], a1 = yr[k + 1];
            uy[i] = f32x4{a0.x, a0.y, a1.x, a1.y};
          } else if (k <= K - 1) {
            const float2 a0 = yr[k];
            uy[i] = f32x4{a0.x, a0.y, 0.f, 0.f};
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int e = tid + NT * i;
      const int row = e / (GD_CB / 2), q = e % (GD_CB / 2);
      sv[i] = *reinterpret_cast<const f32x4*>(S + static_cast<int64_t>(row) * (2 * Kb) + 2 * c * GD_CB + 4 * q);
    }
  };
  auto lstore = [&](const f32x4 (&uy)[UPT], const f32x4 (&sv)[SPT]) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int e = tid + NT * i;
      if (e < uitems) {
        const int row = e / (GD_CB / 2), b2 = e % (GD_CB / 2);
        const float2 u0 = unit_phase(make_float2(uy[i].x, uy[i].y)), u1 = unit_phase(make_float2(uy[i].z, uy[i].w));
        *reinterpret_cast<f32x4*>(u_lds + row * GD_ROWB + 16 * b2) = f32x4{u0.x, u0.y, u1.x, u1.y};
      }
    }
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int e = tid + NT * i;
      const int row = e / (GD_CB / 2), q = e % (GD_CB / 2);
      *reinterpret_cast<f32x4*>(s_lds + row * GD_ROWB + 16 * q) = sv[i];
    }
  };
  static_assert(sitems % NT == 0, "table pieces must tile the threads");

  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  auto multiply = [&]() {
    if (SPLIT && tlive) {
      // split BF16 on v_mfma_f32_32x32x16_bf16: step j covers 8 bins of the
      // wave's quarter, k slot kq its bins 4 kq .. 4 kq + 3 (Re, Im of
      // each); psi = ah + al and the table's (hi, lo) halves give
      // ah th + ah tl + al th, all products exact in FP32, the dropped
      // al tl and the rounding of al leave ~2^-16 of each term
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = 8 * (8 * j + 4 * kq);
        const f32x4 x0 = *reinterpret_cast<const f32x4*>(u_lds + ta + o);
        const f32x4 x1 = *reinterpret_cast<const f32x4*>(u_lds + ta + o + 16);
        const f32x4 y0 = *reinterpret_cast<const f32x4*>(u_lds + tb + o);
        const f32x4 y1 = *reinterpret_cast<const f32x4*>(u_lds + tb + o + 16);
        const i32x4 th = *reinterpret_cast<const i32x4*>(s_lds + tcol + o);
        const i32x4 tl = *reinterpret_cast<const i32x4*>(s_lds + tcol + o + 16);
        float a[8];
        // psi = u_m conj(u_m') of four bins
        a[0] = __builtin_fmaf(x0.x, y0.x, x0.y * y0.y);
        a[1] = __builtin_fmaf(x0.y, y0.x, -(x0.x * y0.y));
        a[2] = __builtin_fmaf(x0.z, y0.z, x0.w * y0.w);
        a[3] = __builtin_fmaf(x0.w, y0.z, -(x0.z * y0.w));
        a[4] = __builtin_fmaf(x1.x, y1.x, x1.y * y1.y);
        a[5] = __builtin_fmaf(x1.y, y1.x, -(x1.x * y1.y));
        a[6] = __builtin_fmaf(x1.z, y1.z, x1.w * y1.w);
        a[7] = __builtin_fmaf(x1.w, y1.z, -(x1.z * y1.w));
        bf16x8 ah, al;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          ah[i] = static_cast<__bf16>(a[i]);
          al[i] = static_cast<__bf16>(a[i] - static_cast<float>(ah[i]));
        }
        const bf16x8 bh = __builtin_bit_cast(bf16x8, th), bl = __builtin_bit_cast(bf16x8, tl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
      }
    } else if (tlive) {
      // k slot kq of four steps covers bins b + 2 kq and b + 2 kq + 1 (Re,
      // then Im of each): a lane reads its own two bins of u_m, u_m' and of
      // its lag's table row, 16 bytes each per four products
      const int kb = 16 * kq;
#pragma unroll 8
      for (int b = 0; b < GD_CB / 4; b += 4) {
        const f32x4 x = *reinterpret_cast<const f32x4*>(u_lds + ta + 8 * b + kb);
        const f32x4 y = *reinterpret_cast<const f32x4*>(u_lds + tb + 8 * b + kb);
        const f32x4 sc = *reinterpret_cast<const f32x4*>(s_lds + tcol + 8 * b + kb);
        // psi = u_m conj(u_m')
        const float re0 = __builtin_fmaf(x.x, y.x, x.y * y.y), im0 = __builtin_fmaf(x.y, y.x, -(x.x * y.y));
        const float re1 = __builtin_fmaf(x.z, y.z, x.w * y.w), im1 = __builtin_fmaf(x.w, y.z, -(x.z * y.w));
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(re0, sc.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(im0, sc.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(re1, sc.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(im1, sc.w, acc, 0, 0, 0);
      }
    }
  };
  gload(0, uy, sv);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // the previous chunk's reads are done
    lstore(uy, sv);
    __syncthreads();
    if (c + 1 < nchunks) gload(c + 1, uy, sv);
    multiply();
  }
  // the other quarters' partial tiles through LDS (the u buffer is free now)
  __syncthreads();
  f32x16* red = reinterpret_cast<f32x16*>(gd_lds);
  if (half >= 1 && tlive) red[((half - 1) * 4 + (wave & 3)) * 64 + lane] = acc;
  __syncthreads();
  if (half >= 1 || !tlive) return;
  for (int q = 0; q < 3; ++q) {
    const f32x16 o = red[(q * 4 + wave) * 64 + lane];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] += o[v];
  }
  // 32 x 32 accumulator layout: register v of lane i holds row
  // 8 (v / 4) + 4 (i / 32) + v % 4 and column i % 32
  const int rt = t / nct, ct = t % nct;
  const int n = ct * 32 + r32 - max_np;  // lag of this lane's column
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rho = rt * 32 + 8 * (v / 4) + 4 * kq + (v % 4);
    if (rho >= ft * P) continue;
    const int fl = rho / P, p = rho % P;
    const int64_t f = fbase + fl;
    const int npp = np[p];
    if (f < L && n >= -npp && n <= npp) xiT[static_cast<int64_t>(off[p] + n + npp) * ldxi + f] = acc[v];
  }
}

// Per-pair SLRI fat stage on the matrix cores, g[l][p R + r] = gscale_p
// sum_n V_p[n][r] xi_p[l][n] (eq. (57)): one wave per (pair, 16 frames, 16
// columns of R) on v_mfma_f32_16x16x4_f32, A = xi^T rows of the pair's lags
// (frames contiguous), B = V_p; eight steps of loads are issued ahead of
// their products.  Block = four waves, the pair's next four frame tiles;
// pair index P zero-fills g's padding columns.
template <typename TG>
__global__ __launch_bounds__(256) void slri_fat_mfma(const float* __restrict__ xiT, int64_t ldxi, int L,
                                                     const int32_t* __restrict__ np, const int32_t* __restrict__ off,
                                                     const float* __restrict__ V, int vrows, int R,
                                                     const float* __restrict__ gscale, int P, TG* __restrict__ g,
                                                     int Kc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = blockIdx.y;
  const int64_t l0 = static_cast<int64_t>(blockIdx.x) * 64 + wave * 16;
  if (p == P) {  // uniform over the block
    const int pad = Kc - P * R;
    for (int e = lane; e < 16 * pad; e += 64) {
      const int64_t l = l0 + e / pad;
      if (l < L) g[l * Kc + P * R + e % pad] = cvt<TG>(0.0f);
    }
    return;
  }
  const int r16 = lane & 15, kk = lane >> 4;
  const int nrows = 2 * np[p] + 1;
  const float* xs = xiT + static_cast<int64_t>(off[p]) * ldxi + l0 + r16;
  const float* Vp = V + static_cast<int64_t>(p) * vrows * R;
  const float sc = gscale[p];
  const int nsteps = (nrows + 3) / 4;
  for (int c0 = 0; c0 < R; c0 += 16) {
    const int col = c0 + r16;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    constexpr int U = 8;
    for (int s0 = 0; s0 < nsteps; s0 += U) {
      float a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int n = 4 * (s0 + u) + kk;
        const bool ok = n < nrows;
        a[u] = ok ? xs[static_cast<int64_t>(n) * ldxi] : 0.0f;
        b[u] = ok && col < R ? Vp[n * R + col] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
    }
    // 16 x 16 accumulator layout: register v of lane i holds row (frame)
    // 4 (i / 16) + v and column i % 16
    if (col < R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t l = l0 + 4 * kk + v;
        if (l < L) g[l * Kc + p * R + col] = cvt<TG>(acc[v] * sc);
      }
    }
  }
}

// Global SLRI fat stage g = Lambda_fat xi (eq. (57) with the stacked fit of
// (54)): g[l][c] = scale * sum_a V[a][c] xi[l][a] over all PN stacked
// samples.  A wave holds 64 consecutive frames (coalesced xi rows) and 4
// columns per lane (one 16-byte V load, uniform over the wave); a block is
// 64 frames x 16 columns.  V is zero-padded to Kc columns, so the padding
// columns come out zero.
// The same product on the matrix cores: a block owns 32 frames x 32
// columns of g; its eight waves take the lag pairs (a, a + 1) of every
// eighth v_mfma_f32_32x32x2_f32 step (a = 16 t + 2 w), reading xi^T rows
// (frames contiguous) and V rows (columns contiguous) straight from memory
// twelve steps ahead, and the eight partial tiles are added in LDS in wave
// order (deterministic).  Lags past PN read as zero.
template <typename TG>
__global__ __launch_bounds__(512) void slri_fat_global_mfma(const float* __restrict__ xiT, int64_t ldxi, int L,
                                                            int PN, const float* __restrict__ V, int Kc,
                                                            const float* __restrict__ gscale, TG* __restrict__ g) {
  constexpr int NW = 8;
  __shared__ f32x16 red[NW - 1][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r32 = lane & 31, kq = lane >> 5;
  const int64_t l0 = static_cast<int64_t>(blockIdx.x) * 32;
  const int c0 = blockIdx.y * 32;
  const float* xs = xiT + l0 + r32;
  const float* vs = V + c0 + r32;
  // two accumulators (even and odd steps) so consecutive products are
  // independent; added at the end
  f32x16 acc, acc1;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = acc1[v] = 0.0f;
  constexpr int U = 12;
  const int nsteps = (PN + 1) / 2;
  for (int s0 = wave; s0 < nsteps; s0 += NW * U) {
    float a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a_ = 2 * (s0 + NW * u) + kq;
      const bool ok = s0 + NW * u < nsteps && a_ < PN;
      a[u] = ok ? xs[static_cast<int64_t>(a_) * ldxi] : 0.0f;
      b[u] = ok ? vs[static_cast<int64_t>(a_) * Kc] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; u += 2) {
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], acc, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u + 1], b[u + 1], acc1, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] += acc1[v];
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
  for (int q = 0; q < NW - 1; ++q) {
    const f32x16 o = red[q][lane];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] += o[v];
  }
  // accumulator layout: register v of lane i holds row (frame)
  // 8 (v / 4) + 4 (i / 32) + v % 4 and column i % 32
  const float sc = gscale[0];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t l = l0 + 8 * (v / 4) + 4 * kq + (v % 4);
    if (l < L) g[l * Kc + c0 + r32] = cvt<TG>(acc[v] * sc);
  }
}

// ====================================================== SLRI tall stream ===
//
// z[l][j] = alpha * sum_c g[l][c] U[j][c] (the tall stage of eq. (57)) for
// FP32, 16-bit and FP8 operands with rows of at most 1 KB (16-bit rows up to
// 1280 bytes on six compute waves, whose registers then hold the longer U
// rows).  Warp-specialised
// streaming: one loader wave brings the g rows of the next groups of 32
// frames straight into LDS (global_load_lds, no register round trip) up to
// four groups ahead, as many as the load counter and LDS hold, while CW
// compute waves (32 candidates each) multiply the current group and store
// it.  vmcnt is per wave and counts stores as well as loads, so keeping
// every global load out of the compute waves means they never wait for their
// own map stores, and the loader only ever waits for its loads; the
// barriers are plain s_barrier (a workgroup fence would make the loader
// drain its loads at every group).  The loads still queue behind the CU's
// map stores, so a block covers 32 CW candidates to read each g row as few
// times as possible.  Block b owns 32 CW candidates and one of nsplit
// contiguous ranges of frame groups; the splits of a candidate tile run back
// to back on one XCD (xcd_tile), so the U rows they share are fetched from
// HBM once.

template <typename T, int NS, int CW, bool CT>
__global__ __launch_bounds__(64 * (CW + 1)) void tall_ws(const T* __restrict__ g, int64_t ldg, int grows,
                                               const T* __restrict__ U, int64_t ldu,
                                               float* __restrict__ z, int64_t ldz, int L, int64_t J,
                                               float alpha, int njt, int nsplit, int gps,
                                               const int32_t* __restrict__ ctab,
                                               const int32_t* __restrict__ tlist) {
  constexpr int STEP = Mfma<T>::STEP;
  constexpr int LB = STEP / 2;
  constexpr int NV = LB / 16;
  constexpr int ROWP = NS * STEP + 16;  // padded LDS row (bytes)
  constexpr int CPR = NS * STEP / 16;   // 16-byte chunks per g row
  // buffers: the group being multiplied plus up to four in flight, as many
  // as the load counter (63 loads, NI per group) and 150 KB of LDS allow
  constexpr int NI = (32 * (CPR + 1) + 63) / 64;  // loads per group (a row's pad unit included)
  constexpr int DV = 1 + 63 / NI;
  constexpr int DL = (150 * 1024) / (32 * ROWP) - 1;
  constexpr int NBUF = 1 + (DV < DL ? (DV < 4 ? DV : 4) : (DL < 4 ? DL : 4));
  __shared__ __attribute__((aligned(16))) unsigned char gs[NBUF][32 * ROWP];
  int jt, sp;
  if (!xcd_tile(njt, nsplit, jt, sp)) return;
  if (tlist) jt = tlist[jt];  // njt counts the listed tiles
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g0 = sp * gps;
  const int ng = std::min((L + 31) / 32, g0 + gps) - g0;  // groups of this block
  if (ng <= 0) return;  // block-uniform

  if (wave == CW) {
    // loader: direct loads into LDS, D = NBUF - 1 groups in flight.  Load k
    // of a group fills 16-byte slots 64 k .. 64 k + 63 of its buffer (lane
    // l: slot 64 k + l).  A row's pad unit and the chunks of table entry -1
    // are filled from the row's first chunk (finite samples; entry -1 meets
    // zero weights), so that only lanes past the buffer are masked, every
    // load has an active lane, each group counts exactly NI loads and the
    // waits below are exact.
    const unsigned char* gb = reinterpret_cast<const unsigned char*>(g);
    constexpr int SLOTS = 32 * (CPR + 1);
    constexpr int D = NBUF - 1;
    static_assert((D - 1) * NI < 64, "vmcnt holds at most 63 loads");
    int32_t dcol[NI];
    int drow[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int q = 64 * k + lane;
      const int r = q / (CPR + 1), s = q % (CPR + 1);
      drow[k] = r;
      dcol[k] = q < SLOTS ? 0 : -1;
      if (q < SLOTS && s < CPR) {
        if constexpr (CT) {
          const int32_t cc = ctab[static_cast<int64_t>(jt) * CPR + s];
          dcol[k] = cc >= 0 ? cc * static_cast<int32_t>(sizeof(T)) : 0;
        } else {
          dcol[k] = 16 * s;
        }
      }
    }
    auto issue = [&](int i) {
      unsigned char* base = &gs[i % NBUF][0];
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        // rows past the ones g holds repeat its last row (their frames are
        // never stored)
        const int row = min((g0 + i) * 32 + drow[k], grows - 1);
        if (dcol[k] >= 0)
          __builtin_amdgcn_global_load_lds(
              (const __attribute__((address_space(1))) void*)(gb + static_cast<int64_t>(row) * ldg * sizeof(T) + dcol[k]),
              (__attribute__((address_space(3))) void*)(base + 1024 * k), 16, 0, 0);
      }
    };
    for (int i = 0; i < D && i < ng; ++i) issue(i);
    if (ng >= D)
      wait_vm<(D - 1) * NI>();
    else
      wait_vm<0>();
    asm volatile("s_barrier" ::: "memory");
    for (int i = 0; i < ng; ++i) {
      if (i + D < ng) {
        issue(i + D);
        wait_vm<(D - 1) * NI>();  // group i + 1 has landed
      } else {
        wait_vm<0>();
      }
      asm volatile("s_barrier" ::: "memory");
    }
    return;
  }

  const int r32 = lane & 31, gq = lane >> 5;
  const int64_t j0 = static_cast<int64_t>(jt) * (32 * CW) + wave * 32;
  // U rows of this lane's candidate (zeros past J: the last tile may reach
  // beyond the padded rows of U)
  const bool jok = j0 + r32 < J;
  i32x4 uf[NS][NV];
  {
    const unsigned char* ur =
        reinterpret_cast<const unsigned char*>(U) + (jok ? j0 + r32 : 0) * ldu * static_cast<int64_t>(sizeof(T)) + gq * LB;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v)
        uf[s][v] = jok ? *reinterpret_cast<const i32x4*>(ur + s * STEP + 16 * v) : i32x4{0, 0, 0, 0};
  }
  asm volatile("s_barrier" ::: "memory");
  // element offset of this lane inside a group's rows: row 4 gq, column r32
  // (the host keeps 36 ldz below 2^31)
  const uint32_t loff = static_cast<uint32_t>(4 * gq * ldz + r32);
  for (int i = 0; i < ng; ++i) {
    const int grp = g0 + i;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const unsigned char* ar = &gs[i % NBUF][r32 * ROWP + gq * LB];
    if constexpr (NS <= 16) {
      i32x4 af[NS][NV];
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < NV; ++v) af[s][v] = *reinterpret_cast<const i32x4*>(ar + s * STEP + 16 * v);
#pragma unroll
      for (int s = 0; s < NS; ++s) Mfma<T>::run(af[s], uf[s], acc);
    } else {
      // long rows: U alone takes 4 NS registers, so the g fragments are
      // read CHK steps at a time (a quarter of the row past 1 KB, whose step
      // count is even but need not divide by four)
      constexpr int CHK = NS * STEP > 1024 ? (NS + 3) / 4 : NS / 2;
#pragma unroll
      for (int s0 = 0; s0 < NS; s0 += CHK) {
        i32x4 af[CHK][NV];
#pragma unroll
        for (int s = 0; s < CHK; ++s)
          if (s0 + s < NS)
#pragma unroll
            for (int v = 0; v < NV; ++v) af[s][v] = *reinterpret_cast<const i32x4*>(ar + (s0 + s) * STEP + 16 * v);
#pragma unroll
        for (int s = 0; s < CHK; ++s)
          if (s0 + s < NS) Mfma<T>::run(af[s], uf[s0 + s], acc);
      }
    }
    // rows (frames) 8 (v / 4) + 4 gq + v % 4 of the group, column j0 + r32:
    // a uniform row pointer plus the lane's 32-bit offset
    float* zg = z + static_cast<int64_t>(grp) * 32 * ldz + j0;
    if (grp * 32 + 32 <= L) {
      if (jok) {
#pragma unroll
        for (int v = 0; v < 16; ++v) zg[(8 * (v / 4) + (v % 4)) * ldz + loff] = alpha * acc[v];
      }
    } else if (jok) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int l = grp * 32 + 8 * (v / 4) + 4 * gq + (v % 4);
        if (l < L) zg[(8 * (v / 4) + (v % 4)) * ldz + loff] = alpha * acc[v];
      }
    }
    asm volatile("s_barrier" ::: "memory");
  }
}

// Dense-window SSPI operand: B[j][kpos(t, p) + (lag - a0(t, p))] = the tap
// weights of candidate j and pair p (eq. (58) per (j, p)), from the gather
// records (absolute start of tap 0 and Qs weights); every other entry of B
// stays zero.  kpos and a0 (first lag of the window) place pair p's window
// inside the contraction of candidate tile t = j / 256.
template <typename TW>
__global__ __launch_bounds__(256) void sspi_dense_weights(const int32_t* __restrict__ start,
                                                          const TW* __restrict__ w, int Qs, int Q, int64_t J,
                                                          const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ a0,
                                                          const int32_t* __restrict__ kpos, int P,
                                                          const int32_t* __restrict__ tiles,
                                                          TW* __restrict__ B, int kmax) {
  const int64_t t = tiles[blockIdx.x];  // one block per listed tile
  const int64_t j = t * 256 + threadIdx.x;
  const int p = blockIdx.y;
  if (j >= J) return;
  const int64_t rec = static_cast<int64_t>(p) * J + j;
  const int rel = start[rec] - off[p];  // tap 0 within the pair's lags
  const int k0 = kpos[t * P + p] + rel - a0[t * P + p];
  // the pair's slot of the contraction ends where the next pair's begins;
  // only zero-weighted taps (past the pair's lags) fall beyond it
  const int kend = p + 1 < P ? kpos[t * P + p + 1] : kmax;
  for (int q = 0; q < Q; ++q) {
    const TW v = w[rec * Qs + q];
    if (static_cast<float>(v) != 0.0f && k0 + q < kend) B[j * kmax + k0 + q] = v;
  }
}

// Frame-major samples for the dense-window SSPI, in 8 copies shifted by
// c = 0..7 columns so that every window can start on a 16-byte chunk:
// xf[l][c XW + a] = xi^T[colmap[a - c]][l] for 0 <= a - c < PNA (0 elsewhere
// and where colmap < 0), narrowed to the operand type.  A block owns 32
// columns a of every copy and 32 frames: it stages the 39 source columns
// those reach (a - 7 .. a + 31) once in LDS and writes all 8 copies.
template <typename T>
__global__ __launch_bounds__(256) void xi_to_frames(const float* __restrict__ xiT, int64_t ldxi, int L, int PNA,
                                                    int XW, const int32_t* __restrict__ colmap,
                                                    T* __restrict__ xf, int64_t ldf) {
  __shared__ float t[39][33];
  const int a0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 39; r += 8) {
    const int a = a0 - 7 + r, l = l0 + tx;
    float x = 0.0f;
    if (a >= 0 && a < PNA && l < L) {
      const int n = colmap[a];
      if (n >= 0) x = xiT[static_cast<int64_t>(n) * ldxi + l];
    }
    t[r][tx] = x;
  }
  __syncthreads();
  const int a = a0 + tx;
  if (a >= XW) return;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    for (int r = ty; r < 32; r += 8) {
      const int l = l0 + r;
      if (l < L) xf[static_cast<int64_t>(l) * ldf + c * XW + a] = cvt<T>(t[tx + 7 - c][r]);
    }
}

// ========================================================= SSPI gather ===
//
// z[l][j] = sum_p sum_{q < Q} w[p][j][q] xi[start(p, j) + q][l].
// One lane per candidate location j (256 per block) and FT frames per block,
// accumulated in registers.  The GCC samples of the frame tile are staged in
// LDS lag-major ([lag][FT frames], rows padded by 4 words so that lanes
// reading nearby lags hit different banks), one chunk of pairs at a time;
// each lane gathers the rows of its own Q-tap windows with 16-byte reads
// (4 frames each).  Starts and weights are per-lane coalesced vector loads.
//
// PAIRS = true (16-bit and FP8 weights): LDS holds packed FP16 "sliding
// pairs" E[n][l] = (xi[n][l], xi[n+1][l]) and two taps are applied by one
// v_dot2_f32_f16 with FP32 accumulation, halving LDS bytes per FMA.
//
// Blocks are ordered for the 8 XCDs (workgroups are dispatched round-robin
// over XCDs): XCD x walks a contiguous range of location tiles with the
// frame tiles innermost, so a tile's starts and weights stay in that XCD's
// L2 across all frame tiles.

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
constexpr int SSPI_MAX_CHUNK = 512;  // pairs per staged chunk of the SSPI gather
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename TW>
__device__ inline float wdecode(TW w);
template <>
__device__ inline float wdecode<float>(float w) { return w; }
template <>
__device__ inline float wdecode<__bf16>(__bf16 w) { return static_cast<float>(w); }
template <>
__device__ inline float wdecode<_Float16>(_Float16 w) { return static_cast<float>(w); }
template <>
__device__ inline float wdecode<fp8>(fp8 w) {
  // E4M3 -> FP32: exponent bias 7 -> 127; subnormals m * 2^-9
  const uint32_t c = w.bits;
  const uint32_t sg = (c & 0x80u) << 24;
  const uint32_t em = c & 0x7Fu;
  const float mag = (em >> 3) ? __uint_as_float(((em << 20) + (120u << 23))) : static_cast<float>(em) * 0x1p-9f;
  return __uint_as_float(__float_as_uint(mag) | sg);
}

// Tap i of a weight record held as 32-bit words (no type punning through
// pointers: the element is extracted by shifts and bit casts).
template <typename TW>
__device__ inline float tap(const uint32_t* wv, int i) {
  if constexpr (sizeof(TW) == 4) {
    return __uint_as_float(wv[i]);
  } else if constexpr (sizeof(TW) == 2) {
    const uint16_t b = static_cast<uint16_t>(wv[i / 2] >> (16 * (i % 2)));
    return wdecode<TW>(__builtin_bit_cast(TW, b));
  } else {
    const uint8_t b = static_cast<uint8_t>(wv[i / 4] >> (8 * (i % 4)));
    return wdecode<TW>(fp8{b});
  }
}

__device__ inline uint32_t pack_h2(float a, float b) {
  const h2 v = {static_cast<_Float16>(a), static_cast<_Float16>(b)};
  return __builtin_bit_cast(uint32_t, v);
}

template <typename TW, int Q, int FT, bool PAIRS>
__global__ __launch_bounds__(256) void sspi_gather(const float* __restrict__ xiT, int64_t ldxi,
                                                   int PN, const int32_t* __restrict__ start,
                                                   const TW* __restrict__ w, int Qs,
                                                   const int2* __restrict__ win, int cap, int P,
                                                   int64_t J, int L, int nftiles,
                                                   float* __restrict__ z, int64_t ldz,
                                                   const int32_t* __restrict__ tlist, int ntl) {
  constexpr int STRIDE = FT + 4;  // LDS row stride in 32-bit words
  constexpr int QP = PAIRS ? (Q + 1) / 2 : Q;
  constexpr int C4 = FT / 4;      // 16-byte pieces per staged row
  extern __shared__ __attribute__((aligned(16))) uint32_t xs[];
  __shared__ int pbase[SSPI_MAX_CHUNK + 1];
  // every location tile, or the ntl tiles listed
  const int nj = tlist ? ntl : static_cast<int>((J + 255) / 256);
  int jt, ft;
  if (!xcd_tile(nj, nftiles, jt, ft)) return;
  if (tlist) jt = tlist[jt];
  const int tid = threadIdx.x;
  const int64_t j = static_cast<int64_t>(jt) * 256 + tid;
  const bool live = j < J;
  const int64_t jc = live ? j : J - 1;  // dead lanes read a valid record of this tile
  const int64_t l0 = static_cast<int64_t>(ft) * FT;
  constexpr int WORDS = (Q * static_cast<int>(sizeof(TW)) + 3) / 4;
  const int2* wt = win + static_cast<int64_t>(jt) * P;  // (first row, rows) per pair

  float acc[FT];
#pragma unroll
  for (int f = 0; f < FT; ++f) acc[f] = 0.0f;

  for (int p0 = 0; p0 < P;) {
    // chunk: consecutive pairs whose windows fit `cap` rows (one always fits)
    int rows = 0, p1 = p0;
    while (p1 < P && p1 - p0 < SSPI_MAX_CHUNK) {
      const int c = wt[p1].y;
      if (p1 > p0 && rows + c > cap) break;
      rows += c;
      ++p1;
    }
    __syncthreads();
    if (tid == 0) {
      int b = 0;
      for (int q = p0; q < p1; ++q) {
        pbase[q - p0] = b;
        b += wt[q].y;
      }
      pbase[p1 - p0] = b;
    }
    __syncthreads();
    // stage the windows, four 16-byte pieces in flight per thread; a row's
    // pair is found by bisection over the window offsets
    const int items = rows * C4;
    for (int e0 = 0; e0 < items; e0 += 4 * 256) {
      f32x4 a[4], bb[4];
      int dst[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * 256 + tid;
        a[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        bb[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        dst[u] = -1;
        if (e < items) {
          const int row = e / C4, c4 = e % C4;
          int lo = 0, hi = p1 - p0;  // pbase[lo] <= row < pbase[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pbase[mid] <= row) lo = mid; else hi = mid;
          }
          const int n = wt[p0 + lo].x + (row - pbase[lo]);
          const float* src = xiT + static_cast<int64_t>(n) * ldxi + l0 + 4 * c4;
          if (n >= 0 && n < PN) a[u] = *reinterpret_cast<const f32x4*>(src);
          if (PAIRS && n + 1 >= 0 && n + 1 < PN) bb[u] = *reinterpret_cast<const f32x4*>(src + ldxi);
          dst[u] = row * STRIDE + 4 * c4;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (dst[u] < 0) continue;
        u32x4 v;
        if (PAIRS) {
          v.x = pack_h2(a[u].x, bb[u].x);
          v.y = pack_h2(a[u].y, bb[u].y);
          v.z = pack_h2(a[u].z, bb[u].z);
          v.w = pack_h2(a[u].w, bb[u].w);
        } else {
          v = __builtin_bit_cast(u32x4, a[u]);
        }
        *reinterpret_cast<u32x4*>(xs + dst[u]) = v;
      }
    }
    __syncthreads();
    // starts and weights of the next group of GP pairs are loaded while the
    // current group is applied
    constexpr int GP = 4;
    int s_cur[GP], s_nxt[GP];
    uint32_t w_cur[GP][WORDS], w_nxt[GP][WORDS];
    auto fetch = [&](int pg, int (&sv)[GP], uint32_t (&wv)[GP][WORDS]) {
#pragma unroll
      for (int u = 0; u < GP; ++u) {
        const int p = min(pg + u, p1 - 1);  // past the chunk: a valid record, not applied
        const int64_t rec = static_cast<int64_t>(p) * J + jc;
        sv[u] = start[rec];
        const uint32_t* wsrc = reinterpret_cast<const uint32_t*>(w + rec * Qs);
#pragma unroll
        for (int i = 0; i < WORDS; ++i) wv[u][i] = wsrc[i];
      }
    };
    fetch(p0, s_cur, w_cur);
    for (int pg = p0; pg < p1; pg += GP) {
      if (pg + GP < p1) fetch(pg + GP, s_nxt, w_nxt);
#pragma unroll
      for (int u = 0; u < GP; ++u) {
        const int p = pg + u;
        if (p >= p1) break;  // uniform
        const int s = s_cur[u] - wt[p].x + pbase[p - p0];  // LDS row of tap 0
        const uint32_t* wv = w_cur[u];
        const uint32_t* rowp = xs + s * STRIDE;
        if (PAIRS) {
#pragma unroll
          for (int q2 = 0; q2 < QP; ++q2) {
            const float wa = tap<TW>(wv, 2 * q2);
            const float wb = 2 * q2 + 1 < Q ? tap<TW>(wv, 2 * q2 + 1) : 0.0f;
            const h2 wp = __builtin_bit_cast(h2, pack_h2(wa, wb));
            const uint32_t* r = rowp + 2 * q2 * STRIDE;
#pragma unroll
            for (int f4 = 0; f4 < FT / 4; ++f4) {
              const u32x4 e4 = *reinterpret_cast<const u32x4*>(r + 4 * f4);
              // elements are copied to scalars before the bit cast: hipcc 7.2
              // lowers __builtin_bit_cast of a vector swizzle (e4.y) to e4.x
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const uint32_t word = e4[i];
                acc[4 * f4 + i] = __builtin_amdgcn_fdot2(wp, __builtin_bit_cast(h2, word), acc[4 * f4 + i], false);
              }
            }
          }
        } else {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const float wq = tap<TW>(wv, q);
            const uint32_t* r = rowp + q * STRIDE;
#pragma unroll
            for (int f4 = 0; f4 < FT / 4; ++f4) {
              const f32x4 e4 = *reinterpret_cast<const f32x4*>(r + 4 * f4);
              acc[4 * f4 + 0] = __builtin_fmaf(wq, e4.x, acc[4 * f4 + 0]);
              acc[4 * f4 + 1] = __builtin_fmaf(wq, e4.y, acc[4 * f4 + 1]);
              acc[4 * f4 + 2] = __builtin_fmaf(wq, e4.z, acc[4 * f4 + 2]);
              acc[4 * f4 + 3] = __builtin_fmaf(wq, e4.w, acc[4 * f4 + 3]);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < GP; ++u) {
        s_cur[u] = s_nxt[u];
#pragma unroll
        for (int i = 0; i < WORDS; ++i) w_cur[u][i] = w_nxt[u][i];
      }
    }
    p0 = p1;
  }
  if (!live) return;
  constexpr float zs = 1.0f / sspi_wscale<TW>();
#pragma unroll
  for (int f = 0; f < FT; ++f) {
    const int64_t l = l0 + f;
    if (l < L) z[l * ldz + j] = acc[f] * zs;
  }
}

// ===================================================== SSPI band product ===
//
// z[l][j] = sum_p sum_{q < Q} w[p][j][q] xi[start(p, j) + q][l] (eq. (58))
// on the matrix cores, for apertures whose per-tile lag windows are too wide
// for the dense-window contraction.  For 256-candidate tile t and pair p the
// taps of the tile's candidates fall in the band of columns
// [A_tp, A_tp + W_tp) of the frame-major FP16 samples xb[l][n] (A_tp on a
// multiple of 8, n the stacked lag index), and those of 32-candidate
// subtile s in the narrower band [A_tp + o_tps, A_tp + o_tps + 16 k_tps).
// Tiles and subtiles are runs of a compact candidate order (balanced k-d
// splits of the grid, weighted by how fast the TDOAs change along each
// axis), which narrows the bands; the maps are written through that order.
// A block owns one tile and 128 frames (64 when a band is too wide for
// that).  Pairs go in passes (precomputed per
// tile) whose bands and records fit SB_LDS: a pass's bands for the 64
// frames, its candidates' tap records (tile-major copies made at plan time)
// and the next pass's band descriptors are loaded straight from global
// memory into LDS, every load in flight at once.  Wave s then multiplies,
// pair by pair, its subtile's band on v_mfma_f32_32x32x16_f16: A = 16 band
// columns of 32 frames, B = the 16 x 32 matrix holding each candidate's Q
// FP16 tap weights at its own rows and zeros elsewhere.  A lane shifts its
// packed taps once per pair into the two 8-row blocks they can touch and
// selects its block for each step; every frame group of the block uses it.  Every frame row goes through the same sequence of products, so
// a frame's map does not depend on the other frames of the block.
constexpr int SB_LDS = 72 * 1024;  // bands and records of one pass (two blocks per CU)
constexpr int SB_MAXPP = 32;    // pairs per pass at most (one descriptor load)

// Band descriptor of (tile, pair): the band (A, W) and per subtile s the
// offset o / 8 and 16-column steps k as sub[s] = (o / 8) | (k << 8)
// (k = 0: no live candidate).
struct BandDesc {
  int32_t A, W;
  uint16_t sub[8];
  uint32_t pad[2];
};
static_assert(sizeof(BandDesc) == 32, "two descriptors per 64-byte load pair");

// LDS row of a staged band of W columns, in 16-byte units: W + 16 columns
// (a subtile's steps reach up to 16 columns past W), made odd so that the 32
// rows of one read spread over the banks; every unit holds staged samples
// (the band is read that many columns wide)
__host__ __device__ constexpr int band_units(int W) { return ((W + 16) / 8) | 1; }

// LDS bytes of one pair in a pass: its band for the block's FR frames, the
// starts and the taps (QW 32-bit words) of the tile's 256 candidates
__host__ __device__ constexpr int band_pair_bytes(int W, int QW, int FR) {
  return FR * 16 * band_units(W) + 256 * 4 * (1 + QW);
}

typedef unsigned long long u64;

// One candidate's column of B holds its taps (packed FP16, tap i at bits
// 16 i of the 128-bit lo:hi) at rows rel .. rel + Q - 1 and zeros elsewhere,
// so only the 8-row blocks rel / 8 and rel / 8 + 1 can be non-zero: the tap
// vector shifted by 16 (rel % 8) bits, low 128 bits in f0, the rest in f1.
// Explicit selects for shifts of 64 bits and more (the hardware takes
// 64-bit shift amounts modulo 64).
__device__ inline void band_blocks(u64 lo, u64 hi, int d, i32x4& f0, i32x4& f1) {
  const int sh = 16 * d;  // 0 .. 112
  u64 a, b, c, e;
  if (sh == 0) {
    a = lo;
    b = hi;
    c = e = 0;
  } else if (sh < 64) {
    a = lo << sh;
    b = (hi << sh) | (lo >> (64 - sh));
    c = hi >> (64 - sh);
    e = 0;
  } else if (sh == 64) {
    a = 0;
    b = lo;
    c = hi;
    e = 0;
  } else {
    a = 0;
    b = lo << (sh - 64);
    c = (hi << (sh - 64)) | (lo >> (128 - sh));
    e = hi >> (128 - sh);
  }
  f0 = i32x4{static_cast<int>(a), static_cast<int>(a >> 32), static_cast<int>(b), static_cast<int>(b >> 32)};
  f1 = i32x4{static_cast<int>(c), static_cast<int>(c >> 32), static_cast<int>(e), static_cast<int>(e >> 32)};
}

__device__ inline void lds_dma16(const void* src, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

template <int QW, int FR>
__global__ __launch_bounds__(512) void sspi_band(const _Float16* __restrict__ xb, int64_t ldb, int Lrows,
                                                 const int32_t* __restrict__ rstart,
                                                 const uint32_t* __restrict__ rtaps,
                                                 const BandDesc* __restrict__ desc,
                                                 const uint16_t* __restrict__ bnext,
                                                 const int32_t* __restrict__ order, int P, int64_t J, int L,
                                                 int nftiles, float* __restrict__ z, int64_t ldz) {
  static_assert(QW == 2 || QW == 4, "taps are packed in two or four words");
  static_assert(FR == 64 || FR == 128, "two or four frame groups of 32");
  constexpr int NG = FR / 32;
  extern __shared__ __attribute__((aligned(16))) unsigned char sb_lds[];
  unsigned char* dbuf = sb_lds;                              // [2][SB_MAXPP] descriptors
  unsigned char* region = sb_lds + 2 * SB_MAXPP * sizeof(BandDesc);
  const int njt = static_cast<int>((J + 255) / 256);
  int jt, ft;
  if (!xcd_tile(njt, nftiles, jt, ft)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r32 = lane & 31, kq = lane >> 5;
  const int cand = wave * 32 + r32;
  const int64_t pos = static_cast<int64_t>(jt) * 256 + cand;  // position in the compact order
  const bool live = pos < J;
  const int64_t l0 = static_cast<int64_t>(ft) * FR;
  const int64_t tp0 = static_cast<int64_t>(jt) * P;  // (tile, pair 0)
  const int64_t ndesc = static_cast<int64_t>(njt) * P;
  const uint16_t* nx = bnext + tp0;
  // descriptors of the first pass
  if (wave == 0 && 2 * tp0 + lane < 2 * ndesc)
    lds_dma16(reinterpret_cast<const unsigned char*>(desc + tp0) + 16 * lane, dbuf);

  f32x16 acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[g][v] = 0.0f;
  int cur = 0;
  for (int p0 = 0; p0 < P; cur ^= 1) {
    const int p1 = nx[p0];
    const int np = p1 - p0;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // the previous pass's reads are done; this pass's descriptors are in
    const BandDesc* dc = reinterpret_cast<const BandDesc*>(dbuf + cur * SB_MAXPP * sizeof(BandDesc));
    // bands: pair q's band is u 16-byte pieces per frame, item i = f u + c at
    // byte 16 i of its part of the region; each wave issues every 8th chunk
    // of 64 items
    int off = 0;
    for (int k = 0; k < np; ++k) {
      const int A = dc[k].A, u = band_units(dc[k].W);
      const int items = FR * u;
      const float inv = 1.0f / static_cast<float>(u);
      for (int c0 = 64 * wave; c0 < items; c0 += 512) {
        const int i = c0 + lane;
        // i / u exactly: i < 128 u and the quotient's fraction is >= 1 / (2 u)
        const int f = static_cast<int>((static_cast<float>(i) + 0.5f) * inv);
        const int c = i - f * u;
        const int64_t row = min(l0 + f, static_cast<int64_t>(Lrows - 1));  // rows past the frames are not stored
        if (i < items) lds_dma16(xb + row * ldb + A + 8 * c, region + off + 16 * c0);
      }
      off += 16 * items;
    }
    // records: starts (1 KB per pair) and taps (QW KB per pair), contiguous
    // for the pass's pairs in the tile-major copies
    unsigned char* rs = region + off;
    unsigned char* rw = rs + 1024 * np;
    const unsigned char* gs = reinterpret_cast<const unsigned char*>(rstart + (tp0 + p0) * 256);
    const unsigned char* gw = reinterpret_cast<const unsigned char*>(rtaps + (tp0 + p0) * 256 * QW);
    for (int c0 = wave; c0 < np * (1 + QW); c0 += 8) {
      if (c0 < np)
        lds_dma16(gs + 1024 * c0 + 16 * lane, rs + 1024 * c0);
      else
        lds_dma16(gw + 1024 * (c0 - np) + 16 * lane, rw + 1024 * (c0 - np));
    }
    // descriptors of the next pass (32, past P harmless)
    if (wave == 0 && p1 < P && 2 * (tp0 + p1) + lane < 2 * ndesc)
      lds_dma16(reinterpret_cast<const unsigned char*>(desc + tp0 + p1) + 16 * lane,
                dbuf + (cur ^ 1) * SB_MAXPP * sizeof(BandDesc));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    off = 0;
    for (int k = 0; k < np; ++k) {
      const int A = dc[k].A, u = band_units(dc[k].W);
      const uint32_t e = dc[k].sub[wave];
      const int o = 8 * static_cast<int>(e & 0xffu), ks = static_cast<int>(e >> 8);
      const int s_c = reinterpret_cast<const int32_t*>(rs)[k * 256 + cand];
      u64 lo = 0, hi = 0;
      if constexpr (QW == 2) {
        lo = reinterpret_cast<const u64*>(rw)[k * 256 + cand];
      } else {
        lo = reinterpret_cast<const u64*>(rw)[2 * (k * 256 + cand)];
        hi = reinterpret_cast<const u64*>(rw)[2 * (k * 256 + cand) + 1];
      }
      const int rel = s_c - A - o;  // row of tap 0 in the subtile's band (>= 0)
      i32x4 f0, f1;
      band_blocks(lo, hi, rel & 7, f0, f1);
      const int b0 = rel >> 3;  // the 8-row block of f0
      const unsigned char* ar = region + off + r32 * u * 16 + (o + 8 * kq) * 2;
      for (int kk = 0; kk < ks; ++kk) {
        const int bi = 2 * kk + kq;  // this lane's 8-row block of the step
        i32x4 bf;
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) bf[e2] = bi == b0 ? f0[e2] : (bi == b0 + 1 ? f1[e2] : 0);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const i32x4 af = *reinterpret_cast<const i32x4*>(ar + g * 32 * u * 16 + 32 * kk);
          acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, af),
                                                          __builtin_bit_cast(f16x8, bf), acc[g], 0, 0, 0);
        }
      }
      off += FR * 16 * u;
    }
    p0 = p1;
  }
  if (!live) return;
  const int64_t j = order[pos];
  // register v of lane i: frame 8 (v / 4) + 4 (i / 32) + v % 4 of the group,
  // candidate i % 32
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t l = l0 + 32 * g + 8 * (v / 4) + 4 * kq + (v % 4);
      if (l < L) z[l * ldz + j] = acc[g][v];
    }
}

// Band descriptors from the tile-major records: block (t, p), one thread per
// candidate of tile t.  A rounded down and A + W up to multiples of 8; subtile s's taps
// lie in [A + o, A + o + 16 k), o a multiple of 8.
__global__ __launch_bounds__(256) void sspi_band_tables(const int32_t* __restrict__ rstart, int64_t J, int Q,
                                                        int P, BandDesc* __restrict__ desc) {
  __shared__ int lo_s[8], hi_s[8];
  const int t = blockIdx.x, p = blockIdx.y;
  const int tid = threadIdx.x;
  const bool live = static_cast<int64_t>(t) * 256 + tid < J;
  const int s = live ? rstart[(static_cast<int64_t>(t) * P + p) * 256 + tid] : 0;
  int lo = live ? s : INT_MAX, hi = live ? s + Q : INT_MIN;
  // min / max over each 32-candidate subtile
  for (int m = 16; m >= 1; m >>= 1) {
    lo = min(lo, __shfl_xor(lo, m, 32));
    hi = max(hi, __shfl_xor(hi, m, 32));
  }
  if ((tid & 31) == 0) {
    lo_s[tid >> 5] = lo;
    hi_s[tid >> 5] = hi;
  }
  __syncthreads();
  int blo = INT_MAX, bhi = INT_MIN;
  for (int i = 0; i < 8; ++i) {
    blo = min(blo, lo_s[i]);
    bhi = max(bhi, hi_s[i]);
  }
  // tile t holds at least one live candidate, so blo <= bhi
  const int A = blo - blo % 8;  // starts are >= 0
  const int W = (bhi - A + 7) / 8 * 8;
  BandDesc* d = desc + static_cast<int64_t>(t) * P + p;
  if (tid == 0) {
    d->A = A;
    d->W = W;
    d->pad[0] = d->pad[1] = 0u;
  }
  if (tid < 8) {
    const int sl = lo_s[tid], sh = hi_s[tid];
    uint16_t e = 0;
    if (sl <= sh) {
      const int o = (sl - A) / 8 * 8;
      const int k = (sh - A - o + 15) / 16;
      e = static_cast<uint16_t>((o / 8) | (k << 8));
    }
    d->sub[tid] = e;
  }
}

// Passes of the band product: per tile, consecutive pairs (at most
// SB_MAXPP) whose bands and records fit SB_LDS (one always does);
// bnext[t][p0] = the first pair after the pass that starts at p0.  One
// thread per tile.
__global__ __launch_bounds__(256) void sspi_band_passes(const BandDesc* __restrict__ desc, int njt, int P, int QW,
                                                        int FR, uint16_t* __restrict__ bnext) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= njt) return;
  const BandDesc* dt = desc + static_cast<int64_t>(t) * P;
  for (int p0 = 0; p0 < P;) {
    int bytes = 0, p1 = p0;
    while (p1 < P && p1 - p0 < SB_MAXPP) {
      const int b = band_pair_bytes(dt[p1].W, QW, FR);
      if (p1 > p0 && bytes + b > SB_LDS) break;
      bytes += b;
      ++p1;
    }
    bnext[static_cast<int64_t>(t) * P + p0] = static_cast<uint16_t>(p1);
    p0 = p1;
  }
}

// Tile-major records of the band product: rstart[t][p][c] and the taps as
// packed FP16, QW words each, of candidate order[t 256 + c] (zeros for
// positions past J and taps past Q).
template <typename TW>
__global__ __launch_bounds__(256) void sspi_band_records(const int32_t* __restrict__ start,
                                                         const TW* __restrict__ w, int Qs, int Q, int64_t J,
                                                         int P, int QW, const int32_t* __restrict__ order,
                                                         int32_t* __restrict__ rstart,
                                                         uint32_t* __restrict__ rtaps) {
  const int t = blockIdx.x, p = blockIdx.y, c = threadIdx.x;
  const int64_t pos = static_cast<int64_t>(t) * 256 + c;
  const int64_t dst = (static_cast<int64_t>(t) * P + p) * 256 + c;
  uint32_t v[4] = {0u, 0u, 0u, 0u};
  int s = 0;
  if (pos < J) {
    const int64_t j = order[pos];
    const int64_t rec = static_cast<int64_t>(p) * J + j;
    s = start[rec];
    for (int i = 0; i < Q; ++i) {
      const _Float16 h = static_cast<_Float16>(static_cast<float>(w[rec * Qs + i]));
      v[i / 2] |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h)) << (16 * (i % 2));
    }
  }
  rstart[dst] = s;
  for (int k = 0; k < QW; ++k) rtaps[dst * QW + k] = v[k];
}

// xb[l][n] = xi[n][l] in FP16 for n < PN, zero for PN <= n < XB (frame-major
// samples of the band product), from the lag-major samples xiT [PN][ldxi].
__global__ __launch_bounds__(256) void xi_rows16(const float* __restrict__ xiT, int64_t ldxi, int L, int PN,
                                                 int XB, _Float16* __restrict__ xb, int64_t ldb) {
  __shared__ float t[32][33];
  const int n0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int n = n0 + r, l = l0 + tx;
    t[r][tx] = (n < PN && l < L) ? xiT[static_cast<int64_t>(n) * ldxi + l] : 0.0f;
  }
  __syncthreads();
  const int n = n0 + tx;
  if (n >= XB) return;
  for (int r = ty; r < 32; r += 8) {
    const int l = l0 + r;
    if (l < L) xb[static_cast<int64_t>(l) * ldb + n] = static_cast<_Float16>(t[tx][r]);
  }
}

// The same from the frame-major samples of the iFFT kernel, part [L][PN].
__global__ __launch_bounds__(256) void rows_to_f16(const float* __restrict__ part, int64_t ldp, int L, int PN,
                                                   int XB, _Float16* __restrict__ xb, int64_t ldb) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t l = i / XB, n = i % XB;
  if (l >= L) return;
  xb[l * ldb + n] = n < PN ? static_cast<_Float16>(part[l * ldp + n]) : static_cast<_Float16>(0.0f);
}

// ================================================== plan-time kernels =====

// sinc(x - n) for integer n with the argument reduced exactly: x = k0 + r,
// |r| <= 1/2, sin(pi (x - n)) = (-1)^(k0 + n) sin(pi r).  sr = sin(pi r)
// is shared by every n of one x.
__device__ inline double sinc_red(double x, double k0, double sr, int n) {
  const double d = x - static_cast<double>(n);
  if (d == 0.0) return 1.0;
  const long long par = (static_cast<long long>(k0) + n) & 1LL;
  return (par ? -sr : sr) / (M_PI * d);
}

// Gram matrices G_p = Lambda_p^T Lambda_p (eq. (54) per pair: its right
// singular vectors are the eigenvectors of G_p) in FP64 on
// v_mfma_f64_16x16x4_f64, Lambda_p[j][a] = sinc(x_p(j) - (a - N_p))
// generated in registers.  Block = one 64 x 64 tile (ta <= tb) of one pair,
// looping over all J; both the tile and its mirror are written to
// G [P][nmax][nmax].  Lane i supplies row i % 16 and k slot (candidate)
// i / 16 of each 4-candidate step; accumulator register v of lane i holds
// row 4 v + i / 16, column i % 16.
__global__ __launch_bounds__(256) void gram_f64(const double* __restrict__ x, int64_t J,
                                                const int32_t* __restrict__ np, int nmax, int ntile,
                                                double* __restrict__ G) {
  int t = blockIdx.x, ta = 0;
  while (t >= ntile - ta) {
    t -= ntile - ta;
    ++ta;
  }
  const int tb = ta + t;
  const int p = blockIdx.y;
  const int npp = np[p], n = 2 * npp + 1;
  if (tb * 64 >= n) return;  // block-uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wx = (wave >> 1) * 32, ww = (wave & 1) * 32;
  const int r16 = lane & 15, g = lane >> 4;
  int ra[2], cb[2];
  for (int a = 0; a < 2; ++a) ra[a] = ta * 64 + wx + a * 16 + r16;
  for (int b = 0; b < 2; ++b) cb[b] = tb * 64 + ww + b * 16 + r16;
  f64x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  const double* xp = x + static_cast<int64_t>(p) * J;
  for (int64_t j0 = 0; j0 < J; j0 += 4) {
    const int64_t j = j0 + g;
    const bool ok = j < J;
    const double xv = ok ? xp[j] : 0.0;
    const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
    double fa[2], fb[2];
    for (int a = 0; a < 2; ++a) fa[a] = (ok && ra[a] < n) ? sinc_red(xv, k0, sr, ra[a] - npp) : 0.0;
    for (int b = 0; b < 2; ++b) fb[b] = (ok && cb[b] < n) ? sinc_red(xv, k0, sr, cb[b] - npp) : 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  double* Gp = G + static_cast<int64_t>(p) * nmax * nmax;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int col = cb[b];
      if (col >= n) continue;
      for (int v = 0; v < 4; ++v) {
        const int row = ta * 64 + wx + a * 16 + 4 * v + g;
        if (row >= n) continue;
        Gp[static_cast<int64_t>(row) * nmax + col] = acc[a][b][v];
        Gp[static_cast<int64_t>(col) * nmax + row] = acc[a][b][v];
      }
    }
}

// U_p = Lambda_p V_p (eq. (54): left singular vectors times singular values)
// into the FP32 staging matrix Us [Jpad][Kc] at columns p R + r.  One thread
// per candidate; V_p is staged in LDS 512 rows x 8 columns at a time; FP64
// sums.
__global__ __launch_bounds__(256) void slri_u_f64(const double* __restrict__ x, int64_t J,
                                                  const int32_t* __restrict__ np, int nmax, int R,
                                                  const double* __restrict__ V, float* __restrict__ Us, int Kc) {
  constexpr int AR = 512;
  __shared__ double vs[AR * 8];
  const int p = blockIdx.y;
  const int npp = np[p], n = 2 * npp + 1;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const double xv = j < J ? x[static_cast<int64_t>(p) * J + j] : 0.0;
  const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
  const double* Vp = V + static_cast<int64_t>(p) * nmax * R;
  for (int r0 = 0; r0 < R; r0 += 8) {
    const int rc = min(8, R - r0);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a0 = 0; a0 < n; a0 += AR) {
      const int an = min(AR, n - a0);
      __syncthreads();
      for (int e = threadIdx.x; e < an * 8; e += 256) {
        const int a = e / 8, c = e % 8;
        vs[e] = c < rc ? Vp[static_cast<int64_t>(a0 + a) * R + r0 + c] : 0.0;
      }
      __syncthreads();
      if (j < J) {
        for (int a = 0; a < an; ++a) {
          const double lam = sinc_red(xv, k0, sr, a0 + a - npp);
#pragma unroll
          for (int c = 0; c < 8; ++c) acc[c] = fma(lam, vs[a * 8 + c], acc[c]);
        }
      }
    }
    if (j < J) {
      float* dst = Us + j * Kc + p * R + r0;
      for (int c = 0; c < rc; ++c) dst[c] = static_cast<float>(acc[c]);
    }
  }
}

// Gram matrix G = Lambda^T Lambda of the stacked J x PN interpolation
// matrix (43) for the global fit of (54).  Same tiling and MFMA lane layout
// as gram_f64; stacked column a belongs to pair pa[a] at lag la[a], so every
// lane evaluates its own rows' sinc from that pair's TDOA.  Block = one
// 64 x 64 tile (ta <= tb) over candidates [j0, j1) of split blockIdx.y;
// partial tiles go to G [split][PN][PN] (summed on the host).
__global__ __launch_bounds__(256) void gram_global_f64(const double* __restrict__ x, int64_t J,
                                                       const int32_t* __restrict__ pa,
                                                       const int32_t* __restrict__ la, int PN, int ntile,
                                                       int64_t jchunk, double* __restrict__ G) {
  int t = blockIdx.x, ta = 0;
  while (t >= ntile - ta) {
    t -= ntile - ta;
    ++ta;
  }
  const int tb = ta + t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wx = (wave >> 1) * 32, ww = (wave & 1) * 32;
  const int r16 = lane & 15, g = lane >> 4;
  int ra[2], cb[2];
  const double* xa[2];
  const double* xb[2];
  int na[2], nb[2];
  for (int a = 0; a < 2; ++a) {
    ra[a] = ta * 64 + wx + a * 16 + r16;
    const int rr = min(ra[a], PN - 1);
    xa[a] = x + static_cast<int64_t>(pa[rr]) * J;
    na[a] = la[rr];
  }
  for (int b = 0; b < 2; ++b) {
    cb[b] = tb * 64 + ww + b * 16 + r16;
    const int cc = min(cb[b], PN - 1);
    xb[b] = x + static_cast<int64_t>(pa[cc]) * J;
    nb[b] = la[cc];
  }
  f64x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * jchunk;
  const int64_t j1 = min(J, j0 + jchunk);
  for (int64_t jb = j0; jb < j1; jb += 4) {
    const int64_t j = jb + g;
    const bool ok = j < j1;
    double fa[2], fb[2];
    for (int a = 0; a < 2; ++a) {
      const double xv = ok ? xa[a][j] : 0.0;
      const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
      fa[a] = (ok && ra[a] < PN) ? sinc_red(xv, k0, sr, na[a]) : 0.0;
    }
    for (int b = 0; b < 2; ++b) {
      const double xv = ok ? xb[b][j] : 0.0;
      const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
      fb[b] = (ok && cb[b] < PN) ? sinc_red(xv, k0, sr, nb[b]) : 0.0;
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  double* Gs = G + static_cast<int64_t>(blockIdx.y) * PN * PN;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int col = cb[b];
      if (col >= PN) continue;
      for (int v = 0; v < 4; ++v) {
        const int row = ta * 64 + wx + a * 16 + 4 * v + g;
        if (row >= PN) continue;
        Gs[static_cast<int64_t>(row) * PN + col] = acc[a][b][v];
        Gs[static_cast<int64_t>(col) * PN + row] = acc[a][b][v];
      }
    }
}

// U = Lambda V for the global fit (left singular vectors times singular
// values) into the FP32 staging matrix Us [Jpad][Kc], columns 0..R-1.  One
// thread per candidate and 8 columns per pass; pair by pair, the TDOA and
// its reduced sine are formed once and V's rows of that pair staged in LDS.
__global__ __launch_bounds__(256) void slri_u_global_f64(const double* __restrict__ x, int64_t J,
                                                         const int32_t* __restrict__ np,
                                                         const int32_t* __restrict__ off, int P, int R,
                                                         const double* __restrict__ V, float* __restrict__ Us,
                                                         int Kc) {
  constexpr int AR = 576;  // >= 2 N_p + 1 of every pair (checked on the host)
  __shared__ double vs[AR * 8];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int r0 = blockIdx.y * 8;
  const int rc = min(8, R - r0);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = 0; p < P; ++p) {
    const int npp = np[p], n = 2 * npp + 1;
    __syncthreads();
    for (int e = threadIdx.x; e < n * 8; e += 256) {
      const int a = e / 8, c = e % 8;
      vs[e] = c < rc ? V[static_cast<int64_t>(off[p] + a) * R + r0 + c] : 0.0;
    }
    __syncthreads();
    if (j < J) {
      const double xv = x[static_cast<int64_t>(p) * J + j];
      const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
      for (int a = 0; a < n; ++a) {
        const double lam = sinc_red(xv, k0, sr, a - npp);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fma(lam, vs[a * 8 + c], acc[c]);
      }
    }
  }
  if (j < J) {
    float* dst = Us + j * Kc + r0;
    for (int c = 0; c < rc; ++c) dst[c] = static_cast<float>(acc[c]);
  }
}

// C = Lambda B (TR = false: M = J candidates, K = stacked lags) or
// C = Lambda^T B (TR = true: M = stacked lags, K = candidates) in FP64 on
// v_mfma_f64_16x16x4_f64, with Lambda[j][a] = sinc(x_p(j) - n) of (43)
// generated in registers: the products of the randomized global fit.  The
// stacked lag axis is padded per pair to 16-slot chunks (chunk c: pair
// cpair[c], lags clag0[c] .. clag0[c] + 15, valid up to N_p = cnp[c];
// padding slots are zero), so a 16-deep K chunk (TR = false) or a 16-row
// group (TR = true) belongs to one pair.  Block = one 64 x 64 tile of C,
// four waves of 32 x 32 (2 x 2 MFMA tiles); B rows staged through LDS per
// 16-deep chunk.  TR = false: each lane forms x, its rounding and
// sin(pi r) once per chunk for its two rows; TR = true: the chunk's
// (x, k0, sin pi r) for each row group's pair and each of the 16
// candidates are formed once in LDS.  Lane i supplies row i % 16 and k slot
// i / 16 of each 4-deep step; accumulator register v of lane i holds row
// 4 v + i / 16, column i % 16.  Rows of B past K hold zeros.
template <bool TR>
__global__ __launch_bounds__(256) void lam_gemm_f64(const double* __restrict__ x, int64_t J,
                                                    const int32_t* __restrict__ cpair,
                                                    const int32_t* __restrict__ clag0,
                                                    const int32_t* __restrict__ cnp, int64_t M, int64_t Kd,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ C, int64_t ldc, int ntn) {
  __shared__ double bs[16][64 + 2];
  __shared__ double gxs[4][16], gks[4][16], gss[4][16];
  const int tn = static_cast<int>(blockIdx.x % ntn);
  const int64_t m0 = static_cast<int64_t>(blockIdx.x / ntn) * 64;
  const int n0 = tn * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int r16 = lane & 15, kq = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  // TR: this lane's two rows (stacked slots): pair and lag, fixed
  int tpair[2] = {0, 0}, tlag[2] = {0, 0};
  bool tval[2] = {false, false};
  if constexpr (TR) {
#pragma unroll
    for (int ms = 0; ms < 2; ++ms) {
      const int64_t a = m0 + wm * 32 + ms * 16 + r16;
      if (a < M) {
        const int64_t c = a / 16;
        tpair[ms] = cpair[c];
        tlag[ms] = clag0[c] + static_cast<int>(a % 16);
        tval[ms] = tlag[ms] <= cnp[c];
      }
    }
  }
  for (int64_t k0 = 0; k0 < Kd; k0 += 16) {
    __syncthreads();
    {
      const int r = tid >> 4, cc = 4 * (tid & 15);
      const double* src = B + (k0 + r) * ldb + n0 + cc;
#pragma unroll
      for (int e = 0; e < 4; ++e) bs[r][cc + e] = src[e];
    }
    double xv[2] = {0.0, 0.0}, kr[2] = {0.0, 0.0}, sr[2] = {0.0, 0.0};
    int lag0 = 0, npp = 0;
    if constexpr (!TR) {
      const int64_t c = k0 / 16;
      const int p = cpair[c];
      lag0 = clag0[c];
      npp = cnp[c];
#pragma unroll
      for (int ms = 0; ms < 2; ++ms) {
        const int64_t j = m0 + wm * 32 + ms * 16 + r16;
        xv[ms] = j < J ? x[static_cast<int64_t>(p) * J + j] : 0.0;
        kr[ms] = rint(xv[ms]);
        sr[ms] = sin(M_PI * (xv[ms] - kr[ms]));
      }
    } else {
      if (tid < 64) {
        const int g = tid >> 4, jj = tid & 15;
        const int64_t a = m0 + 16 * g, j = k0 + jj;
        double v = 0.0;
        if (a < M && j < J) v = x[static_cast<int64_t>(cpair[a / 16]) * J + j];
        gxs[g][jj] = v;
        gks[g][jj] = rint(v);
        gss[g][jj] = sin(M_PI * (v - rint(v)));
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double av[2], bv[2];
#pragma unroll
      for (int ms = 0; ms < 2; ++ms) {
        if constexpr (!TR) {
          const int64_t j = m0 + wm * 32 + ms * 16 + r16;
          const int n = lag0 + 4 * s + kq;
          av[ms] = (j < J && n <= npp) ? sinc_red(xv[ms], kr[ms], sr[ms], n) : 0.0;
        } else {
          const int g = 2 * wm + ms, jj = 4 * s + kq;
          av[ms] = (tval[ms] && k0 + jj < J) ? sinc_red(gxs[g][jj], gks[g][jj], gss[g][jj], tlag[ms]) : 0.0;
        }
      }
#pragma unroll
      for (int ns = 0; ns < 2; ++ns) bv[ns] = bs[4 * s + kq][wn * 32 + ns * 16 + r16];
#pragma unroll
      for (int ms = 0; ms < 2; ++ms)
#pragma unroll
        for (int ns = 0; ns < 2; ++ns)
          acc[ms][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ms], bv[ns], acc[ms][ns], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ms = 0; ms < 2; ++ms)
#pragma unroll
    for (int ns = 0; ns < 2; ++ns)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 32 + ms * 16 + 4 * v + kq;
        const int col = n0 + wn * 32 + ns * 16 + r16;
        if (row < M) C[row * ldc + col] = acc[ms][ns][v];
      }
}

// max |U_p| over the staged columns of pair p (per-pair FP8 scale).
__global__ __launch_bounds__(256) void pair_absmax(const float* __restrict__ Us, int64_t J, int Kc, int R,
                                                   float* __restrict__ out) {
  __shared__ float red[256];
  const int p = blockIdx.x;
  float m = 0.0f;
  for (int64_t e = threadIdx.x; e < J * R; e += 256)
    m = fmaxf(m, fabsf(Us[(e / R) * Kc + p * R + e % R]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = red[0];
}

// Us[:, p R .. p R + R) *= inv_sigma[p]
__global__ void scale_pairs(float* __restrict__ Us, int64_t rows, int Kc, int R, int P,
                            const float* __restrict__ inv_sigma) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= rows * Kc) return;
  const int col = static_cast<int>(i % Kc);
  if (col < P * R) Us[i] *= inv_sigma[col / R];
}

// SSPI windows (eq. (55) per row and pair): the Q_p integers nearest to x,
// clamped to [-N_p, N_p], start = clamp(ceil(x - Q_p / 2), -N_p,
// N_p - Q_p + 1), weights sinc(x - n) in FP64 rounded once to FP32 and then
// to the weight type; records [P][J] (absolute stacked lag) and [P][J][Qs].
// A block covers the 256 candidates of one gather tile and one pair and also
// writes the tile's lag window win[tile][p] = (first row, rows): every row a
// candidate of the tile reads.
template <typename TW>
__global__ __launch_bounds__(256) void sspi_windows(const double* __restrict__ x, int64_t J,
                                                    const int32_t* __restrict__ np, const int32_t* __restrict__ off,
                                                    int Qsel, int Q, int Qs, int P, int td,
                                                    const int32_t* __restrict__ gstart,
                                                    const int32_t* __restrict__ gcount, int32_t* __restrict__ start,
                                                    TW* __restrict__ w, int2* __restrict__ win) {
  __shared__ int rlo[256], rhi[256];
  const int p = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int npp = np[p];
  int q = min(Qsel, 2 * npp + 1);
  int sabs_lo = 0x7fffffff, sabs_hi = -0x7fffffff;
  if (j < J) {
    const double xv = x[static_cast<int64_t>(p) * J + j];
    const int64_t rec = static_cast<int64_t>(p) * J + j;
    double s = ceil(xv - 0.5 * q);
    s = fmin(fmax(s, static_cast<double>(-npp)), static_cast<double>(npp - q + 1));
    // conv. TD-SRP (23): the lag nearest to x, half away from zero, kept in
    // the sampled range [-N_p, N_p] (with N_aux = 0 an endfire candidate can
    // round to N_p + 1)
    if (td) s = fmin(fmax(copysign(floor(fabs(xv) + 0.5), xv), static_cast<double>(-npp)),
                     static_cast<double>(npp));
    // global selection: the window chosen on the host
    if (gstart) {
      s = gstart[rec];
      q = gcount[rec];
    }
    const int si = static_cast<int>(s);
    const int sabs = off[p] + si + npp;
    start[rec] = sabs;
    sabs_lo = sabs_hi = sabs;
    const double k0 = rint(xv), sr = sin(M_PI * (xv - k0));
    for (int t2 = 0; t2 < Qs; ++t2) {
      float v = t2 < q ? static_cast<float>(sinc_red(xv, k0, sr, si + t2)) : 0.0f;
      if (td) v = t2 == 0 ? 1.0f : 0.0f;
      w[rec * Qs + t2] = cvt<TW>(v * sspi_wscale<TW>());
    }
  }
  rlo[threadIdx.x] = sabs_lo;
  rhi[threadIdx.x] = sabs_hi;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      rlo[threadIdx.x] = min(rlo[threadIdx.x], rlo[threadIdx.x + h]);
      rhi[threadIdx.x] = max(rhi[threadIdx.x], rhi[threadIdx.x + h]);
    }
    __syncthreads();
  }
  // the gather reads Q taps from every start (taps past q_p carry zero
  // weight), so the staged window covers Q rows past the last start; rows
  // past PN are staged as zeros
  if (threadIdx.x == 0) win[static_cast<int64_t>(blockIdx.x) * P + p] = make_int2(rlo[0], rhi[0] + Q - rlo[0]);
}

// Steering operand of conv. FD-SRP: H[j * ldh + p Kp + 2 (k-1) + {0,1}] =
// (cos theta, -sin theta), theta = pi k x_p(j) / K (eq. (19) with (14)),
// row-major, or tile-major (fd16_tiled) for the FD GEMM (FP32, 16-bit, FP8).  The
// phase is reduced in FP64: theta = 2 pi (t - rint(t)), t = k x / (2K), and
// sin/cos come from the FP64 sincospi.  Rows j >= J and slots k >= K are 0.
template <typename T>
__global__ void build_steering(const double* __restrict__ x, int P, int64_t J, int K, int Kp, int64_t ldh,
                               bool tiled, T* __restrict__ H) {
  const int64_t j = blockIdx.x;
  const int slots = Kp / 2;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= P * slots) return;
  const int p = e / slots, kk = e % slots;
  const int k = kk + 1;
  double c = 0.0, s = 0.0;
  if (j < J && k <= K - 1) {
    const double t = static_cast<double>(k) * x[static_cast<int64_t>(p) * J + j] / (2.0 * K);
    const double r = t - rint(t);
    sincospi(2.0 * r, &s, &c);
  }
  // (re, im) share a 16-byte chunk, so the tiled layout keeps them adjacent
  const int64_t e0 = static_cast<int64_t>(p) * Kp + 2 * kk;
  T* h = tiled ? reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(H) +
                                      fd16_tiled(j, e0 * static_cast<int64_t>(sizeof(T)), ldh * static_cast<int64_t>(sizeof(T))))
               : H + j * ldh + e0;
  h[0] = cvt64<T>(c);
  h[1] = cvt64<T>(-s);
}

// The complex steering matrix of LR-SRP in FP64, H[j][p (K-1) + k - 1] =
// exp(i theta), theta = pi k x_p(j) / K (eq. (19)), reduced as in
// build_steering; row-major [J][P (K-1)] (a column-major P (K-1) x J matrix
// for the BLAS calls of the fit).
__global__ void build_h_c64(const double* __restrict__ x, int P, int64_t J, int K, double2* __restrict__ H) {
  const int64_t j = blockIdx.x;
  const int n = P * (K - 1);
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= n) return;
  const int p = e / (K - 1), k = e % (K - 1) + 1;
  const double t = static_cast<double>(k) * x[static_cast<int64_t>(p) * J + j] / (2.0 * K);
  const double r = t - rint(t);
  double sn, cs;
  sincospi(2.0 * r, &sn, &cs);
  H[j * n + e] = make_double2(cs, sn);
}

// dst = src * s, narrowed to the operand type (the LR fat-stage output).
template <typename T>
__global__ void scale_convert(const float* __restrict__ src, T* __restrict__ dst, int64_t n, float s) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) dst[i] = cvt<T>(src[i] * s);
}

template <typename T>
__global__ void convert_f32(const float* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) dst[i] = cvt<T>(src[i]);
}

// xi^T [PN][ld] -> xi [L][PN]
__global__ void transpose_xi(const float* __restrict__ xiT, int64_t ld, int PN, int L,
                             float* __restrict__ xi) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= static_cast<int64_t>(PN) * L) return;
  const int64_t l = i / PN, n = i % PN;
  xi[i] = xiT[n * ld + l];
}

// ================================================================ host ====

namespace {

size_t dsize(int dtype) {
  switch (dtype) {
    case SRP_F32: return 4;
    case SRP_BF16: return 2;
    case SRP_F16: return 2;
    case SRP_FP8_E4M3: return 1;
    case SRP_F64: return 8;
  }
  return 4;
}

template <typename T>
void launch_steering(const double* d_x, const HostPlan& hp, int Kp, int64_t Jpad, int64_t ldh, void* H) {
  // the FP32, 16-bit and FP8 GEMM (gemm_fd16) reads the tile-major layout
  const bool tiled = sizeof(T) <= 4;
  if (tiled && ((ldh * static_cast<int64_t>(sizeof(T))) % FD16_SB != 0 || Jpad % FD16_TILE != 0))
    throw Error{SRP_E_UNSUPPORTED, "steering rows are not whole 64-byte stages of 256-row tiles"};
  dim3 grid(static_cast<unsigned>(Jpad), (hp.P * (Kp / 2) + 255) / 256);
  hipLaunchKernelGGL(build_steering<T>, grid, dim3(256), 0, 0, d_x, hp.P, hp.J, hp.K, Kp, ldh, tiled,
                     static_cast<T*>(H));
  check_launch("build_steering");
}

template <typename T>
void launch_convert(const float* src, void* dst, int64_t n) {
  hipLaunchKernelGGL(convert_f32<T>, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, 0,
                     src, static_cast<T*>(dst), n);
  check_launch("convert_f32");
}

void convert_dtype(int dtype, const float* src, void* dst, int64_t n) {
  switch (dtype) {
    case SRP_F32: HIP_OK(hipMemcpy(dst, src, n * 4, hipMemcpyDeviceToDevice)); break;
    case SRP_BF16: launch_convert<__bf16>(src, dst, n); break;
    case SRP_F16: launch_convert<_Float16>(src, dst, n); break;
    case SRP_FP8_E4M3: launch_convert<fp8>(src, dst, n); break;
    default: throw Error{SRP_E_UNSUPPORTED, "dtype not supported here"};
  }
}

struct Alloc {
  DevicePlan& dp;
  size_t budget;
  void* get(size_t bytes) {
    if (budget && dp.resident_bytes + bytes > budget)
      throw Error{SRP_E_BUDGET, "plan exceeds the HBM budget (" + std::to_string(dp.resident_bytes + bytes) +
                                    " > " + std::to_string(budget) + " bytes)"};
    void* p = nullptr;
    HIP_OK(hipMalloc(&p, std::max<size_t>(bytes, 256)));
    dp.resident_bytes += bytes;
    return p;
  }
};

// BF16 of an FP32 value, round to nearest even (finite inputs), and back
inline uint16_t bf16_rne(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
inline float bf16_float(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}

template <typename T>
void upload(void* dst, const std::vector<T>& v) {
  HIP_OK(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// tile shapes of the launch configurations
// FD GEMM (FP32, 16-bit and FP8), C = alpha X W^T (X: cross-spectra rows, W:
// steering rows, both tile-major as fd16_tiled lays them out): 256 x 256 tiles, 2 x 2 waves of 4 x 4 MFMA
// blocks (accumulators in AccVGPRs, one block per CU).  K streams in 64-byte
// stages straight into a ring of NBUF LDS stage buffers (global_load_lds, no
// register staging), each refilled as soon as the barrier after its last
// read has passed; one plain s_barrier per stage publishes it once every
// wave has waited for its own loads of it.  A stage row holds four 16-byte
// chunks, chunk c of row r at position c ^ f(r mod 16) with f(r) =
// ((r >> 1) ^ (r >> 3)) & 3, so that the fragment reads of 8 or 16
// consecutive rows at one chunk fall in distinct banks (32 or 64 banks).
// Both operands are stored tile-major (fd16_tiled: a 256-row tile's 64-byte
// stage pieces contiguous, already in the swizzled order), so one load is
// 1 KB contiguous and fills 16 rows of the stage; row-major operands, whose
// stages are scattered 64-byte pieces of rows tens of KB apart, kept the
// loads at a fraction of the L2's rate.  The MFMA steps are software-pipelined (the next step's fragments
// are read during the current step's MFMAs), since with one wave per SIMD
// nothing else hides the LDS latency.  Blocks are grouped per XCD with the
// frame tiles innermost (xcd_tile), so a steering tile is fetched from HBM
// once.  With blockIdx.z > 0 the contraction is split: split z covers
// elements [z kdim, (z + 1) kdim) and writes rows [z cz_rows, ...) of C.
template <typename T>
__global__ __launch_bounds__(256) void gemm_fd16(const T* __restrict__ X, int64_t ldx,
                                                 const T* __restrict__ W, int64_t ldw,
                                                 float* __restrict__ C, int64_t ldc, int nx, int nw,
                                                 int kdim, float alpha, int nw_tiles, int nx_tiles,
                                                 int64_t cz_rows) {
  constexpr int STEP = Mfma<T>::STEP;  // bytes of a row per MFMA step
  constexpr int LB = STEP / 2;         // bytes per lane per step
  constexpr int NV = LB / 16;
  constexpr int KS = FD16_SB / STEP;   // MFMA steps per stage
  static_assert(FD16_SB == 64, "four chunks per stage row");
  static_assert(FD16_NBUF * FD16_STAGE <= 160 * 1024, "LDS");
  static_assert((FD16_NBUF - 1) * FD16_NI < 64, "vmcnt holds at most 63 loads");
  __shared__ __attribute__((aligned(16))) unsigned char lds[FD16_NBUF * FD16_STAGE];

  int wt, xt;
  if (!xcd_tile(nw_tiles, nx_tiles, wt, xt)) return;  // uniform over the block
  const int x0 = xt * FD16_TILE, w0 = wt * FD16_TILE;
  if (x0 >= nx) return;
  const int64_t kz = static_cast<int64_t>(blockIdx.z) * kdim * static_cast<int64_t>(sizeof(T));
  C += static_cast<int64_t>(blockIdx.z) * cz_rows * ldc;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (SGPR)
  // loads: waves 0, 1 fill frame rows 128 wave .. + 127, waves 2, 3 the
  // candidate rows 128 (wave - 2) ..; load i covers 16 of them
  // both operands are tile-major with the swizzle applied (fd16_tiled): a
  // load is 1 KB contiguous, lane l's 16 bytes landing at byte 16 l
  const bool xside = wave < 2;
  const int64_t nstg = (xside ? ldx : ldw) * static_cast<int64_t>(sizeof(T)) / FD16_SB;  // stages per full row
  const unsigned char* src =
      reinterpret_cast<const unsigned char*>(xside ? static_cast<const void*>(X) : static_cast<const void*>(W)) +
      ((static_cast<int64_t>(xside ? xt : wt) * nstg + kz / FD16_SB) * FD16_TILE + (wave & 1) * 128) * FD16_SB +
      16 * lane;
  constexpr int64_t step16 = 1024, sstride = FD16_TILE * FD16_SB;
  const int ns = static_cast<int>(kdim * static_cast<int64_t>(sizeof(T)) / FD16_SB);
  // stage s >= ns reloads the last stage (a valid address) into a spent
  // buffer, so that every wait below counts the same loads
  auto issue = [&](int s) {
    unsigned char* dst = lds + (s % FD16_NBUF) * FD16_STAGE + wave * FD16_NI * 1024;
    const unsigned char* sp = src + static_cast<int64_t>(min(s, ns - 1)) * sstride;
#pragma unroll
    for (int i = 0; i < FD16_NI; ++i)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(sp + i * step16),
                                       (__attribute__((address_space(3))) void*)(dst + 1024 * i), 16, 0, 0);
  };

  const int r32 = lane & 31, g = lane >> 5;
  const int wy = wave >> 1, wx = wave & 1;
  f32x16 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;

  // fragment rows: frames wy 128 + 32 a + r32, candidates 256 + wx 128 +
  // 32 b + r32 (all with r mod 16 = r32 mod 16); logical chunk c of step t
  // is t STEP / 16 + g NV + v.  FP8 fragments are 8 registers (two chunks),
  // loaded in place so that the MFMA takes them without copies.
  using F = typename std::conditional<NV == 2, i32x8, i32x4>::type;
  const int sw = fd16_swz(r32 & 15);
  const int xrow = (wy * 128 + r32) * FD16_SB, wrow = (FD16_TILE + wx * 128 + r32) * FD16_SB;
  auto ld = [&](const unsigned char* p) { return *reinterpret_cast<const i32x4*>(p); };
  auto frags = [&](int s, auto tc, F (&fa)[4], F (&fb)[4]) {
    constexpr int t = decltype(tc)::value;
    const unsigned char* bs = lds + (s % FD16_NBUF) * FD16_STAGE;
    const int p0 = 16 * (((t * STEP) / 16 + g * NV) ^ sw);
    if constexpr (NV == 1) {
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = ld(bs + xrow + p0 + a * 32 * FD16_SB);
#pragma unroll
      for (int b = 0; b < 4; ++b) fb[b] = ld(bs + wrow + p0 + b * 32 * FD16_SB);
    } else {
      const int p1 = 16 * (((t * STEP) / 16 + g * NV + 1) ^ sw);
#pragma unroll
      for (int a = 0; a < 4; ++a)
        fa[a] = __builtin_shufflevector(ld(bs + xrow + p0 + a * 32 * FD16_SB), ld(bs + xrow + p1 + a * 32 * FD16_SB),
                                        0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        fb[b] = __builtin_shufflevector(ld(bs + wrow + p0 + b * 32 * FD16_SB), ld(bs + wrow + p1 + b * 32 * FD16_SB),
                                        0, 1, 2, 3, 4, 5, 6, 7);
    }
  };
  auto mfmas = [&](const F (&fa)[4], const F (&fb)[4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if constexpr (std::is_same<T, float>::value)
          Mfma<float>::run(&fa[a], &fb[b], acc[a][b]);  // four 32x32x2 steps per 16-byte chunk
        else if constexpr (std::is_same<T, fp8>::value)
          // E4M3 operands (format 0), E8M0 scales 127 = 2^0
          acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[a], fb[b], acc[a][b], 0, 0, 0, 127, 0, 127);
        else if constexpr (std::is_same<T, __bf16>::value)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[a]),
                                                              __builtin_bit_cast(bf16x8, fb[b]), acc[a][b], 0, 0, 0);
        else
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, fa[a]),
                                                             __builtin_bit_cast(f16x8, fb[b]), acc[a][b], 0, 0, 0);
      }
  };
  // MFMA step t of stage s with the fragments in (ca, cb); reads the next
  // step's fragments into (na, nb) first.  At a stage's last step every
  // fragment of the stage is already in registers (and this wave's reads
  // are done): after the barrier that publishes stage s + 1, whose loads
  // this wave has waited for (the NBUF - 2 later stages stay in flight),
  // the buffer of stage s takes the loads of stage s + NBUF.
  auto step = [&](int s, auto tc, F (&ca)[4], F (&cb)[4], F (&na)[4], F (&nb)[4]) {
    constexpr int t = decltype(tc)::value;
    constexpr int NR = 8 * NV;  // LDS reads of a step's fragments
    // this step's fragments were read one step ago
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));
    if constexpr (t + 1 < KS) {
      frags(s, std::integral_constant<int, t + 1>{}, na, nb);
      mfmas(ca, cb);
      // one MFMA, one LDS read, ...
#pragma unroll
      for (int i = 0; i < NR && i < 16; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
    } else {
      // unconditional, so that the loop body is one basic block and the
      // register sets need no copies: after the last stage the barrier,
      // reloads and reads of a spent buffer are harmless and unused
      wait_vm_lds<(FD16_NBUF - 2) * FD16_NI>();
      asm volatile("s_barrier" ::: "memory");
      issue(s + FD16_NBUF);
      frags(s + 1, std::integral_constant<int, 0>{}, na, nb);
      mfmas(ca, cb);
      // the loads of stage s + NBUF and the next fragment reads interleaved
      // with this step's MFMAs
#pragma unroll
      for (int i = 0; i < FD16_NI; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x004, 2, 0);  // SALU
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
      }
#pragma unroll
      for (int i = 0; i < NR && i < 16 - FD16_NI; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  for (int s = 0; s < FD16_NBUF; ++s) issue(s);
  wait_vm_lds<(FD16_NBUF - 1) * FD16_NI>();  // stage 0 has landed
  asm volatile("s_barrier" ::: "memory");
  F fa0[4], fb0[4], fa1[4], fb1[4];
  frags(0, std::integral_constant<int, 0>{}, fa0, fb0);
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  // two stages per iteration so that the register sets alternate at compile
  // time (step q = s KS + t multiplies set q & 1); ns is even
  for (int s = 0; s < ns; s += 2) {
    if constexpr (KS == 2) {
      step(s, I0{}, fa0, fb0, fa1, fb1);
      step(s, I1{}, fa1, fb1, fa0, fb0);
      step(s + 1, I0{}, fa0, fb0, fa1, fb1);
      step(s + 1, I1{}, fa1, fb1, fa0, fb0);
    } else {
      static_assert(KS == 1, "one or two MFMA steps per stage");
      step(s, I0{}, fa0, fb0, fa1, fb1);
      step(s + 1, I0{}, fa1, fb1, fa0, fb0);
    }
  }
  wait_vm_lds<0>();  // the reloads past the last stage

  // 32 x 32 accumulator layout: register v of lane i holds row
  // 8 (v / 4) + 4 (i / 32) + v % 4 and column i % 32
  const int rbase = x0 + wy * 128 + 4 * g;
  float* cp = C + static_cast<int64_t>(rbase) * ldc + w0 + wx * 128 + r32;
  const int cbase = w0 + wx * 128 + r32;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ro = a * 32 + 8 * (v / 4) + (v % 4);
      if (rbase + ro >= nx) continue;
      float* rp = cp + ro * ldc;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (cbase + b * 32 < nw) rp[b * 32] = alpha * acc[a][b][v];
    }
}

// General FP32 GEMM tile (the LR-SRP fat product): 128 x 128 per block,
// 2 x 2 waves, 256-byte K slices (128 bytes for FP8).  As the FP32 FD GEMM it
// beat 256 x 128 tiles with 128-byte slices (55.0 vs 58.6 ms at 125,000
// candidates and 1000 frames) but hit L2 on 12 % of reads and fetched ~200 GB
// per 1000 maps; gemm_fd16's tile-major 256 x 256 tiles replaced it there
// (52.5 ms, 23.8 GB).
constexpr int BIG_BX = 128, BIG_BW = 128, BIG_WGX = 2;
template <typename T>
constexpr int big_bkb() {
  return sizeof(T) == 1 ? 128 : 256;
}
// FD runs gemm_fd16 (256 x 256 tiles) in FP32, 16-bit and FP8.  At 16-bit and FP8 MFMA rates
// 2 x 2 blocks of 32 x 32 per wave read ~16 MACs per byte of LDS fragments,
// which saturates LDS; 4 x 4 blocks per wave (accumulators in AccVGPRs)
// halve that.  Measured at 125,000 x 1000 x 28,672, BF16 / FP8 ms per call:
// 128 x 128 tiles 11.2 / 5.0; 256 x 256 with register-staged K slices
// 8.1 / 3.9; direct-to-LDS stage ring with pipelined MFMA steps 7.4 / 3.75;
// tile-major operands 6.1 / 3.2; FP32 55.0 (128 x 128 row-major tiles) -> 52.5.
// candidate rows of the resident operands are padded to the widest W tile
constexpr int JPAD_ROWS = 256;
// workspace frame rows are padded to whole 256-frame tiles, the largest
// frame tile any kernel reads (fd_gen)
constexpr int LPAD_ROWS = 256;
// Row pitch of the FD operands (steering H and the cross-spectra psi): P Kp
// elements plus FD_ROW_PAD_BYTES.  Padding by 128 or 256 bytes changed
// neither the time nor the L2 hit rate of the 128 x 128 tiles, so it is 0.
constexpr int FD_ROW_PAD_BYTES = 0;
inline int64_t fd_ld(const HostPlan& hp, const DevicePlan& dp, size_t es) {
  return static_cast<int64_t>(hp.P) * dp.Kp + FD_ROW_PAD_BYTES / static_cast<int64_t>(es);
}
// general tall GEMM for FP32 rows past the streaming kernel's 1 KB
constexpr int TALL_BX = 256, TALL_BW = 128, TALL_WGX = 2, TALL_BKB = 128;
// the same for 16-bit and FP8 rows past the streaming kernel's limit (2 m
// disc: 3968 columns; SI): 128 x 128 tiles with 256-byte slices, 0.53
// against 0.67 ms on the 2 m disc (FP32 kept the 256 x 128 / 128-byte tile,
// which was 6 % faster there)
constexpr int TALL16_BX = 128, TALL16_BW = 128, TALL16_WGX = 2, TALL16_BKB = 256;
constexpr int tall_bkb(int dtype) { return dtype == SRP_F32 ? TALL_BKB : TALL16_BKB; }
constexpr int TALL_STEP_BYTES(int dtype) { return dtype == SRP_FP8_E4M3 ? 64 : 32; }  // Mfma<T>::STEP
// longest 16-bit U row of the streaming tall kernel (rows past 1 KB run on
// TALL_CW_LONG compute waves)
constexpr int TALL_ROW_MAX16 = 1280;
// Columns Kc of the tall operands for `raw` columns of data: a multiple of
// four MFMA steps when the 16-bit / FP8 rows fit the streaming kernel (at
// most 1 KB), else a whole K slice of the general GEMM that runs instead.
inline int tall_cols(int dtype, int64_t raw) {
  const int es = static_cast<int>(dsize(dtype));
  if (dtype != SRP_F32) {
    const int64_t ws = round_up(raw, 4 * TALL_STEP_BYTES(dtype) / es);
    if (ws * es <= 1024) return static_cast<int>(ws);
    // 16-bit rows past 1 KB: pairs of MFMA steps (32 columns, the global fat
    // stage's tile; the long-row kernel takes 34 to 40 steps)
    const int64_t wl = round_up(raw, 2 * TALL_STEP_BYTES(dtype) / es);
    if (es == 2 && wl * es <= TALL_ROW_MAX16) return static_cast<int>(wl);
  }
  return static_cast<int>(round_up(raw, tall_bkb(dtype) / es));
}
constexpr int TALL_CW = 8;       // compute waves per block of the tall kernel (256 candidates)
// the same for 16-bit rows of 1 KB to 1280 bytes (192 candidates; two waves
// per SIMD, each with 256 registers for its U rows).  Measured on per-pair
// SLRI R = 21 at 125,000 candidates x 1000 frames: 4 / 6 / 7 compute waves
// 0.304 / 0.279 / 0.288 ms per call (each g row feeds more candidates)
constexpr int TALL_CW_LONG = 6;
constexpr int SSPI_FT = 32;                       // frames per SSPI block

}  // namespace

// Plan-time device temporary, freed on every exit path.
// The gather is instantiated for Q = 1..8, 10, 12 and 16 taps; a selection
// of q taps runs on the smallest instance with at least q (the extra taps
// carry zero weight).
int gather_q(int q) {
  if (q <= 8) return std::max(q, 1);
  if (q <= 10) return 10;
  if (q <= 12) return 12;
  if (q <= 16) return 16;
  throw Error{SRP_E_UNSUPPORTED, "SSPI with more than 16 taps per (location, pair) is not built"};
}

struct TmpBuf {
  void* p = nullptr;
  explicit TmpBuf(size_t bytes) { HIP_OK(hipMalloc(&p, std::max<size_t>(bytes, 1))); }
  ~TmpBuf() {
    if (p) (void)hipFree(p);
  }
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

int host_threads() {
  const unsigned n = std::thread::hardware_concurrency();
  return static_cast<int>(std::min(std::max(n, 1u), 16u));
}

// Global SLRI operands (eq. (54) over the stacked Lambda): the PN x PN Gram
// matrix on the device in FP64 (candidate range split across blocks, the
// partial sums added on the host), its eigenvectors on the host, then
// U = Lambda V on the device; a single FP8 weight scale and activation
// scale, as for one pair.
static void fit_slri_global_rand(HostPlan& hp, const double* dx);
static void fit_slri_global_gram(HostPlan& hp, const double* dx);
static void build_slri_global_operands(HostPlan& hp, DevicePlan& dp, Alloc& A, const double* dx);

static void build_slri_global_device(HostPlan& hp, DevicePlan& dp, Alloc& A, const double* dx) {
  if (2 * hp.max_np + 1 > 576) throw Error{SRP_E_UNSUPPORTED, "global SLRI stages at most 576 lags per pair"};
  if (hp.global_rand)
    fit_slri_global_rand(hp, dx);
  else
    fit_slri_global_gram(hp, dx);
  build_slri_global_operands(hp, dp, A, dx);
}

// V and the singular values of the global fit from the PN x PN Gram matrix
// (exact, PN <= 4096).
static void fit_slri_global_gram(HostPlan& hp, const double* dx) {
  const int PN = hp.PN, P = hp.P;
  std::vector<int32_t> pa(PN), la(PN);
  for (int p = 0; p < P; ++p)
    for (int i = 0; i < 2 * hp.np[p] + 1; ++i) {
      pa[hp.off[p] + i] = p;
      la[hp.off[p] + i] = i - hp.np[p];
    }
  TmpBuf dpa(PN * 4), dla(PN * 4);
  upload(static_cast<int32_t*>(dpa.p), pa);
  upload(static_cast<int32_t*>(dla.p), la);
  const int ntile = (PN + 63) / 64;
  const int tiles = ntile * (ntile + 1) / 2;
  // enough candidate splits to give every CU a few blocks, within ~1 GB of partials
  int splits = std::max(1, std::min<int>(static_cast<int>((hp.J + 4095) / 4096), (1024 + tiles - 1) / tiles));
  while (splits > 1 && static_cast<double>(splits) * PN * PN * 8 > 1e9) --splits;
  const int64_t jchunk = round_up((hp.J + splits - 1) / splits, 4);
  const size_t gn = static_cast<size_t>(splits) * PN * PN;
  TmpBuf dg(gn * sizeof(double));
  hipLaunchKernelGGL(gram_global_f64, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(splits)), dim3(256), 0,
                     0, dx, hp.J, dpa.as<int32_t>(), dla.as<int32_t>(), PN, ntile, jchunk, dg.as<double>());
  check_launch("gram_global_f64");
  std::vector<double> gall(gn);
  HIP_OK(hipMemcpy(gall.data(), dg.p, gn * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> G(static_cast<size_t>(PN) * PN, 0.0);
  parallel_for(PN, host_threads(), [&](int a) {
    for (int sidx = 0; sidx < splits; ++sidx) {
      const double* src = &gall[(static_cast<size_t>(sidx) * PN + a) * PN];
      double* dst = &G[static_cast<size_t>(a) * PN];
      for (int b = 0; b < PN; ++b) dst[b] += src[b];
    }
  });
  std::vector<double>().swap(gall);
  slri_fit_global(hp, G);
}

// U = Lambda V and the runtime operands of the global fit from hp.V.
static void build_slri_global_operands(HostPlan& hp, DevicePlan& dp, Alloc& A, const double* dx) {
  const int PN = hp.PN, R = hp.R, P = hp.P;
  // U = Lambda V, staged in FP32 as [Jpad][Kc]
  const size_t ucount = static_cast<size_t>(dp.Jpad) * dp.Kc;
  TmpBuf dv(hp.V.size() * sizeof(double));
  upload(dv.p, hp.V);
  TmpBuf us(ucount * sizeof(float));
  HIP_OK(hipMemset(us.p, 0, ucount * sizeof(float)));
  hipLaunchKernelGGL(slri_u_global_f64, dim3(static_cast<unsigned>((hp.J + 255) / 256), static_cast<unsigned>((R + 7) / 8)),
                     dim3(256), 0, 0, dx, hp.J, dp.d_np, dp.d_off, P, R, dv.as<double>(), us.as<float>(), dp.Kc);
  check_launch("slri_u_global_f64");
  float sigma = 1.0f;
  if (hp.dtype == SRP_FP8_E4M3) {
    TmpBuf um(sizeof(float));
    hipLaunchKernelGGL(pair_absmax, dim3(1), dim3(256), 0, 0, us.as<float>(), hp.J, dp.Kc, R, um.as<float>());
    check_launch("pair_absmax");
    float umax = 0.0f;
    HIP_OK(hipMemcpy(&umax, um.p, sizeof(float), hipMemcpyDeviceToHost));
    if (umax > 0) sigma = static_cast<float>(std::exp2(std::ceil(std::log2(umax / 448.0))));
    std::vector<float> inv(1, 1.0f / sigma);
    TmpBuf di(sizeof(float));
    upload(di.as<float>(), inv);
    hipLaunchKernelGGL(scale_pairs, dim3(static_cast<unsigned>((ucount + 255) / 256)), dim3(256), 0, 0,
                       us.as<float>(), dp.Jpad, dp.Kc, R, 1, di.as<float>());
    check_launch("scale_pairs");
    HIP_OK(hipDeviceSynchronize());
  }
  // activation bound: |g_c| <= sigma * sum_a |V[a][c]| * 2 (K - 1)
  double vl1 = 0;
  for (int r = 0; r < R; ++r) {
    double sum = 0;
    for (int a = 0; a < PN; ++a) sum += std::fabs(hp.V[static_cast<size_t>(a) * R + r]);
    vl1 = std::max(vl1, sum);
  }
  const double amax_act = sigma * vl1 * 2.0 * (hp.K - 1);
  double act = 1.0;
  if (hp.dtype == SRP_FP8_E4M3) act = std::exp2(std::ceil(std::log2(amax_act / 448.0)));
  if (hp.dtype == SRP_F16 && amax_act > 60000.0) act = std::exp2(std::ceil(std::log2(amax_act / 60000.0)));
  std::vector<float> gscale(1, static_cast<float>(sigma / act));
  dp.tall_alpha = static_cast<float>(act);
  dp.d_U = A.get(ucount * dsize(hp.dtype));
  convert_dtype(hp.dtype, us.as<float>(), dp.d_U, static_cast<int64_t>(ucount));
  HIP_OK(hipDeviceSynchronize());
  // V as FP32 [PN][Kc], zero past column R
  std::vector<float> Vf(static_cast<size_t>(PN) * dp.Kc, 0.0f);
  for (int a = 0; a < PN; ++a)
    for (int r = 0; r < R; ++r) Vf[static_cast<size_t>(a) * dp.Kc + r] = static_cast<float>(hp.V[static_cast<size_t>(a) * R + r]);
  dp.d_V = static_cast<float*>(A.get(Vf.size() * 4));
  upload(dp.d_V, Vf);
  dp.d_gscale = static_cast<float*>(A.get(4));
  upload(dp.d_gscale, gscale);
}

// LR-SRP operands (eqs. (26)-(29)).  The truncated SVD of the complex
// steering matrix H (J x n, n = P (K-1)) is taken through the smaller of
// its two Gram matrices, in FP64 on the device: H is materialised
// (build_h_c64), the Gram matrix formed by rocBLAS zherk and decomposed by
// rocSOLVER zheevd.  Viewing H's row-major storage as the column-major
// n x J matrix X = H^T:
//   n <= J: X X^H = conj(H^H H); its eigenvectors z give V = conj(z), and
//           H_tall = H V (zgemm: T^T = V^T X);
//   J <  n: X^H X = conj(H H^H); U = conj(z), H_tall = U Sigma, and
//           conj(H^H U) = X conj(U) = X z (zgemm), V = H^H U / sigma.
// Runtime operands: F (rows 2r, 2r+1 hold (Re V, Im V) and (-Im V, Re V) in
// the interleaved (Re, Im) slots of psi, so psi F^T gives Re and Im of
// (V^H psi)_r) and the tall operand (columns 2 Re T, -2 Im T), so that the
// tall product is 2 Re[T g].
struct Blas {
  rocblas_handle h = nullptr;
  Blas() {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{SRP_E_HIP, "rocblas_create_handle failed"};
  }
  ~Blas() {
    if (h) (void)rocblas_destroy_handle(h);
  }
  Blas(const Blas&) = delete;
  Blas& operator=(const Blas&) = delete;
};

static void blas_ok(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    throw Error{SRP_E_HIP, std::string(what) + " failed: " + rocblas_status_to_string(st)};
}

// Global SLRI fit (54) by randomized subspace iteration (Halko, Martinsson
// and Tropp, SIAM Review 53 (2011), Alg. 4.4 with the SVD of Alg. 5.1), for
// stacked Lambda too wide for the Gram eigendecomposition: with l = R + p
// columns (p = max(16, R / 8), l rounded up to 64), Omega Gaussian (seeded),
//   Y = Lambda Omega, Q = orth(Y); q = 2 times: Z = orth(Lambda^T Q),
//   Q = orth(Lambda Z); then B^T = Lambda^T Q (PN x l) and the eigenpairs
// (W, sigma^2) of B B^T give V = B^T W sigma^-1 and the singular values.
// Every product runs in FP64 with Lambda generated (lam_gemm_f64); orth is
// the Householder LQ of the l x n row block (rocSOLVER dgelqf / dorglq),
// B B^T by rocBLAS dsyrk, its eigenpairs by rocSOLVER dsyevd.  The
// singular values past the l computed are reported as zero.
static void fit_slri_global_rand(HostPlan& hp, const double* dx) {
  const int P = hp.P, PN = hp.PN, R = hp.R;
  const int64_t J = hp.J;
  // stacked lags padded to 16-slot chunks per pair
  std::vector<int32_t> cpair, clag0, cnp, pbase(P);
  for (int p = 0; p < P; ++p) {
    pbase[p] = static_cast<int32_t>(16 * cpair.size());
    const int n = 2 * hp.np[p] + 1;
    for (int c = 0; c < (n + 15) / 16; ++c) {
      cpair.push_back(p);
      clag0.push_back(-hp.np[p] + 16 * c);
      cnp.push_back(hp.np[p]);
    }
  }
  const int64_t PNA = 16 * static_cast<int64_t>(cpair.size());
  // l sample columns: R plus oversampling, at most the rows of either side
  const int l = static_cast<int>(
      std::min<int64_t>(round_up(R + std::max(16, R / 8), 64), std::min<int64_t>(PNA, J) / 64 * 64));
  if (l < R) throw Error{SRP_E_UNSUPPORTED, "randomized global SLRI needs R well below PN and J"};
  const int64_t Jk = round_up(J, 64);  // rows of Y / Q (zeros past J)
  TmpBuf dcp(cpair.size() * 4), dcl(clag0.size() * 4), dcn(cnp.size() * 4);
  upload(static_cast<int32_t*>(dcp.p), cpair);
  upload(static_cast<int32_t*>(dcl.p), clag0);
  upload(static_cast<int32_t*>(dcn.p), cnp);
  TmpBuf dy(static_cast<size_t>(Jk) * l * 8), dz(static_cast<size_t>(PNA) * l * 8);
  HIP_OK(hipMemset(dy.p, 0, static_cast<size_t>(Jk) * l * 8));
  // Omega [PNA][l]: standard normal by Box-Muller from a seeded 64-bit
  // generator; padding rows zero
  {
    std::vector<double> om(static_cast<size_t>(PNA) * l, 0.0);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    auto next = [&]() {  // splitmix64
      st += 0x9E3779B97F4A7C15ull;
      uint64_t zz = st;
      zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
      zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
      return zz ^ (zz >> 31);
    };
    for (int p = 0; p < P; ++p)
      for (int i = 0; i < 2 * hp.np[p] + 1; ++i) {
        double* row = &om[static_cast<size_t>(pbase[p] + i) * l];
        for (int c = 0; c < l; c += 2) {
          const double u1 = (static_cast<double>(next() >> 11) + 0.5) * 0x1p-53;
          const double u2 = static_cast<double>(next() >> 11) * 0x1p-53;
          const double rr = std::sqrt(-2.0 * std::log(u1));
          row[c] = rr * std::cos(2.0 * M_PI * u2);
          if (c + 1 < l) row[c + 1] = rr * std::sin(2.0 * M_PI * u2);
        }
      }
    upload(dz.as<double>(), om);
  }
  const int ntn = l / 64;
  auto lam = [&](const double* Bm, double* Cm) {  // Y = Lambda Z
    hipLaunchKernelGGL(lam_gemm_f64<false>, dim3(static_cast<unsigned>((J + 63) / 64 * ntn)), dim3(256), 0, 0, dx, J,
                       dcp.as<int32_t>(), dcl.as<int32_t>(), dcn.as<int32_t>(), J, PNA, Bm,
                       static_cast<int64_t>(l), Cm, static_cast<int64_t>(l), ntn);
    check_launch("lam_gemm_f64");
  };
  auto lamt = [&](const double* Bm, double* Cm) {  // Z = Lambda^T Y
    hipLaunchKernelGGL(lam_gemm_f64<true>, dim3(static_cast<unsigned>(PNA / 64 * ntn + (PNA % 64 ? ntn : 0))),
                       dim3(256), 0, 0, dx, J, dcp.as<int32_t>(), dcl.as<int32_t>(), dcn.as<int32_t>(), PNA,
                       round_up(J, 16), Bm, static_cast<int64_t>(l), Cm, static_cast<int64_t>(l), ntn);
    check_launch("lam_gemm_f64");
  };
  Blas blas;
  TmpBuf tau(static_cast<size_t>(l) * 8);
  // orthonormal basis of the column space of the n x l matrix held
  // row-major [n][l] (= the column-major l x n matrix A): A = L Q' (LQ),
  // Q' overwrites A
  auto orth = [&](double* Am, int64_t n) {
    blas_ok(rocsolver_dgelqf(blas.h, l, static_cast<rocblas_int>(n), Am, l, tau.as<double>()), "rocsolver_dgelqf");
    blas_ok(rocsolver_dorglq(blas.h, l, static_cast<rocblas_int>(n), l, Am, l, tau.as<double>()), "rocsolver_dorglq");
  };
  lam(dz.as<double>(), dy.as<double>());
  orth(dy.as<double>(), J);
  for (int it = 0; it < 2; ++it) {
    lamt(dy.as<double>(), dz.as<double>());
    orth(dz.as<double>(), PNA);
    lam(dz.as<double>(), dy.as<double>());
    orth(dy.as<double>(), J);
  }
  lamt(dy.as<double>(), dz.as<double>());  // B^T = Lambda^T Q, [PNA][l]
  TmpBuf dg(static_cast<size_t>(l) * l * 8), dd(static_cast<size_t>(l) * 8), de(static_cast<size_t>(l) * 8),
      dinfo(sizeof(rocblas_int));
  const double one = 1.0, zero = 0.0;
  blas_ok(rocblas_dsyrk(blas.h, rocblas_fill_upper, rocblas_operation_none, l, static_cast<rocblas_int>(PNA), &one,
                        dz.as<double>(), l, &zero, dg.as<double>(), l),
          "rocblas_dsyrk");
  blas_ok(rocsolver_dsyevd(blas.h, rocblas_evect_original, rocblas_fill_upper, l, dg.as<double>(), l,
                           dd.as<double>(), de.as<double>(), dinfo.as<rocblas_int>()),
          "rocsolver_dsyevd");
  rocblas_int info = 0;
  HIP_OK(hipMemcpy(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost));
  if (info != 0) throw Error{SRP_E_HIP, "rocsolver_dsyevd did not converge (info " + std::to_string(info) + ")"};
  // V^T (R x PNA, column-major) = W_R^T B^T with W_R the eigenvectors of
  // the R largest eigenvalues (the last R columns, ascending order)
  TmpBuf dvt(static_cast<size_t>(R) * PNA * 8);
  blas_ok(rocblas_dgemm(blas.h, rocblas_operation_transpose, rocblas_operation_none, R,
                        static_cast<rocblas_int>(PNA), l, &one, dg.as<double>() + static_cast<size_t>(l - R) * l, l,
                        dz.as<double>(), l, &zero, dvt.as<double>(), R),
          "rocblas_dgemm");
  std::vector<double> ev(l), vt(static_cast<size_t>(R) * PNA);
  HIP_OK(hipMemcpy(ev.data(), dd.p, ev.size() * 8, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(vt.data(), dvt.p, vt.size() * 8, hipMemcpyDeviceToHost));
  std::fill(hp.sv.begin(), hp.sv.end(), 0.0);
  for (int i = 0; i < l && i < PN; ++i) hp.sv[i] = std::sqrt(std::max(0.0, ev[l - 1 - i]));
  // column r of V (descending sigma) is row R - 1 - r of V^T, over sigma_r
  for (int p = 0; p < P; ++p)
    for (int i = 0; i < 2 * hp.np[p] + 1; ++i) {
      const size_t a = static_cast<size_t>(hp.off[p] + i), ap = static_cast<size_t>(pbase[p] + i);
      for (int r = 0; r < R; ++r) {
        const double sg = hp.sv[r];
        hp.V[a * R + r] = sg > 0 ? vt[ap * R + (R - 1 - r)] / sg : 0.0;
      }
    }
}

static void build_lr_device(HostPlan& hp, DevicePlan& dp, Alloc& A, const double* dx) {
  const int P = hp.P, K = hp.K, R = hp.RH;
  const int64_t J = hp.J, n = static_cast<int64_t>(P) * (K - 1);
  const int64_t m = std::min(J, n);
  if (m > 16384) throw Error{SRP_E_UNSUPPORTED, "LR-SRP needs min(J, P (K - 1)) <= 16384 for its Gram matrix"};
  if (static_cast<double>(J) * n * 16 > 48e9) throw Error{SRP_E_UNSUPPORTED, "LR-SRP fit: H above 48 GB"};
  TmpBuf dh(static_cast<size_t>(J) * n * sizeof(double2));
  hipLaunchKernelGGL(build_h_c64, dim3(static_cast<unsigned>(J), static_cast<unsigned>((n + 255) / 256)), dim3(256),
                     0, 0, dx, P, J, K, dh.as<double2>());
  check_launch("build_h_c64");
  HIP_OK(hipDeviceSynchronize());
  Blas blas;
  auto* X = reinterpret_cast<rocblas_double_complex*>(dh.p);
  const bool nroute = n <= J;
  TmpBuf dg(static_cast<size_t>(m) * m * sizeof(double2));
  auto* G = reinterpret_cast<rocblas_double_complex*>(dg.p);
  const double one = 1.0, zero = 0.0;
  blas_ok(rocblas_zherk(blas.h, rocblas_fill_lower, nroute ? rocblas_operation_none : rocblas_operation_conjugate_transpose,
                        static_cast<rocblas_int>(m), static_cast<rocblas_int>(nroute ? J : n), &one, X,
                        static_cast<rocblas_int>(n), &zero, G, static_cast<rocblas_int>(m)),
          "rocblas_zherk");
  TmpBuf dd(m * sizeof(double)), de(m * sizeof(double)), dinfo(sizeof(rocblas_int));
  blas_ok(rocsolver_zheevd(blas.h, rocblas_evect_original, rocblas_fill_lower, static_cast<rocblas_int>(m), G,
                           static_cast<rocblas_int>(m), dd.as<double>(), de.as<double>(), dinfo.as<rocblas_int>()),
          "rocsolver_zheevd");
  HIP_OK(hipDeviceSynchronize());
  rocblas_int info = 0;
  HIP_OK(hipMemcpy(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost));
  if (info != 0) throw Error{SRP_E_HIP, "rocsolver_zheevd did not converge (info " + std::to_string(info) + ")"};
  std::vector<double> lam(m);
  HIP_OK(hipMemcpy(lam.data(), dd.p, m * sizeof(double), hipMemcpyDeviceToHost));
  // eigenvalues ascending: the R largest are the last R columns of z
  const double2* zR = reinterpret_cast<const double2*>(dg.p) + static_cast<int64_t>(m - R) * m;
  hp.lr_s.assign(R, 0.0);
  for (int r = 0; r < R; ++r) hp.lr_s[r] = std::sqrt(std::max(0.0, lam[m - 1 - r]));
  const double smin = 1e-12 * (hp.lr_s.empty() ? 0.0 : hp.lr_s[0]);
  // T [J][R] and V [n][R] on the host, column r = the r-th largest
  std::vector<double2> T(static_cast<size_t>(J) * R), V(static_cast<size_t>(n) * R);
  const rocblas_double_complex c1{1.0, 0.0}, c0{0.0, 0.0};
  if (nroute) {
    std::vector<double2> zh(static_cast<size_t>(m) * R);
    HIP_OK(hipMemcpy(zh.data(), zR, zh.size() * sizeof(double2), hipMemcpyDeviceToHost));
    std::vector<double2> vcm(static_cast<size_t>(n) * R);  // column-major n x R, V = conj(z)
    for (int r = 0; r < R; ++r)
      for (int64_t i = 0; i < n; ++i) {
        const double2 z = zh[static_cast<size_t>(R - 1 - r) * m + i];
        vcm[static_cast<size_t>(r) * n + i] = make_double2(z.x, -z.y);
        V[static_cast<size_t>(i) * R + r] = make_double2(z.x, -z.y);
      }
    TmpBuf dv(vcm.size() * sizeof(double2)), dt(T.size() * sizeof(double2));
    upload(dv.p, vcm);
    blas_ok(rocblas_zgemm(blas.h, rocblas_operation_transpose, rocblas_operation_none, R, static_cast<rocblas_int>(J),
                          static_cast<rocblas_int>(n), &c1, dv.as<rocblas_double_complex>(), static_cast<rocblas_int>(n),
                          X, static_cast<rocblas_int>(n), &c0, dt.as<rocblas_double_complex>(), R),
            "rocblas_zgemm");
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(T.data(), dt.p, T.size() * sizeof(double2), hipMemcpyDeviceToHost));
  } else {
    std::vector<double2> zh(static_cast<size_t>(m) * R);
    HIP_OK(hipMemcpy(zh.data(), zR, zh.size() * sizeof(double2), hipMemcpyDeviceToHost));
    for (int r = 0; r < R; ++r) {
      const double sg = hp.lr_s[r] > smin ? hp.lr_s[r] : 0.0;
      for (int64_t j = 0; j < J; ++j) {
        const double2 z = zh[static_cast<size_t>(R - 1 - r) * m + j];
        T[static_cast<size_t>(j) * R + r] = make_double2(z.x * sg, -z.y * sg);  // U sigma, U = conj(z)
      }
    }
    // conj(H^H U) = X z, for the R columns of z (ascending order)
    TmpBuf dw(static_cast<size_t>(n) * R * sizeof(double2));
    blas_ok(rocblas_zgemm(blas.h, rocblas_operation_none, rocblas_operation_none, static_cast<rocblas_int>(n), R,
                          static_cast<rocblas_int>(J), &c1, X, static_cast<rocblas_int>(n),
                          reinterpret_cast<const rocblas_double_complex*>(zR), static_cast<rocblas_int>(m), &c0,
                          dw.as<rocblas_double_complex>(), static_cast<rocblas_int>(n)),
            "rocblas_zgemm");
    HIP_OK(hipDeviceSynchronize());
    std::vector<double2> w(static_cast<size_t>(n) * R);
    HIP_OK(hipMemcpy(w.data(), dw.p, w.size() * sizeof(double2), hipMemcpyDeviceToHost));
    for (int r = 0; r < R; ++r) {
      const double inv = hp.lr_s[r] > smin ? 1.0 / hp.lr_s[r] : 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const double2 c = w[static_cast<size_t>(R - 1 - r) * n + i];
        V[static_cast<size_t>(i) * R + r] = make_double2(c.x * inv, -c.y * inv);
      }
    }
  }
  // runtime operands
  dp.Kc = static_cast<int>(round_up(tall_cols(hp.dtype, 2 * R), 32));
  dp.Fpad = static_cast<int>(round_up(dp.Kc, BIG_BW));
  const int64_t ldf = static_cast<int64_t>(P) * dp.Kp;
  std::vector<float> F(static_cast<size_t>(dp.Fpad) * ldf, 0.0f);
  double act_max = 0;
  for (int r = 0; r < R; ++r) {
    float* f0 = &F[static_cast<size_t>(2 * r) * ldf];
    float* f1 = &F[static_cast<size_t>(2 * r + 1) * ldf];
    double l1a = 0, l1b = 0;
    for (int p = 0; p < P; ++p)
      for (int k = 1; k < K; ++k) {
        const double2 v = V[static_cast<size_t>(p * (K - 1) + k - 1) * R + r];
        const size_t e = static_cast<size_t>(p) * dp.Kp + 2 * (k - 1);
        f0[e] = static_cast<float>(v.x);
        f0[e + 1] = static_cast<float>(v.y);
        f1[e] = static_cast<float>(-v.y);
        f1[e + 1] = static_cast<float>(v.x);
        l1a += std::fabs(v.x) + std::fabs(v.y);
      }
    l1b = l1a;
    act_max = std::max(act_max, std::max(l1a, l1b));  // |Re g|, |Im g| <= sum |V| since |psi| <= 1
  }
  dp.d_F = static_cast<float*>(A.get(F.size() * 4));
  upload(dp.d_F, F);
  const size_t ucount = static_cast<size_t>(dp.Jpad) * dp.Kc;
  std::vector<float> Us(ucount, 0.0f);
  double umax = 0;
  for (int64_t j = 0; j < J; ++j)
    for (int r = 0; r < R; ++r) {
      const double2 t = T[static_cast<size_t>(j) * R + r];
      Us[static_cast<size_t>(j) * dp.Kc + 2 * r] = static_cast<float>(2.0 * t.x);
      Us[static_cast<size_t>(j) * dp.Kc + 2 * r + 1] = static_cast<float>(-2.0 * t.y);
      umax = std::max(umax, 2.0 * std::max(std::fabs(t.x), std::fabs(t.y)));
    }
  double sigma = 1.0, act = 1.0;
  if (hp.dtype == SRP_FP8_E4M3) {
    if (umax > 0) sigma = std::exp2(std::ceil(std::log2(umax / 448.0)));
    if (act_max > 0) act = std::exp2(std::ceil(std::log2(act_max / 448.0)));
    for (float& u : Us) u = static_cast<float>(u / sigma);
  }
  if (hp.dtype == SRP_F16 && act_max > 60000.0) act = std::exp2(std::ceil(std::log2(act_max / 60000.0)));
  dp.lr_gscale = static_cast<float>(1.0 / act);
  dp.tall_alpha = static_cast<float>(act * sigma);
  TmpBuf us(ucount * 4);
  upload(us.p, Us);
  dp.d_U = A.get(ucount * dsize(hp.dtype));
  convert_dtype(hp.dtype, us.as<float>(), dp.d_U, static_cast<int64_t>(ucount));
  HIP_OK(hipDeviceSynchronize());
}

// Dense-window SSPI (16-bit weights).  For candidate tile t (256
// candidates, the tiles of sspi_windows and of the streaming tall kernel)
// and pair p the taps fall inside the lag window win[t][p]; rounded up to
// whole 8-lag chunks and stacked over pairs, these windows form a
// contraction of K_t <= kmax columns, so that
//   z[l][j] = sum_k xf[l][col_t(k)] B[j][k]
// with B holding each candidate's tap weights at its lags' positions (zeros
// elsewhere) and xf the samples frame-major, each pair's lags starting on an
// 8-element boundary, in 8 copies shifted by 0..7 columns so that a window
// starting at any lag is read in whole 16-byte chunks from one of them (the
// lags a chunk reads past the window meet zero weights).  On the matrix
// cores this costs K_t MACs per candidate
// and frame instead of the gather's P Q, but runs at the MFMA rate.  Tiles
// whose K_t fits the streaming kernel's 1 KB rows go to the matrix cores,
// the rest stay on the gather; built when at least half the tiles fit.
static void build_sspi_dense(HostPlan& hp, DevicePlan& dp, Alloc& A, const std::vector<int2>& wins, int njt,
                             int Qs) {
  const int P = hp.P;
  const int es = static_cast<int>(dsize(hp.dtype));
  const int kcap = 1024 / es;  // the streaming kernel's row limit in elements
  std::vector<int32_t> offA(P + 1, 0);
  for (int p = 0; p < P; ++p) offA[p + 1] = offA[p] + static_cast<int32_t>(round_up(2 * hp.np[p] + 1, 8));
  const int PNA = offA[P];
  std::vector<int32_t> a0(static_cast<size_t>(njt) * P), kpos(static_cast<size_t>(njt) * P), kt(njt);
  std::vector<int32_t> dtiles, gtiles;
  int kmax = 0;
  for (int t = 0; t < njt; ++t) {
    int k = 0;
    for (int p = 0; p < P; ++p) {
      const int2 w = wins[static_cast<size_t>(t) * P + p];
      const int lo = w.x - hp.off[p];  // first staged lag within the pair
      // taps past the pair's 2 N_p + 1 lags (a gather width above the lag
      // count) carry zero weight and are left out
      const int len = std::max(0, std::min(w.y, 2 * hp.np[p] + 1 - lo));
      a0[static_cast<size_t>(t) * P + p] = lo;
      kpos[static_cast<size_t>(t) * P + p] = k;
      k += static_cast<int>(round_up(len, 8));
    }
    kt[t] = k;
    if (k <= kcap) {
      dtiles.push_back(t);
      kmax = std::max(kmax, k);
    } else {
      gtiles.push_back(t);
    }
  }
  // worth it only when most tiles move to the matrix cores
  if (2 * dtiles.size() < static_cast<size_t>(njt)) return;
  kmax = static_cast<int>(round_up(kmax, 4 * TALL_STEP_BYTES(hp.dtype) / es));
  // chunk columns of each dense tile in the frame-major samples: the window
  // of pair p starting at lag lo is read from the copy shifted by
  // c = (8 - lo % 8) % 8, where it starts on a chunk boundary; its last chunk
  // ends before column offA[p + 1] + 14 <= XW of that copy
  const int XW = PNA + 16;
  const int cpr = kmax / 8;
  std::vector<int32_t> ctab(static_cast<size_t>(njt) * cpr, -1);
  for (int t : dtiles)
    for (int p = 0; p < P; ++p) {
      const int lo = a0[static_cast<size_t>(t) * P + p];
      const int k0 = kpos[static_cast<size_t>(t) * P + p];
      const int kn = (p + 1 < P ? kpos[static_cast<size_t>(t) * P + p + 1] : kt[t]) - k0;
      const int c = (8 - lo % 8) % 8;
      for (int m = 0; m < kn / 8; ++m) {
        const int col = offA[p] + lo + c + 8 * m;
        if (col % 8 != 0 || col + 8 > XW)
          throw Error{SRP_E_UNSUPPORTED, "dense-window SSPI: chunk outside its copy"};
        ctab[static_cast<size_t>(t) * cpr + k0 / 8 + m] = c * XW + col;
      }
    }
  std::vector<int32_t> colmap(PNA, -1);
  for (int p = 0; p < P; ++p)
    for (int r = 0; r < 2 * hp.np[p] + 1; ++r) colmap[offA[p] + r] = hp.off[p] + r;
  TmpBuf da0(a0.size() * 4), dkpos(kpos.size() * 4);
  upload(da0.p, a0);
  upload(dkpos.p, kpos);
  dp.d_dtiles = static_cast<int32_t*>(A.get(dtiles.size() * 4));
  upload(dp.d_dtiles, dtiles);
  if (!gtiles.empty()) {
    dp.d_gtiles = static_cast<int32_t*>(A.get(gtiles.size() * 4));
    upload(dp.d_gtiles, gtiles);
  }
  const size_t bbytes = static_cast<size_t>(dp.Jpad) * kmax * es;
  dp.d_B = A.get(bbytes);
  HIP_OK(hipMemset(dp.d_B, 0, bbytes));
  const dim3 gw(static_cast<unsigned>(dtiles.size()), static_cast<unsigned>(P));
  if (hp.dtype == SRP_BF16)
    hipLaunchKernelGGL(sspi_dense_weights<__bf16>, gw, dim3(256), 0, 0, dp.d_start, static_cast<const __bf16*>(dp.d_w),
                       Qs, dp.sspi_q, hp.J, dp.d_off, da0.as<int32_t>(), dkpos.as<int32_t>(), P, dp.d_dtiles,
                       static_cast<__bf16*>(dp.d_B), kmax);
  else
    hipLaunchKernelGGL(sspi_dense_weights<_Float16>, gw, dim3(256), 0, 0, dp.d_start,
                       static_cast<const _Float16*>(dp.d_w), Qs, dp.sspi_q, hp.J, dp.d_off, da0.as<int32_t>(),
                       dkpos.as<int32_t>(), P, dp.d_dtiles, static_cast<_Float16*>(dp.d_B), kmax);
  check_launch("sspi_dense_weights");
  // one launch over every dense tile at the widest contraction (tiles in
  // width classes of 64 columns, one launch each, measured slower: 0.253
  // against 0.215 ms per 1000 maps at Q = 3, the launches' tails cost more
  // than the narrower classes save)
  dp.d_ctab = static_cast<int32_t*>(A.get(ctab.size() * 4));
  upload(dp.d_ctab, ctab);
  dp.d_colmap = static_cast<int32_t*>(A.get(colmap.size() * 4));
  upload(dp.d_colmap, colmap);
  HIP_OK(hipDeviceSynchronize());
  dp.sspi_dense = true;
  dp.sspi_kmax = kmax;
  dp.sspi_pna = PNA;
  dp.sspi_xw = XW;
  dp.n_dtiles = static_cast<int>(dtiles.size());
  dp.n_gtiles = static_cast<int>(gtiles.size());
}

// SSPI band product (the matrix cores for wide windows): descriptors and
// passes per tile on the device, then tile-major FP16 copies of the records,
// which replace the pair-major ones (the band product is then the only
// consumer).  Used when every pair's band fits one pass.
template <typename TW>
static void build_sspi_band(HostPlan& hp, DevicePlan& dp, Alloc& A, int njt, int Qs) {
  const int P = hp.P, Q = dp.sspi_q;
  const int QW = Q <= 4 ? 2 : 4;
  const size_t nd = static_cast<size_t>(njt) * P;
  if (P > 65535) return;
  // compact order and tile-major records
  std::vector<int32_t> order = compact_order(hp, 256, 32);
  order.resize(static_cast<size_t>(njt) * 256, 0);
  const size_t nr = nd * 256;
  std::unique_ptr<TmpBuf> ord(new TmpBuf(order.size() * 4)), rs(new TmpBuf(nr * 4)), rw(new TmpBuf(nr * 4 * QW));
  upload(static_cast<int32_t*>(ord->p), order);
  hipLaunchKernelGGL(sspi_band_records<TW>, dim3(static_cast<unsigned>(njt), static_cast<unsigned>(P)), dim3(256), 0,
                     0, dp.d_start, static_cast<const TW*>(dp.d_w), Qs, Q, hp.J, P, QW, ord->as<int32_t>(),
                     rs->as<int32_t>(), static_cast<uint32_t*>(rw->p));
  check_launch("sspi_band_records");
  TmpBuf dd(nd * sizeof(BandDesc));
  hipLaunchKernelGGL(sspi_band_tables, dim3(static_cast<unsigned>(njt), static_cast<unsigned>(P)), dim3(256), 0, 0,
                     rs->as<int32_t>(), hp.J, Q, P, static_cast<BandDesc*>(dd.p));
  check_launch("sspi_band_tables");
  std::vector<BandDesc> descs(nd);
  HIP_OK(hipMemcpy(descs.data(), dd.p, nd * sizeof(BandDesc), hipMemcpyDeviceToHost));
  int widest = 0, last = 0;
  for (const BandDesc& d : descs) {
    widest = std::max(widest, d.W);
    last = std::max(last, d.A + 8 * band_units(d.W));
  }
  // 128 frames per block when the widest band fits a pass, else 64
  const int FR = band_pair_bytes(widest, QW, 128) <= SB_LDS ? 128 : 64;
  if (band_pair_bytes(widest, QW, FR) > SB_LDS) return;  // the gather takes wide bands
  dp.d_bdesc = A.get(nd * sizeof(BandDesc));
  HIP_OK(hipMemcpy(dp.d_bdesc, dd.p, nd * sizeof(BandDesc), hipMemcpyDeviceToDevice));
  dp.d_bnext = static_cast<uint16_t*>(A.get(nd * sizeof(uint16_t)));
  hipLaunchKernelGGL(sspi_band_passes, dim3(static_cast<unsigned>((njt + 255) / 256)), dim3(256), 0, 0,
                     static_cast<const BandDesc*>(dp.d_bdesc), njt, P, QW, FR, dp.d_bnext);
  check_launch("sspi_band_passes");
  int32_t* rstart = static_cast<int32_t*>(A.get(nr * 4));
  uint32_t* rtaps = static_cast<uint32_t*>(A.get(nr * 4 * QW));
  dp.d_border = static_cast<int32_t*>(A.get(order.size() * 4));
  HIP_OK(hipMemcpy(rstart, rs->p, nr * 4, hipMemcpyDeviceToDevice));
  HIP_OK(hipMemcpy(rtaps, rw->p, nr * 4 * QW, hipMemcpyDeviceToDevice));
  HIP_OK(hipMemcpy(dp.d_border, ord->p, order.size() * 4, hipMemcpyDeviceToDevice));
  rs.reset();
  rw.reset();
  HIP_OK(hipDeviceSynchronize());
  // the pair-major records are not read again
  const size_t es = dsize(hp.dtype);
  HIP_OK(hipFree(dp.d_start));
  HIP_OK(hipFree(dp.d_w));
  dp.resident_bytes -= static_cast<size_t>(hp.J) * P * 4 + static_cast<size_t>(hp.J) * P * Qs * es;
  dp.d_start = rstart;
  dp.d_w = rtaps;
  dp.sspi_qw = QW;
  dp.sspi_fr = FR;
  // a band of W columns is staged band_units(W) pieces of 8 columns wide
  dp.sspi_xb = static_cast<int>(round_up(std::max<int64_t>(hp.PN, last) + 32, 8));
  dp.sspi_band = true;
}

void device_build(HostPlan& hp, DevicePlan& dp, int64_t frame_tile, size_t budget) {
  (void)frame_tile;
  dp.device = -1;
  HIP_OK(hipGetDevice(&dp.device));
  Alloc A{dp, budget};
  const int P = hp.P;
  // per-pair cross-spectrum slot: 2 (K - 1) reals padded to 128 elements
  dp.Kp = static_cast<int>(round_up(2 * (hp.K - 1), 128));
  dp.Jpad = round_up(hp.J, JPAD_ROWS);
  dp.d_pm = static_cast<int32_t*>(A.get(P * 4));
  dp.d_pmp = static_cast<int32_t*>(A.get(P * 4));
  dp.d_np = static_cast<int32_t*>(A.get(P * 4));
  dp.d_off = static_cast<int32_t*>(A.get(P * 4));
  upload(dp.d_pm, hp.pair_m);
  upload(dp.d_pmp, hp.pair_mp);
  upload(dp.d_np, hp.np);
  upload(dp.d_off, hp.off);

  if (hp.variant == SRP_LR) {
    if (hp.dtype == SRP_F64) throw Error{SRP_E_UNSUPPORTED, "LR-SRP has no FP64 path"};
    TmpBuf dx(hp.x.size() * sizeof(double));
    upload(dx.p, hp.x);
    build_lr_device(hp, dp, A, dx.as<double>());
    return;
  }

  if (hp.variant == SRP_FD) {
    const size_t es = dsize(hp.dtype);
    const size_t hbytes = static_cast<size_t>(dp.Jpad) * fd_ld(hp, dp, es) * es;
    // resident H up to 16 GiB (and within the budget); beyond, the steering
    // is generated on the fly from the FP64 TDOAs, once per call.  (A 48 GiB
    // cap doubled the serving mix's resident bytes for no throughput: a
    // resident 33 GB H is re-read from HBM on every small batch, which costs
    // about what generating it does.)
    const bool fits = hbytes <= (size_t(16) << 30) && (budget == 0 || hbytes + dp.resident_bytes <= budget);
    dp.fd_gen = hp.fd_steering == 2 || (hp.fd_steering == 0 && !fits);
    if (dp.fd_gen) {
      if (hp.dtype == SRP_F64) throw Error{SRP_E_UNSUPPORTED, "FP64 FD needs the resident steering operand"};
      dp.d_xg = static_cast<double*>(A.get(hp.x.size() * sizeof(double)));
      upload(dp.d_xg, hp.x);
      // few candidate tiles: split the contraction at pair boundaries so that
      // a frame tile has ~512 blocks (up to 8 splits of at least 4 pairs)
      const int64_t nwt = (hp.J + 255) / 256;
      int ks = 1;
      while (ks < 8 && nwt * ks * 2 <= 512 && P / (ks * 2) >= 4) ks *= 2;
      if (ks == 1) {
        // many tiles: balance the last round of the one-block-per-CU launch
        // (fd_gen16) by up to 8 splits of at least 4 pairs (2 m disc: 782
        // tiles in 4 rounds, 3.06 of work; 4 splits: 13 rounds of a quarter,
        // 96.4 ms per 256 frames; 8 splits: 25 rounds of an eighth, 93.1 ms
        // with the larger partial sums)
        int cus = 0;
        HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dp.device));
        cus = std::max(cus, 1);
        double best = std::ceil(static_cast<double>(nwt) / cus);
        for (int k = 2; k <= 8 && P / k >= 4; ++k) {
          const double cost = std::ceil(static_cast<double>(nwt) * k / cus) / k;
          if (cost < 0.99 * best) {
            best = cost;
            ks = k;
          }
        }
      }
      dp.fd_ksplit = ks;
      return;
    }
    dp.d_H = A.get(hbytes);
    // few candidate tiles (small grids, long contractions): split the
    // contraction over blockIdx.z so that the GEMM has ~512 blocks per frame
    // tile; a plan constant, so a frame's map does not depend on its batch
    const int64_t nwt = dp.Jpad / FD16_TILE;
    if (hp.dtype != SRP_F64 && nwt < 64) {
      const int64_t slices = static_cast<int64_t>(P) * dp.Kp * static_cast<int64_t>(es) / (2 * FD16_SB);
      int ks = 1;
      while (ks < 64 && nwt * ks * 2 <= 512 && slices % (ks * 2) == 0 && slices / (ks * 2) >= 16) ks *= 2;
      dp.fd_ksplit = ks;
    }
    double* d_x = nullptr;
    HIP_OK(hipMalloc(&d_x, hp.x.size() * sizeof(double)));
    try {
      upload(d_x, hp.x);
      switch (hp.dtype) {
        case SRP_F32: launch_steering<float>(d_x, hp, dp.Kp, dp.Jpad, fd_ld(hp, dp, es), dp.d_H); break;
        case SRP_BF16: launch_steering<__bf16>(d_x, hp, dp.Kp, dp.Jpad, fd_ld(hp, dp, es), dp.d_H); break;
        case SRP_F16: launch_steering<_Float16>(d_x, hp, dp.Kp, dp.Jpad, fd_ld(hp, dp, es), dp.d_H); break;
        case SRP_FP8_E4M3: launch_steering<fp8>(d_x, hp, dp.Kp, dp.Jpad, fd_ld(hp, dp, es), dp.d_H); break;
        case SRP_F64: launch_steering<double>(d_x, hp, dp.Kp, dp.Jpad, fd_ld(hp, dp, es), dp.d_H); break;
      }
      HIP_OK(hipDeviceSynchronize());
    } catch (...) {
      (void)hipFree(d_x);
      throw;
    }
    HIP_OK(hipFree(d_x));
    return;
  }

  if (hp.fft) {
    // iFFT sampling (46): twiddles of the length-K complex inverse FFT and
    // the factors exp(i pi k / K) that fold the length-2K real transform
    // into it, evaluated in FP64 and rounded once
    dp.logk = 0;
    while ((1 << dp.logk) < hp.K) ++dp.logk;
    std::vector<float2> tw(hp.K / 2), w2(hp.K);
    for (int t = 0; t < hp.K / 2; ++t)
      tw[t] = make_float2(static_cast<float>(std::cos(2.0 * M_PI * t / hp.K)),
                          static_cast<float>(std::sin(2.0 * M_PI * t / hp.K)));
    for (int k = 0; k < hp.K; ++k)
      w2[k] = make_float2(static_cast<float>(std::cos(M_PI * k / hp.K)),
                          static_cast<float>(std::sin(M_PI * k / hp.K)));
    dp.d_tw = static_cast<float2*>(A.get(tw.size() * sizeof(float2)));
    upload(dp.d_tw, tw);
    dp.d_w2 = static_cast<float2*>(A.get(w2.size() * sizeof(float2)));
    upload(dp.d_w2, w2);
  } else {
    // the iDFT table shared by every pair: row j holds lag n = j - max_np,
    // (2 cos, -2 sin)(pi k n / K) in slots 2 (k - 1), 2 (k - 1) + 1, the
    // angle pi (k n mod 2K) / K reduced exactly in integers, then evaluated
    // in FP64; rows past 2 max_np + 1 and bins past K - 1 are zero
    dp.gd_kb = static_cast<int>(round_up(hp.K - 1, GD_CB));
    dp.gd_nct = (2 * hp.max_np + 1 + 31) / 32;
    if (dp.gd_nct > GD_NCT) throw Error{SRP_E_UNSUPPORTED, "too many lags for the direct sampling kernel"};
    if (dp.gd_nct == 3) dp.gd_nct = 4;  // the kernel stages 32, 64 or 128 table rows
    std::vector<float> S(static_cast<size_t>(dp.gd_nct) * 32 * 2 * dp.gd_kb, 0.0f);
    for (int i = 0; i < 2 * hp.max_np + 1; ++i) {
      const int64_t n = i - hp.max_np;
      for (int k = 1; k < hp.K; ++k) {
        int64_t m = (static_cast<int64_t>(k) * n) % (2 * hp.K);
        if (m < 0) m += 2 * hp.K;
        const double ang = M_PI * static_cast<double>(m) / hp.K;
        S[static_cast<size_t>(i) * 2 * dp.gd_kb + 2 * (k - 1)] = static_cast<float>(2.0 * std::cos(ang));
        S[static_cast<size_t>(i) * 2 * dp.gd_kb + 2 * (k - 1) + 1] = static_cast<float>(-2.0 * std::sin(ang));
      }
    }
    dp.d_S = static_cast<float*>(A.get(S.size() * 4));
    upload(dp.d_S, S);
    if (hp.dtype != SRP_F32 && hp.dtype != SRP_F64) {
      // BF16 (hi, lo) halves for the split products: per 4 bins (8 values)
      // 16 bytes of hi then 16 of lo, the FP32 table's byte layout
      std::vector<uint16_t> S16(S.size() * 2);
      for (size_t q = 0; q < S.size() / 8; ++q)
        for (int i = 0; i < 8; ++i) {
          const float v = S[8 * q + i];
          const uint16_t h = bf16_rne(v);
          S16[16 * q + i] = h;
          S16[16 * q + 8 + i] = bf16_rne(v - bf16_float(h));
        }
      dp.d_S16 = A.get(S16.size() * 2);
      upload(static_cast<uint16_t*>(dp.d_S16), S16);
    }
    // frames per block: about four 32-row tiles of (frame, pair) rows, at
    // most GD_FM (frame, microphone) rows of u in LDS
    dp.gd_ft = std::max(1, std::min(128 / P, GD_FM / hp.M));
  }

  if (hp.variant == SRP_SLRI) {
    if (hp.dtype == SRP_F64) throw Error{SRP_E_UNSUPPORTED, "SLRI has no FP64 path"};
    const int R = hp.R;
    const int vrows = 2 * hp.max_np + 1;
    // padded to a whole K slice of the FP32 GEMM and, for the 16-bit and
    // FP8 operands, to a multiple of four MFMA steps of the tall kernel
    dp.Kc = tall_cols(hp.dtype, static_cast<int64_t>(hp.global_fit ? 1 : P) * R);
    TmpBuf dx(hp.x.size() * sizeof(double));
    upload(dx.p, hp.x);
    if (hp.global_fit) {
      build_slri_global_device(hp, dp, A, dx.as<double>());
      return;
    }
    // Gram matrices on the device (FP64 MFMA), eigenvectors on the host
    // (SI keeps every lag: V = I from the host plan, no fit)
    if (hp.form != SRP_SI) {
      const int ntile = (vrows + 63) / 64;
      const size_t gn = static_cast<size_t>(P) * vrows * vrows;
      TmpBuf dg(gn * sizeof(double));
      HIP_OK(hipMemset(dg.p, 0, gn * sizeof(double)));
      hipLaunchKernelGGL(gram_f64, dim3(static_cast<unsigned>(ntile * (ntile + 1) / 2), static_cast<unsigned>(P)),
                         dim3(256), 0, 0, dx.as<double>(), hp.J, dp.d_np, vrows, ntile, dg.as<double>());
      check_launch("gram_f64");
      std::vector<double> gall(gn);
      HIP_OK(hipMemcpy(gall.data(), dg.p, gn * sizeof(double), hipMemcpyDeviceToHost));
      parallel_for(P, host_threads(), [&](int p) {
        const int n = 2 * hp.np[p] + 1;
        std::vector<double> gp(static_cast<size_t>(n) * n);
        const double* src = &gall[static_cast<size_t>(p) * vrows * vrows];
        for (int a = 0; a < n; ++a)
          std::copy(src + static_cast<size_t>(a) * vrows, src + static_cast<size_t>(a) * vrows + n,
                    gp.begin() + static_cast<size_t>(a) * n);
        slri_fit_pair(hp, p, gp);
      });
    }
    // U = Lambda V on the device, staged in FP32 as [Jpad][Kc]
    const size_t ucount = static_cast<size_t>(dp.Jpad) * dp.Kc;
    TmpBuf dv(hp.V.size() * sizeof(double));
    upload(dv.p, hp.V);
    TmpBuf us(ucount * sizeof(float));
    HIP_OK(hipMemset(us.p, 0, ucount * sizeof(float)));
    hipLaunchKernelGGL(slri_u_f64, dim3(static_cast<unsigned>((hp.J + 255) / 256), static_cast<unsigned>(P)),
                       dim3(256), 0, 0, dx.as<double>(), hp.J, dp.d_np, vrows, R, dv.as<double>(), us.as<float>(),
                       dp.Kc);
    check_launch("slri_u_f64");
    // per-pair weight scale (FP8 only) and a power-of-two activation scale
    // bounding |g| by the format's range: |xi| <= 2 (K - 1) since |psi| <= 1
    std::vector<float> sigma(P, 1.0f), gscale(P, 1.0f);
    if (hp.dtype == SRP_FP8_E4M3) {
      TmpBuf um(P * sizeof(float));
      hipLaunchKernelGGL(pair_absmax, dim3(P), dim3(256), 0, 0, us.as<float>(), hp.J, dp.Kc, R, um.as<float>());
      check_launch("pair_absmax");
      std::vector<float> umax(P);
      HIP_OK(hipMemcpy(umax.data(), um.p, P * sizeof(float), hipMemcpyDeviceToHost));
      std::vector<float> inv(P, 1.0f);
      for (int p = 0; p < P; ++p) {
        if (umax[p] > 0) sigma[p] = static_cast<float>(std::exp2(std::ceil(std::log2(umax[p] / 448.0))));
        inv[p] = 1.0f / sigma[p];
      }
      TmpBuf di(P * sizeof(float));
      upload(di.p, inv);
      hipLaunchKernelGGL(scale_pairs, dim3(static_cast<unsigned>((ucount + 255) / 256)), dim3(256), 0, 0,
                         us.as<float>(), dp.Jpad, dp.Kc, R, P, di.as<float>());
      check_launch("scale_pairs");
      HIP_OK(hipDeviceSynchronize());
    }
    double amax_act = 0;
    for (int p = 0; p < P; ++p) {
      double vl1 = 0;
      for (int r = 0; r < R; ++r) {
        double sum = 0;
        for (int i = 0; i < vrows; ++i) sum += std::fabs(hp.V[(static_cast<size_t>(p) * vrows + i) * R + r]);
        vl1 = std::max(vl1, sum);
      }
      amax_act = std::max(amax_act, sigma[p] * vl1 * 2.0 * (hp.K - 1));
    }
    double act = 1.0;
    if (hp.dtype == SRP_FP8_E4M3) act = std::exp2(std::ceil(std::log2(amax_act / 448.0)));
    if (hp.dtype == SRP_F16 && amax_act > 60000.0) act = std::exp2(std::ceil(std::log2(amax_act / 60000.0)));
    for (int p = 0; p < P; ++p) gscale[p] = static_cast<float>(sigma[p] / act);
    dp.tall_alpha = static_cast<float>(act);
    dp.d_U = A.get(ucount * dsize(hp.dtype));
    convert_dtype(hp.dtype, us.as<float>(), dp.d_U, static_cast<int64_t>(ucount));
    HIP_OK(hipDeviceSynchronize());
    std::vector<float> Vf(hp.V.begin(), hp.V.end());
    dp.d_V = static_cast<float*>(A.get(Vf.size() * 4));
    upload(dp.d_V, Vf);
    dp.d_gscale = static_cast<float*>(A.get(P * 4));
    upload(dp.d_gscale, gscale);
    return;
  }

  // SSPI
  if (hp.dtype == SRP_F64) throw Error{SRP_E_UNSUPPORTED, "SSPI has no FP64 path"};
  {
    const int Q = gather_q(hp.Q);  // taps the gather kernel reads (zero-weighted past the selection)
    dp.sspi_q = Q;
    const int es = static_cast<int>(dsize(hp.dtype));
    const int Qs = static_cast<int>(round_up(Q * es, 4) / es);
    std::unique_ptr<TmpBuf> dgs, dgc;
    if (hp.global_fit) {
      dgs.reset(new TmpBuf(hp.gstart.size() * 4));
      dgc.reset(new TmpBuf(hp.gcount.size() * 4));
      upload(dgs->p, hp.gstart);
      upload(dgc->p, hp.gcount);
    }
    // device layouts are pair-major ([P][J] and [P][J][Qs]) so that lanes
    // (consecutive locations) load consecutive records
    TmpBuf dx(hp.x.size() * sizeof(double));
    upload(dx.p, hp.x);
    dp.d_start = static_cast<int32_t*>(A.get(static_cast<size_t>(hp.J) * P * 4));
    dp.d_w = A.get(static_cast<size_t>(hp.J) * P * Qs * es);
    const int njt = static_cast<int>((hp.J + 255) / 256);
    dp.d_win = static_cast<int2*>(A.get(static_cast<size_t>(njt) * P * sizeof(int2)));
    const dim3 gw(static_cast<unsigned>(njt), static_cast<unsigned>(P));
#define SRP_WIN(TW)                                                                                           \
  hipLaunchKernelGGL(sspi_windows<TW>, gw, dim3(256), 0, 0, dx.as<double>(), hp.J, dp.d_np, dp.d_off, hp.Q, Q, \
                     Qs, P, hp.form == SRP_TD ? 1 : 0, dgs ? dgs->as<int32_t>() : nullptr,                     \
                     dgc ? dgc->as<int32_t>() : nullptr, dp.d_start, static_cast<TW*>(dp.d_w), dp.d_win)
    switch (hp.dtype) {
      case SRP_F32: SRP_WIN(float); break;
      case SRP_BF16: SRP_WIN(__bf16); break;
      case SRP_F16: SRP_WIN(_Float16); break;
      case SRP_FP8_E4M3: SRP_WIN(fp8); break;
    }
#undef SRP_WIN
    check_launch("sspi_windows");
    // LDS rows per staged chunk: 32 KB worth (five blocks per CU), or the
    // widest window
    std::vector<int2> wins(static_cast<size_t>(njt) * P);
    HIP_OK(hipMemcpy(wins.data(), dp.d_win, wins.size() * sizeof(int2), hipMemcpyDeviceToHost));
    int widest = 0;
    for (const int2& v : wins) widest = std::max(widest, v.y);
    dp.sspi_cap = std::max(widest, 32 * 1024 / ((SSPI_FT + 4) * 4));
    if (static_cast<size_t>(dp.sspi_cap) * (SSPI_FT + 4) * 4 > 150 * 1024)
      throw Error{SRP_E_UNSUPPORTED, "a candidate tile spans too many lags of one pair for the SSPI tile"};
    if (hp.dtype == SRP_BF16 || hp.dtype == SRP_F16) {
      build_sspi_dense(hp, dp, A, wins, njt, Qs);
      if (!dp.sspi_dense && Q <= 8) {
        if (hp.dtype == SRP_BF16)
          build_sspi_band<__bf16>(hp, dp, A, njt, Qs);
        else
          build_sspi_band<_Float16>(hp, dp, A, njt, Qs);
      }
    }
  }
}

void device_profile_collect(DevicePlan& dp,
                            std::vector<std::pair<std::string, std::pair<double, int64_t>>>& out) {
  out.clear();
  for (const auto& sp : dp.spans) {
    HIP_OK(hipEventSynchronize(sp.stop));
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, sp.start, sp.stop));
    auto it = std::find_if(out.begin(), out.end(), [&](const auto& e) { return e.first == sp.name; });
    if (it == out.end()) {
      out.push_back({sp.name, {0.0, 0}});
      it = out.end() - 1;
    }
    it->second.first += ms;
    it->second.second += 1;
    dp.event_pool.push_back(sp.start);
    dp.event_pool.push_back(sp.stop);
  }
  dp.spans.clear();
}

// Peak picking (10)-(11): one block per map; each thread keeps its best
// (value, index) over a strided sweep (the first index wins among equal
// values), then a tree reduction with the same order.
template <typename T>
__global__ __launch_bounds__(256) void argmax_rows(const T* __restrict__ z, int64_t J, int64_t ld,
                                                   int64_t* __restrict__ idx, double* __restrict__ val) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const T* row = z + static_cast<int64_t>(blockIdx.x) * ld;
  double best = 0.0;
  int64_t bj = -1;
  for (int64_t j = threadIdx.x; j < J; j += 256) {
    const double v = static_cast<double>(row[j]);
    if (v == v && (bj < 0 || v > best)) {
      best = v;
      bj = j;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bj;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double v2 = bv[threadIdx.x + h];
      const int64_t j2 = bi[threadIdx.x + h];
      const int64_t j1 = bi[threadIdx.x];
      if (j2 >= 0 && (j1 < 0 || v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && j2 < j1))) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    idx[blockIdx.x] = bi[0];
    val[blockIdx.x] = bi[0] >= 0 ? bv[0] : 0.0;
  }
}

void device_argmax(const void* maps, bool f64, int64_t L, int64_t J, int64_t ld, int64_t* idx, double* val,
                   hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(argmax_rows<double>, dim3(static_cast<unsigned>(L)), dim3(256), 0, st,
                       static_cast<const double*>(maps), J, ld, idx, val);
  else
    hipLaunchKernelGGL(argmax_rows<float>, dim3(static_cast<unsigned>(L)), dim3(256), 0, st,
                       static_cast<const float*>(maps), J, ld, idx, val);
  check_launch("argmax_rows");
}

void device_free(DevicePlan& dp) {
  for (const auto& sp : dp.spans) {
    (void)hipEventDestroy(sp.start);
    (void)hipEventDestroy(sp.stop);
  }
  for (hipEvent_t e : dp.event_pool) (void)hipEventDestroy(e);
  void* ptrs[] = {dp.d_pm, dp.d_pmp, dp.d_np, dp.d_off, dp.d_H, dp.d_S, dp.d_S16, dp.d_tw, dp.d_w2,
                  dp.d_U, dp.d_V, dp.d_gscale, dp.d_F, dp.d_start, dp.d_w, dp.d_win, dp.d_xg, dp.d_B,
                  dp.d_ctab, dp.d_colmap, dp.d_dtiles, dp.d_gtiles, dp.d_bdesc, dp.d_bnext, dp.d_border, dp.ws};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  dp = DevicePlan{};
}

namespace {

struct WsLayout {
  int64_t Lc = 0, Lpad = 0;
  size_t psi = 0, xi = 0, part = 0, g = 0, g32 = 0, xf = 0, total = 0;
};

WsLayout ws_layout(const HostPlan& hp, const DevicePlan& dp, int64_t L, int64_t frame_tile) {
  WsLayout w;
  w.Lc = std::max<int64_t>(1, std::min(L, frame_tile));
  w.Lpad = round_up(w.Lc, LPAD_ROWS);
  size_t off = 0;
  w.psi = off;
  if (hp.variant == SRP_FD) off = align256(off + static_cast<size_t>(w.Lpad) * fd_ld(hp, dp, dsize(hp.dtype)) * dsize(hp.dtype));
  if (hp.variant == SRP_FD && dp.fd_ksplit > 1) {
    // partial products of the split contraction, [ksplit][Lpad][Jpad]
    w.part = off;
    off = align256(off + static_cast<size_t>(dp.fd_ksplit) * w.Lpad * dp.Jpad * 4);
  }
  if (hp.variant == SRP_LR) {
    // FP32 cross-spectra, the FP32 fat-stage output and its narrowed copy
    off = align256(off + static_cast<size_t>(w.Lpad) * fd_ld(hp, dp, 4) * 4);
    w.g32 = off;
    off = align256(off + static_cast<size_t>(w.Lpad) * dp.Kc * 4);
    w.g = off;
    off = align256(off + static_cast<size_t>(w.Lpad) * dp.Kc * dsize(hp.dtype));
  }
  if (hp.variant != SRP_FD && hp.variant != SRP_LR) {
    // lag-major samples [PN][Lpad] (not needed when the band product reads
    // the iFFT's frame-major samples)
    w.xi = off;
    if (!(hp.variant == SRP_SSPI && dp.sspi_band && hp.fft)) off = align256(off + static_cast<size_t>(hp.PN) * w.Lpad * 4);
    w.part = off;
    // frame-major samples of the iFFT kernel, [Lc][PN]
    if (hp.fft) off = align256(off + static_cast<size_t>(w.Lc) * hp.PN * 4);
  }
  if (hp.variant == SRP_SLRI) {
    w.g = off;
    off = align256(off + static_cast<size_t>(w.Lpad) * dp.Kc * dsize(hp.dtype));
  }
  if (hp.variant == SRP_SSPI && dp.sspi_dense) {
    w.xf = off;  // frame-major samples of the dense-window path (8 shifted copies)
    off = align256(off + static_cast<size_t>(w.Lpad) * 8 * dp.sspi_xw * dsize(hp.dtype));
  }
  if (hp.variant == SRP_SSPI && dp.sspi_band) {
    w.xf = off;  // frame-major FP16 samples of the band product, [Lc][sspi_xb]
    off = align256(off + static_cast<size_t>(w.Lc) * dp.sspi_xb * 2);
  }
  w.total = off;
  return w;
}

template <typename TO, typename TC>
void launch_phat(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L, TO* out,
                 int64_t ld_l, int64_t ld_p, int kslots, hipStream_t st, bool tiled = false) {
  if (L == 0) return;
  dim3 grid((kslots + 63) / 64, static_cast<unsigned>(L));
  const size_t lds = 2 * static_cast<size_t>(hp.M) * 64 * sizeof(TC);
  TRACED(dp, "phat", st,
         hipLaunchKernelGGL((phat_kernel<TO, TC>), grid, dim3(64), lds, st,
                            static_cast<const float2*>(frames), hp.M, hp.K, hp.P, dp.d_pm, dp.d_pmp, out,
                            ld_l, ld_p, kslots, tiled));
  check_launch("phat_kernel");
}

void phat_dispatch(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L,
                   void* out, int dtype, hipStream_t st) {
  const int64_t ld_l = fd_ld(hp, dp, dsize(dtype));
  const int kslots = dp.Kp / 2;
  // the resident-steering GEMM (gemm_fd16: FP32, 16-bit, FP8) and the 16-bit
  // generated-steering kernel (fd_gen16) read psi tile-major
  const bool tiled = hp.variant == SRP_FD && (dp.fd_gen ? dsize(dtype) == 2 : dsize(dtype) <= 4);
  switch (dtype) {
    case SRP_F32: launch_phat<float, float>(hp, dp, frames, L, static_cast<float*>(out), ld_l, dp.Kp, kslots, st, tiled); break;
    case SRP_BF16: launch_phat<__bf16, float>(hp, dp, frames, L, static_cast<__bf16*>(out), ld_l, dp.Kp, kslots, st, tiled); break;
    case SRP_F16: launch_phat<_Float16, float>(hp, dp, frames, L, static_cast<_Float16*>(out), ld_l, dp.Kp, kslots, st, tiled); break;
    case SRP_FP8_E4M3: launch_phat<fp8, float>(hp, dp, frames, L, static_cast<fp8*>(out), ld_l, dp.Kp, kslots, st, tiled); break;
    case SRP_F64: launch_phat<double, double>(hp, dp, frames, L, static_cast<double*>(out), ld_l, dp.Kp, kslots, st); break;
  }
}

// C = alpha X W^T; with ksplit > 1 the contraction (kdim elements) is split
// into ksplit equal parts whose products go to row blocks of cz_rows rows of
// C (partial sums, reduced by the caller).
template <typename T, int BX, int BW, int WGX, int BKB>
void launch_gemm(DevicePlan& dp, const char* kname, const void* X, int64_t ldx, const void* W, int64_t ldw,
                 float* C, int64_t ldc, int nx, int nw, int kdim, float alpha, int64_t Lpad, hipStream_t st,
                 int64_t wrows = 0, int ksplit = 1, int64_t cz_rows = 0) {
  const int nwt = static_cast<int>((wrows ? wrows : dp.Jpad) / BW);
  const int nxt = static_cast<int>(Lpad / BX);
  const int blocks = static_cast<int>(round_up(static_cast<int64_t>(nwt) * nxt, 8));
  TRACED(dp, kname, st,
         hipLaunchKernelGGL((gemm_nt<T, BX, BW, WGX, BKB, false>), dim3(blocks, 1, ksplit), dim3(256), 0, st,
                            static_cast<const GemmBatch*>(nullptr), static_cast<const T*>(X), ldx,
                            static_cast<const T*>(W), ldw, C, ldc, nw, kdim / ksplit, alpha, nx, nwt, nxt,
                            cz_rows));
}

template <typename T>
void launch_big_gemm(DevicePlan& dp, const char* kname, const void* X, int64_t ldx, const void* W, int64_t ldw,
                     float* C, int64_t ldc, int nx, int nw, int kdim, float alpha, int64_t Lpad,
                     hipStream_t st, int ksplit = 1, int64_t cz_rows = 0) {
  {
    // rows of X and W are read up to whole 256-row tiles (Lpad, Jpad rows
    // are allocated)
    // the kernel takes two 64-byte stages per iteration
    if ((static_cast<int64_t>(kdim / ksplit) * static_cast<int64_t>(sizeof(T))) % (2 * FD16_SB) != 0 || kdim % ksplit != 0)
      throw Error{SRP_E_UNSUPPORTED, "FD contraction is not whole 128-byte rows"};
    const int nwt = static_cast<int>(dp.Jpad / FD16_TILE);
    const int nxt = static_cast<int>(Lpad / FD16_TILE);
    const int blocks = static_cast<int>(round_up(static_cast<int64_t>(nwt) * nxt, 8));
    TRACED(dp, kname, st,
           hipLaunchKernelGGL((gemm_fd16<T>), dim3(blocks, 1, ksplit), dim3(256), 0, st, static_cast<const T*>(X),
                              ldx, static_cast<const T*>(W), ldw, C, ldc, nx, nw, kdim / ksplit, alpha, nwt, nxt,
                              cz_rows));
  }
}

// z[l][j] = alpha sum_s part[s][l][j] over the ksplit partial products of
// a split FD contraction, in split order.
__global__ __launch_bounds__(256) void split_reduce(const float* __restrict__ part, int ksplit, int64_t cz_rows,
                                                    int64_t ldp, int L, int64_t J, float alpha,
                                                    float* __restrict__ z, int64_t ldz) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= static_cast<int64_t>(L) * J) return;
  const int64_t l = i / J, j = i % J;
  float s = 0.0f;
  for (int q = 0; q < ksplit; ++q) s += part[(q * cz_rows + l) * ldp + j];
  z[l * ldz + j] = alpha * s;
}

// Frame splits of the tall kernel: the number of ranges per candidate tile
// (1..8, at least four groups each) that minimises rounds x (groups per
// block + 2), where rounds = blocks / resident block slots rounded up (the
// last, partial round leaves slots idle) and the 2 stands for a block's
// fixed cost (its U rows and the first staged groups).
void tall_split(DevicePlan& dp, const void* kern, int threads, int njt, int ngroups, int& nsplit, int& gps) {
  int slots = 0;
  for (const auto& ks : dp.tall_slots)
    if (ks.first == kern) slots = ks.second;
  if (slots == 0) {
    int per_cu = 0, cus = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dp.device));
    slots = std::max(1, per_cu) * std::max(1, cus);
    dp.tall_slots.emplace_back(kern, slots);
  }
  nsplit = 1;
  int64_t best = -1;
  for (int s = 1; s <= 8 && (s == 1 || ngroups / s >= 4); ++s) {
    const int64_t rounds = (static_cast<int64_t>(njt) * s + slots - 1) / slots;
    const int64_t cost = rounds * ((ngroups + s - 1) / s + 2);
    if (best < 0 || cost < best) {
      best = cost;
      nsplit = s;
    }
  }
  gps = (ngroups + nsplit - 1) / nsplit;
  nsplit = (ngroups + gps - 1) / gps;
}

// FD with generated steering: 256-frame tiles (waves 2 x 2) for large
// batches, 64-frame tiles (waves 1 x 4) for small ones.
template <typename T>
void launch_fd_gen(const HostPlan& hp, DevicePlan& dp, const void* psi, int64_t ldpsi, int64_t kfd, float* z,
                   int64_t ldz, int64_t Lc, int64_t Lpad, float* part, hipStream_t st) {
  const int nw = static_cast<int>((hp.J + 255) / 256);  // fd_gen's 256-candidate tiles
  const int kdim = static_cast<int>(kfd);
  // split contraction (a plan constant, so a frame's map does not depend on
  // its batch): partial products into the workspace, then a fixed-order
  // reduction
  const int ks = dp.fd_ksplit;
  const int pps = (hp.P + ks - 1) / ks;
  float* c = ks > 1 ? part : z;
  const int64_t ldc = ks > 1 ? dp.Jpad : ldz;
  const float alpha = ks > 1 ? 1.0f : 2.0f;
  if constexpr (std::is_same<T, float>::value) {
    // FP32: 64-frame tiles at every batch size, with per-pair accumulators
    // (the FP32 matrix cores, not the tile's operand reuse, bound this form)
    const int nxt = static_cast<int>((Lc + 63) / 64);
    const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(nw) * nxt, 8));
    TRACED(dp, "fd_gen", st,
           hipLaunchKernelGGL((fd_gen<T, 64, 1, true>), dim3(blocks, ks), dim3(256), 0, st,
                              static_cast<const T*>(psi), ldpsi, dp.d_xg, hp.J, hp.K, dp.Kp, c, ldc,
                              static_cast<int>(Lc), kdim, alpha, nw, nxt, pps, Lpad));
  } else if (sizeof(T) == 2) {
    // 16-bit: generation overlapped with the MFMAs, 256- or 64-frame tiles
    if constexpr (sizeof(T) == 2) {
      if ((static_cast<int64_t>(dp.Kp) * 2) % (2 * FD16_SB) != 0 || ldpsi * 2 % FD16_SB != 0)
        throw Error{SRP_E_UNSUPPORTED, "FD pair slots are not whole 128-byte rows"};
      const int bxf = Lc > 128 ? 256 : 64;
      const int nxt = static_cast<int>((Lc + bxf - 1) / bxf);
      const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(nw) * nxt, 8));
      if (bxf == 256)
        TRACED(dp, "fd_gen", st,
               hipLaunchKernelGGL((fd_gen16<T, 256>), dim3(blocks, ks), dim3(256), 0, st, static_cast<const T*>(psi),
                                  ldpsi, dp.d_xg, hp.J, hp.K, dp.Kp, c, ldc, static_cast<int>(Lc), hp.P, alpha, nw, nxt,
                                  pps, Lpad));
      else
        TRACED(dp, "fd_gen", st,
               hipLaunchKernelGGL((fd_gen16<T, 64>), dim3(blocks, ks), dim3(256), 0, st, static_cast<const T*>(psi),
                                  ldpsi, dp.d_xg, hp.J, hp.K, dp.Kp, c, ldc, static_cast<int>(Lc), hp.P, alpha, nw, nxt,
                                  pps, Lpad));
    }
  } else if (Lc > 128) {
    const int nxt = static_cast<int>((Lc + 255) / 256);
    const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(nw) * nxt, 8));
    TRACED(dp, "fd_gen", st,
           hipLaunchKernelGGL((fd_gen<T, 256, 2>), dim3(blocks, ks), dim3(256), 0, st, static_cast<const T*>(psi),
                              ldpsi, dp.d_xg, hp.J, hp.K, dp.Kp, c, ldc, static_cast<int>(Lc), kdim, alpha, nw, nxt,
                              pps, Lpad));
  } else {
    const int nxt = static_cast<int>((Lc + 63) / 64);
    const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(nw) * nxt, 8));
    TRACED(dp, "fd_gen", st,
           hipLaunchKernelGGL((fd_gen<T, 64, 1>), dim3(blocks, ks), dim3(256), 0, st, static_cast<const T*>(psi),
                              ldpsi, dp.d_xg, hp.J, hp.K, dp.Kp, c, ldc, static_cast<int>(Lc), kdim, alpha, nw, nxt,
                              pps, Lpad));
  }
  if (ks > 1) {
    const int64_t n = Lc * hp.J;
    TRACED(dp, "split_reduce", st,
           hipLaunchKernelGGL(split_reduce, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, part, ks,
                              Lpad, dp.Jpad, static_cast<int>(Lc), hp.J, 2.0f, z, ldz));
  }
}

template <typename T>
void launch_tall_gemm(DevicePlan& dp, const void* X, int64_t ldx, const void* W, int64_t ldw, float* C,
                      int64_t ldc, int nx, int nw, int kdim, float alpha, int64_t Lpad, hipStream_t st,
                      const int32_t* ctab = nullptr, const int32_t* tlist = nullptr, int ntl = 0) {
  const int steps = kdim * static_cast<int>(sizeof(T)) / Mfma<T>::STEP;
  const int rowb = kdim * static_cast<int>(sizeof(T));
  // rows of at most 1 KB (16-bit: 1280 bytes, past 1 KB on six compute waves
  // and without tile lists): U rows in registers, g streamed through LDS by
  // the loader wave; anything else takes the general MFMA GEMM.  FP32 rows
  // run on v_mfma_f32_32x32x2f32 with the same sums as the general GEMM
  // (maps bitwise equal; per-pair SLRI R = 8 at 125,000 x 1000: 0.633 ->
  // 0.561 ms per call)
  const bool longrow = sizeof(T) == 2 && rowb > 1024 && rowb <= TALL_ROW_MAX16 && !ctab && !tlist;
  {
    if ((rowb <= 1024 || longrow) && (steps % 4 == 0 || (longrow && steps % 2 == 0)) && rowb % Mfma<T>::STEP == 0 &&
        36 * ldc < (int64_t(1) << 31)) {
      const int ngroups = (nx + 31) / 32;
#define SRP_WS(NSV, CW, CT)                                                                                   \
  case NSV:                                                                                                   \
    if constexpr (NSV * Mfma<T>::STEP <= (sizeof(T) == 2 ? TALL_ROW_MAX16 : 1024)) {                          \
    const int njt = tlist ? ntl : static_cast<int>((nw + 32 * CW - 1) / (32 * CW));                           \
    auto kern = ctab ? &tall_ws<T, NSV, CW, CT> : &tall_ws<T, NSV, CW, false>;                                \
    int nsplit, gps;                                                                                          \
    tall_split(dp, reinterpret_cast<const void*>(kern), 64 * (CW + 1), njt, ngroups, nsplit, gps);            \
    const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(njt) * nsplit, 8));          \
    TRACED(dp, ctab ? "sspi_dense" : "gemm_tall", st,                                                         \
           hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * (CW + 1)), 0, st, static_cast<const T*>(X), ldx,  \
                              static_cast<int>(Lpad), static_cast<const T*>(W), ldw, C, ldc, nx,               \
                              static_cast<int64_t>(nw), alpha, njt, nsplit, gps, ctab, tlist));                \
    return;                                                                                                   \
    }                                                                                                         \
    break;
      // chunk tables (dense-window SSPI) come with 16-bit operands only
      constexpr bool CT = !std::is_same<T, float>::value;
      if (!longrow) {
        switch (steps) {
          SRP_WS(4, TALL_CW, CT) SRP_WS(8, TALL_CW, CT) SRP_WS(12, TALL_CW, CT) SRP_WS(16, TALL_CW, CT)
          SRP_WS(20, TALL_CW, CT) SRP_WS(24, TALL_CW, CT) SRP_WS(28, TALL_CW, CT) SRP_WS(32, TALL_CW, CT)
          default: break;
        }
      } else {
        switch (steps) {
          // never with a chunk table (longrow excludes it)
          SRP_WS(34, TALL_CW_LONG, false) SRP_WS(36, TALL_CW_LONG, false) SRP_WS(38, TALL_CW_LONG, false)
          SRP_WS(40, TALL_CW_LONG, false)
          default: break;
        }
      }
#undef SRP_WS
    }
  }
  if (ctab || tlist) throw Error{SRP_E_UNSUPPORTED, "dense-window SSPI needs the streaming tall kernel"};
  if constexpr (std::is_same<T, float>::value)
    launch_gemm<T, TALL_BX, TALL_BW, TALL_WGX, TALL_BKB>(dp, "gemm_tall", X, ldx, W, ldw, C, ldc, nx, nw, kdim, alpha,
                                                        Lpad, st);
  else
    launch_gemm<T, TALL16_BX, TALL16_BW, TALL16_WGX, TALL16_BKB>(dp, "gemm_tall", X, ldx, W, ldw, C, ldc, nx, nw, kdim,
                                                                alpha, Lpad, st);
}

// Direct GCC sampling (40) straight from the frames into xi^T [PN][ldxi].
void launch_slices(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t Lc, float* xiT, int64_t ldxi,
                   hipStream_t st, bool exact) {
  // split BF16 products for 16-bit and FP8 plans (not for the FP32 export)
  const bool split = !exact && dp.d_S16 != nullptr;
  const int ft = dp.gd_ft;
  const int nrt = (ft * hp.P + 31) / 32;
  const int ntiles = nrt * dp.gd_nct;
  const dim3 grid(static_cast<unsigned>((Lc + ft - 1) / ft), static_cast<unsigned>((ntiles + GD_TILES - 1) / GD_TILES));
  const int NCT = dp.gd_nct <= 1 ? 1 : (dp.gd_nct <= 2 ? 2 : 4);
  const size_t lds = static_cast<size_t>(GD_FM + 1 + 32 * NCT) * GD_ROWB;
#define SRP_GD(NC)                                                                                            \
  do {                                                                                                        \
    auto kern = split ? &gcc_direct<NC, true> : &gcc_direct<NC, false>;                                      \
    if (lds > 65536)                                                                                          \
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),                                         \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));         \
    TRACED(dp, "gcc_direct", st,                                                                              \
           hipLaunchKernelGGL(kern, grid, dim3(1024), lds, st, static_cast<const float2*>(frames), hp.M, hp.K,  \
                              static_cast<int>(Lc), hp.P, dp.d_pm, dp.d_pmp, dp.d_np, dp.d_off, hp.max_np,    \
                              split ? static_cast<const float*>(dp.d_S16) : dp.d_S, dp.gd_kb, ft, nrt,       \
                              dp.gd_nct, xiT, ldxi));                                                         \
  } while (0)
  if (NCT == 1)
    SRP_GD(1);
  else if (NCT == 2)
    SRP_GD(2);
  else
    SRP_GD(4);
#undef SRP_GD
}

// SLRI fat stage g_p = V_p^T xi_p (eq. (57)) for every frame of the tile.
template <typename TG>
void launch_fat(const HostPlan& hp, DevicePlan& dp, const float* xiT, int64_t ldxi, int64_t Lc, void* g,
                hipStream_t st) {
  if (hp.global_fit) {
    if (dp.Kc % 32 != 0) throw Error{SRP_E_UNSUPPORTED, "global SLRI needs the tall width in 32-column tiles"};
    const dim3 g2(static_cast<unsigned>((Lc + 31) / 32), static_cast<unsigned>(dp.Kc / 32));
    TRACED(dp, "slri_fat", st,
           hipLaunchKernelGGL(slri_fat_global_mfma<TG>, g2, dim3(512), 0, st, xiT, ldxi, static_cast<int>(Lc),
                              hp.PN, dp.d_V, dp.Kc, dp.d_gscale, static_cast<TG*>(g)));
    return;
  }
  const int vrows = 2 * hp.max_np + 1;
  const dim3 g2(static_cast<unsigned>((Lc + 63) / 64), static_cast<unsigned>(hp.P + 1));
  TRACED(dp, "slri_fat", st,
         hipLaunchKernelGGL(slri_fat_mfma<TG>, g2, dim3(256), 0, st, xiT, ldxi, static_cast<int>(Lc), dp.d_np,
                            dp.d_off, dp.d_V, vrows, hp.R, dp.d_gscale, hp.P, static_cast<TG*>(g), dp.Kc));
}

template <int MODE, typename TG>
void launch_front(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t Lc, float* xiT, int64_t ldxi,
                  float* part, void* g, hipStream_t st, bool lag_major = true, bool exact = false) {
  if (hp.fft) {
    const dim3 grid(static_cast<unsigned>(Lc * hp.P));
#define SRP_FFT(LK)                                                                                           \
  case LK:                                                                                                    \
    TRACED(dp, "gcc_fft", st,                                                                                 \
           hipLaunchKernelGGL(gcc_fft<LK>, grid, dim3(256), 0, st, static_cast<const float2*>(frames), hp.M,  \
                              hp.P, dp.d_pm, dp.d_pmp, dp.d_np, dp.d_off, dp.d_tw, dp.d_w2, part,             \
                              static_cast<int64_t>(hp.PN)));                                                  \
    break;
    switch (dp.logk) {
      SRP_FFT(2) SRP_FFT(3) SRP_FFT(4) SRP_FFT(5) SRP_FFT(6) SRP_FFT(7) SRP_FFT(8) SRP_FFT(9) SRP_FFT(10)
      SRP_FFT(11)
      default: throw Error{SRP_E_UNSUPPORTED, "iFFT sampling needs N a power of two, at most 4096"};
    }
#undef SRP_FFT
    if (!lag_major) return;  // the caller reads the frame-major samples in part
    const dim3 tgrid(static_cast<unsigned>((hp.PN + 31) / 32), static_cast<unsigned>((Lc + 31) / 32));
    TRACED(dp, "transpose_lp", st,
           hipLaunchKernelGGL(transpose_lp, tgrid, dim3(256), 0, st, part, static_cast<int64_t>(hp.PN),
                              static_cast<int>(Lc), hp.PN, xiT, ldxi));
  } else {
    launch_slices(hp, dp, frames, Lc, xiT, ldxi, st, exact);
  }
  if constexpr (MODE == 1) {
    launch_fat<TG>(hp, dp, xiT, ldxi, Lc, g, st);
  }
}


template <typename TW, int Q>
void launch_sspi_q(const HostPlan& hp, DevicePlan& dp, const float* xiT, int64_t Lpad,
                   int64_t Lc, float* z, int64_t ldz, hipStream_t st) {
  constexpr bool PAIRS = !std::is_same<TW, float>::value;
  const int es = static_cast<int>(sizeof(TW));
  const int Qs = static_cast<int>(round_up(Q * es, 4) / es);
  const size_t lds = static_cast<size_t>(dp.sspi_cap) * (SSPI_FT + 4) * 4;
  auto kern = &sspi_gather<TW, Q, SSPI_FT, PAIRS>;
  if (lds > 60 * 1024)
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(lds)));
  // with the dense-window path only the tiles it left over
  const int32_t* tl = dp.sspi_dense ? dp.d_gtiles : nullptr;
  const int nj = dp.sspi_dense ? dp.n_gtiles : static_cast<int>((hp.J + 255) / 256);
  if (nj == 0) return;
  const int nf = static_cast<int>((Lc + SSPI_FT - 1) / SSPI_FT);
  const int blocks = static_cast<int>(round_up(static_cast<int64_t>(nj) * nf, 8));
  TRACED(dp, "sspi_gather", st,
         hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, xiT, Lpad, hp.PN, dp.d_start,
                            static_cast<const TW*>(dp.d_w), Qs, dp.d_win, dp.sspi_cap, hp.P, hp.J,
                            static_cast<int>(Lc), nf, z, ldz, tl, nj));
}

template <int QW, int FR>
void launch_band_qw(const HostPlan& hp, DevicePlan& dp, const _Float16* xb, int64_t Lc, float* z, int64_t ldz,
                    hipStream_t st) {
  auto kern = &sspi_band<QW, FR>;
  const int lds = SB_LDS + 2 * SB_MAXPP * static_cast<int>(sizeof(BandDesc));
  HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  const int njt = static_cast<int>((hp.J + 255) / 256);
  const int nf = static_cast<int>((Lc + FR - 1) / FR);
  const unsigned blocks = static_cast<unsigned>(round_up(static_cast<int64_t>(njt) * nf, 8));
  TRACED(dp, "sspi_band", st,
         hipLaunchKernelGGL(kern, dim3(blocks), dim3(512), lds, st, xb, static_cast<int64_t>(dp.sspi_xb),
                            static_cast<int>(Lc), dp.d_start, static_cast<const uint32_t*>(dp.d_w),
                            static_cast<const BandDesc*>(dp.d_bdesc), dp.d_bnext, dp.d_border, hp.P, hp.J,
                            static_cast<int>(Lc), nf, z, ldz));
}

// SSPI band product of the frame tile: frame-major FP16 samples, then the
// band kernel over every candidate tile.
void launch_band(const HostPlan& hp, DevicePlan& dp, const float* xiT, int64_t Lpad, const float* part,
                 _Float16* xb, int64_t Lc, float* z, int64_t ldz, hipStream_t st) {
  const int XB = dp.sspi_xb;
  if (hp.fft) {
    const int64_t n = Lc * XB;
    TRACED(dp, "xi_to_frames", st,
           hipLaunchKernelGGL(rows_to_f16, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, part,
                              static_cast<int64_t>(hp.PN), static_cast<int>(Lc), hp.PN, XB, xb,
                              static_cast<int64_t>(XB)));
  } else {
    const dim3 gt(static_cast<unsigned>((XB + 31) / 32), static_cast<unsigned>((Lc + 31) / 32));
    TRACED(dp, "xi_to_frames", st,
           hipLaunchKernelGGL(xi_rows16, gt, dim3(256), 0, st, xiT, Lpad, static_cast<int>(Lc), hp.PN, XB, xb,
                              static_cast<int64_t>(XB)));
  }
  if (dp.sspi_qw == 2) {
    if (dp.sspi_fr == 128)
      launch_band_qw<2, 128>(hp, dp, xb, Lc, z, ldz, st);
    else
      launch_band_qw<2, 64>(hp, dp, xb, Lc, z, ldz, st);
  } else {
    if (dp.sspi_fr == 128)
      launch_band_qw<4, 128>(hp, dp, xb, Lc, z, ldz, st);
    else
      launch_band_qw<4, 64>(hp, dp, xb, Lc, z, ldz, st);
  }
}

template <typename TW>
void launch_sspi(const HostPlan& hp, DevicePlan& dp, const float* xiT, int64_t Lpad, int64_t Lc,
                 float* z, int64_t ldz, hipStream_t st) {
  switch (dp.sspi_q) {
    case 1: launch_sspi_q<TW, 1>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 2: launch_sspi_q<TW, 2>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 3: launch_sspi_q<TW, 3>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 4: launch_sspi_q<TW, 4>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 5: launch_sspi_q<TW, 5>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 6: launch_sspi_q<TW, 6>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 7: launch_sspi_q<TW, 7>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 8: launch_sspi_q<TW, 8>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 10: launch_sspi_q<TW, 10>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 12: launch_sspi_q<TW, 12>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    case 16: launch_sspi_q<TW, 16>(hp, dp, xiT, Lpad, Lc, z, ldz, st); break;
    default: throw Error{SRP_E_UNSUPPORTED, "SSPI gather with this Q is not built"};
  }
}

}  // namespace

size_t workspace_bytes(const HostPlan& hp, const DevicePlan& dp, int64_t L, int64_t frame_tile) {
  return ws_layout(hp, dp, L, frame_tile).total;
}

static void* ensure_ws(DevicePlan& dp, void* ws, size_t ws_bytes, size_t need) {
  if (ws) {
    if (ws_bytes < need)
      throw Error{SRP_E_INVALID, "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need)};
    if (reinterpret_cast<uintptr_t>(ws) & 255) throw Error{SRP_E_INVALID, "workspace must be 256-byte aligned"};
    return ws;
  }
  if (dp.ws_bytes < need) {
    if (dp.ws) HIP_OK(hipFree(dp.ws));
    dp.ws = nullptr;
    dp.ws_bytes = 0;
    HIP_OK(hipMalloc(&dp.ws, need));
    dp.ws_bytes = need;
  }
  return dp.ws;
}

void device_compute(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L, void* maps,
                    int64_t ldm, void* ws, size_t ws_bytes, int64_t frame_tile, hipStream_t st) {
  if (L <= 0) return;
  const WsLayout lay = ws_layout(hp, dp, L, frame_tile);
  unsigned char* base = static_cast<unsigned char*>(ensure_ws(dp, ws, ws_bytes, lay.total));
  const int64_t frame_elems = static_cast<int64_t>(hp.M) * (hp.K + 1);  // complex per frame
  const int64_t kfd = static_cast<int64_t>(hp.P) * dp.Kp;           // FD contraction length
  const int64_t ldpsi = fd_ld(hp, dp, dsize(hp.dtype));              // row pitch of psi and H
  for (int64_t l0 = 0; l0 < L; l0 += lay.Lc) {
    const int64_t Lc = std::min(lay.Lc, L - l0);
    const void* fr = static_cast<const float2*>(frames) + l0 * frame_elems;
    void* psi = base + lay.psi;
    if (hp.variant == SRP_LR) {
      // eq. (29): g = H_fat psi as the real product psi F^T (FP32 operands,
      // MFMA), narrowed to the operand type, then z = 2 Re[H_tall g]
      phat_dispatch(hp, dp, fr, Lc, psi, SRP_F32, st);
      float* g32 = reinterpret_cast<float*>(base + lay.g32);
      float* z = static_cast<float*>(maps) + l0 * ldm;
      launch_gemm<float, BIG_BX, BIG_BW, BIG_WGX, big_bkb<float>()>(dp, "lr_fat", psi, fd_ld(hp, dp, 4), dp.d_F, kfd,
                                                                   g32, dp.Kc, (int)Lc, dp.Kc, (int)kfd, 1.0f,
                                                                   lay.Lpad, st, dp.Fpad);
      void* g = base + lay.g;
      const int64_t ng = Lc * dp.Kc;
      const dim3 cg(static_cast<unsigned>((ng + 255) / 256));
      switch (hp.dtype) {
        case SRP_F32:
          launch_tall_gemm<float>(dp, g32, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_BF16:
          TRACED(dp, "lr_narrow", st, hipLaunchKernelGGL(scale_convert<__bf16>, cg, dim3(256), 0, st, g32, static_cast<__bf16*>(g), ng, dp.lr_gscale));
          launch_tall_gemm<__bf16>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_F16:
          TRACED(dp, "lr_narrow", st, hipLaunchKernelGGL(scale_convert<_Float16>, cg, dim3(256), 0, st, g32, static_cast<_Float16*>(g), ng, dp.lr_gscale));
          launch_tall_gemm<_Float16>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_FP8_E4M3:
          TRACED(dp, "lr_narrow", st, hipLaunchKernelGGL(scale_convert<fp8>, cg, dim3(256), 0, st, g32, static_cast<fp8*>(g), ng, dp.lr_gscale));
          launch_tall_gemm<fp8>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
      }
      continue;
    }
    if (hp.variant == SRP_FD) {
      phat_dispatch(hp, dp, fr, Lc, psi, hp.dtype, st);
      if (hp.dtype == SRP_F64) {
        double* z = static_cast<double*>(maps) + l0 * ldm;
        dim3 grid(static_cast<unsigned>((hp.J + 63) / 64), static_cast<unsigned>((Lc + 63) / 64));
        TRACED(dp, "gemm_fd_f64", st,
               hipLaunchKernelGGL(gemm_nt_f64, grid, dim3(256), 0, st, static_cast<const double*>(psi), ldpsi,
                                  static_cast<const double*>(dp.d_H), ldpsi, z, ldm, static_cast<int>(Lc),
                                  static_cast<int>(hp.J), static_cast<int>(kfd), 2.0));
        check_launch("gemm_nt_f64");
        continue;
      }
      float* z = static_cast<float*>(maps) + l0 * ldm;
      if (dp.fd_gen) {
        float* part = reinterpret_cast<float*>(base + lay.part);
        switch (hp.dtype) {
          case SRP_F32: launch_fd_gen<float>(hp, dp, psi, ldpsi, kfd, z, ldm, Lc, lay.Lpad, part, st); break;
          case SRP_BF16: launch_fd_gen<__bf16>(hp, dp, psi, ldpsi, kfd, z, ldm, Lc, lay.Lpad, part, st); break;
          case SRP_F16: launch_fd_gen<_Float16>(hp, dp, psi, ldpsi, kfd, z, ldm, Lc, lay.Lpad, part, st); break;
          case SRP_FP8_E4M3: launch_fd_gen<fp8>(hp, dp, psi, ldpsi, kfd, z, ldm, Lc, lay.Lpad, part, st); break;
        }
        continue;
      }
      {
        // split contraction: partial products into the workspace, then a
        // fixed-order reduction
        const int ks = dp.fd_ksplit;
        float* part = reinterpret_cast<float*>(base + lay.part);
        float* c = ks > 1 ? part : z;
        const int64_t ldc = ks > 1 ? dp.Jpad : ldm;
        const float a = ks > 1 ? 1.0f : 2.0f;
        switch (hp.dtype) {
          case SRP_F32: launch_big_gemm<float>(dp, "gemm_fd", psi, ldpsi, dp.d_H, ldpsi, c, ldc, (int)Lc, (int)hp.J, (int)kfd, a, lay.Lpad, st, ks, lay.Lpad); break;
          case SRP_BF16: launch_big_gemm<__bf16>(dp, "gemm_fd", psi, ldpsi, dp.d_H, ldpsi, c, ldc, (int)Lc, (int)hp.J, (int)kfd, a, lay.Lpad, st, ks, lay.Lpad); break;
          case SRP_F16: launch_big_gemm<_Float16>(dp, "gemm_fd", psi, ldpsi, dp.d_H, ldpsi, c, ldc, (int)Lc, (int)hp.J, (int)kfd, a, lay.Lpad, st, ks, lay.Lpad); break;
          case SRP_FP8_E4M3: launch_big_gemm<fp8>(dp, "gemm_fd", psi, ldpsi, dp.d_H, ldpsi, c, ldc, (int)Lc, (int)hp.J, (int)kfd, a, lay.Lpad, st, ks, lay.Lpad); break;
        }
        if (ks > 1) {
          const int64_t n = Lc * hp.J;
          TRACED(dp, "split_reduce", st,
                 hipLaunchKernelGGL(split_reduce, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, part,
                                    ks, lay.Lpad, dp.Jpad, static_cast<int>(Lc), hp.J, 2.0f, z, ldm));
        }
      }
      continue;
    }
    // SLRI and SSPI: PHAT + sampling (+ fat stage) straight from the frames
    float* xiT = reinterpret_cast<float*>(base + lay.xi);
    float* part = reinterpret_cast<float*>(base + lay.part);
    float* z = static_cast<float*>(maps) + l0 * ldm;
    if (hp.variant == SRP_SLRI) {
      void* g = base + lay.g;
      switch (hp.dtype) {
        case SRP_F32:
          launch_front<1, float>(hp, dp, fr, Lc, xiT, lay.Lpad, part, g, st);
          launch_tall_gemm<float>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_BF16:
          launch_front<1, __bf16>(hp, dp, fr, Lc, xiT, lay.Lpad, part, g, st);
          launch_tall_gemm<__bf16>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_F16:
          launch_front<1, _Float16>(hp, dp, fr, Lc, xiT, lay.Lpad, part, g, st);
          launch_tall_gemm<_Float16>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
        case SRP_FP8_E4M3:
          launch_front<1, fp8>(hp, dp, fr, Lc, xiT, lay.Lpad, part, g, st);
          launch_tall_gemm<fp8>(dp, g, dp.Kc, dp.d_U, dp.Kc, z, ldm, (int)Lc, (int)hp.J, dp.Kc, dp.tall_alpha, lay.Lpad, st);
          break;
      }
    } else {
      if (dp.sspi_band) {
        // band product on the matrix cores; the iFFT's frame-major samples
        // feed it directly
        launch_front<0, float>(hp, dp, fr, Lc, xiT, lay.Lpad, part, nullptr, st, !hp.fft);
        _Float16* xb = reinterpret_cast<_Float16*>(base + lay.xf);
        launch_band(hp, dp, xiT, lay.Lpad, part, xb, Lc, z, ldm, st);
        continue;
      }
      launch_front<0, float>(hp, dp, fr, Lc, xiT, lay.Lpad, part, nullptr, st);
      if (dp.sspi_dense) {
        // dense windows on the matrix cores: frame-major samples, then the
        // streaming tall kernel with the per-tile chunk table
        void* xf = base + lay.xf;
        const int64_t ldf = 8 * static_cast<int64_t>(dp.sspi_xw);
        const dim3 gt(static_cast<unsigned>((dp.sspi_xw + 31) / 32), static_cast<unsigned>((Lc + 31) / 32));
        if (hp.dtype == SRP_BF16) {
          TRACED(dp, "xi_to_frames", st,
                 hipLaunchKernelGGL(xi_to_frames<__bf16>, gt, dim3(256), 0, st, xiT, lay.Lpad, static_cast<int>(Lc),
                                    dp.sspi_pna, dp.sspi_xw, dp.d_colmap, static_cast<__bf16*>(xf), ldf));
          launch_tall_gemm<__bf16>(dp, xf, ldf, dp.d_B, dp.sspi_kmax, z, ldm, (int)Lc, (int)hp.J,
                                 dp.sspi_kmax, 1.0f, lay.Lpad, st, dp.d_ctab, dp.d_dtiles, dp.n_dtiles);
          if (dp.n_gtiles) launch_sspi<__bf16>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st);
        } else {
          TRACED(dp, "xi_to_frames", st,
                 hipLaunchKernelGGL(xi_to_frames<_Float16>, gt, dim3(256), 0, st, xiT, lay.Lpad, static_cast<int>(Lc),
                                    dp.sspi_pna, dp.sspi_xw, dp.d_colmap, static_cast<_Float16*>(xf), ldf));
          launch_tall_gemm<_Float16>(dp, xf, ldf, dp.d_B, dp.sspi_kmax, z, ldm, (int)Lc, (int)hp.J,
                                 dp.sspi_kmax, 1.0f, lay.Lpad, st, dp.d_ctab, dp.d_dtiles, dp.n_dtiles);
          if (dp.n_gtiles) launch_sspi<_Float16>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st);
        }
        continue;
      }
      switch (hp.dtype) {
        case SRP_F32: launch_sspi<float>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st); break;
        case SRP_BF16: launch_sspi<__bf16>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st); break;
        case SRP_F16: launch_sspi<_Float16>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st); break;
        case SRP_FP8_E4M3: launch_sspi<fp8>(hp, dp, xiT, lay.Lpad, Lc, z, ldm, st); break;
      }
    }
  }
}

void device_crossspec(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L, void* psi,
                      hipStream_t st) {
  const int64_t ld_p = 2 * (hp.K - 1);
  launch_phat<float, float>(hp, dp, frames, L, static_cast<float*>(psi), hp.P * ld_p, ld_p, hp.K - 1, st);
}

// ------------------------------------------------ static scratch workspace --
//
// The workspace of srp_compute_static: a fixed array in device memory, one
// copy per GPU (held until the process ends).  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is kept per device.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

static void* scratch_address(int device) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) throw Error{SRP_E_INVALID, "static scratch needs a device plan"};
  if (static_cast<size_t>(device) >= addr.size()) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != device) HIP_OK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      throw Error{SRP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    addr[device] = p;
  }
  return addr[device];
}

void device_compute_static(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L, void* maps,
                           int64_t ldm, int64_t frame_tile, hipStream_t st) {
  if (L <= 0) return;
  // the largest frame tile (at most the plan's) whose workspace fits; below
  // the row padding of the workspace a smaller tile saves nothing
  int64_t tile = std::min(L, frame_tile);
  while (tile > LPAD_ROWS && workspace_bytes(hp, dp, tile, tile) > STATIC_SCRATCH_BYTES) tile = (tile + 1) / 2;
  const size_t need = workspace_bytes(hp, dp, tile, tile);
  if (need > STATIC_SCRATCH_BYTES)
    throw Error{SRP_E_UNSUPPORTED, "workspace of " + std::to_string(need) + " bytes for a " + std::to_string(tile) +
                                       "-frame tile exceeds the static scratch of " +
                                       std::to_string(STATIC_SCRATCH_BYTES) + " bytes; use srp_compute"};
  device_compute(hp, dp, frames, L, maps, ldm, scratch_address(dp.device), STATIC_SCRATCH_BYTES, tile, st);
}

void device_gcc_samples(const HostPlan& hp, DevicePlan& dp, const void* frames, int64_t L, float* xi,
                        void* ws, size_t ws_bytes, int64_t frame_tile, hipStream_t st) {
  if (L <= 0) return;
  const WsLayout lay = ws_layout(hp, dp, L, frame_tile);
  unsigned char* base = static_cast<unsigned char*>(ensure_ws(dp, ws, ws_bytes, lay.total));
  const int64_t frame_elems = static_cast<int64_t>(hp.M) * (hp.K + 1);
  for (int64_t l0 = 0; l0 < L; l0 += lay.Lc) {
    const int64_t Lc = std::min(lay.Lc, L - l0);
    const void* fr = static_cast<const float2*>(frames) + l0 * frame_elems;
    float* xiT = reinterpret_cast<float*>(base + lay.xi);
    float* part = reinterpret_cast<float*>(base + lay.part);
    launch_front<0, float>(hp, dp, fr, Lc, xiT, lay.Lpad, part, nullptr, st, true, true);  // FP32 samples
    const int64_t n = static_cast<int64_t>(hp.PN) * Lc;
    TRACED(dp, "transpose_xi", st,
           hipLaunchKernelGGL(transpose_xi, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                              xiT, lay.Lpad, hp.PN, static_cast<int>(Lc), xi + l0 * hp.PN));
    check_launch("transpose_xi");
  }
}

}  // namespace srp
