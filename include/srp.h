/*
 * srp.h -- C ABI of the MI355X (gfx950) SRP-map library.
 *
 * Computes steered response power (SRP) maps from multichannel STFT frames,
 * following Dietzen, De Sena and van Waterschoot, "Scalable-Complexity
 * Steered Response Power based on Low-Rank and Sparse Interpolation"
 * (arXiv 2306.08514), in three forms:
 *
 *   SRP_FD    conv. FD-SRP, the dense transform z = 2 Re[H psi]
 *             (Sec. II-D, eq. (22));
 *   SRP_SLRI  sampling of each pair's GCC (Sec. III-B3, eqs. (40), (46)-(48))
 *             followed by low-rank interpolation z = sum_p U_p (V_p^T xi_p),
 *             the rank-R truncated SVD of each pair's sinc interpolation
 *             matrix Lambda_p (Sec. IV-A, eqs. (54), (56), (57));
 *   SRP_SSPI  the same sampling followed by sparse interpolation keeping the Q
 *             largest-magnitude entries of every row of every Lambda_p
 *             (Sec. IV-A, eqs. (55), (58)).
 *
 * Conventions used by every entry point:
 *   - N is the DFT length 2K of the STFT; frames hold bins 0..K; the map uses
 *     bins 1..K-1 and treats DC and Nyquist as zero (Sec. II-D).
 *   - Pairs p <-> (m, m'), m > m', are enumerated with m' in the outer and m
 *     in the inner loop (the double sum of eq. (8)).
 *   - PHAT weighting psi = y_m y_m'^* / |y_m y_m'^*| (eq. (2)), 0 where the
 *     product vanishes.
 *   - TDOAs are near-field (eq. (3)), in samples x_p(j) = Delta t_p(j) fs,
 *     computed in FP64 on the host; N_p = floor(d_p fs / c) + N_aux (eq. (33)).
 *   - sinc is the normalised sinc of Whittaker-Shannon interpolation
 *     (eq. (31), (42)).
 *   - Map scale: z = 2 Re[H psi] exactly as in eq. (22); the GCC samples are
 *     the unnormalised inverse DFT xi_p[n] = 2 Re sum_k psi_p[k] e^{j pi k n/K}
 *     (eq. (40)).
 *
 * Memory: host pointers are read during the call and copied; device pointers
 * must stay valid until the work enqueued on the given stream completes.
 * A plan owns its device memory until srp_destroy.  No entry point
 * synchronises the stream except where stated.
 *
 * Errors: every entry point returns an srp_status; on failure
 * srp_last_error() returns a message for the calling thread.  A failed
 * srp_plan leaves *out == NULL and leaks nothing.  No C++ exception crosses
 * the ABI.
 */
#ifndef SRP_H_
#define SRP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srp_plan_s* srp_plan_t;

typedef enum {
  SRP_OK = 0,
  SRP_E_INVALID = -1,     /* bad argument or geometry */
  SRP_E_NOMEM = -2,       /* host or device allocation failed */
  SRP_E_UNSUPPORTED = -3, /* variant/dtype combination not built */
  SRP_E_HIP = -4,         /* a HIP runtime call failed */
  SRP_E_BUDGET = -5       /* plan or workspace exceeds opts.hbm_budget */
} srp_status;

typedef enum {
  SRP_FD = 0,    /* conv. FD-SRP, eq. (22) */
  SRP_SLRI = 1,  /* SLRI-SRP, eq. (57) */
  SRP_SSPI = 2,  /* SSPI-SRP, eq. (58) */
  SRP_SI = 3,    /* SI-SRP, eq. (44): every lag of every pair interpolated;
                    rank_or_q ignored */
  SRP_TD = 4,    /* conv. TD-SRP, eq. (23): the GCC read at the TDOA rounded
                    to the nearest sample (half away from zero); rank_or_q
                    ignored */
  SRP_LR = 5     /* LR-SRP, eqs. (26)-(29): z = 2 Re[H_tall (H_fat psi)]
                    from the rank-R_H truncated SVD of the steering matrix H
                    (J x P(K-1)); rank_or_q = R_H <= min(J, P(K-1), 1024).
                    The fit runs on the device (FP64, through the smaller
                    Gram matrix of H, min(J, P(K-1)) <= 16384); no host-only
                    plans */
} srp_variant;

/* Operand precision of the dominant contraction (steering matrix for FD, the
 * tall factor U for SLRI, the interpolation weights for SSPI).  Accumulation
 * is FP32 (FP64 for SRP_F64).  Cross-spectra, GCC samples and the SLRI fat
 * stage are computed in FP32 for every dtype, except that with 16-bit or FP8
 * operands the direct sampling (40) multiplies split BF16 (hi, lo) halves of
 * the cross-spectra and of its table on the matrix cores (FP32 accumulation,
 * ~1e-5 relative per term; srp_gcc_samples always returns the FP32
 * products); the SLRI fat stage's output g is then narrowed to the operand
 * type.  SSPI with 16-bit or FP8 weights
 * reads the GCC samples narrowed to 16 bits: BF16 (BF16 weights) or FP16
 * (FP16 weights) frame-major copies where a candidate tile runs on the
 * matrix cores, FP16 sample pairs in the gather.  FP8 is OCP E4M3: SLRI
 * scales U per pair by a power of two (undone in the fat stage) and g by
 * one activation scale; SSPI stores its weights (|w| <= 1, the same bound
 * for every pair) times 2^8, undone exactly on the sums, so taps down to
 * 2^-14 stay normal; FD steering (|h| <= 1) is unscaled. */
typedef enum {
  SRP_F32 = 0,
  SRP_BF16 = 1,
  SRP_F16 = 2,
  SRP_FP8_E4M3 = 3,
  SRP_F64 = 4
} srp_dtype;

typedef struct {
  double c;              /* speed of sound in m/s (default 343.0) */
  int n_aux;             /* auxiliary lags N_aux of eq. (33) (default 2) */
  srp_dtype dtype;       /* operand precision (default SRP_F32) */
  int device;            /* HIP device ordinal; -1 builds the host plan only
                            (no device memory; srp_compute is then invalid) */
  int64_t frame_tile;    /* frames per internal tile (default 1024) */
  size_t hbm_budget;     /* max device bytes for the plan, 0 = unlimited */
  int sampling;          /* GCC sampling of SLRI/SSPI (Sec. III-B2, eq. (49)):
                            0 = whichever of the two forms costs fewer
                            operations by (49), 1 = the direct product
                            2 Re[S_p psi_p] of (40), 2 = the iFFT of (46)
                            (N must be a power of two, at most 4096) */
  int fd_steering;       /* steering operand of conv. FD-SRP (eq. (22)):
                            0 = resident when it takes at most 16 GiB and
                            fits the budget, else generated; 1 = resident
                            J x 2P(K-1) matrix; 2 = generated on the fly
                            from the FP64 TDOAs inside the product (not for
                            SRP_F64) */
  int far_field;         /* 1: grid rows are unit directions u pointing from
                            the array towards the source (Sec. II-A, the far
                            limit of (3)): x_p = -(r_m - r_m')^T u fs / c;
                            rows must have unit length (|1 - |u|| <= 1e-6) */
  int global_fit;        /* 1: the paper's global forms over the stacked
                            J x PN Lambda of (43) instead of one fit per
                            pair (0, the default).  SLRI (54): one rank-R
                            truncated SVD, rank_or_q = R_Lambda, the total
                            rank: exact through the PN x PN Gram matrix for
                            PN <= 4096, by FP64 randomized subspace
                            iteration on the device above (host-only plans:
                            PN <= 4096); 2: SLRI by the randomized fit at
                            any PN.  SSPI (55): the Q_Lambda =
                            rank_or_q * J * P largest-magnitude entries
                            (rank_or_q = mean taps per location and pair;
                            every entry at or above the Q_Lambda-th largest
                            magnitude is kept; at most 16 per location and
                            pair).  Other variants: SRP_E_INVALID */
} srp_opts;

typedef struct {
  int M, P, K;           /* microphones, pairs, half DFT length */
  int64_t J;             /* candidate locations */
  int PN;                /* stacked GCC samples sum_p (2 N_p + 1) */
  int max_np;            /* max_p N_p */
  int rank_or_q;         /* effective R (SLRI) or Q (SSPI), 0 for FD */
  srp_variant variant;
  srp_dtype dtype;
  double mean_n;         /* N of eq. (35) */
  double macs_per_map;   /* run-time MACs per map: C (24), C_slri (61),
                            C_sspi (62) (global forms: R_Lambda (J + PN),
                            the kept entries Q_Lambda) or C_lr (30); the
                            sampling term is the form that runs, 2PN(K-1)
                            or 8PK log2(2K) (49) */
  size_t device_bytes;   /* resident device memory owned by the plan */
  double plan_seconds;   /* wall time of plan construction */
  int64_t map_pitch;     /* recommended row pitch of the maps in elements:
                            J rounded up to 128, so that every row starts on
                            a 512-byte boundary and the map stores write
                            whole cache lines */
  int sampling_fft;      /* 1 if SLRI/SSPI sample the GCCs by the iFFT of
                            (46), 0 for the direct product of (40) */
  int fd_generated;      /* 1 if the FD steering is generated on the fly */
  int sspi_dense_tiles;  /* SSPI with 16-bit weights: 256-candidate tiles
                            whose lag windows (each rounded up to 8 lags,
                            stacked over pairs) fit 512 columns and run as
                            a dense contraction on the matrix cores; 0
                            otherwise */
  int sspi_gather_tiles; /* SSPI tiles evaluated by the gather of (58) */
  int sspi_band_tiles;   /* SSPI with 16-bit weights and at most 8 taps when
                            the dense windows do not fit (large apertures):
                            256-candidate tiles run as the band product of
                            (58) on the matrix cores (every tile, or none) */
} srp_plan_info;

/* Fills *opts with the defaults listed above. */
void srp_default_opts(srp_opts* opts);

/* Builds a plan (Sec. IV-B: everything that depends only on geometry and
 * frequency resolution is computed upfront, in FP64).
 *   mics      host, M x 3 row-major, metres (M >= 2)
 *   grid      host, J x 3 row-major (J >= 1): candidate positions in metres,
 *             or unit source directions with opts->far_field
 *   fs        sampling rate in Hz (> 0)
 *   N         DFT length 2K (even, >= 8); requires 2 N_p + 1 <= N for every
 *             pair (lag aliasing, Sec. III-B2 footnote)
 *   variant   SRP_FD, SRP_SLRI, SRP_SSPI, SRP_SI, SRP_TD or SRP_LR
 *   rank_or_q R per pair (SLRI, <= 32) or Q per (location, pair) (SSPI,
 *             <= 16), >= 1, clamped per pair to 2 N_p + 1; with
 *             opts->global_fit the total rank R_Lambda (SLRI) or the mean
 *             taps per (location, pair) (SSPI); R_H for LR; ignored for
 *             FD, SI and TD
 *   opts      NULL for defaults
 *   out       receives the plan, NULL on failure
 * Returns SRP_E_INVALID for bad geometry or arguments, SRP_E_UNSUPPORTED for
 * a dtype the variant does not offer, SRP_E_BUDGET when the resident operands
 * exceed opts->hbm_budget, SRP_E_NOMEM / SRP_E_HIP on allocation or runtime
 * failures. */
srp_status srp_plan(const double* mics, int M, const double* grid, int64_t J,
                    double fs, int N, srp_variant variant, int rank_or_q,
                    const srp_opts* opts, srp_plan_t* out);

/* Bytes of device workspace srp_compute needs for L frames. */
srp_status srp_workspace_size(srp_plan_t plan, int64_t L, size_t* bytes);

/* Computes one SRP map per frame.
 *   frames    device, complex64 [L][M][N/2 + 1] (interleaved re, im float32)
 *   L         number of frames (>= 0; 0 is a no-op)
 *   maps      device, float32 (float64 for SRP_F64 plans): map l occupies
 *             elements [l * ld_maps, l * ld_maps + J); the elements past J
 *             in each row are not written
 *   ld_maps   row pitch of maps in elements, >= J; 0 means J (dense
 *             [L][J]).  srp_plan_info.map_pitch gives the pitch at which
 *             the map stores run fastest (rows on 512-byte boundaries)
 *   workspace device, >= srp_workspace_size(L) bytes, 256-byte aligned; NULL
 *             uses a plan-owned buffer (then at most one call per plan may be
 *             in flight at a time)
 *   stream    hipStream_t to enqueue on (NULL = the null stream)
 * Returns SRP_E_INVALID for ld_maps in (0, J).  Asynchronous: returns after
 * enqueueing. */
srp_status srp_compute(srp_plan_t plan, const void* frames, int64_t L,
                       void* maps, int64_t ld_maps, void* workspace,
                       size_t ws_bytes, void* stream);

/* srp_compute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same maps, bit for bit, with no workspace argument and no allocation.
 * The workspace is a static scratch array of SRP_STATIC_SCRATCH_BYTES in
 * device memory, one per GPU, held until the process ends; the frames are
 * processed in the largest frame tile (at most the plan's frame_tile)
 * whose workspace fits it.
 *   frames, L, maps, ld_maps, stream  as for srp_compute
 * SRP_STATIC_SCRATCH_BYTES is 128 MiB.  Returns SRP_E_UNSUPPORTED when
 * even the smallest frame tile (256 frames of workspace rows) needs more
 * than the scratch (e.g. FD on 496 pairs with 2048-point frames: 520 MB of
 * BF16 cross-spectra), SRP_E_INVALID as srp_compute does.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap in time on one GPU (other streams,
 * other threads, other plans) race and must be serialised by the caller.
 * The scratch keeps the last call's contents; nothing read from it needs
 * to start at zero.  With profiling on (srp_profile_enable) the spans
 * create HIP events. */
#define SRP_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
srp_status srp_compute_static(srp_plan_t plan, const void* frames, int64_t L,
                              void* maps, int64_t ld_maps, void* stream);

/* Peak picking of (10)-(11) on the device: for each of L maps (row pitch
 * ld_maps >= J elements, float32 or float64 as given by dtype = SRP_F32 or
 * SRP_F64), the candidate with the largest value, ties to the smallest
 * index; NaN never wins.
 *   maps  device, as written by srp_compute
 *   idx   device, int64 [L]: the candidate index (-1 if every value is NaN)
 *   val   device, float64 [L]: its value
 * Asynchronous on `stream`.  SRP_E_INVALID for J < 1, ld_maps < J or another
 * dtype. */
srp_status srp_argmax(const void* maps, srp_dtype dtype, int64_t L, int64_t J, int64_t ld_maps,
                      int64_t* idx, double* val, void* stream);

/* Stage entry point: PHAT-weighted cross-spectra (eq. (2)) of L frames.
 *   psi  device, complex64 [L][P][K-1] */
srp_status srp_crossspec(srp_plan_t plan, const void* frames, int64_t L,
                         void* psi, void* stream);

/* Stage entry point: GCC samples xi_p[n], n = -N_p..N_p, of L frames
 * (eq. (40)), pairs stacked in order, lags in natural order, from FP32
 * products whatever the plan's dtype.
 *   xi   device, float32 [L][PN]
 * Only for SLRI and SSPI plans (the sampling stage exists only there). */
srp_status srp_gcc_samples(srp_plan_t plan, const void* frames, int64_t L,
                           float* xi, void* stream);

srp_status srp_plan_info_get(srp_plan_t plan, srp_plan_info* info);

/* Host-side plan data, for inspection (no device access):
 *   what = "tdoa"     double [P][J]   x_p(j) in samples
 *          "np"       int32  [P]      N_p
 *          "pairs"    int32  [P][2]   (m, m')
 *          "slri_u"   double [P][J][R]  U_p = Lambda_p V_p (FP64, before cast)
 *          "slri_v"   double [P][maxlag][R] V_p, rows n = -N_p..N_p, padded
 *                                      to 2 max_np + 1 rows with zeros
 *          "slri_s"   double [P][2 max_np + 1] singular values, descending
 *          "sspi_start" int32 [J][P]  first lag s of the window (-N_p..)
 *          "sspi_w"   double [J][P][Q] weights sinc(x - s - q), zero past
 *                                      the window's taps
 *          "lr_s"     double [R_H]   the R_H largest singular values of H
 *                                      (LR-SRP)
 * With global_fit, "slri_u" is [J][R_Lambda], "slri_v" [PN][R_Lambda] and
 * "slri_s" [PN] (the stacked fit of (54); the randomized fit reports its
 * l = R + max(16, R / 8) (rounded up to 64) leading values and zeros past
 * them); global SSPI exports its variable
 * windows in the same [J][P][Q] layout, Q the widest window.
 * "tdoa", "slri_u", "sspi_start" and "sspi_w" are kept only by host-only
 * plans (device = -1): a device plan fits these on the device and frees the
 * host copies.  bytes: size of dst; *needed receives the required size.  dst
 * may be NULL to query the size.  SRP_E_INVALID if the plan has no such
 * data. */
srp_status srp_plan_export(srp_plan_t plan, const char* what, void* dst,
                           size_t bytes, size_t* needed);

/* Per-kernel timing.  While enabled, srp_compute, srp_crossspec and
 * srp_gcc_samples record a pair of HIP events around every kernel they
 * launch, on the caller's stream.  srp_profile_collect waits for the
 * recorded events and returns, per kernel name, the total time in ms and the
 * number of launches since the previous collect, then clears them.  A plan
 * with profiling enabled must be driven from one host thread at a time.
 *   out       host array of `capacity` entries; *count receives the number of
 *             kernel names (entries beyond capacity are dropped). */
typedef struct {
  char name[32];
  double total_ms;
  int64_t launches;
} srp_kernel_time;

srp_status srp_profile_enable(srp_plan_t plan, int enable);
srp_status srp_profile_collect(srp_plan_t plan, srp_kernel_time* out, int capacity,
                               int* count);

/* Frees the plan and all device memory it owns; safe on NULL.  The caller
 * must make sure no work using the plan is still in flight. */
void srp_destroy(srp_plan_t plan);

/* Message describing the last failure on the calling thread ("" if none). */
const char* srp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRP_H_ */
