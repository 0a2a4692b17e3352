/*
 * cpi.h -- C ABI of the MI355X (gfx950) correlation plenoptic imaging library.
 *
 * The library computes the two steps of correlation plenoptic imaging (CPI):
 *
 *  1. the 4-D correlation function of Eq. (1) (Section "CPI algorithm",
 *     item 1):  Gamma(rho_a, rho_b) = <A(rho_a) B(rho_b)> - <A(rho_a)><B(rho_b)>
 *     over N frame pairs, both averages normalised by N.  It is evaluated
 *     exactly: numer = N * S_ab - S_a * S_b in int64 (S_ab the sum of
 *     products, S_a and S_b the per-pixel sums, S_ab contracted on matrix
 *     cores: binary frames as FP4 (E2M1) 0/1 operands with FP32 sums, or as
 *     int8 with int32 sums, byte frames as int8; every partial sum is an
 *     exact integer), then gamma = fl64(fl64(numer) / fl64(N*N));
 *
 *  2. refocusing (Section "CPI algorithm", item 2; refocusing optimisation in
 *     Section 4.1): for each plane parameter alpha and output pixel (x_r, y_r)
 *       u_x = alpha*(x_r - ca_x) + ca_x + (1 - alpha)*mag_x*(x_b - cb_x)
 *       u_y = alpha*(y_r - ca_y) + ca_y + (1 - alpha)*mag_y*(y_b - cb_y)
 *       I_alpha(x_r, y_r) = sum over detector-B pixels (x_b, y_b) of the
 *         bilinear sample of the view Gamma(., rho_b) at (u_x, u_y),
 *     corners outside the Ha x Wa view contributing zero.  Interpolation
 *     coordinates are built on the device from FP64 per-plane tables; samples
 *     are weighted and summed in FP32.
 *
 * Conventions shared by every entry point
 *  - Pixel index rho = y * W + x (0-based) on both detectors.
 *  - Frames are frame-major: frame i occupies bytes [i*FB, (i+1)*FB) with
 *      FB = P          for CPI_FRAMES_U8   (one byte per pixel), or
 *      FB = ceil(P/8)  for CPI_FRAMES_BIT1 (pixel 8j+k in bit k of byte j,
 *                                           padding bits of the last byte ignored).
 *  - Gamma storage: CPI_GAMMA_VIEW_MAJOR  -> element (rho_a, rho_b) at rho_b*Pa + rho_a
 *                   CPI_GAMMA_PIXEL_MAJOR -> element (rho_a, rho_b) at rho_a*Pb + rho_b
 *  - Ownership: frame, Gamma, output and workspace pointers are DEVICE
 *    pointers owned by the caller; the library never allocates or frees device
 *    memory.  Geometry and alpha pointers are HOST pointers, read before the
 *    call returns.  Device pointers must be 16-byte aligned.
 *  - Asynchrony: after validation every call only enqueues work on `stream`
 *    (a hipStream_t, NULL = the null stream); results are valid once the
 *    stream has reached that point.  Calls on distinct streams with distinct
 *    workspaces may run concurrently.  cpi_autotune_refocus and the stream
 *    save/load calls synchronise the stream.
 *  - Errors: every entry point returns a cpi_status and never aborts.  Invalid
 *    arguments are rejected before anything is enqueued; cpi_last_error()
 *    returns this thread's text for the last failure.
 */
#ifndef CPI_H
#define CPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPI_OK = 0,
  CPI_ERR_INVALID_ARG = 1,  /* null/misaligned pointer, bad size, bad enum, non-finite alpha */
  CPI_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement */
  CPI_ERR_OVERFLOW = 3,     /* N^2 * max|a| * max|b| >= 2^63 or N^2 >= 2^53 */
  CPI_ERR_WORKSPACE = 4,    /* workspace smaller than the *_workspace_size figure */
  CPI_ERR_DEVICE = 5,       /* HIP runtime or launch failure (text in cpi_last_error) */
  CPI_ERR_NOT_READY = 6     /* stream handle has no frames yet */
} cpi_status;

typedef enum { CPI_FRAMES_U8 = 0, CPI_FRAMES_BIT1 = 1 } cpi_frame_format;

typedef enum { CPI_GAMMA_VIEW_MAJOR = 0, CPI_GAMMA_PIXEL_MAJOR = 1 } cpi_gamma_layout;

/* Refocus geometry.  wa x ha: detector A (spatial, Da); wb x hb: detector B
 * (lens plane, Db); mag_*: magnification from Db to Da pixel units; ca_*,
 * cb_*: optical-axis centres on Da and Db in pixels; out_w x out_h: output
 * grid, whose pixel (x_r, y_r) sits at Da coordinates (x_r, y_r). */
typedef struct {
  int32_t wa, ha, wb, hb;
  double mag_x, mag_y;
  double ca_x, ca_y, cb_x, cb_y;
  int32_t out_w, out_h;
} cpi_geometry;

/* Library version string (static storage). */
const char* cpi_version(void);
/* Name of a status code (static storage). */
const char* cpi_status_string(cpi_status s);
/* Detail text of the last failed call on this thread ("" if none). */
const char* cpi_last_error(void);

/* Default geometry: mag = wa/wb and ha/hb, centres (w-1)/2 and (h-1)/2,
 * output grid = the Da grid.  `out` is a host pointer. */
cpi_status cpi_geometry_default(int32_t wa, int32_t ha, int32_t wb, int32_t hb,
                                cpi_geometry* out);

/* ---------------------------------------------------------------------------
 * Correlation function, Eq. (1), exact.
 *
 * cpi_correlate_workspace_size: bytes of device workspace cpi_correlate needs
 *   for these sizes in one shot (written to *bytes, a host pointer); when the
 *   environment variable CPI_WORKSPACE_LIMIT (bytes) is below that, the size
 *   of the blocked plan that fits the limit (see below).
 *
 * cpi_correlate: Gamma for n frame pairs.
 *   frames_a  n frames of pa pixels (detector A), format `fmt`
 *   frames_b  n frames of pb pixels (detector B), format `fmt`
 *   gamma     nullable, pa*pb doubles in `layout`: fl64(numer)/fl64(n*n)
 *   gamma_f32 nullable, pa*pb floats in `layout`:  fl32(gamma)
 *   numer     nullable, pa*pb int64 in `layout`:   n*S_ab - S_a*S_b
 *   sum_a     nullable, pa int64: S_a;  sum_b nullable, pb int64: S_b
 *   At least one of gamma, gamma_f32, numer must be non-null.
 *   Binary data (every byte 0 or 1, or CPI_FRAMES_BIT1) is contracted from
 *   packed bits; other uint8 data from bytes (offset by -128 when a value
 *   exceeds 127, which leaves numer unchanged); int32 partial sums are folded
 *   into int64 whenever the next block of frames could overflow them.
 *   Memory-adaptive blocking (Section 4.1 splits the work into blocks sized
 *   by the memory available): when workspace_bytes, capped by
 *   CPI_WORKSPACE_LIMIT if set, is below the one-shot size, the frames are
 *   folded in blocks of F frames through the running sums of the streaming
 *   calls (F the largest multiple of 512 whose state fits: the int32 or int64
 *   S_ab, the sums and one block's operands, without the streaming calls'
 *   FP32 Gamma buffer); the results are identical and the call stays
 *   asynchronous (one push per block is enqueued).  Blocks only pay when the
 *   frames' operands outweigh S_ab (n above about 32 * pa * pb / (pa + pb)
 *   frames for 1-bit data: 1.05e6 at 65536 x 65536 pixels).  A workspace
 *   below the state for F = 512 gives CPI_ERR_WORKSPACE.  Inputs longer than
 *   one ingest pass (n above 2^24 - 512 = 16776704 frames) are always folded
 *   this way, in blocks of at most that many frames; for them
 *   cpi_correlate_workspace_size reports the state for such blocks.
 *   Errors: CPI_ERR_INVALID_ARG (null frames/workspace, n, pa or pb <= 0,
 *   bad enum, misalignment, all outputs null), CPI_ERR_OVERFLOW (n*n*255*255
 *   >= 2^63 for U8, n*n >= 2^53 for either format), CPI_ERR_WORKSPACE,
 *   CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
cpi_status cpi_correlate_workspace_size(int64_t n, int64_t pa, int64_t pb,
                                        cpi_frame_format fmt, size_t* bytes);
cpi_status cpi_correlate(const void* frames_a, const void* frames_b, int64_t n,
                         int64_t pa, int64_t pb, cpi_frame_format fmt,
                         cpi_gamma_layout layout, double* gamma, float* gamma_f32,
                         int64_t* numer, int64_t* sum_a, int64_t* sum_b,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Plain FP32 correlator, the comparison path for the int8 one: frames are
 * unpacked to FP32, S_ab, S_a and S_b are FP32 sums (FMA), and
 *   gamma_f32 = fl32(S_ab/n) - fl32(fl32(S_a/n) * fl32(S_b/n))   (FP32 ops).
 * Same inputs, layout and errors as cpi_correlate; gamma_f32 must be non-null. */
cpi_status cpi_correlate_f32_plain_workspace_size(int64_t n, int64_t pa, int64_t pb,
                                                  cpi_frame_format fmt, size_t* bytes);
cpi_status cpi_correlate_f32_plain(const void* frames_a, const void* frames_b,
                                   int64_t n, int64_t pa, int64_t pb,
                                   cpi_frame_format fmt, cpi_gamma_layout layout,
                                   float* gamma_f32, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Refocusing (shift-and-sum of perspective views).
 *
 * gamma    Gamma as FP32 in CPI_GAMMA_VIEW_MAJOR storage: Pb = wb*hb views of
 *          ha x wa pixels (device)
 * g        geometry (host)
 * alphas   n_alpha plane parameters (host, finite), 1 <= n_alpha <= 4096
 * out      n_alpha * out_h * out_w floats, plane-major then row-major (device)
 *
 * cpi_refocus runs the batched kernel (many planes per launch) with the tile
 * configuration cached by cpi_autotune_refocus for this shape, or a default.
 * cpi_refocus_plain runs one plane per launch with direct gathers.
 * cpi_autotune_refocus times the candidate configurations on these inputs,
 * caches the fastest (in memory and, if CPI_AUTOTUNE_CACHE names a file, on
 * disk), synchronises `stream`, and leaves the refocused stack in `out`.
 * Errors: CPI_ERR_INVALID_ARG (null pointers, non-positive sizes, non-finite
 * geometry or alpha, n_alpha out of range), CPI_ERR_WORKSPACE, CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
cpi_status cpi_refocus_workspace_size(const cpi_geometry* g, int32_t n_alpha,
                                      size_t* bytes);
cpi_status cpi_refocus(const float* gamma, const cpi_geometry* g,
                       const double* alphas, int32_t n_alpha, float* out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* cpi_refocus without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture into a HIP graph, serving loops,
 * harnesses that forbid allocation).  The workspace is a 128 MiB array in the
 * library's device memory, one per device, held until the process ends; the
 * call allocates nothing.  It uses the configuration cpi_refocus would,
 * except that the row-lane kernel is replaced by the column-sum kernel and
 * view-row splits are halved until the tables and partial sums fit the
 * array: the result is that of cpi_refocus_tiled with that configuration.
 * Every call on one device shares its array, so calls that overlap on one
 * device (other streams, other threads) race; serialise them.  Nothing in
 * the array needs clearing between calls.
 * Errors: those of cpi_refocus; CPI_ERR_WORKSPACE before any launch when the
 * tables alone exceed 128 MiB (about n_alpha * hb * out_h * 16 bytes). */
cpi_status cpi_refocus_noalloc(const float* gamma, const cpi_geometry* g,
                               const double* alphas, int32_t n_alpha, float* out,
                               void* stream);
cpi_status cpi_refocus_plain(const float* gamma, const cpi_geometry* g,
                             const double* alphas, int32_t n_alpha, float* out,
                             void* workspace, size_t workspace_bytes, void* stream);
cpi_status cpi_autotune_refocus(const float* gamma, const cpi_geometry* g,
                                const double* alphas, int32_t n_alpha, float* out,
                                void* workspace, size_t workspace_bytes,
                                void* stream);
/* The batched-kernel configuration cpi_refocus uses for this shape on the
 * current device: planes per work-group, output rows per wave and view-row
 * splits (host pointers). */
cpi_status cpi_refocus_config(const cpi_geometry* g, int32_t n_alpha,
                              int32_t* planes_per_group, int32_t* rows_per_wave,
                              int32_t* view_splits);

/* Kernels of the batched refocus path.  All evaluate the same sum (the
 * bilinear sample of every view at the plane's shifted point, summed over
 * the views); they differ in summation order only.
 *   CPI_REFOCUS_ROWS: every output row interpolates its two view rows, for
 *     every view, and sums over the views.
 *   CPI_REFOCUS_COLUMN_SUMS: for each lens-plane row y_b, the column
 *     interpolants of every view row the tile touches are summed over x_b
 *     first; the row weights (which depend on y_b and the output row, not on
 *     x_b) are applied once per y_b.
 *   CPI_REFOCUS_VIEW_ROWS: the same two sums as CPI_REFOCUS_COLUMN_SUMS in
 *     two passes: the column interpolants of every view row, summed over x_b,
 *     are written to the workspace for each (plane, y_b), then the row
 *     weights fold them over y_b.  Lanes are view rows, so column cells and
 *     weights are shared by a wave.  Takes views of at most 256 rows and
 *     plane groups whose sample columns, for the chosen output columns per
 *     work-group, span at most 64 view columns; cpi_refocus uses the
 *     column-sum kernel where it does not apply. */
typedef enum {
  CPI_REFOCUS_ROWS = 0,
  CPI_REFOCUS_COLUMN_SUMS = 1,
  CPI_REFOCUS_VIEW_ROWS = 2
} cpi_refocus_kernel;

/* A batched-refocus configuration: planes per work-group and output rows per
 * tile, (4, 8), (4, 16), (8, 8), (8, 16), (8, 32), (16, 8), (16, 16) for
 * both CPI_REFOCUS_ROWS and CPI_REFOCUS_COLUMN_SUMS and also (1, 16),
 * (2, 16), (2, 32), (4, 32) for CPI_REFOCUS_COLUMN_SUMS; view-row splits
 * (1..16); the kernel (cpi_refocus_kernel) and, for CPI_REFOCUS_COLUMN_SUMS,
 * the number of view windows staged in LDS (2, 3 or 4, and 2 or 3 for 8
 * planes x 32 rows, whose four windows exceed a CU's LDS; ignored by the
 * other kernels, and reported as 0 for them).  For CPI_REFOCUS_VIEW_ROWS,
 * rows_per_wave holds the output columns per work-group instead, with
 * (planes, columns) in (8, 8), (4, 16), (8, 16), (16, 16), (8, 32), and
 * view_splits is ignored. */
typedef struct {
  int32_t planes_per_group;
  int32_t rows_per_wave;
  int32_t view_splits;
  int32_t kernel;
  int32_t stages;
} cpi_refocus_tiles;

/* The configuration cpi_refocus uses for this shape on the current device
 * (cached by cpi_autotune_refocus, or the default).  `out` is a host pointer. */
cpi_status cpi_refocus_get_tiles(const cpi_geometry* g, int32_t n_alpha,
                                 cpi_refocus_tiles* out);
/* cpi_refocus with an explicit configuration `tiles` (host pointer) instead
 * of the cached one.  Errors: CPI_ERR_INVALID_ARG for a null `tiles` and the
 * argument errors of cpi_refocus; CPI_ERR_UNSUPPORTED for a configuration
 * that is not built, or a CPI_REFOCUS_VIEW_ROWS configuration that does not
 * apply to the geometry and planes; all before any launch.  Results are bitwise
 * reproducible for a given configuration. */
cpi_status cpi_refocus_tiled(const float* gamma, const cpi_geometry* g,
                             const double* alphas, int32_t n_alpha, float* out,
                             const cpi_refocus_tiles* tiles, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Matrix-core encoding of binary frames (CPI_FRAMES_BIT1, and CPI_FRAMES_U8
 * data whose bytes are all 0 or 1).
 *   CPI_MMA_AUTO (default): FP4 (E2M1) operands with FP32 accumulation when
 *     one contraction pass covers at most 2^24 frames (every partial sum is
 *     then an integer below 2^24, exact in FP32), int8 operands with int32
 *     sums otherwise;
 *   CPI_MMA_INT8: int8 operands with int32 sums always.
 * Both give identical, exact results.  The setting is process-wide and
 * applies to calls enqueued after it returns (cpi_correlate, cpi_stream_push);
 * the environment variable CPI_GEMM_ENC=int8 sets CPI_MMA_INT8 at load time.
 * Errors: CPI_ERR_INVALID_ARG for an unknown value. */
typedef enum { CPI_MMA_AUTO = 0, CPI_MMA_INT8 = 1 } cpi_mma_encoding;

cpi_status cpi_set_mma_encoding(cpi_mma_encoding enc);
cpi_mma_encoding cpi_get_mma_encoding(void);

/* ---------------------------------------------------------------------------
 * Refocusing with a resampled lens-plane grid: the general form of the
 * multilinear interpolation of Gamma (Section 4.1, refocusing optimisation),
 * in which the lens-plane coordinate rho_b is also interpolated.  The sum over
 * detector-B pixels becomes a sum over the sample points
 *   x_b(i) = ox + i * sx (i < nx),   y_b(j) = oy + j * sy (j < ny)
 * (detector-B pixel units, sx, sy > 0), u_x, u_y are formed with these
 * fractional x_b, y_b, and every sample is the 4-D multilinear interpolant of
 * Gamma at (u_x, u_y, x_b, y_b): 16 corners weighted by products of linear
 * weights, corners outside either detector contributing zero.  The integer
 * grid (0, 0, 1, 1, Wb, Hb) gives cpi_refocus.
 *
 * Because the interpolant is linear in Gamma, it is computed in two steps:
 *   cpi_resample_views: views[j * nx + i][.] (FP32, nx * ny views of Pa values)
 *     = the bilinear interpolant along rho_b of the views of gamma (FP32
 *     view-major) at (x_b(i), y_b(j)); independent of alpha;
 *   refocusing of those views (cpi_refocus, batched) under the geometry of
 *     cpi_lens_sampling_geometry: Wb -> nx, Hb -> ny, mag -> mag * s,
 *     cb -> (cb - o) / s.
 * cpi_refocus_resampled does both; its workspace holds the views first.
 * Errors: CPI_ERR_INVALID_ARG (bad sample grid: counts outside [1, 65536],
 *   spacings not positive, non-finite or |value| >= 2^20; as cpi_refocus),
 *   CPI_ERR_WORKSPACE, CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny;     /* sample counts along x_b and y_b */
  double ox, oy;      /* first sample point */
  double sx, sy;      /* sample spacing (> 0) */
} cpi_lens_sampling;

cpi_status cpi_lens_sampling_geometry(const cpi_geometry* g, const cpi_lens_sampling* s,
                                      cpi_geometry* out);
cpi_status cpi_resample_views(const float* gamma, const cpi_geometry* g,
                              const cpi_lens_sampling* s, float* views, void* stream);
cpi_status cpi_refocus_resampled_workspace_size(const cpi_geometry* g, const cpi_lens_sampling* s,
                                                int32_t n_alpha, size_t* bytes);
cpi_status cpi_refocus_resampled(const float* gamma, const cpi_geometry* g,
                                 const cpi_lens_sampling* s, const double* alphas,
                                 int32_t n_alpha, float* out, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Streaming: frame chunks folded into device-resident sums as rank-k updates
 * (the sums of Eq. (1) are additive over frames), so Gamma for all frames so
 * far is available after every chunk.
 *
 * cpi_stream_workspace_size: device bytes a stream needs for pa, pb, fmt and
 *   chunks of at most max_chunk frames (max_chunk at most 131008 for
 *   CPI_FRAMES_U8 and 16776704, one ingest pass, for CPI_FRAMES_BIT1; larger
 *   values give CPI_ERR_INVALID_ARG).
 * cpi_stream_create: builds a handle over caller workspace (device) on `stream`;
 *   the handle owns host-side state only.  Sums start at zero.
 * cpi_stream_push: folds k <= max_chunk frame pairs (device pointers, format
 *   fmt) into S_ab, S_a, S_b and refreshes the handle's FP32 Gamma.
 * cpi_stream_push_host: the same for host chunks (pinned memory gives an
 *   asynchronous copy; pageable memory is copied synchronously).  The copy
 *   runs on a copy stream the library keeps per device (made at the first
 *   handle), into one of two device staging buffers of the handle, so that it
 *   overlaps the work on the previous chunk; the handle's stream waits for
 *   it.
 * cpi_stream_frames: frames folded so far (host pointer).
 * cpi_stream_gamma: writes Gamma for all frames so far (each output nullable).
 * cpi_stream_gamma_f32_ptr: device address of the handle's FP32 view-major
 *   Gamma, refreshed by every push.
 * cpi_stream_refocus: refocuses the current Gamma (as cpi_refocus).
 * cpi_stream_state_size / save / load: checkpoint of (N, S_a, S_b, S_ab) in a
 *   host buffer; both synchronise the stream.  A checkpoint loads only into a
 *   stream of the same pa, pb and fmt.
 * cpi_stream_destroy: frees the handle (not the workspace).
 *
 * Overlapping a refocus with the next update: cpi_stream_workspace_size_ex /
 * cpi_stream_create_ex take gamma_buffers (1 or 2); with 2 the handle holds
 * two FP32 Gamma buffers and push k writes buffer k % 2 (one more pa * pb * 4
 * bytes of workspace).  cpi_stream_refocus_async enqueues the refocus of the
 * latest push's Gamma on refocus_stream (a second stream of the same device):
 * that stream first waits for the push; the next push that writes the same
 * buffer waits on the handle's stream for the refocus.  Every other call
 * keeps its meaning (cpi_stream_gamma_f32_ptr names the latest push's
 * buffer).  With 2 buffers, update k + 1 runs on the handle's stream while
 * refocus k runs on refocus_stream; results are those of the serial calls.
 * The out and workspace buffers of an asynchronous refocus are in use until
 * refocus_stream has reached it.  The handle and its events belong to one
 * host thread at a time.
 * Errors: CPI_ERR_INVALID_ARG, CPI_ERR_OVERFLOW (N would break the bounds of
 *   cpi_correlate), CPI_ERR_NOT_READY (gamma requested before any frame),
 *   CPI_ERR_WORKSPACE, CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
typedef struct cpi_stream_s* cpi_stream_t;

cpi_status cpi_stream_workspace_size(int64_t pa, int64_t pb, cpi_frame_format fmt,
                                     int64_t max_chunk, size_t* bytes);
cpi_status cpi_stream_create(int64_t pa, int64_t pb, cpi_frame_format fmt,
                             int64_t max_chunk, void* workspace, size_t bytes,
                             void* stream, cpi_stream_t* out);
cpi_status cpi_stream_workspace_size_ex(int64_t pa, int64_t pb, cpi_frame_format fmt,
                                        int64_t max_chunk, int32_t gamma_buffers,
                                        size_t* bytes);
cpi_status cpi_stream_create_ex(int64_t pa, int64_t pb, cpi_frame_format fmt,
                                int64_t max_chunk, int32_t gamma_buffers, void* workspace,
                                size_t bytes, void* stream, cpi_stream_t* out);
cpi_status cpi_stream_push(cpi_stream_t s, const void* chunk_a, const void* chunk_b,
                           int64_t k);
cpi_status cpi_stream_push_host(cpi_stream_t s, const void* chunk_a,
                                const void* chunk_b, int64_t k);
cpi_status cpi_stream_frames(cpi_stream_t s, int64_t* n);
cpi_status cpi_stream_gamma(cpi_stream_t s, cpi_gamma_layout layout, double* gamma,
                            float* gamma_f32, int64_t* numer, int64_t* sum_a,
                            int64_t* sum_b);
cpi_status cpi_stream_gamma_f32_ptr(cpi_stream_t s, const float** gamma_f32);
cpi_status cpi_stream_refocus(cpi_stream_t s, const cpi_geometry* g,
                              const double* alphas, int32_t n_alpha, float* out,
                              void* workspace, size_t workspace_bytes);
cpi_status cpi_stream_refocus_async(cpi_stream_t s, const cpi_geometry* g,
                                    const double* alphas, int32_t n_alpha, float* out,
                                    void* workspace, size_t workspace_bytes,
                                    void* refocus_stream);
cpi_status cpi_stream_state_size(cpi_stream_t s, size_t* bytes);
cpi_status cpi_stream_save(cpi_stream_t s, void* host_buf, size_t bytes);
cpi_status cpi_stream_load(cpi_stream_t s, const void* host_buf, size_t bytes);
cpi_status cpi_stream_destroy(cpi_stream_t s);

/* ---------------------------------------------------------------------------
 * Raw sensor frames holding both detectors side by side, the paper's input
 * (Section "Input Dataset"): frames of 256 rows x 512 pixels at 1 bit per
 * pixel, the left 256 columns imaging detector A and the right 256 detector
 * B; files of 512 such frames back to back, no header.
 *
 * cpi_sidebyside: frame_w x frame_h pixels per raw frame (frame_w even) and
 *   the region of interest, roi_w x roi_h at (roi_x, roi_y) inside each half,
 *   taken from both halves.  A raw frame is ceil(frame_w*frame_h/8) bytes with
 *   pixel (y, x) at bit (y*frame_w + x) % 8 of byte (y*frame_w + x) / 8 (the
 *   least-significant-bit-first reading of the 1-bit format).
 * cpi_split_sidebyside: n raw frames (device) -> n CPI_FRAMES_BIT1 frames of
 *   roi_w*roi_h pixels per detector (device, ceil(roi_w*roi_h/8) bytes each),
 *   enqueued on `stream`.
 * cpi_file_frames: number of whole raw frames in a file (host only).
 * cpi_stream_ingest_files: folds every frame of the listed files, in order,
 *   into a CPI_FRAMES_BIT1 stream whose pa and pb both equal roi_w*roi_h.  The
 *   calling thread reads pieces of at most min(max_chunk, host_bytes / raw
 *   frame, dev_bytes / raw frame) frames into host_a and host_b in turn (host
 *   memory of host_bytes each; pinned memory lets the read of one piece
 *   overlap the device work on the previous one), copies each into dev_raw
 *   (caller device scratch of dev_bytes), splits it into the stream's chunk
 *   buffers and pushes it.  Returns once the last piece is enqueued, with the
 *   number of frames ingested in *frames (host); host_a, host_b and dev_raw
 *   stay in use until the stream has reached that point.
 * Errors: CPI_ERR_INVALID_ARG (null pointers, sizes, a region outside the
 *   half, a stream whose format or pixel counts do not match, buffers smaller
 *   than one raw frame, a missing or unreadable file, a file that is not a
 *   whole number of frames: all files are checked before any is read),
 *   CPI_ERR_DEVICE, CPI_ERR_OVERFLOW as for cpi_stream_push.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t frame_w, frame_h;
  int32_t roi_x, roi_y, roi_w, roi_h;
} cpi_sidebyside;

cpi_status cpi_split_sidebyside(const void* frames, int64_t n, const cpi_sidebyside* f,
                                void* frames_a, void* frames_b, void* stream);
cpi_status cpi_file_frames(const char* path, const cpi_sidebyside* f, int64_t* frames);
cpi_status cpi_stream_ingest_files(cpi_stream_t s, const char* const* paths, int32_t n_paths,
                                   const cpi_sidebyside* f, void* host_a, void* host_b,
                                   size_t host_bytes, void* dev_raw, size_t dev_bytes,
                                   int64_t* frames);

/* ---------------------------------------------------------------------------
 * Measured peaks of the current device, to set beside the vendor figures the
 * rooflines are quoted against: matrix-core ops/s of register-only loops of
 * the two ops the contraction uses (int8 16x16x64 with int32 sums, FP4
 * 16x16x128 with FP32 sums, on binary-like operands), and bytes/s read plus
 * written by a device copy of copy_bytes.
 * cpi_measure_peaks_scratch_size: device scratch needed for copy_bytes.
 * cpi_measure_peaks: runs the three measurements on `stream` (synchronises
 *   it); outputs are host pointers.
 * Errors: CPI_ERR_INVALID_ARG (null pointers, copy_bytes not a positive
 *   multiple of 16), CPI_ERR_WORKSPACE, CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
cpi_status cpi_measure_peaks_scratch_size(size_t copy_bytes, size_t* bytes);
cpi_status cpi_measure_peaks(void* scratch, size_t scratch_bytes, size_t copy_bytes,
                             double* int8_ops_per_s, double* fp4_ops_per_s,
                             double* copy_bytes_per_s, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (tracing).  While recording is on, every entry point brackets
 * each group of kernels it enqueues with a pair of HIP events on the caller's
 * stream.  Group names: "ingest" (sums and operand transposition), "gemm"
 * (matrix-core contraction with its epilogue), "unpack_f32", "sgemm_f32",
 * "refocus_tables", "refocus_batched" (including the reduction of split
 * partial sums), "refocus_plain", "refocus_resample", "state_gamma".
 * cpi_profile_begin clears earlier records and starts recording;
 * cpi_profile_end stops it; cpi_profile_query waits for the recorded events
 * and returns the number of launches and their summed duration for one group.
 * Recording adds one event pair per group and call; it is meant for
 * measurement runs.  Not thread-safe with concurrent calls on other threads.
 * ------------------------------------------------------------------------- */
cpi_status cpi_profile_begin(void);
cpi_status cpi_profile_end(void);
cpi_status cpi_profile_query(const char* group, int64_t* launches, double* total_ms);

/* ---------------------------------------------------------------------------
 * Learned denoiser.  Not part of the paper: a small network trained on the
 * pipeline's own output that maps a plane refocused from few frames to the
 * same plane refocused from many frames; the plain pipeline stays the
 * reference it is judged against and the fallback where it does not help.
 *
 * Model.  Each input plane p is normalised by its own mean mu and population
 * standard deviation sigma (sigma = 1 for a constant plane):
 * x = (p - mu) / sigma.  A four-level convolutional encoder-decoder f
 * (U-Net form, widths 32, 64, 128, 256) computes a correction and the output
 * is (x + f(x)) * sigma + mu.  Encoder levels: two 3x3 convolutions (zero
 * padding) each followed by ReLU, levels joined by 2x2 max-pooling; decoder
 * levels: nearest 2x upsampling, concatenation [upsampled, encoder output of
 * the level] along channels, two 3x3 convolutions with ReLU; then a 1x1
 * convolution to one channel.  Training minimises the mean squared error of
 * x + f(x) against the target plane normalised with the input's (mu, sigma),
 * over every pixel of the batch, with Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected moments).
 *
 * Precision.  Convolutions run on BF16 matrix cores with FP32 sums;
 * activations and their gradients are stored as bfloat16 (round to nearest
 * even), the output convolution and the loss in FP32; master weights, their
 * gradients (FP32 atomics) and the Adam moments are FP32.
 *
 * Parameters: one FP32 device array of cpi_denoiser_param_count floats.
 * Layer i (cpi_denoiser_layer_info, execution order) holds its weights
 * w[cout][ks][ks][cin] at weight_offset and its biases b[cout] at
 * bias_offset.  Channel counts are stored padded (the first layer's input to
 * 8 channels, the output layer to 32); weights of unused channels
 * (cin_used <= ci < cin, cout_used <= co < cout) must be zero and stay zero
 * under training.  The caller initialises the parameters and the two Adam
 * moment arrays (same size, zero at the start).
 *
 * Planes: FP32 device arrays [batch][h][w]; h and w positive multiples of 8,
 * batch * h * w <= 2^26.  Workspace: caller-owned device memory of at least
 * cpi_denoiser_workspace_size(batch, h, w, train) bytes (train != 0 for
 * cpi_denoiser_train_step and cpi_denoiser_gradients).
 *
 * cpi_denoiser_forward: out = denoised planes (out may not alias planes).
 * cpi_denoiser_train_step: one Adam step (step number >= 1) on one batch of
 *   (planes, targets); *loss (device float) receives the batch loss of the
 *   parameters before the step.  Updates params, adam_m, adam_v in place.
 * cpi_denoiser_gradients: the batch loss and the gradient of every parameter
 *   (into grads, same layout as params) without an update.
 * cpi_image_quality: per plane b, psnr[b] = 10 log10(R^2 / MSE) with R the
 *   target plane's max - min (+inf when the planes are equal) and ssim[b] =
 *   mean SSIM over every position of an 11 x 11 Gaussian window (sigma 1.5,
 *   normalised to sum 1) that fits in the plane, both planes mapped by the
 *   target's minimum and range to [0, 1] (range 1 for a constant target),
 *   K1 = 0.01, K2 = 0.03; FP64; planes at least 11 x 11; psnr and ssim are
 *   device arrays of batch doubles.
 * Errors: CPI_ERR_INVALID_ARG (null or misaligned pointers, bad sizes, step
 *   < 1, non-positive learning rate), CPI_ERR_WORKSPACE, CPI_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[16];
  int32_t cin, cout, ks;        /* stored channel counts and kernel size */
  int32_t cin_used, cout_used;  /* channels that carry data */
  int64_t weight_offset;        /* floats from the start of the parameters */
  int64_t bias_offset;
} cpi_denoiser_layer;

cpi_status cpi_denoiser_layer_count(int32_t* count);
cpi_status cpi_denoiser_layer_info(int32_t index, cpi_denoiser_layer* out);
cpi_status cpi_denoiser_param_count(int64_t* count);
cpi_status cpi_denoiser_workspace_size(int32_t batch, int32_t h, int32_t w, int32_t train,
                                       size_t* bytes);
cpi_status cpi_denoiser_forward(const float* params, int32_t batch, int32_t h, int32_t w,
                                const float* planes, float* out, void* workspace,
                                size_t workspace_bytes, void* stream);
cpi_status cpi_denoiser_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                                   float lr, int32_t batch, int32_t h, int32_t w,
                                   const float* planes, const float* targets, float* loss,
                                   void* workspace, size_t workspace_bytes, void* stream);
cpi_status cpi_denoiser_gradients(const float* params, int32_t batch, int32_t h, int32_t w,
                                  const float* planes, const float* targets, float* loss,
                                  float* grads, void* workspace, size_t workspace_bytes,
                                  void* stream);
cpi_status cpi_image_quality(const float* pred, const float* target, int32_t batch, int32_t h,
                             int32_t w, double* psnr, double* ssim, void* stream);

/* ---------------------------------------------------------------------------
 * The denoiser's kernels one at a time (each used by the network above).
 * Tensors are NHWC [b][h][w][c] bfloat16 (raw uint16 bits) device arrays,
 * 16-byte aligned.  All calls only enqueue work on `stream`.
 *
 * cpi_nn_pack_weights: FP32 w[cout][ks][ks][cin] -> bfloat16 rows
 *   w_packed[cout][kpad] (k = (ky*ks + kx)*cin + ci, zero for k >= ks*ks*cin,
 *   kpad = ks*ks*cin rounded up to a multiple of 32) and, if w_packed_t is not
 *   null, the backward-data weights w_packed_t[cin][kpad_t] with
 *   k = (ks*ks - 1 - tap)*cout + co (kpad_t = ks*ks*cout rounded up to 32).
 * cpi_nn_conv2d: out[p][co] = act(b[co] + sum over taps and ci of
 *   w[co][tap][ci] * x[p + tap offset][ci]) (zero padding), act = ReLU
 *   if relu != 0; then zeroed where mask[p][co] <= 0 (mask nullable; bias
 *   nullable).  Output to out (bfloat16) and/or out_f32 (FP32).  cin % 8 == 0,
 *   cout % 32 == 0, ks 1 or 3.  With (dy, w_packed_t, cin := cout, cout := cin,
 *   kpad := kpad_t) it is the gradient with respect to the input.
 * cpi_nn_conv2d_wgrad: dw[co][tap][ci] += sum over pixels p of
 *   dy[p][co] * x[p + tap offset][ci] (FP32, accumulated into dw), and, if db
 *   is not null, db[co] += sum over pixels of dy[p][co].  The pixels are
 *   split over work-groups.  With a workspace (device memory, 16-byte
 *   aligned, at least cpi_nn_conv2d_wgrad_workspace_size bytes, owned by the
 *   caller and free again when the stream has run the call) each split
 *   stores its partial sums there and one more kernel adds them to dw and db
 *   in split order, so the result is reproducible bit for bit; with a null
 *   workspace the splits add with FP32 atomics (order not fixed).  A
 *   workspace smaller than the size query gives CPI_ERR_WORKSPACE.
 * cpi_nn_bias_grad: db[c] += sum over pixels of dy[p][c].
 * cpi_nn_maxpool2 / _grad: 2x2 maximum (h, w even); the gradient goes to the
 *   first maximal position in the order (0,0), (0,1), (1,0), (1,1).
 * cpi_nn_upsample2 / _grad: nearest 2x upsampling of [b][h][w][c]; the
 *   gradient sums the four copies and is zeroed where mask <= 0 (nullable).
 * cpi_nn_concat / cpi_nn_split: out[p] = [a[p], b[p]] and its inverse.
 * cpi_nn_upsample2_concat / _grad: out = [upsample2(low) (c1 channels),
 *   skip (c2 channels)] for low [b][h][w][c1] and skip [b][2h][2w][c2]
 *   (c1, c2 multiples of 8); the gradient gives dskip and dlow (the four
 *   copies summed, zeroed where mask <= 0, mask nullable).
 * cpi_nn_add_mask: x = x + add (nullable), zeroed where mask <= 0 (nullable).
 * cpi_nn_mse: z[p] = y[p][0] + residual[p] (y with c FP32 channels per pixel,
 *   residual nullable); *loss += sum (z - t)^2 / pixels (loss nullable) and
 *   dy[p][0] = 2 (z - t) / pixels, dy[p][c > 0] = 0 (bfloat16, nullable).
 * cpi_nn_adam: one Adam step on FP32 arrays (bias correction with `step`).
 * ------------------------------------------------------------------------- */
cpi_status cpi_nn_pack_weights(const float* w, int32_t cout, int32_t cin, int32_t ks,
                               uint16_t* w_packed, uint16_t* w_packed_t, void* stream);
cpi_status cpi_nn_conv2d(const uint16_t* x, const uint16_t* w_packed, const float* bias,
                         const uint16_t* mask, int32_t relu, int32_t b, int32_t h, int32_t w,
                         int32_t cin, int32_t cout, int32_t ks, int32_t kpad, uint16_t* out,
                         float* out_f32, void* stream);
cpi_status cpi_nn_conv2d_wgrad_workspace_size(int32_t b, int32_t h, int32_t w, int32_t cin,
                                              int32_t cout, int32_t ks, size_t* bytes);
cpi_status cpi_nn_conv2d_wgrad(const uint16_t* x, const uint16_t* dy, int32_t b, int32_t h,
                               int32_t w, int32_t cin, int32_t cout, int32_t ks, float* dw,
                               float* db, void* workspace, size_t workspace_bytes,
                               void* stream);
cpi_status cpi_nn_bias_grad(const uint16_t* dy, int64_t pixels, int32_t c, float* db,
                            void* stream);
cpi_status cpi_nn_maxpool2(const uint16_t* x, int32_t b, int32_t h, int32_t w, int32_t c,
                           uint16_t* out, void* stream);
cpi_status cpi_nn_maxpool2_grad(const uint16_t* x, const uint16_t* dout, int32_t b, int32_t h,
                                int32_t w, int32_t c, uint16_t* dx, void* stream);
cpi_status cpi_nn_upsample2(const uint16_t* x, int32_t b, int32_t h, int32_t w, int32_t c,
                            uint16_t* out, void* stream);
cpi_status cpi_nn_upsample2_grad(const uint16_t* dout, int32_t b, int32_t h, int32_t w, int32_t c,
                                 const uint16_t* mask, uint16_t* dx, void* stream);
cpi_status cpi_nn_concat(const uint16_t* a, const uint16_t* b, int64_t pixels, int32_t ca,
                         int32_t cb, uint16_t* out, void* stream);
cpi_status cpi_nn_upsample2_concat(const uint16_t* low, const uint16_t* skip, int32_t b, int32_t h,
                                  int32_t w, int32_t c1, int32_t c2, uint16_t* out, void* stream);
cpi_status cpi_nn_upsample2_concat_grad(const uint16_t* d, int32_t b, int32_t h, int32_t w,
                                       int32_t c1, int32_t c2, const uint16_t* mask,
                                       uint16_t* dlow, uint16_t* dskip, void* stream);
cpi_status cpi_nn_split(const uint16_t* d, int64_t pixels, int32_t ca, int32_t cb, uint16_t* da,
                        uint16_t* db, void* stream);
cpi_status cpi_nn_add_mask(uint16_t* x, const uint16_t* add, const uint16_t* mask, int64_t count,
                           void* stream);
cpi_status cpi_nn_mse(const float* y, int32_t c, const float* residual, const float* target,
                      int64_t pixels, float* loss, uint16_t* dy, void* stream);
cpi_status cpi_nn_adam(float* w, const float* g, float* m, float* v, int64_t count, int64_t step,
                       float lr, float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CPI_H */
