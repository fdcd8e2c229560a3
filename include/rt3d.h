/*
 * rt3d.h -- C ABI of librt3d.so, an MI355X (gfx950) implementation of the
 * per-iteration body of the plug-and-play point-cloud reconstruction of
 * single-photon lidar data (Tachella et al., "Real-time 3D reconstruction
 * from single-photon lidar data using plug-and-play point cloud denoisers").
 *
 * Problem (Results, "Observation model"): a lidar cube Z of rows x cols
 * pixels and T histogram bins holds Poisson counts with mean
 *     lambda[i,j,t] = g[i,j] * ( sum_{n in pixel (i,j)} r_n h(t - t_n) + b[i,j] ),
 * h the known impulse response (IRF), g the detector gain (0 = dead pixel),
 * t_n / r_n the depth (bins) and intensity (photons) of point n, b the
 * background (photons per bin).  The library returns, per pixel, the points
 * (depth, intensity) and the background that the reconstruction loop of
 * Results, "Reconstruction algorithm" reaches: gradient steps on t, r and b,
 * each followed by a denoiser (APSS point-cloud denoising for depth, a
 * manifold nearest-neighbour low-pass plus a minimum-intensity threshold for
 * intensity, a 2-D image filter for background).
 *
 * Conventions
 *   - bins are 0-based; depth is the real-valued bin of the IRF origin;
 *   - pixel p = (frame * rows + i) * cols + j; P = frames * rows * cols;
 *   - every pointer called `dev_*` or documented as device memory is HIP
 *     device memory owned by the caller; the library never frees it;
 *   - every call that takes `hip_stream` only enqueues work on that stream
 *     (a hipStream_t, NULL = the default stream) and returns; inputs must stay
 *     valid and outputs untouched until the stream has passed that point;
 *   - a context is used by one host thread at a time; contexts are
 *     independent.  No C++ exception crosses this interface.
 *
 * Errors: every call returns rt3d_status; on failure rt3d_last_error(ctx)
 * gives a message (valid until the next call on that context).  Errors found
 * on the device (capacity overflow, invalid events, non-finite output values)
 * are sticky in the context's workspace and reported by rt3d_query(); when
 * several occur, the word holds one of them.
 */
#ifndef RT3D_H
#define RT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt3d_status;
#define RT3D_OK             0
#define RT3D_E_INVALID     -1   /* bad argument: null, zero size, bad IRF, misaligned pointer */
#define RT3D_E_NOMEM       -2   /* workspace missing or too small */
#define RT3D_E_DEVICE      -3   /* a HIP call failed; message has its text */
#define RT3D_E_CAPACITY    -4   /* entry or point capacity exceeded; outputs truncated */
#define RT3D_E_STATE       -5   /* call not valid in the context's state */
#define RT3D_E_UNSUPPORTED -6   /* valid request this build does not handle */
#define RT3D_E_NONFINITE   -7   /* a non-finite depth, intensity or background reached the output
                                   (e.g. an intensity beyond FP32 range from a tiny gain) */

#define RT3D_K_MAX 4            /* compile-time slot capacity per pixel */

/* Depth denoiser plugged into the depth block. */
#define RT3D_DENOISE_NONE 0
#define RT3D_DENOISE_APSS 1
#define RT3D_DENOISE_CNN  2   /* learned network for pixels with <= 3 points, APSS for the rest */

/* Algorithm parameters.  Defaults (rt3d_params_default) are the readings of
 * the paper's unstated constants; `struct_size` must be sizeof(rt3d_params). */
typedef struct rt3d_params {
    uint32_t struct_size;
    int32_t  n_iter;     /* iterations of the loop (20) */
    int32_t  k_max;      /* slots per pixel, <= RT3D_K_MAX (4) */
    int32_t  k_init;     /* peaks sought per pixel at initialisation, <= k_max (3) */
    double   p_xy;       /* world units per pixel (1) */
    double   dz;         /* world units per bin (0.1) */
    double   h_apss;     /* APSS kernel support, world units (2) */
    double   h_int;      /* intensity graph radius, world units (2) */
    double   beta_t;     /* depth step scale in units of 1/(g r I_h), I_h the IRF's shift
                            Fisher information per photon (0.5) */
    double   dmax;       /* depth step clip in bins; <= 0: max(0.5, 1/sqrt(I_h)) */
    double   beta_r;     /* intensity step scale (1) */
    double   beta_b;     /* background step scale (1) */
    double   r_min;      /* minimum admissible intensity, photons (1) */
    double   d_merge;    /* in-pixel merge distance, bins; <= 0: max(1, sigma_h) */
    double   sigma_b;    /* background Gaussian filter, pixels; 0 = identity (2) */
    double   b_min;      /* background floor, photons/bin (1e-8) */
    double   sbr_guess;  /* log-matched filter floor eps = 1/(sbr_guess T) (1) */
    int32_t  r_init;     /* initialisation photon pooling radius, pixels (0) */
    int32_t  n_min;      /* minimum photons in a peak window (2) */
    double   kappa;      /* peak acceptance in background standard deviations (3) */
    int32_t  w_nms;      /* peak suppression half width, bins; <= 0: ceil(max(1, 2 sigma_h)) */
    int32_t  m_min;      /* minimum APSS neighbours (3) */
    int32_t  denoiser;   /* RT3D_DENOISE_APSS (default), RT3D_DENOISE_CNN or RT3D_DENOISE_NONE */
    int32_t  fused_loop; /* with APSS, a batch of frames of one size of at most 4096 pixels can run
                          * all iterations in one launch (one workgroup per frame, steps separated
                          * by workgroup barriers) instead of one launch per step.  1: always
                          * (when eligible); 0: never; -1 (default): the choice rt3d_autotune
                          * measured for this batch shape, else when the batch holds at least
                          * 64 frames (fewer frames leave most compute units idle) */
    int32_t  sr;         /* super-resolution factor s, 1..4 (1): the point cloud is estimated on a
                          * grid s times finer than the lidar pixels (Results, dynamic scenes: the
                          * map f sends s x s point-grid pixels to one lidar pixel, whose Poisson
                          * intensity adds all their points; gain and background stay per lidar
                          * pixel).  With s > 1: rows and cols of rt3d_input, the histograms, CSR,
                          * gain, events and rt3d_set_workspace are the lidar's; the output's
                          * pt_off has F (rows s) (cols s) + 1 entries over point-grid pixels
                          * (pixel (f, i, j) of the (rows s) x (cols s) frames) and its background
                          * F rows cols; p_xy is the point grid's pitch; the initialisation runs on
                          * the lidar grid and every point-grid pixel starts from its lidar pixel's
                          * points with 1/s^2 of the intensity.  Frames of one size only
                          * (E_UNSUPPORTED with frame_rows / frame_cols), no learned denoiser
                          * (E_UNSUPPORTED at create), per-step kernels only (fused_loop ignored). */
    double   persp;      /* camera model of the map f (Results, "Observation model": camera parameters
                          * such as the focal length).  0 (default): orthographic, X = j p_xy,
                          * Y = i p_xy, Z = t dz.  > 0: a pinhole camera at the origin looking along
                          * +Z; pixel (i, j) of a rows x cols frame sees along the unit ray of
                          * (persp (j - cx), persp (i - cy), 1), cx = (cols - 1)/2, cy = (rows - 1)/2
                          * (persp: the tangent of one pixel's angle, pixel pitch / focal length),
                          * and depth t is the range t dz along that ray.  APSS, the intensity graph
                          * and the initial normals then use these positions, APSS moves a point
                          * along its own ray and normals face the sensor.  p_xy still sets the
                          * neighbour window, R = ceil(h_apss / p_xy): set it to the smallest
                          * lateral pixel footprint (range x persp) of the scene.  E_UNSUPPORTED
                          * when that window's tile does not fit the APSS kernel's LDS (R > 5);
                          * per-step kernels only (fused_loop ignored). */
    int32_t  ilp_box;    /* divisor of the intensity low-pass (Results, "Reconstruction algorithm",
                          * intensity update: only points of one surface are correlated).  0 (default):
                          * r_new = (r + sum of the neighbours found) / (1 + their number), the mean
                          * over the point's surface, a pixel without a point of that surface taking
                          * no part; 1: divided by 1 + the number of surrounding pixels inside the
                          * image (a 3 x 3 box in which a missing neighbour counts as zero intensity,
                          * which attenuates isolated points).  E_INVALID for other values. */
    int32_t  lanes_per_pixel; /* lanes that share one pixel's active bins in the gradient steps: 4 or
                          * 8; 0 (default): rt3d_autotune's choice for the batch shape, else 8 below
                          * 131,072 pixels per call (four would leave most of the chip idle) and 4
                          * from there on.  The results do not depend on it beyond FP32 summation
                          * order; a frame gives the same bits in every batch only where this is
                          * fixed (4 or 8), as the default follows the batch's size.  E_INVALID for
                          * other values. */
} rt3d_params;

/* Input kinds. */
#define RT3D_IN_HIST_U16   0   /* dense histograms */
#define RT3D_IN_PHOTON_CSR 1   /* active-bin lists, as rt3d_debug_compact writes them */
#define RT3D_IN_PHOTON_EVENTS 2 /* unordered photon events (pixel, bin) */

typedef struct rt3d_input {
    uint32_t struct_size;      /* sizeof(rt3d_input) */
    int32_t  kind;             /* RT3D_IN_* */
    uint32_t frames, rows, cols;
    /* RT3D_IN_HIST_U16: device uint16 [frames][rows][cols][bins], 16-byte aligned. */
    const uint16_t* hist;
    /* RT3D_IN_PHOTON_CSR: device off[P + 1] and ent[off[P]]; entry = (bin << 16) | count,
     * bins strictly ascending within a pixel, counts >= 1. */
    const uint32_t* off;
    const uint32_t* ent;
    /* Optional device float gain[P] (g of the observation model); NULL = 1.
     * 0 marks a dead pixel; a gain that is not a finite number >= 0 is treated
     * as 0 and leaves RT3D_E_INVALID for rt3d_query. */
    const float* gain;
    /* RT3D_IN_PHOTON_EVENTS: n_events (< 2^31) photons, in any order; device
     * ev_pixel[n_events] = f * rows * cols + i * cols + j and ev_bin[n_events] = bin.
     * ev_scratch is caller-owned device memory of n_events uint32, overwritten.
     * An event with pixel >= P or bin >= bins is dropped and a bin receiving more
     * than 65535 photons is stored as 65535; both leave RT3D_E_INVALID for rt3d_query. */
    const uint32_t* ev_pixel;
    const uint16_t* ev_bin;
    uint32_t* ev_scratch;
    uint64_t n_events;
    /* Frames of different sizes in one call (both NULL: every frame is rows x cols).
     * Host arrays of `frames` entries: frame f is frame_rows[f] x frame_cols[f]
     * pixels and its pixels follow those of frame f - 1 (pixel-major within the
     * frame), in the histograms, the CSR, the gain, the output and the event
     * pixel numbers alike; rows and cols are then ignored and P is the sum of
     * the frames' pixels (the workspace must be sized for at least that many).
     * Consecutive frames of one size are processed as one group (the learned
     * denoiser runs once per group).  E_INVALID for a zero or oversized frame. */
    const uint32_t* frame_rows;
    const uint32_t* frame_cols;
    /* RT3D_FLAG_* bits. */
    uint32_t flags;
    /* Per-pixel IRFs h_ij (Results, "Observation model": the response is known
     * per pixel): optional device uint8 irf_class[P], the class (0 = the IRF of
     * rt3d_create, k = the k-th rt3d_add_irf) of every pixel; numbers the
     * context has no IRF for count as 0.  NULL: class 0 everywhere.  Each
     * IRF-dependent kernel then runs once per class of the context.
     * E_UNSUPPORTED with super-resolution or the learned denoiser. */
    const uint8_t* irf_class;
} rt3d_input;

/* Warm start (video): skip the initialisation; the iterations start from the
 * point state and background the previous reconstruction on this context left
 * (its output), for new photon data of the same frames and frame sizes.
 * E_STATE when the context holds no such state (no earlier call, a different
 * batch shape, or a step-by-step call in between). */
#define RT3D_FLAG_WARM_START 1u

typedef struct rt3d_output {
    uint32_t struct_size;      /* sizeof(rt3d_output) */
    uint32_t capacity;         /* points the per-point arrays can hold (P * RT3D_K_MAX always suffices) */
    uint32_t* pt_off;          /* device [P + 1]: points of pixel p are pt_off[p] .. pt_off[p+1]-1 */
    double*   depth;           /* device [capacity]: depth in bins, ascending within a pixel */
    float*    intensity;       /* device [capacity]: intensity in photons */
    float*    normal;          /* device [capacity * 3] or NULL: unit surface normal (x, y, z) */
    float*    background;      /* device [P]: background in photons per bin */
    double*   world_z;         /* device [capacity] or NULL: the point's world Z coordinate, depth x dz
                                  (orthographic) or depth x dz x the z component of the pixel's unit
                                  ray (params.persp > 0); Results, "Observation model": the map f */
} rt3d_output;
/* struct_size: sizeof(rt3d_output), or offsetof(rt3d_output, world_z) for
 * callers built before world_z existed (no world_z output then). */
/* (With params.sr = s > 1, P above is the point grid's pixel count for pt_off
 * and the lidar's for background; see rt3d_params.sr.) */

/* Per-point state in device memory, slot-major structure of arrays, as the
 * library keeps it between steps; used by the step-by-step entry points. */
typedef struct rt3d_state {
    uint32_t frames, rows, cols;
    double*  t;     /* [RT3D_K_MAX][P] depth, bins */
    float*   r;     /* [RT3D_K_MAX][P] intensity */
    float*   n;     /* [3][RT3D_K_MAX][P] normal components x, y, z */
    uint8_t* cnt;   /* [P] live slots 0..cnt-1, ascending depth */
    float*   b;     /* [P] background */
} rt3d_state;
/* With params.sr = s > 1 a state describes the point grid (rows and cols are
 * the point grid's, multiples of s) and b[0 .. frames (rows/s) (cols/s) - 1]
 * holds the lidar pixels' background (the rest of b is unused). */

typedef struct rt3d_stats {
    uint32_t struct_size;      /* sizeof(rt3d_stats) */
    int32_t  device_error;     /* sticky RT3D_E_* found on the device, or RT3D_OK */
    uint64_t entries;          /* active entries of the last compaction */
    uint64_t points;           /* points in the last output */
} rt3d_stats;

typedef struct rt3d_ctx rt3d_ctx;

/* Fill every field of *p with its default. */
void rt3d_params_default(rt3d_params* p);

/* Create a context for histograms of `bins` bins and the IRF irf[0..irf_len-1]
 * (host memory, copied): samples at integer lags, normalised here to unit sum,
 * origin sample `irf_origin` (< 0: the argmax, smallest index on ties).  The
 * continuous h is the Catmull-Rom interpolant of the samples (zero outside,
 * clamped at zero), so h and h' are continuous (Results, "Observation model":
 * h is known).
 * Requirements: 1 <= irf_len <= bins <= 65535, samples finite and >= 0 with
 * positive sum.  Uses the current HIP device; uploads small tables (blocking).
 * E_INVALID on bad arguments, E_DEVICE on a HIP failure. */
rt3d_status rt3d_create(const double* irf, uint32_t irf_len, int32_t irf_origin, uint32_t bins,
                        const rt3d_params* p, rt3d_ctx** out);

/* Per-pixel IRFs: adds IRF class *id (1, 2, ... < RT3D_MAX_IRFS) to the
 * context, with the same rules and the same model as rt3d_create's IRF (its
 * own length and origin; every table derived from it: S, the Fisher
 * information and so the depth step and its clip, the peak windows and
 * suppression width, the merge distance).  rt3d_input.irf_class names each
 * pixel's class.  Uploads the tables (blocking, on the context's device).
 * A graph recorded before this call keeps the classes it was recorded with
 * (its launches cover those classes only; higher numbers count as 0 there).
 * E_INVALID for a rejected IRF or a full context, E_UNSUPPORTED with
 * super-resolution or the learned denoiser, E_DEVICE on a HIP failure. */
#define RT3D_MAX_IRFS 16
rt3d_status rt3d_add_irf(rt3d_ctx* ctx, const double* irf, uint32_t irf_len, int32_t irf_origin, int32_t* id);

/* Destroy a context (NULL allowed).  Caller memory is not freed. */
void rt3d_destroy(rt3d_ctx* ctx);

/* Last error message of the context ("" if none). */
const char* rt3d_last_error(const rt3d_ctx* ctx);

/* IRF variance sigma_h^2 (bins^2) and model facts of the context. */
double rt3d_sigma2(const rt3d_ctx* ctx);

/* Bytes of device workspace needed for batches of up to frames x rows x cols
 * pixels with up to max_entries (< 2^32) active entries after compaction.
 * rt3d_set_workspace binds such a block (device memory owned by the caller,
 * 256-byte aligned, at least rt3d_workspace_bytes for the same arguments;
 * it clears the block's error word, synchronously).  The block must stay
 * valid while work that uses it is in flight; one workspace serves one stream
 * at a time.  E_INVALID on a NULL/misaligned pointer or max_entries >= 2^32,
 * E_NOMEM when `bytes` is too small. */
size_t rt3d_workspace_bytes(const rt3d_ctx* ctx, uint32_t frames, uint32_t rows, uint32_t cols,
                            uint64_t max_entries);
rt3d_status rt3d_set_workspace(rt3d_ctx* ctx, void* dev_ptr, size_t bytes, uint32_t frames,
                               uint32_t rows, uint32_t cols, uint64_t max_entries);

/* Whole reconstruction (all of the loop: compaction of histograms into active
 * bins, log-matched-filter initialisation, n_iter iterations of depth,
 * intensity and background updates, output packing) for a batch of frames.
 * Asynchronous on hip_stream; no host synchronisation inside.  E_INVALID /
 * E_NOMEM / E_UNSUPPORTED are found on the host before anything is enqueued. */
rt3d_status rt3d_reconstruct(rt3d_ctx* ctx, const rt3d_input* in, rt3d_output* out,
                             void* hip_stream);

/* Replayable reconstruction: one rt3d_reconstruct call recorded into a HIP
 * graph (its ~140 kernel launches become one graph launch).  The graph keeps
 * the call's pointers -- input, output, gain and the context's workspace --
 * so each replay repeats exactly that call on whatever the buffers then hold;
 * the caller refills the input between replays and must not rebind the
 * workspace or destroy the context while the graph exists.  Recording
 * enqueues nothing; E_STATE while kernel timing (rt3d_profile) is on; the
 * argument checks of rt3d_reconstruct apply.  rt3d_graph_launch is
 * asynchronous on hip_stream.  rt3d_graph_destroy accepts NULL. */
typedef struct rt3d_graph rt3d_graph;
rt3d_status rt3d_graph_create(rt3d_ctx* ctx, const rt3d_input* in, rt3d_output* out, rt3d_graph** graph);
rt3d_status rt3d_graph_launch(rt3d_graph* graph, void* hip_stream);
void rt3d_graph_destroy(rt3d_graph* graph);

/* Synchronise hip_stream, then report device-side errors, entry and point
 * counts of the last calls.  Returns the sticky device error (or OK). */
rt3d_status rt3d_query(rt3d_ctx* ctx, void* hip_stream, rt3d_stats* st);

/* Kernel timing.  rt3d_profile(ctx, id) makes every later launch of kernel
 * group `id` (RT3D_KERNEL_*) on any stream be bracketed by HIP events
 * recorded on that stream; id < 0 switches timing off.  rt3d_profile_read
 * waits for the recorded events, returns the summed milliseconds and the
 * number of timed launches, and clears them.  The events are created once and
 * reused (at most 4096 launches are kept between reads; later ones are not
 * timed).  E_INVALID for an unknown id, E_DEVICE on a HIP failure. */
#define RT3D_KERNEL_COMPACT   0   /* histogram -> active bins (count, scan, fill) */
#define RT3D_KERNEL_INIT      1   /* log-matched-filter initialisation */
#define RT3D_KERNEL_NORMALS   2   /* initial normals */
#define RT3D_KERNEL_DEPTH     3   /* depth gradient step */
#define RT3D_KERNEL_APSS      4   /* APSS */
#define RT3D_KERNEL_MERGE     5   /* in-pixel merge launched alone (the step entry point only) */
#define RT3D_KERNEL_INTENSITY 6   /* in-pixel merge fused with the intensity gradient step */
#define RT3D_KERNEL_IFILTER   7   /* intensity low-pass and threshold */
#define RT3D_KERNEL_BKG       8   /* background gradient step */
#define RT3D_KERNEL_BFILTER   9   /* background filter (row and column passes) */
#define RT3D_KERNEL_OUTPUT   10   /* output packing (count, scan, pack) */
#define RT3D_KERNEL_CNN      11   /* learned denoiser forward (features + four convolutions) */
#define RT3D_KERNEL_LOOP     12   /* every iteration in one launch (params.fused_loop) */
#define RT3D_KERNEL_COUNT    13
/* Autotuning.  Times a reconstruction of this input in each mapping of the
 * loop onto the GPU the batch admits -- one launch per step with 4 lanes per
 * pixel in the gradient steps, the same with 8 lanes, and all iterations in one
 * launch (one workgroup per frame; frames of one size up to 4096 pixels with
 * APSS) -- and keeps the fastest for this batch shape (frames x rows x cols) in
 * the context, where params.fused_loop = -1 and params.lanes_per_pixel = 0 use
 * it.  Synchronises the stream; the output holds the last timed
 * reconstruction.  *fused (may be NULL) receives 1 for the one-launch loop, 0
 * for one launch per step.  Batches of several frame sizes keep the defaults
 * (nothing is timed).  Not while a graph is being recorded.
 * rt3d_mapping reports the mapping rt3d_reconstruct would take for this input
 * (*fused as above, *lanes the lanes per pixel of the per-step gradient
 * kernels); no GPU work. */
rt3d_status rt3d_autotune(rt3d_ctx* ctx, const rt3d_input* in, rt3d_output* out, void* hip_stream,
                          int32_t* fused);
rt3d_status rt3d_mapping(rt3d_ctx* ctx, const rt3d_input* in, int32_t* fused, int32_t* lanes);
rt3d_status rt3d_profile(rt3d_ctx* ctx, int32_t id);
rt3d_status rt3d_profile_read(rt3d_ctx* ctx, double* total_ms, uint64_t* launches);

/* ---------------------------------------------------------------------------
 * Step-by-step entry points (each row of the loop alone, for testing and
 * for callers composing their own loop).  All asynchronous on hip_stream.
 * ------------------------------------------------------------------------- */

/* Histogram -> active-bin lists (Methods: cost linear in bins with non-zero
 * counts).  hist: device uint16 [P][bins], 16-byte aligned; off: device
 * [P + 1]; ent: device [capacity].  Entries beyond capacity are dropped and
 * E_CAPACITY becomes the sticky device error.  Needs the workspace. */
rt3d_status rt3d_debug_compact(rt3d_ctx* ctx, const uint16_t* hist, uint32_t npix,
                               uint32_t* off, uint32_t* ent, uint64_t capacity, void* hip_stream);

/* The same histogram -> active-bin lists as rt3d_debug_compact, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): it allocates nothing and
 * needs no workspace.  The per-pixel counts and the scan's tile prefixes live
 * in a fixed device array of the library, one per GPU (RT3D_NOALLOC_SCRATCH_BYTES,
 * held until the process ends); every histogram is read twice (no staging).
 * npix <= RT3D_NOALLOC_MAX_PIXELS, else E_INVALID; hist: device uint16
 * [npix][bins], 16-byte aligned; off: device [npix + 1]; ent: device
 * [capacity] (capacity > 0).  Entries beyond capacity are dropped and
 * E_CAPACITY is written to *dev_err (caller-owned device int32, never
 * cleared by the call; NULL: not reported).  Asynchronous on hip_stream.
 * Calls that overlap on one GPU (other streams or host threads) share the
 * array and race: the caller orders them. */
#define RT3D_NOALLOC_MAX_PIXELS 4194304u
#define RT3D_NOALLOC_SCRATCH_BYTES 16810248u
rt3d_status rt3d_compact_noalloc(rt3d_ctx* ctx, const uint16_t* hist, uint32_t npix, uint32_t* off,
                                 uint32_t* ent, uint64_t capacity, int32_t* dev_err, void* hip_stream);

/* Photon events -> the same active-bin lists (the photons a time-tagged
 * detector reports, counted per (pixel, bin); Methods: only bins with non-zero
 * counts are kept).  ev_pixel / ev_bin: device [n_events] (n_events < 2^31, any
 * order; pixel < npix, bin < bins); ev_scratch: caller-owned device
 * [n_events] uint32, overwritten.  off: device [npix + 1]; ent: device
 * [capacity].  The output does not depend on the event order.  Out-of-range
 * events are dropped and a count above 65535 is stored as 65535, each leaving
 * E_INVALID as the sticky device error; entries beyond capacity are dropped
 * with E_CAPACITY.  Needs the workspace. */
rt3d_status rt3d_debug_compact_events(rt3d_ctx* ctx, const uint32_t* ev_pixel, const uint16_t* ev_bin,
                                      uint64_t n_events, uint32_t npix, uint32_t* ev_scratch, uint32_t* off,
                                      uint32_t* ent, uint64_t capacity, void* hip_stream);

/* Steps.  `in` is read, `out` is written in full (it must not alias `in`);
 * off/ent are the active-bin lists, gain may be NULL.  With params.sr = s > 1
 * the states are point-grid states (see rt3d_state), off/ent/gain the lidar
 * pixels'; the gradient steps use the super-resolved lambda, the background
 * filter acts on the lidar background, and the initialisation runs on the
 * lidar grid before its points spread over the point grid (it needs a
 * workspace for the lidar frames).  Without super-resolution the
 * initialisation uses a bound workspace that covers the frames for its list
 * of pixels whose pooled window holds more than 608 active bins, which are
 * then scored from LDS; without one they take a slower search from HBM with
 * the same result. */
#define RT3D_STEP_INIT       0  /* log-matched-filter initialisation + initial normals (reads no state) */
#define RT3D_STEP_DEPTH      1  /* gradient step on depth */
#define RT3D_STEP_APSS       2  /* APSS depth denoiser */
#define RT3D_STEP_MERGE      3  /* in-pixel merge of coincident points */
#define RT3D_STEP_INTENSITY  4  /* gradient step on intensity */
#define RT3D_STEP_IFILTER    5  /* intensity low-pass, threshold, slot compaction */
#define RT3D_STEP_BKG        6  /* gradient step on background */
#define RT3D_STEP_BFILTER    7  /* background image filter */
#define RT3D_STEP_ITERATION  8  /* one whole iteration (steps 1..7) */
rt3d_status rt3d_debug_step(rt3d_ctx* ctx, int32_t step, const uint32_t* off, const uint32_t* ent,
                            const float* gain, const rt3d_state* in, rt3d_state* out,
                            void* hip_stream);

/* Raw partial derivatives of the negative log-likelihood (Results,
 * "Observation model"): gt, gr device float [RT3D_K_MAX][P] (slots >= cnt
 * written 0), gb device float [P] (with params.sr = s > 1: P point-grid
 * pixels for gt, gr and the lidar pixels for gb). */
rt3d_status rt3d_debug_gradients(rt3d_ctx* ctx, const uint32_t* off, const uint32_t* ent,
                                 const float* gain, const rt3d_state* st,
                                 float* gt, float* gr, float* gb, void* hip_stream);

/* The per-pixel IRF classes (device uint8 [P], as rt3d_input.irf_class) that
 * rt3d_debug_step and rt3d_debug_gradients use from now on; NULL: class 0
 * everywhere.  The array must stay valid while those calls use it. */
rt3d_status rt3d_debug_irf_class(rt3d_ctx* ctx, const uint8_t* irf_class);

/* ---------------------------------------------------------------------------
 * Learned depth denoiser.  The paper lets any denoiser act as the proximal
 * step of the depth block (Results, "Reconstruction algorithm"; Discussion).
 * With p->denoiser == RT3D_DENOISE_CNN the depth block runs, after the depth
 * gradient step, a four-layer 3x3 convolutional network on the per-pixel
 * slot maps (features of slots 0..2: (t - 5x5 mean of the slot)/sigma_h
 * clipped to [-8, 8], log(1 + r), valid flag; channels 16 -> 32 -> 32 -> 32
 * -> 3, ReLU between layers, zero padding), FP16 matrix-core arithmetic with
 * FP32 accumulation, and moves slot k by sigma_h * output_k; pixels with four
 * points use APSS.  Weights: RT3D_CNN_PARAMS FP32 values, layer by layer
 * w[ky][kx][cin][cout] then bias[cout] for (cin, cout) = (16, 32), (32, 32),
 * (32, 32), (32, 3).  The workspace of a CNN context holds the training
 * buffers (size it with rt3d_workspace_bytes on that context).
 * ------------------------------------------------------------------------- */
#define RT3D_CNN_PARAMS 24003

typedef struct rt3d_adam {
    uint32_t struct_size;      /* sizeof(rt3d_adam) */
    float lr;                  /* >= 0; 0 computes loss and gradient, weights stay */
    float beta1, beta2;        /* in [0, 1) */
    float eps;                 /* > 0 */
} rt3d_adam;

/* Host FP32 weights in / out (synchronous on the null stream).  Setting the
 * weights clears the Adam moments and step.  E_INVALID when n != RT3D_CNN_PARAMS. */
/* Checkpoint of the network and its optimiser, so training resumes exactly:
 * rt3d_denoiser_save writes (synchronously, after the device is idle) a
 * little-endian file: the 8 bytes "RT3DCNN\0", uint32 version (1), uint32
 * RT3D_CNN_PARAMS, uint32 layer count (4) and each layer's input and output
 * channels, int64 Adam step, then FP32 master weights, Adam first moments and
 * Adam second moments (RT3D_CNN_PARAMS each, in the weight layout above), and
 * a uint64 FNV-1a hash of every byte before it.  rt3d_denoiser_load reads such
 * a file into the context (weights, moments and step; blocking) and marks the
 * network loaded.  E_INVALID for a NULL path, a file that is not such a
 * checkpoint (magic, version, sizes, hash, non-finite values: the context is
 * left unchanged), E_DEVICE on an I/O or HIP failure, E_STATE when the context
 * was not created with RT3D_DENOISE_CNN. */
rt3d_status rt3d_denoiser_save(rt3d_ctx* ctx, const char* path);
rt3d_status rt3d_denoiser_load(rt3d_ctx* ctx, const char* path);
rt3d_status rt3d_cnn_set_weights(rt3d_ctx* ctx, const float* host, size_t n);
rt3d_status rt3d_cnn_get_weights(rt3d_ctx* ctx, float* host, size_t n);

/* FP32 gradient of the last rt3d_cnn_train_step (in the weight layout above),
 * synchronous, for testing.  E_STATE without a CNN workspace. */
rt3d_status rt3d_cnn_last_gradient(rt3d_ctx* ctx, float* host, size_t n);

/* Network output for a state: y device float [3][P] (corrections in sigma_h
 * units for slots 0..2; pixels with four points included).  Needs a CNN
 * context and its workspace. */
rt3d_status rt3d_cnn_forward(rt3d_ctx* ctx, const rt3d_state* st, float* y, void* hip_stream);

/* One training step on a state (the depth block's input) and its true depths
 * truth: device float [n_surf][P], NaN where a pixel has no such surface.
 * Targets: slot k < min(cnt, 3) takes the nearest true depth of its pixel
 * within 3 sigma_h; loss = mean squared error of the outputs over matched
 * slots.  Backward pass on the matrix cores, deterministic weight-gradient
 * reduction, Adam on the FP32 master weights.  loss: device float [2] =
 * (loss, matched slots).  Asynchronous on hip_stream. */
rt3d_status rt3d_cnn_train_step(rt3d_ctx* ctx, const rt3d_state* st, const float* truth, uint32_t n_surf,
                                const rt3d_adam* opt, float* loss, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
