/*
 * dptrack.h - C ABI of the MI355X (gfx950) direct photometric tracker.
 *
 * Pose-only direct photometric tracking of a frame against a sparse map
 * (paper Sec. IV): an image pyramid, an inverse-compositional (IC) precompute
 * per reference frame, and a per-frame coarse-to-fine Gauss-Newton track whose
 * normal equations are reduced and solved on the GPU.
 *
 * Conventions shared by every entry point
 *   - Return value: DPT_OK (0) or a negative dpt_error.  dpt_last_error() gives a
 *     message for the calling thread, valid until that thread's next call.
 *     Nothing throws across the ABI and nothing aborts.
 *   - A tracking failure is not an API error: dpt_track_frame returns DPT_OK and
 *     reports it in dpt_result.status together with the best pose reached.
 *   - Poses are world -> camera, row-major 4x4 doubles (Eq.(1): u = pi(T P)).
 *   - Images are uint8 grayscale, row-major, with a row pitch in bytes >= width.
 *     Pixel centres sit at integer coordinates.
 *   - The caller owns every input buffer; it is only borrowed for the duration
 *     of the call.  A context copies what it keeps into device memory it owns.
 *   - "on_device" flags say whether a pointer is device memory (1, HIP) or host
 *     memory (0); any other value is DPT_E_ARG.  Device inputs must stay valid
 *     until the call returns.
 *   - All GPU work of a context is ordered on the HIP stream given at creation
 *     (NULL = the null stream).  Calls that return host results synchronise that
 *     stream before returning.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef DPTRACK_H
#define DPTRACK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPT_OK = 0,
  DPT_E_ARG = -1,   /* invalid argument: NULL pointer, size or flag out of range */
  DPT_E_HIP = -2,   /* a HIP runtime call or kernel launch failed */
  DPT_E_STATE = -3, /* call out of order (no pyramid / no reference points yet) */
  DPT_E_OOM = -4    /* device or pinned host allocation failed */
} dpt_error;

/* dpt_result.status */
enum {
  DPT_TRACK_OK = 0,             /* converged at level 0 */
  DPT_TRACK_MAX_ITERS = 1,      /* level 0 used all max_iters iterations (pose still returned) */
  DPT_TRACK_TOO_FEW_POINTS = 2, /* fewer than min_points valid points at some iteration */
  DPT_TRACK_NOT_PD = 3,         /* normal matrix not positive definite (Cholesky pivot too small) */
  DPT_TRACK_TIMEOUT = 4         /* a cooperative wait gave up (dpt_set_spin_limit); the pose is not valid */
};

/* dpt_params.precision */
enum { DPT_PREC_FP32 = 0, DPT_PREC_MIXED = 1 };

/* dpt_params.flags
 *   DPT_FLAG_FIXED_H  the paper's own inverse-compositional track (Sec. IV-B,
 *                     Sec. IV-C precompute and track): per level, H = sum of J^T J
 *                     over every reference-valid point and sample is reduced
 *                     once when the reference is set, and each iteration reduces
 *                     only b = -sum J^T r over the points valid in the current
 *                     frame; no robust weights (huber_k is ignored, the cost is
 *                     r^2/2).  FP32 precision only. */
enum { DPT_FLAG_FIXED_H = 1 };
/*   DPT_FLAG_GAUSS_F32  track on the paper's floating-point Gaussian pyramid
 *                     (Sec. IV-C, image pyramids) instead of the uint8 box
 *                     pyramid: level 0 is the frame as FP32, each coarser level
 *                     blurs the previous one by a vertical and then a horizontal
 *                     pass of the binomial kernel [1 3 3 1]/8 (samples 2y-1 ..
 *                     2y+2, clamped to the level) and keeps every second sample,
 *                     so pixel centres and per-level intrinsics are those of the
 *                     box pyramid.  Point selection still reads the uint8 frame.
 *                     FP32 precision only. */
enum { DPT_FLAG_GAUSS_F32 = 2 };

/* pyramid slots */
enum { DPT_SLOT_REF = 0, DPT_SLOT_CUR = 1 };

/* Level-0 pinhole camera: u = fx X/Z + cx, v = fy Y/Z + cy.  Level l uses
 * f/2^l and (c + 0.5)/2^l - 0.5, consistent with the 2x2 box pyramid. */
typedef struct {
  int32_t width, height; /* 16 <= width, height <= 8192 */
  double fx, fy, cx, cy;
} dpt_camera;

typedef struct {
  int32_t levels;       /* pyramid levels, 1..8; level l is floor(W/2^l) x floor(H/2^l) */
  int32_t max_iters;    /* Gauss-Newton iterations per level, 1..100 */
  float huber_k;        /* Huber threshold in intensity levels; <= 0 = plain least squares */
  float step_eps;       /* a level ends when max_j |delta_j| < step_eps (rad, m) */
  float z_min;          /* points with camera depth <= z_min (m) are invalid */
  int32_t min_points;   /* fewer valid points: DPT_TRACK_TOO_FEW_POINTS */
  int32_t n_pattern;    /* patch samples per point K, 1..128 */
  int8_t pattern[256];  /* K (dx, dy) offsets in level pixels, |d| <= 16, same at every level */
  int32_t precision;    /* DPT_PREC_FP32 */
  int32_t flags;        /* 0, or DPT_FLAG_FIXED_H and/or DPT_FLAG_GAUSS_F32 */
} dpt_params;

typedef struct {
  double T_cw[16];             /* world -> current camera */
  double final_cost;           /* mean Huber cost over the valid level-0 samples at T_cw (0 if none) */
  int32_t iterations;          /* Gauss-Newton updates applied, all levels */
  int32_t iters_per_level[8];  /* updates per level (index = level) */
  int32_t n_valid_points;      /* valid level-0 points at T_cw */
  int32_t status;              /* DPT_TRACK_* */
  int64_t samples;             /* residual samples evaluated, all passes */
} dpt_result;

typedef struct dpt_ctx dpt_ctx;

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* dpt_last_error(void);

/* Create a single-stream tracker.  max_points bounds every later reference map
 * (1..65536).  hip_stream: a hipStream_t, or NULL.  Allocates all device memory
 * the context needs: two pyramids, the per-level IC cache (12 bytes per sample
 * and level), staging buffers.  *out receives the context. */
int dpt_create(const dpt_camera* cam, const dpt_params* prm, int32_t max_points, void* hip_stream, dpt_ctx** out);

/* Release a context and all its memory (NULL is a no-op). */
void dpt_destroy(dpt_ctx* ctx);

/* Build the uint8 pyramid of one slot from an image (paper Sec. IV-C, "Image
 * pyramids"; read here as 2x2 box means rounded half up, floor sizes).
 * slot: DPT_SLOT_REF or DPT_SLOT_CUR.  img: width x height bytes, row pitch
 * `pitch` >= width, in device memory if img_on_device else host memory.
 * Building the REF slot invalidates the reference points. */
int dpt_build_pyramid(dpt_ctx* ctx, int32_t slot, const uint8_t* img, int64_t pitch, int32_t img_on_device);

/* Copy level `level` of a slot's pyramid (floor(W/2^l) x floor(H/2^l), packed
 * rows) to host memory.  Test hook for bit-exact comparison. */
int dpt_get_pyramid(dpt_ctx* ctx, int32_t slot, int32_t level, uint8_t* host_dst);
/* DPT_FLAG_GAUSS_F32 contexts: level `level` of the slot's floating-point
 * Gaussian pyramid, W_l x H_l floats, into host memory (waits for the stream). */
int dpt_get_pyramid_f32(dpt_ctx* ctx, int32_t slot, int32_t level, float* host_dst);

/* Map-point selection on the REF slot's level 0 (stand-in for the map points the
 * indirect pipeline provides, Sec. III): the n pixels with the largest integer
 * score (I[y][x+1]-I[y][x-1])^2 + (I[y+1][x]-I[y-1][x])^2 inside
 * margin <= x <= W-1-margin, margin <= y <= H-1-margin (margin >= 1), ties to the
 * smaller linear index y*W+x.  Writes min(n, candidates) indices in ascending
 * order to host_idx (capacity n) and their count to *n_out. */
int dpt_select_points(dpt_ctx* ctx, int32_t n, int32_t margin, int32_t* host_idx, int32_t* n_out);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the selection of
 * dpt_select_points on a device image the caller passes, needing no context
 * and allocating nothing.  Its histograms, completion counter and per-chunk
 * counts live in a static device array of the library (about 36 KB per GPU,
 * held until the process ends) instead of context memory; the call only
 * enqueues kernels on hip_stream (a kernel clears the array first) and never
 * waits.  img: device uint8 image width x height, rows `pitch` bytes apart
 * (width <= pitch < 2^31); idx: device int32[n], receives min(n, candidates)
 * indices y*width+x in ascending order; count: device int32, receives their
 * number.  The outputs are complete once the stream has run the call.
 * width * height <= 4096 * 4096 (DPT_E_ARG beyond, before any device work);
 * n and margin as in dpt_select_points.  All calls on one GPU share the array:
 * calls that overlap on one GPU (two streams, two threads) race and may return
 * wrong selections; serialise them. */
int dpt_select_points_noalloc(const uint8_t* img, int32_t width, int32_t height, int64_t pitch, int32_t n,
                              int32_t margin, int32_t* idx, int32_t* count, void* hip_stream);

/* Set the reference map and run the IC precompute on the REF pyramid (Sec.
 * IV-C "Precompute Inverse Compositional", Eq.(6)): for each level and point,
 * x0 = T_rw P, the patch intensities I0 and reference-side gradients are cached;
 * the Jacobian is rebuilt from them and x0 during tracking.
 * xyz_world: n x 3 floats (device memory if xyz_on_device).  T_rw: world ->
 * reference camera.  0 <= n <= max_points. */
int dpt_set_reference_points(dpt_ctx* ctx, const float* xyz_world, int32_t n, const double T_rw[16],
                             int32_t xyz_on_device);

/* Reference update from a depth map, all on the stream with no host round trip
 * (the RGB-D form of the reference update: the map points of Sec. IV-A come
 * from the reference frame's own depth instead of the indirect pipeline).
 * Selects n points on the REF level 0 exactly as dpt_select_points, turns each
 * selected pixel (x, y) with depth z into P = T_rw^-1 (z K^-1 [x, y, 1]^T)
 * (FP64, rounded to FP32) and runs the IC precompute of
 * dpt_set_reference_points on them.  The map holds n points: a selected pixel
 * without a positive finite depth, and the entries past the selection count
 * (only when fewer than n candidates exist), are points that are never valid.
 * depth: level-0 depths in metres, rows of depth_pitch floats (>= width),
 * device memory if depth_on_device (else copied, synchronously).
 * 1 <= n <= max_points; margin as in dpt_select_points. */
int dpt_set_reference_from_depth(dpt_ctx* ctx, int32_t n, int32_t margin, const float* depth, int64_t depth_pitch,
                                 int32_t depth_on_device, const double T_rw[16]);

/* Track the CUR pyramid against the reference (Sec. IV-C "Track"; Eq.(2)-(5)):
 * coarse to fine, per level up to max_iters Huber-weighted Gauss-Newton steps,
 * the 21 + 6 normal-equation terms reduced on the GPU, a Cholesky solve and the
 * inverse-compositional update T_rel <- T_rel exp(delta)^-1 on the GPU, then a
 * cost-only pass at level 0.  T_cw_init: start pose.  Synchronises the stream
 * and fills *out. */
int dpt_track_frame(dpt_ctx* ctx, const double T_cw_init[16], dpt_result* out);

/* Start pose of an enqueued track. */
enum { DPT_INIT_GIVEN = 0, DPT_INIT_CONST_VELOCITY = 1, DPT_INIT_PROPOSED = 2 };

/* Most tracks (frames) enqueued and not yet synchronised, per context or batch. */
#define DPT_MAX_IN_FLIGHT 256

/* Run reference updates on a second stream (hip_stream; NULL or the context's
 * own stream: back to one stream), so that a keyframe's reference update (the
 * reference pyramid, selection, back-projection and IC precompute of
 * Sec. IV-C) overlaps the tracks of the previous keyframe's frames.  The
 * context then holds two reference banks: an update starts with
 * dpt_build_pyramid(DPT_SLOT_REF) (dpt_set_reference_points and
 * dpt_set_reference_from_depth without one return DPT_E_STATE), writes the bank
 * the tracks do not read once the tracks that read it last have run, and the
 * first track or test hook after it waits (on the context's stream) for the
 * update.  Results are those of the single-stream form.  Inputs of an update
 * (images, depth maps) are read on the reference stream, and so are the
 * device frames of the first window track after it (dpt_track_window_enqueue
 * builds that window's pyramids there, behind the update): the caller orders
 * their producers before it; reading the reference back (dpt_get_pyramid of
 * DPT_SLOT_REF) waits for the reference stream.  The stream stays the
 * caller's and must outlive its use: until the context is destroyed or set
 * back to one stream.  The first call allocates the second bank; the call
 * waits for both streams.  DPT_E_STATE while an update is open. */
int dpt_set_reference_stream(dpt_ctx* ctx, void* hip_stream);

/* A HIP stream for the reference updates: default priority, not ordered with
 * the null stream.  *out receives the stream; the caller destroys it with
 * dpt_stream_destroy (which waits for its work) after every context or batch
 * using it has been destroyed or switched back to one stream.  A process that
 * only needs this one extra stream avoids creating a pool of them. */
int dpt_stream_create(void** out);
int dpt_stream_destroy(void* stream);

/* Asynchronous form of dpt_track_frame (the same computation, Sec. IV-C
 * "Track"): enqueue the track of the CUR pyramid on the context's stream and
 * return at once, so frames can follow each other without the host waiting
 * between them (the paper keeps the tracker on the GPU to avoid CPU-GPU
 * exchange, Sec. IV-C).  The start pose is T_cw_init (DPT_INIT_GIVEN) or the
 * constant-velocity prediction T1 T0^-1 T1 from the context's pose history
 * (DPT_INIT_CONST_VELOCITY, computed on the GPU in FP64; T_cw_init may be NULL),
 * or the learned initialiser's proposal that the last dpt_cnn_propose on this
 * context left in device memory (DPT_INIT_PROPOSED; DPT_E_STATE if none).
 * The history holds the last two poses: dpt_set_pose_history sets it, and every
 * track on the cooperative path appends its result.  The constant-velocity
 * start and the proposed one need that path (launch mode AUTO or COOP; DPT_E_ARG
 * otherwise); on the one-workgroup path a DPT_INIT_GIVEN enqueue runs
 * synchronously.  *out is written by the next dpt_synchronize (or any call
 * that synchronises the context) and must stay valid until then.  At most
 * DPT_MAX_IN_FLIGHT tracks may be in flight (DPT_E_STATE beyond).  Later pyramid builds and
 * reference updates on the same stream are ordered after the enqueued track. */
int dpt_track_enqueue(dpt_ctx* ctx, int32_t init_mode, const double T_cw_init[16], dpt_result* out);

/* Wait for the context's stream and fill the results of every enqueued track.
 * Returns DPT_E_HIP if one of them timed out (its result has status 4).
 * Whatever it returns, no track is in flight afterwards: on a failure of the
 * wait itself every result of a track that finished is filled, every other one
 * gets status DPT_TRACK_TIMEOUT, and the library keeps no pointer to the
 * results or the frames. */
int dpt_synchronize(dpt_ctx* ctx);

/* Fill the results of the oldest n enqueued tracks as soon as they have
 * finished, while the tracks enqueued after them keep the GPU busy: a serving
 * loop collects finished frames without draining the stream.  The host polls
 * the results in host memory (each written last with its sequence number).
 * DPT_E_ARG if fewer than n tracks are in flight; if one of the n timed out,
 * behaves as dpt_synchronize (waits for everything, DPT_E_HIP); DPT_E_HIP if
 * the stream ran dry without the results or none came within 60 s, and then,
 * as after a failed dpt_synchronize, nothing is in flight any more (finished
 * tracks filled, the others DPT_TRACK_TIMEOUT). */
int dpt_collect(dpt_ctx* ctx, int32_t n);

/* Number of enqueued tracks whose results no dpt_synchronize or dpt_collect
 * has filled yet (calls that wait for the stream themselves, such as
 * dpt_track_frame or a launch-configuration change, fill them too), or a
 * negative error code. */
int dpt_tracks_in_flight(dpt_ctx* ctx);

/* Set the pose history used by DPT_INIT_CONST_VELOCITY (row-major 4x4 T_cw,
 * older first), ordered on the stream with the tracks.  Initially identity. */
int dpt_set_pose_history(dpt_ctx* ctx, const double T_older[16], const double T_newer[16]);

/* Most frames one window track may cover. */
#define DPT_MAX_WINDOW 32

/* Window tracking: the tween frames of one reference (Sec. III: the frames the
 * direct tracker handles between two references), n_frames consecutive frames
 * tracked in order against the current reference by one pyramid launch for
 * all of them and one cooperative track launch, the same computation as
 * n_frames dpt_build_pyramid(CUR) + dpt_track_enqueue calls: frame 0 starts
 * from T_cw_init (DPT_INIT_GIVEN) or the constant-velocity prediction of the
 * pose history (DPT_INIT_CONST_VELOCITY), every later frame from the
 * constant-velocity prediction of the two poses before it, and the history
 * ends with the window's last two poses.  The poses are bitwise those of the
 * frame-by-frame calls.  frames: n_frames uint8 W x H images, rows `pitch`
 * bytes apart, frame f at frames + f * frame_stride, in device memory if
 * frames_on_device (1), else host memory (0; copied, and the call then waits
 * for the stream).  out: n_frames results, written by the next
 * dpt_synchronize.  1 <= n_frames <= DPT_MAX_WINDOW; the frames count towards
 * the DPT_MAX_IN_FLIGHT tracks in flight.  The window pyramids are the context's own (the
 * CUR slot is left as it was), allocated on the first call and grown when a
 * longer window comes (the call then first waits for the tracks in flight).
 * Device frames whose rows are W bytes apart (pitch == width) are level 0 of
 * their pyramids as they are: the track launch reads them too, so they must
 * stay unchanged until it has run (work enqueued later on the same stream is
 * ordered after it).
 * DPT_E_ARG for a frame_stride smaller than a frame, the one-workgroup launch
 * mode, or DPT_FLAG_GAUSS_F32; DPT_E_STATE without reference points. */
int dpt_track_window_enqueue(dpt_ctx* ctx, const uint8_t* frames, int64_t pitch, int64_t frame_stride,
                             int32_t n_frames, int32_t frames_on_device, int32_t init_mode,
                             const double T_cw_init[16], dpt_result* out);

/* ------------------------------------------------------------------ tween-window schedule
 * The schedule of Sec. III and Sec. IV-D: direct tracking handles the tween
 * frames between references that the indirect pipeline provides, and hands a
 * frame back to it when
 *   - the track fails (status TOO_FEW_POINTS, NOT_PD or a timeout; a pose that
 *     reached the iteration cap counts as valid),
 *   - its robust error (final_cost, the mean Huber cost) exceeds max_cost,
 *   - the camera centre moved more than max_baseline metres from the
 *     reference's (max_baseline <= 0: no baseline test), or
 *   - max_direct frames were already tracked directly against this reference
 *     (then no direct attempt is made).
 * The paper names a switching and a failure threshold on the error; here they
 * are one value, max_cost.  The indirect side (ORB-SLAM2 in the paper) is the
 * caller: after any decision other than DPT_TWEEN_DIRECT it gives the frame's
 * pose and depth to dpt_tween_anchor, which makes that frame the new reference
 * (selection, back-projection, IC precompute on the device). */
typedef struct {
  float max_cost;      /* accept a direct frame only if final_cost <= max_cost */
  float max_baseline;  /* metres; <= 0: unlimited */
  int32_t max_direct;  /* direct frames per reference, >= 0 */
  int32_t n_points;    /* map points selected at each anchor, 1..max_points */
  int32_t margin;      /* selection margin at each anchor (pixels) */
  int32_t pad;
} dpt_tween_policy;

enum {
  DPT_TWEEN_DIRECT = 0,           /* the direct pose is accepted */
  DPT_TWEEN_INDIRECT_FAILED = 1,  /* the track failed */
  DPT_TWEEN_INDIRECT_COST = 2,    /* final_cost > max_cost */
  DPT_TWEEN_INDIRECT_BASELINE = 3,
  DPT_TWEEN_INDIRECT_MAX_FRAMES = 4
};

typedef struct {
  int32_t decision;          /* DPT_TWEEN_* */
  int32_t direct_since_ref;  /* direct frames accepted against the current reference, this one included */
  int32_t tracked;           /* 1 if a direct track was run (its result is in `track`) */
  int32_t pad;
  double baseline;           /* camera-centre distance of the direct estimate to the reference (m) */
  dpt_result track;
} dpt_tween_result;

/* Set the schedule's policy (copied).  DPT_E_ARG on invalid values. */
int dpt_tween_set_policy(dpt_ctx* ctx, const dpt_tween_policy* policy);

/* Reference from an indirect frame: its image (host or device, `pitch` bytes per
 * row), level-0 depth (as dpt_set_reference_from_depth) and pose T_cw from the
 * indirect pipeline.  Builds the REF pyramid, selects policy.n_points points,
 * back-projects and precomputes, sets the constant-velocity history to (the
 * previous accepted or anchored pose, T_cw) and restarts the direct count.
 * The first anchor of a context uses T_cw as both history entries. */
int dpt_tween_anchor(dpt_ctx* ctx, const uint8_t* img, int64_t pitch, int32_t img_on_device, const float* depth,
                     int64_t depth_pitch, int32_t depth_on_device, const double T_cw[16]);

/* One tween frame: builds the CUR pyramid, tracks from the constant-velocity
 * prediction of the last two accepted or anchored poses and applies the policy.
 * Waits for the result.  After a decision other than DPT_TWEEN_DIRECT the
 * context needs dpt_tween_anchor before the next tween frame (DPT_E_STATE
 * otherwise, and before the first anchor). */
int dpt_tween_frame(dpt_ctx* ctx, const uint8_t* img, int64_t pitch, int32_t img_on_device, dpt_tween_result* out);

/* Test hook: copies of level `level`'s IC cache.  Any pointer may be NULL.
 * valid: n bytes; I0, gx, gy: n*K floats (sample i*K+k); x0: n*3 floats. */
int dpt_get_reference_cache(dpt_ctx* ctx, int32_t level, uint8_t* valid, float* I0, float* gx, float* gy, float* x0);

/* Test hook: one normal-equation pass (Eq.(5), Huber-weighted) at `level` and the
 * relative pose T_rel = T_cw T_rw^-1 (4x4 row-major doubles, used in FP32).
 * H21: upper triangle of H, row-major (H00 H01 .. H05 H11 .. H55); b6; E: sum of
 * Huber costs; n: valid samples; npts: valid points. */
int dpt_normal_equations(dpt_ctx* ctx, int32_t level, const double T_rel[16], float* H21, float* b6, double* E,
                         int64_t* n, int32_t* npts);
/* In the fixed-H mode H21 is the level's precomputed H, and b, E are unweighted. */

/* Fixed-H mode (DPT_FLAG_FIXED_H, Sec. IV-C precompute): the level's H of the
 * current reference as a full symmetric 6x6 row-major (FP64 sum of the FP32
 * per-point terms), and not_pd = 1 when its Cholesky factor failed (a pivot at
 * most 1e-6 of the largest diagonal entry: every track then ends with
 * DPT_TRACK_NOT_PD at that level).  Waits for the stream.  DPT_E_STATE when the
 * context is not in the fixed-H mode or has no reference. */
int dpt_get_fixed_hessian(dpt_ctx* ctx, int32_t level, double H36[36], int32_t* not_pd);

/* Launch configuration of the track kernel.
 *   DPT_LAUNCH_AUTO       cooperative chunks when the GPU supports co-resident
 *                         launches and the map fits, else one workgroup per frame
 *   DPT_LAUNCH_WORKGROUP  one 512-thread workgroup runs the whole frame
 *   DPT_LAUNCH_COOP       the map is split into chunks of `chunk` points (64, 128
 *                         or 256), one workgroup each, synchronised per iteration.
 *                         Patterns other than the 8-pixel one and the Gaussian
 *                         float pyramid use chunks of 64 points, four threads per
 *                         point, whatever `chunk` says
 *   DPT_LAUNCH_COOP_PAIRS as DPT_LAUNCH_COOP with two threads per point, each
 *                         taking four of the 8-pixel pattern's samples: chunks
 *                         of `chunk` points (64 or 128) in 2 x chunk threads.
 *                         Half the work per thread on twice the compute units:
 *                         the faster form for a stream or a small batch that
 *                         leaves most of the GPU idle.  Other patterns and the
 *                         Gaussian float pyramid run as DPT_LAUNCH_COOP
 * Results agree with each other to rounding (the summation order differs).
 *
 * Co-residency.  The chunks of a stream wait for each other's partial sums,
 * so all workgroups of a cooperative track must run at the same time.  A grid
 * larger than a quarter of the device's co-resident capacity (two workgroups
 * per compute unit) goes through the cooperative launch, which the runtime
 * only starts once every workgroup fits.  A smaller grid (one stream of up to
 * 16 chunks, or a small batch) is launched as an ordinary kernel to save the
 * cooperative launch's extra cost; it is co-resident whenever the device has
 * that much room, which holds while this process runs at most three such
 * tracks concurrently and no other work fills the compute units.  If other
 * streams or processes occupy the device so that a chunk cannot start, the
 * waiting chunks give up after the spin limit (dpt_set_spin_limit) and the
 * frame ends with DPT_TRACK_TIMEOUT instead of a pose; nothing hangs.  A caller
 * that shares the device with heavy concurrent work and cannot accept that
 * outcome uses DPT_LAUNCH_WORKGROUP, which never waits across workgroups. */
enum { DPT_LAUNCH_AUTO = 0, DPT_LAUNCH_WORKGROUP = 1, DPT_LAUNCH_COOP = 2, DPT_LAUNCH_COOP_PAIRS = 3 };
int dpt_set_launch_config(dpt_ctx* ctx, int32_t mode, int32_t chunk);

/* Bound of the cooperative track's waits: a chunk that polls the other chunks'
 * partial sums `polls` times without seeing them all gives up, and its frame
 * (and, in a window track, the frames after it) ends with status
 * DPT_TRACK_TIMEOUT; the next synchronisation then reports DPT_E_HIP and resets
 * the exchange, so later tracks start clean.  Default 4194304 (about a second
 * of polling, a poll round being one memory round trip; reached only if the
 * chunks were not co-resident).  polls = 0 makes
 * every cross-chunk wait give up at once, which exercises that path; a map of
 * one chunk never waits.  DPT_E_ARG for polls < 0. */
#define DPT_DEFAULT_SPIN_LIMIT 4194304
int dpt_set_spin_limit(dpt_ctx* ctx, int32_t polls);

/* Cycle split of the cooperative track kernels, for performance work: only a
 * library compiled with -DDPT_CYCLE_PROFILE (paper_2607_16897_amd/build.py
 * --cycles, libdptrack_cycles.so) records it; every other build returns
 * DPT_E_STATE.  For each of the first n_slots workgroup slots of the launch
 * grids, DPT_CYCLE_FIELDS int64 values summed over every launch since the last
 * reset, as seen by thread 0 of the workgroup (shader-clock cycles):
 *   DPT_CYCLE_ACCUMULATE  its own point's residuals and normal-equation terms
 *   DPT_CYCLE_REDUCE      the wave reduction up to the workgroup barrier (waits
 *                         there for the workgroup's slowest wave)
 *   DPT_CYCLE_EXCHANGE    the cross-chunk exchange until the stream totals
 *   DPT_CYCLE_SOLVE       the 6x6 solve and pose update
 *   DPT_CYCLE_ITERATIONS  Gauss-Newton iterations and DPT_CYCLE_LAUNCHES launches
 *   DPT_CYCLE_KERNEL      cycles from the workgroup's start to its end
 *   DPT_CYCLE_REALTIME    the same span in ticks of the 100 MHz constant clock
 *   DPT_CYCLE_PLACE       where the slot's last workgroup ran: XCC id << 32 |
 *                         the HW_ID register (CU, SIMD, shader engine)
 *   DPT_CYCLE_POLLS       poll rounds of the exchanges (one round reads every
 *                         chunk's words once)
 *   DPT_CYCLE_FRAME_START each frame's start (start pose) before its first level
 *   DPT_CYCLE_LEVEL_START each level's start (its points' registers and the
 *                         LDS tile) before its first iteration
 *   DPT_CYCLE_FINAL       the final cost pass with its exchange
 *   DPT_CYCLE_FRAMES      frames tracked
 *   DPT_CYCLE_FRAME_END   window tracks: each frame's end (its pose refined,
 *                         its result written, the history extended)
 * out: n_slots * DPT_CYCLE_FIELDS int64, slot-major.  reset != 0 clears the
 * sums after reading.  Waits for the device.  1 <= n_slots <= 1024. */
#define DPT_CYCLE_FIELDS 16
enum {
  DPT_CYCLE_ACCUMULATE = 0, DPT_CYCLE_REDUCE = 1, DPT_CYCLE_EXCHANGE = 2, DPT_CYCLE_SOLVE = 3,
  DPT_CYCLE_ITERATIONS = 4, DPT_CYCLE_LAUNCHES = 5, DPT_CYCLE_KERNEL = 6, DPT_CYCLE_REALTIME = 7,
  DPT_CYCLE_PLACE = 8, DPT_CYCLE_POLLS = 9, DPT_CYCLE_FRAME_START = 10, DPT_CYCLE_LEVEL_START = 11,
  DPT_CYCLE_FINAL = 12, DPT_CYCLE_FRAMES = 13, DPT_CYCLE_FRAME_END = 14
};
int dpt_cycle_profile(int64_t* out, int32_t n_slots, int32_t reset);

/* Profiling hook: with enable = N > 0, every N-th pyramid build and every
 * N-th track brackets its kernel with HIP events on the context's stream
 * (each event record is a queue marker of a few microseconds, so N > 1 keeps
 * the measurement from slowing the stream much); 0 switches it off (the
 * default), < 0 is DPT_E_ARG.  dpt_last_kernel_ms returns the durations (ms)
 * of the most recent timed pyramid and track kernels (-1 if none was timed);
 * dpt_get_profile the totals (ms) and counts of the timed launches since
 * profiling was enabled.  Both synchronise the context; so does enabling,
 * which also resets the totals. */
int dpt_set_profiling(dpt_ctx* ctx, int32_t enable);
int dpt_last_kernel_ms(dpt_ctx* ctx, float* pyramid_ms, float* track_ms);
int dpt_get_profile(dpt_ctx* ctx, double* pyramid_ms, int64_t* n_pyramid, double* track_ms, int64_t* n_track);

/* ------------------------------------------------------------------ batched streams
 * Many independent camera streams tracked together: one pyramid launch for all
 * streams' images and one cooperative track launch per group of streams that
 * fits the GPU's co-resident capacity (every stream's map split into chunks,
 * Sec. IV-C's per-point work and tree reduction run per chunk), or one
 * workgroup per stream.  Each stream keeps its own camera, pyramids and map;
 * all share dpt_params and the HIP stream.  The per-stream results equal those of
 * dpt_track_frame on a single-stream context to rounding. */
typedef struct dpt_batch dpt_batch;

/* n_streams in 1..4096; cams[s] and max_points[s] (1..65536) per stream. */
int dpt_batch_create(int32_t n_streams, const dpt_camera* cams, const dpt_params* prm, const int32_t* max_points,
                     void* hip_stream, dpt_batch** out);
void dpt_batch_destroy(dpt_batch* b);

/* Build one slot's pyramid for every stream.  imgs[s]: stream s's image (device
 * memory if on_device, else host), row pitch pitches[s] >= its width. */
int dpt_batch_build_pyramids(dpt_batch* b, int32_t slot, const uint8_t* const* imgs, const int64_t* pitches,
                             int32_t on_device);

/* As dpt_select_points / dpt_set_reference_points, for stream `s`. */
int dpt_batch_select_points(dpt_batch* b, int32_t s, int32_t n, int32_t margin, int32_t* host_idx, int32_t* n_out);
int dpt_batch_set_reference_points(dpt_batch* b, int32_t s, const float* xyz_world, int32_t n, const double T_rw[16],
                                   int32_t xyz_on_device);

/* As dpt_set_reference_from_depth, for stream `s`. */
int dpt_batch_set_reference_from_depth(dpt_batch* b, int32_t s, int32_t n, int32_t margin, const float* depth,
                                       int64_t depth_pitch, int32_t depth_on_device, const double T_rw[16]);

/* As dpt_set_reference_from_depth for every stream at once, in one launch
 * sequence for the whole batch (selection, back-projection, IC precompute):
 * n_points[s] points on stream s, depths[s] its level-0 depth map in device
 * memory with rows of depth_pitches[s] floats, T_rw n_streams row-major 4x4. */
int dpt_batch_set_reference_from_depth_all(dpt_batch* b, const int32_t* n_points, int32_t margin,
                                           const float* const* depths, const int64_t* depth_pitches,
                                           const double* T_rw);

/* Copy pyramid level `level` of slot `slot` of every stream, packed, into dst:
 * stream s's level at dst + s * W_l * H_l (all streams must have the same
 * level size).  dst in device memory if dst_on_device, else host. */
int dpt_batch_get_level(dpt_batch* b, int32_t slot, int32_t level, uint8_t* dst, int32_t dst_on_device);

/* Track every stream's CUR pyramid.  T_cw_init: n_streams row-major 4x4
 * doubles; out: n_streams results.  Synchronises the stream. */
int dpt_batch_track(dpt_batch* b, const double* T_cw_init, dpt_result* out);

/* As dpt_set_reference_stream, for every stream of the batch: reference
 * updates (dpt_batch_build_pyramids with DPT_SLOT_REF, which starts one, the
 * per-stream and all-stream reference setters) run on hip_stream into the
 * banks the tracks in flight do not read; the next track orders the batch's
 * stream after the update.  NULL or the batch's stream: one stream again. */
int dpt_batch_set_reference_stream(dpt_batch* b, void* hip_stream);

/* As dpt_track_enqueue / dpt_synchronize / dpt_set_pose_history, for every
 * stream of the batch (T_cw_init: n_streams row-major 4x4 doubles, may be NULL
 * with DPT_INIT_CONST_VELOCITY or DPT_INIT_PROPOSED, the latter starting every
 * stream from the last dpt_cnn_propose_batch; out: n_streams results) or for
 * stream `s`. */
int dpt_batch_track_enqueue(dpt_batch* b, int32_t init_mode, const double* T_cw_init, dpt_result* out);
int dpt_batch_synchronize(dpt_batch* b);
/* As dpt_collect / dpt_tracks_in_flight: the oldest n batched tracks (each
 * n_streams results), and how many are in flight. */
int dpt_batch_collect(dpt_batch* b, int32_t n);
int dpt_batch_tracks_in_flight(dpt_batch* b);
int dpt_batch_set_pose_history(dpt_batch* b, int32_t s, const double T_older[16], const double T_newer[16]);
/* Pose histories of every stream at once (n_streams row-major 4x4 each), one launch. */
int dpt_batch_set_pose_history_all(dpt_batch* b, const double* T_older, const double* T_newer);

/* dpt_track_window_enqueue for every stream of the batch: stream s's frames at
 * frames[s] (pitches[s], frame_strides[s]), all streams n_frames frames, one
 * pyramid launch per 64 streams and one track launch per cooperative group.
 * Each stream advances through its window at its own pace: a stream that needs
 * more iterations on one frame does not hold the others back at every frame.
 * T_cw_init: n_streams row-major 4x4 (DPT_INIT_GIVEN) or NULL; out:
 * n_frames x n_streams results, frame-major (out[f * n_streams + s]). */
int dpt_batch_track_window_enqueue(dpt_batch* b, const uint8_t* const* frames, const int64_t* pitches,
                                   const int64_t* frame_strides, int32_t n_frames, int32_t frames_on_device,
                                   int32_t init_mode, const double* T_cw_init, dpt_result* out);

/* Launch configuration as dpt_set_launch_config, for the whole batch. */
int dpt_batch_set_launch_config(dpt_batch* b, int32_t mode, int32_t chunk);
/* Wait bound as dpt_set_spin_limit, for the whole batch. */
int dpt_batch_set_spin_limit(dpt_batch* b, int32_t polls);

/* Profiling as dpt_set_profiling / dpt_last_kernel_ms / dpt_get_profile: a
 * batched track launch sequence and a batched pyramid launch each count once. */
int dpt_batch_set_profiling(dpt_batch* b, int32_t enable);
int dpt_batch_last_kernel_ms(dpt_batch* b, float* pyramid_ms, float* track_ms);
int dpt_batch_get_profile(dpt_batch* b, double* pyramid_ms, int64_t* n_pyramid, double* track_ms, int64_t* n_track);

/* ------------------------------------------------------------------ learned initialiser
 * A small CNN proposes the reference-to-current twist from the coarsest pyramid
 * pair, as the start pose of the coarse-to-fine Gauss-Newton track (which the
 * paper starts from the previous estimate, Sec. III and Sec. IV-A).  Not in the
 * paper.  Input: the reference and current levels of size 94 x 60, (I - 128)/64.
 * Network: conv 3x3 stride 2 pad 1 + ReLU, 2-16-32-64-64 channels; global
 * average pool; FC 64-64 + ReLU; FC 64-6.  Output: the twist (omega, v) divided
 * by (5 deg x3, 0.1 m x3).  BF16 activations and conv weights, FP32 master
 * weights; the forward and backward convolutions run on the matrix cores
 * (MFMA, FP32 accumulation), the gradients between layers are BF16.
 * Parameters (dpt_cnn_num_params() floats) in tensor order w1 b1 w2 b2 w3 b3 w4
 * b4 fw1 fb1 fw2 fb2, conv weights [co][ci][ky][kx], FC weights [out][in]. */
typedef struct dpt_cnn dpt_cnn;

int32_t dpt_cnn_num_params(void);
/* max_batch: 1..65536 pairs per call.  Parameters start at zero: set them. */
int dpt_cnn_create(int32_t max_batch, void* hip_stream, dpt_cnn** out);
void dpt_cnn_destroy(dpt_cnn* c);
/* host FP32 parameter vectors; set also resets the Adam state */
int dpt_cnn_set_params(dpt_cnn* c, const float* params);
int dpt_cnn_get_params(dpt_cnn* c, float* params);
/* gradients of the last training step, same layout */
int dpt_cnn_get_grads(dpt_cnn* c, float* grads);
/* pairs: B x 2 x 60 x 94 uint8 (reference plane, then current), device memory
 * if on_device.  out_host: B x 6 normalised twists. */
int dpt_cnn_forward(dpt_cnn* c, const uint8_t* pairs, int32_t B, int32_t on_device, float* out_host);
/* One step: forward, mean squared error against targets (B x 6 normalised
 * twists, same memory side as pairs), backward, Adam (beta 0.9/0.999, eps 1e-8)
 * with learning rate lr (lr == 0: gradients only).  *loss_out: the loss. */
int dpt_cnn_train_step(dpt_cnn* c, const uint8_t* pairs, const float* targets, int32_t B, float lr,
                       int32_t on_device, float* loss_out);
/* Test hook: activation of layer l = 1..4 of the last forward (FP32, NHWC), or the
 * network outputs for l = 5. */
int dpt_cnn_get_activation(dpt_cnn* c, int32_t l, int32_t B, float* host_out);
/* Start poses from the network for a single-stream context / every stream of a
 * batch: the REF and CUR pyramids' level (levels-1) must be 94 x 60.  Writes
 * T_cw = exp(xi) T_rw (4x4 row-major doubles per stream). */
int dpt_cnn_predict(dpt_cnn* c, dpt_ctx* ctx, double T_cw_out[16]);
int dpt_cnn_predict_batch(dpt_cnn* c, dpt_batch* b, double* T_cw_out);
/* The same proposal without a host round trip: enqueued on the context's (the
 * batch's) stream, the forward pass on the coarsest REF and CUR levels and the
 * exponential of each twist (FP64), kept in device memory as the start of the
 * next dpt_track_enqueue / dpt_batch_track_enqueue with DPT_INIT_PROPOSED.  The
 * levels are read when the stream reaches the call, so a CUR pyramid built
 * before it on the same stream is the one proposed from.  The network's
 * buffers are used on that stream: the CNN must not run concurrently on
 * another one.  The first call on a context or batch allocates its proposal
 * buffer and uploads its level pointer table (a synchronous copy); later calls
 * neither allocate nor wait.  DPT_E_STATE if a pyramid or the reference is
 * missing, DPT_E_ARG if the coarsest level is not 94 x 60. */
int dpt_cnn_propose(dpt_cnn* c, dpt_ctx* ctx);
int dpt_cnn_propose_batch(dpt_cnn* c, dpt_batch* b);

/* ------------------------------------------------------------------ device characterisation
 * Attainable peaks for the roofline figures, measured on the current device
 * (not part of the method).  Each call allocates, runs two launches on the
 * null stream, times the second with events and frees; it synchronises.
 *
 * dpt_probe_read_bandwidth: 8 workgroups per compute unit, workgroup w reading
 * slice w % n_slices of a zeroed buffer of n_slices x slice_bytes bytes
 * (slice_bytes a positive multiple of 4096, the buffer at most 16 GiB) `reps`
 * times; *gbs = bytes read / time.  One 2 MiB slice stays in every XCD's L2
 * (the L2 read roof); one small slice per workgroup with a footprint between
 * the L2s and the last-level cache gives that cache's roof.
 * dpt_probe_fp32_fma: 8 workgroups per compute unit of 256 threads, each
 * thread 8 independent FP32 FMA chains of `iters` steps, compiled like the
 * library (no packed FP32); *tflops = 2 x FMAs / time.
 * DPT_E_ARG on bad sizes, DPT_E_OOM, DPT_E_HIP. */
int dpt_probe_read_bandwidth(int64_t slice_bytes, int32_t n_slices, int32_t reps, double* gbs);
int dpt_probe_fp32_fma(int32_t iters, double* tflops);

#ifdef __cplusplus
}
#endif

#endif /* DPTRACK_H */
