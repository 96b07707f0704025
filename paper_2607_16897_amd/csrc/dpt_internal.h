// Internal declarations shared by the device kernels and the C-ABI host code.
// Not part of the public ABI (see include/dptrack.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dptrack.h"

#include <algorithm>
#include <vector>

struct dpt_cnn;

namespace dpt {

constexpr int kMaxLevels = 8;
constexpr int kMaxPattern = 128;
constexpr int kTrackThreads = 512;   // one workgroup per tracked frame
constexpr int kRedSlots = 32;        // 21 H + 6 b + E + n + npts, padded to 32

// Upper-triangle order of H used in every reduction: (0,0) (0,1) .. (0,5) (1,1) .. (5,5).
// Slots: [0,21) H, [21,27) b, 27 cost E, 28 valid samples n, 29 valid points.
enum { kSlotB = 21, kSlotE = 27, kSlotN = 28, kSlotPts = 29 };

struct LevelGeom {
  int32_t W, H;
  int64_t off;  // byte offset of the level inside a packed pyramid
  float fx, fy, cx, cy;
};

struct Pattern {
  int32_t K;
  int32_t dx_min, dx_max, dy_min, dy_max;
  int8_t dx[kMaxPattern], dy[kMaxPattern];
};

// Fixed-H mode (Sec. IV-C, precompute and track): the inverse-compositional
// Gauss-Newton matrix of one level, H = sum over every reference-valid point and
// pattern sample of J J^T without weights, reduced once per reference, with its
// Cholesky factor.  The track then reduces only b and the cost.
struct FixedH {
  double H[21];    // upper triangle, tri() order
  float L[21];     // factor L(i, j), i >= j, stored at tri(j, i)
  float invd[6];   // 1 / L(j, j)
  int32_t bad;     // 1: a pivot <= 1e-6 of the largest diagonal entry (not positive definite)
  int32_t pad;
};
static_assert(sizeof(FixedH) % 16 == 0, "FixedH is copied as 16-byte words");

// Slots of the fixed-H reductions: [0,6) b, 6 cost E, 7 valid samples, 8 valid points.
constexpr int kFixSlots = 16;
enum { kFixB = 0, kFixE = 6, kFixN = 7, kFixPts = 8 };

// Reference-side IC cache: per level l, sample s = i*K + k lives at l*cap*K + s.
struct RefCache {
  const float4* x0;         // [cap] reference-camera points (w unused)
  const uint8_t* valid;     // [L][cap]
  const float* I0;          // [L][cap*K]
  const float* gx;          // [L][cap*K]
  const float* gy;          // [L][cap*K]
  const __half* I0h;        // mixed precision: [L][cap*K] template intensity - 128
  const __half2* gh;        // mixed precision: [L][cap*K] (gx, gy)
  const FixedH* fixed;      // fixed-H mode: [L]; null in the robust (IRLS) mode
  int32_t n, cap;
};

// What a track launch writes back (device), read by the host after the stream sync.
struct TrackOut {
  double Td[12];  // mixed precision: final relative pose in FP64
  float T[12];    // final relative pose reference -> current, 3x4 row-major
  float E, n;   // final cost pass: Huber cost sum and valid sample count
  int32_t iterations;
  int32_t iters_per_level[kMaxLevels];
  int32_t n_valid_points;
  int32_t status;
  uint32_t seq;  // written last, after a system-scope fence: the launch's sequence number + frame
  int64_t samples;
};

struct TrackArgs {
  const uint8_t* cur;  // current pyramid base
  const float* curf;   // floating-point Gaussian pyramid of the current frame (same offsets), or null
  LevelGeom lv[kMaxLevels];
  int32_t levels, max_iters, min_points;
  float huber_k, step_eps, z_min;
  Pattern pat;
  RefCache ref;
  float T_init[12];
  TrackOut* out;
  // normal-equation test hook: a single pass at `level` writing kRedSlots floats
  int32_t level;
  float* totals;
};

struct PyrGeom {
  int32_t levels;
  int32_t W[kMaxLevels], H[kMaxLevels];
  int64_t off[kMaxLevels];
};

// Whether the one-thread-per-block pyramid applies: 3 or 4 levels, level-0
// sizes multiples of the block (2^(levels-1)), 8-byte aligned source rows and
// destination.
inline bool pyramid_block_ok(const PyrGeom& g, const void* src, int64_t pitch, const void* dst) {
  if (g.levels != 3 && g.levels != 4) return false;
  const int B = 1 << (g.levels - 1);
  return g.W[0] % B == 0 && g.H[0] % B == 0 && pitch % 8 == 0 && (reinterpret_cast<uintptr_t>(src) & 7) == 0 &&
         (reinterpret_cast<uintptr_t>(dst) & 7) == 0;
}

struct PrecomputeArgs {
  const uint8_t* ref;  // reference pyramid base
  const float* reff;   // floating-point Gaussian pyramid of the reference (same offsets), or null
  LevelGeom lv[kMaxLevels];
  int32_t levels;
  float z_min;
  Pattern pat;
  const float* P;  // [n][3] world points
  float T_rw[12];
  float4* x0;
  uint8_t* valid;
  float *I0, *gx, *gy;
  __half* I0h;   // written when non-null (mixed precision)
  __half2* gh;
  FixedH* fixed;   // fixed-H mode: [L] per-level matrix and factor, else null
  float* hpart;    // fixed-H mode: [L][ceil(cap / 256)][21] per-workgroup partial sums
  int32_t n, cap;
};

// Point selection on one image (candidate c is pixel (m + c % Wc, m + c / Wc)).
struct SelGeom {
  const uint8_t* img;
  int32_t W, m, Wc, C, n;
  float inv_wc;  // 1 / Wc, for the candidate's row
  int32_t pitch, pad;  // bytes between image rows (>= W)
};

// One image's selection: geometry, its scratch (select_scratch_ints ints), the
// output indices and count, and its number of 4096-candidate chunks G.
struct SelJob {
  SelGeom g;
  int32_t* sc;
  int32_t* idx;
  int32_t* count;
  int32_t G, pad;
};

// Map points from selected level-0 pixels and a depth map (device memory).
struct BackprojectArgs {
  const int32_t* idx;    // [n] selected pixel indices y * W + x
  const int32_t* count;  // how many of them are valid selections
  const float* depth;    // level-0 depth in metres, row pitch `pitch` floats
  int64_t pitch;
  int32_t W, n;
  double fx, fy, cx, cy;
  double T_rw[12];       // reference camera <- world, row-major 3x4
  float* P;              // [n][3] world points out
};

// One stream of a cooperative track launch (device array, one entry per stream).
struct CoopStream {
  TrackArgs a;         // a.ref: the reference cache of bank 0
  RefCache ref_alt;    // bank 1 (a reference stream in use), read when the launch's start slot says so
  uint64_t* partials;  // [2][2][n_chunks][32] chunk sums (copy: L2, device scope; parity), word = (tag << 32) | float bits
  double* hist;        // the stream's last two poses T_cw, 2 x 3x4 row-major FP64 (device)
  const uint8_t* win;      // window tracking: the pyramids of consecutive frames, win_stride bytes apart
  const uint8_t* win_alt;  // bank 1's window pyramids, read with bank 1's reference
  int64_t win_stride;
  int32_t n_chunks;
  int32_t pad;
};

// Project the rotation of a row-major 3x4 pose back onto SO(3): two
// Newton-Schulz steps of the polar decomposition, R <- R (3I - R^T R) / 2, each
// squaring the deviation from orthonormality (FP32 updates and products of
// poses leave ~1e-7, which products would otherwise amplify frame by frame).
__host__ __device__ inline void orthonormalize34(double* T) {
  for (int it = 0; it < 2; ++it) {
    double M[9];  // 3I - R^T R
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double rr = T[i] * T[j] + T[4 + i] * T[4 + j] + T[8 + i] * T[8 + j];
        M[3 * i + j] = (i == j ? 3.0 : 0.0) - rr;
      }
    double R[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        R[3 * i + j] = 0.5 * (T[4 * i] * M[j] + T[4 * i + 1] * M[3 + j] + T[4 * i + 2] * M[6 + j]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[4 * i + j] = R[3 * i + j];
  }
}

// Per-launch, per-stream start of a cooperative track (host-mapped, 32 doubles).
struct StartSlot {
  double T_rel[12];  // given start pose relative to the reference (mode kStartGiven)
  double mode;       // kStartGiven, kStartConstVelocity (P1 P0^-1 P1 from the history) or kStartDevice
  // window tracks: level 0 of frame f read at l0 + f * l0_stride (rows W bytes
  // apart) instead of from the window pyramids, or l0 = null
  const uint8_t* l0;
  int64_t l0_stride;
  const double* dev_rel;  // kStartDevice: the start relative to the reference, 3x4 FP64 in device memory
  double T_rw[12];   // reference pose (world -> reference camera), 3x4
  int32_t bank;      // which reference bank of the stream the launch reads (0 or 1)
  int32_t pad2;
  double pad1[3];
};
static_assert(sizeof(StartSlot) == 256, "StartSlot layout");
constexpr int kStartGiven = 0, kStartConstVelocity = 1, kStartDevice = 2;
constexpr int kRing = DPT_MAX_IN_FLIGHT;  // tracks that may be in flight per context or batch

// One image of a batched pyramid launch.
struct PyrJob {
  const uint8_t* src;
  int64_t pitch;
  uint8_t* dst;
  PyrGeom g;
  int32_t vec4;   // width, pitch and addresses multiples of 4
  int32_t vec16;  // ... of 16 (pyramid_tile64v)
};

// Variants of the cooperative track kernel.
// Bits: kCoopMixed and kCoopFixedH as named; kCoopGeneric: any pattern K, four
// lanes per point, kGenericThreads-thread chunks of kGenericThreads / 4 points;
// kCoopFloatPyr (with kCoopGeneric): the floating-point Gaussian pyramid;
// kCoopPairs (8-pixel pattern): two threads per point, chunks of threads / 2 points.
enum { kCoopFP32 = 0, kCoopMixed = 1, kCoopFixedH = 2, kCoopGeneric = 4, kCoopFloatPyr = 8, kCoopPairs = 16 };
constexpr int kGenericThreads = 256;
constexpr int kLanesPerPoint = 4;

// Host-side owner of a cooperative track launch over n streams.  Start slots
// and results live in host-mapped pinned memory that the kernel reads and
// writes directly, in rings of kRing launches, so a launch needs no copy
// commands and up to kRing launches can be in flight.
struct CoopEngine {
  int n = 0, chunk = 256, ppc = 256, work_cap = 0;  // threads and points per chunk
  bool xcd_pack = true, dirty = true;
  hipStream_t stream = nullptr;
  std::vector<CoopStream> h_streams;
  std::vector<int> max_chunks;
  std::vector<int2> h_work;
  CoopStream* d_streams = nullptr;
  int2* d_work = nullptr;
  uint64_t* d_partials = nullptr;
  size_t partial_words = 0;
  uint32_t tag_base = 1;       // epoch tags of the next launch start here; 0 marks a cleared word
  uint32_t seq_next = 1;       // sequence number of the next launch's first frame (never 0)
  uint32_t slot_seq[kRing] = {};  // the sequence number each ring slot's results will carry
  StartSlot* h_start = nullptr;   // [kRing][n], host-mapped
  StartSlot* dv_start = nullptr;  // device view of h_start
  int variant = kCoopFP32;        // kernel variant (kCoop* bits)
  TrackOut* h_out = nullptr;      // [kRing][n] results, host-mapped
  TrackOut* dv_out = nullptr;     // device view of h_out
  hipError_t init(int n_streams, const int* max_points, int chunk, int ppc, bool xcd_pack, hipStream_t s);
  void release();
  // a.ref: the stream's reference bank 0, alt: bank 1 (the same as bank 0 without a reference stream)
  void set_stream(int k, const TrackArgs& a, const RefCache& alt, double* hist, const uint8_t* win,
                  const uint8_t* win_alt, int64_t win_stride);
  hipError_t upload();
  int grid() const;
  StartSlot* start(int slot) { return h_start + (size_t)slot * n; }
  TrackOut* out(int slot) { return h_out + (size_t)slot * n; }
  // Enqueue the track of every stream from start slot `slot`; its results land
  // in out(slot) once the stream reaches this point.  n_frames > 0: track that
  // many consecutive frames of each stream's window pyramids in one launch,
  // frame f's results in out((slot + f) % kRing).
  hipError_t launch(int spin_limit, int slot, int n_frames = 0);
  // Whether every stream's results in ring slot `slot` have arrived (non-blocking).
  bool done(int slot) const;
  hipError_t clear_partials();
  ~CoopEngine() { release(); }
};

// Cycle split of the cooperative track, in builds compiled with
// -DDPT_CYCLE_PROFILE only: per grid slot, summed over every iteration of
// every launch since the last reset, the cycles thread 0 of the workgroup spends
// in each phase of a Gauss-Newton iteration (DPT_CYCLE_* in dptrack.h).
#ifdef DPT_CYCLE_PROFILE
constexpr bool kCycleProfile = true;
#else
constexpr bool kCycleProfile = false;
#endif
constexpr int kCycleSlots = 1024;
hipError_t read_cycle_profile(uint64_t* host, int n_slots, bool reset);  // hipErrorNotSupported without the flag

constexpr int kStatusTimeout = DPT_TRACK_TIMEOUT;  // a cooperative wait gave up (dpt_result.status)
constexpr int kSpinLimit = DPT_DEFAULT_SPIN_LIMIT;  // polls (one round trip to memory each) before a chunk reports a timeout

// Record an error message for dpt_last_error() and return `code`.
int set_error(int code, const char* msg);

// Learned initialiser forward pass on coarsest-level pairs (device pointers).
int cnn_forward_levels(struct ::dpt_cnn* c, const uint8_t* const* refs, const uint8_t* const* curs, int B,
                       float* out_host);
// The same forward pass enqueued on stream s without a host wait: d_lv is a
// device array of B reference then B current level pointers; each pair's
// proposal exp(xi) (the relative start pose, 3x4 FP64) goes to rel + 12 b.
int cnn_propose(struct ::dpt_cnn* c, const uint8_t* const* d_lv, int B, hipStream_t s, double* rel);

// Launchers (kernels.hip, coop.hip).  Each returns the hipError_t of the launch.
hipError_t launch_pyramid(const uint8_t* src, int64_t pitch, uint8_t* dst, const PyrGeom& g, hipStream_t s);
// Floating-point Gaussian pyramid of a uint8 frame (levels at the offsets of g, in floats).
hipError_t launch_pyramid_gauss(const uint8_t* src, int64_t pitch, float* dst, const PyrGeom& g, hipStream_t s);
// Point selection; `scratch` holds select_scratch_ints(W, H) ints of device memory.
int64_t select_scratch_ints(int32_t W, int32_t H);
hipError_t launch_select(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                         int32_t* count, int32_t* scratch, hipStream_t s);
SelJob make_sel_job(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                    int32_t* count, int32_t* scratch);
// Selections of n_img images in one launch sequence; d_jobs in device memory,
// G_max = the largest chunk count among them, any_empty: one has none.  The
// scratch of every image must start zeroed (a fresh one: hipMemset).
hipError_t launch_select_batch(const SelJob* d_jobs, int n_img, int G_max, bool any_empty, hipStream_t s);
// The selection of one device image with its scratch in the library's static
// device array (nothing allocated): images of at most kNoAllocSelectPixels.
constexpr int64_t kNoAllocSelectPixels = 4096 * 4096;
hipError_t launch_select_noalloc(const uint8_t* img, int32_t W, int32_t H, int64_t pitch, int32_t margin, int32_t n,
                                 int32_t* idx, int32_t* count, hipStream_t s);
hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t s);
hipError_t launch_backproject(const BackprojectArgs& a, hipStream_t s);
// Batched forms: one launch over n references / maps (argument arrays in device memory).
hipError_t launch_precompute_batch(const PrecomputeArgs* d_args, int n_ref, int max_samples, int max_levels,
                                   hipStream_t s);
hipError_t launch_backproject_batch(const BackprojectArgs* d_args, int n_maps, int max_n, hipStream_t s);
// Fixed-H mode: per-level H and its factor from a finished precompute (a.fixed, a.hpart set).
hipError_t launch_fixed_h(const PrecomputeArgs& a, hipStream_t s);
hipError_t launch_fixed_h_batch(const PrecomputeArgs* d_args, int n_ref, int max_n, int max_levels, hipStream_t s);
hipError_t launch_track(const TrackArgs& a, hipStream_t s);
// One workgroup per frame; batch[b] describes frame b (device memory).
hipError_t launch_track_batch(const TrackArgs& any, const TrackArgs* batch, int n_frames, int lds_bytes,
                              int max_points, hipStream_t s);
int track_lds_bytes(const LevelGeom* lv, int levels, int pixel_bytes);  // pixel_bytes: 1 uint8, 4 float
hipError_t launch_normal_equations(const TrackArgs& a, hipStream_t s);
// start: the start slots of `slot` (one per stream); out_ring: the kRing x n_out
// result ring (frame f of the launch writes slot (slot + f) % kRing);
// n_frames = 0: one frame from each stream's current pyramid (a.cur / a.curf),
// n_frames > 0: that many frames from the streams' window pyramids.
hipError_t launch_coop_track(const CoopStream* d_streams, const int2* d_work, int n_work, const StartSlot* start,
                             TrackOut* out_ring, int slot, int n_out, int n_frames, uint32_t seq0, uint32_t tag_base,
                             int chunk, int variant, int spin_limit, hipStream_t s);
// Set a pose history (two row-major 4x4 T_cw) on the stream.
hipError_t launch_set_history(double* hist, const double* T0, const double* T1, hipStream_t s);
// Pose histories of n streams: d_vals[24 s ..] = (older, newer) 3x4 into d_hists[s] (device arrays).
hipError_t launch_set_history_batch(double* const* d_hists, const double* d_vals, int n, hipStream_t s);
int coop_max_blocks(int chunk);  // co-resident workgroups of a cooperative launch (0 if unsupported)
hipError_t launch_pyramid_batch(const PyrJob* d_jobs, int n_jobs, int max_w, int max_h, int levels, hipStream_t s);
// Up to kPyrArgJobs images whose sources travel in the kernel arguments; the
// device table holds each job's destination and geometry (src, pitch unused).
constexpr int kPyrArgJobs = 64;
struct PyrSrcArgs {
  const uint8_t* src[kPyrArgJobs];
  int64_t pitch[kPyrArgJobs];
};
// block: every image passes pyramid_block_ok (3 or 4 levels, sizes multiples
// of the block, 8-byte aligned rows): one thread per block of level 0.
hipError_t launch_pyramid_batch_args(const PyrJob* d_static, const PyrSrcArgs& srcs, int n_jobs, int max_w,
                                     int max_h, int levels, bool block, hipStream_t s);
// Window tracking: the box pyramids of n_frames consecutive frames of up to
// kPyrArgJobs streams in one launch.  Frame f of stream s is read from
// src[s] + f * stride[s] (rows pitch[s] apart) and its pyramid written to
// jobs[s].dst + f * jobs[s].dst_stride.
struct WinJob {
  uint8_t* dst;
  int64_t dst_stride;
  PyrGeom g;
};
struct PyrWinSrc {
  const uint8_t* src[kPyrArgJobs];
  int64_t pitch[kPyrArgJobs];
  int64_t stride[kPyrArgJobs];
  int32_t write_l0[kPyrArgJobs];  // 0: the track reads level 0 from the source frames
};
hipError_t launch_pyramid_window(const WinJob* d_jobs, const PyrWinSrc& srcs, int n_streams, int n_frames, int max_w,
                                 int max_h, int levels, bool block, hipStream_t s);

}  // namespace dpt
