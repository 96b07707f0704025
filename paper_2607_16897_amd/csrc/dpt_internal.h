// Internal declarations shared by the device kernels and the C-ABI host code.
// Not part of the public ABI (see include/dptrack.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpt {

constexpr int kMaxLevels = 8;
constexpr int kMaxPattern = 128;
constexpr int kTrackThreads = 1024;  // one workgroup per tracked frame
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

// Reference-side IC cache: per level l, sample s = i*K + k lives at l*cap*K + s.
struct RefCache {
  const float* x0;          // [cap][3] reference-camera points
  const uint8_t* valid;     // [L][cap]
  const float* I0;          // [L][cap*K]
  const float* gx;          // [L][cap*K]
  const float* gy;          // [L][cap*K]
  int32_t n, cap;
};

// What a track launch writes back (device), read by the host after the stream sync.
struct TrackOut {
  float T[12];  // final relative pose reference -> current, 3x4 row-major
  float E, n;   // final cost pass: Huber cost sum and valid sample count
  int32_t iterations;
  int32_t iters_per_level[kMaxLevels];
  int32_t n_valid_points;
  int32_t status;
  int32_t pad;
  int64_t samples;
};

struct TrackArgs {
  const uint8_t* cur;  // current pyramid base
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

struct PrecomputeArgs {
  const uint8_t* ref;  // reference pyramid base
  LevelGeom lv[kMaxLevels];
  int32_t levels;
  float z_min;
  Pattern pat;
  const float* P;  // [n][3] world points
  float T_rw[12];
  float* x0;
  uint8_t* valid;
  float *I0, *gx, *gy;
  int32_t n, cap;
};

// Launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_pyramid(const uint8_t* src, int64_t pitch, uint8_t* dst, const PyrGeom& g, hipStream_t s);
hipError_t launch_select(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                         int32_t* count, hipStream_t s);
hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t s);
hipError_t launch_track(const TrackArgs& a, hipStream_t s);
hipError_t launch_normal_equations(const TrackArgs& a, hipStream_t s);

}  // namespace dpt
