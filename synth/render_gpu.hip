// GPU port of the seeded 3-plane scene renderer (render.c), for generating
// large training sets for the learned initialiser.  Input generation only: the
// same texture model (3-D Gaussian blobs centred on the planes, truncated at
// 4 sigma and binned per plane, plus trilinear value noise from a splitmix64
// lattice hash), evaluated in FP64.  It is never used to produce the oracle's
// inputs or expected values.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

namespace {

constexpr double kCell = 0.25;
constexpr double kReach = 1.6;

struct Grid {
  double lo0, lo1, hi0, hi1;
  int n0, n1;
  const int* start;
  const int* items;
  const double* blobs;  // [n][4] amplitude, sigma, c0, c1
};

struct Scene3 {
  Grid g[3];
  uint64_t seed;
  double noise_amp, noise_cell;
};

__device__ __forceinline__ uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double lattice(uint64_t seed, int64_t ix, int64_t iy, int64_t iz) {
  uint64_t h = mix(seed ^ mix((uint64_t)ix ^ mix((uint64_t)iy ^ mix((uint64_t)iz))));
  return 2.0 * ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

__device__ __forceinline__ double smooth(double t) { return t * t * (3.0 - 2.0 * t); }

__device__ double vnoise(uint64_t seed, double x, double y, double z) {
  double f[3] = {floor(x), floor(y), floor(z)}, p[3] = {x, y, z}, t[3];
  int64_t i[3];
  for (int a = 0; a < 3; ++a) {
    i[a] = (int64_t)f[a];
    t[a] = smooth(p[a] - f[a]);
  }
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
    double w = (dx ? t[0] : 1 - t[0]) * (dy ? t[1] : 1 - t[1]) * (dz ? t[2] : 1 - t[2]);
    acc += w * lattice(seed, i[0] + dx, i[1] + dy, i[2] + dz);
  }
  return acc;
}

__device__ double texture(const Scene3& S, const double* h) {
  double f = 128.0;
  for (int q = 0; q < 3; ++q) {
    const Grid& g = S.g[q];
    double p0, p1, dp;
    if (q == 0) p0 = h[0], p1 = h[2], dp = fabs(h[1] + 1.0);
    else if (q == 1) p0 = h[0], p1 = h[1], dp = fabs(h[2] - 3.0);
    else p0 = h[2], p1 = h[1], dp = fabs(h[0] - 2.0);
    if (dp > kReach || !(p0 >= g.lo0 && p0 < g.hi0 && p1 >= g.lo1 && p1 < g.hi1)) continue;
    int q0 = (int)((p0 - g.lo0) / kCell), q1 = (int)((p1 - g.lo1) / kCell);
    q0 = q0 < g.n0 ? q0 : g.n0 - 1;
    q1 = q1 < g.n1 ? q1 : g.n1 - 1;
    const int c = q1 * g.n0 + q0;
    for (int e = g.start[c]; e < g.start[c + 1]; ++e) {
      const double* bl = g.blobs + 4 * g.items[e];
      const double d0 = p0 - bl[2], d1 = p1 - bl[3], s = bl[1];
      const double d2 = d0 * d0 + d1 * d1 + dp * dp;
      if (d2 <= 16.0 * s * s) f += bl[0] * exp(-d2 / (2.0 * s * s));
    }
  }
  return f + S.noise_amp * vnoise(S.seed, h[0] / S.noise_cell, h[1] / S.noise_cell, h[2] / S.noise_cell);
}

// blockIdx.z = view; poses [views][16] row-major world -> camera
__global__ void render_kernel(Scene3 S, int W, int H, double fx, double fy, double cx, double cy,
                              const double* __restrict__ poses, uint8_t* __restrict__ imgs,
                              float* __restrict__ depths) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y * blockDim.y + threadIdx.y;
  if (u >= W || v >= H) return;
  const double* T = poses + 16 * blockIdx.z;
  const double Rt[9] = {T[0], T[4], T[8], T[1], T[5], T[9], T[2], T[6], T[10]};
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = -(Rt[3 * a] * T[3] + Rt[3 * a + 1] * T[7] + Rt[3 * a + 2] * T[11]);
  const double rc[3] = {(u - cx) / fx, (v - cy) / fy, 1.0};
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = Rt[3 * a] * rc[0] + Rt[3 * a + 1] * rc[1] + Rt[3 * a + 2] * rc[2];
  double best = INFINITY;
  if (d[1] != 0.0) {
    double t = (-1.0 - o[1]) / d[1];
    if (t > 1e-9 && t < best) best = t;
  }
  if (d[2] != 0.0) {
    double t = (3.0 - o[2]) / d[2];
    if (t > 1e-9 && t < best) best = t;
  }
  if (d[0] != 0.0) {
    double t = (2.0 - o[0]) / d[0];
    if (t > 1e-9 && t < best) best = t;
  }
  const size_t pix = (size_t)blockIdx.z * W * H + (size_t)v * W + u;
  if (!(best < INFINITY)) {
    imgs[pix] = 0;
    if (depths) depths[pix] = 0.f;
    return;
  }
  const double h[3] = {o[0] + best * d[0], o[1] + best * d[1], o[2] + best * d[2]};
  double q = rint(texture(S, h));
  q = q < 0 ? 0 : (q > 255 ? 255 : q);
  imgs[pix] = (uint8_t)q;
  if (depths) depths[pix] = (float)best;
}

struct HostGrid {
  double lo0, lo1, hi0, hi1;
  int n0, n1;
  std::vector<int> start, items;
};

void build_grid(HostGrid& g, const double* blobs, int n, const double* win) {
  g.lo0 = win[0] - kReach, g.hi0 = win[1] + kReach, g.lo1 = win[2] - kReach, g.hi1 = win[3] + kReach;
  g.n0 = (int)ceil((g.hi0 - g.lo0) / kCell);
  g.n1 = (int)ceil((g.hi1 - g.lo1) / kCell);
  const int nc = g.n0 * g.n1;
  std::vector<int> count(nc, 0);
  g.start.assign(nc + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int c = 0; c < nc; ++c) g.start[c + 1] = g.start[c] + count[c];
      g.items.assign(g.start[nc] > 0 ? g.start[nc] : 1, 0);
      std::fill(count.begin(), count.end(), 0);
    }
    for (int j = 0; j < n; ++j) {
      double s = blobs[4 * j + 1], c0 = blobs[4 * j + 2], c1 = blobs[4 * j + 3];
      int a0 = (int)floor((c0 - 4 * s - g.lo0) / kCell), b0 = (int)floor((c0 + 4 * s - g.lo0) / kCell);
      int a1 = (int)floor((c1 - 4 * s - g.lo1) / kCell), b1 = (int)floor((c1 + 4 * s - g.lo1) / kCell);
      a0 = a0 < 0 ? 0 : a0, a1 = a1 < 0 ? 0 : a1;
      b0 = b0 >= g.n0 ? g.n0 - 1 : b0, b1 = b1 >= g.n1 ? g.n1 - 1 : b1;
      for (int q1 = a1; q1 <= b1; ++q1)
        for (int q0 = a0; q0 <= b0; ++q0) {
          int c = q1 * g.n0 + q0;
          if (pass == 1) g.items[g.start[c] + count[c]] = j;
          count[c]++;
        }
    }
  }
}

}  // namespace

extern "C" {

// Render `views` poses of one scene into device buffers imgs [views][H][W] and
// optionally depths (camera-frame z, FP32).  poses: host [views][16].
// Returns 0 or a hipError_t code.
int syn_gpu_render(int32_t W, int32_t H, double fx, double fy, double cx, double cy, const double* poses,
                   int32_t views, int32_t n_blobs, const double* blobs, const double* windows, uint64_t seed,
                   double noise_amp, double noise_cell, uint8_t* imgs_dev, float* depths_dev, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  HostGrid hg[3];
  Scene3 S;
  std::vector<void*> owned;
  auto up = [&](const void* src, size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    owned.push_back(p);
    if (hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return nullptr;
    return p;
  };
  int rc = 0;
  for (int q = 0; q < 3; ++q) {
    build_grid(hg[q], blobs + (size_t)q * n_blobs * 4, n_blobs, windows + 4 * q);
    Grid& g = S.g[q];
    g.lo0 = hg[q].lo0, g.lo1 = hg[q].lo1, g.hi0 = hg[q].hi0, g.hi1 = hg[q].hi1, g.n0 = hg[q].n0, g.n1 = hg[q].n1;
    g.start = (const int*)up(hg[q].start.data(), hg[q].start.size() * sizeof(int));
    g.items = (const int*)up(hg[q].items.data(), hg[q].items.size() * sizeof(int));
    g.blobs = (const double*)up(blobs + (size_t)q * n_blobs * 4, (size_t)n_blobs * 4 * sizeof(double));
    if (!g.start || !g.items || !g.blobs) rc = 1;
  }
  const double* dposes = (const double*)up(poses, (size_t)views * 16 * sizeof(double));
  if (!dposes) rc = 1;
  S.seed = seed, S.noise_amp = noise_amp, S.noise_cell = noise_cell;
  if (rc == 0) {
    dim3 blk(32, 8), grd((W + 31) / 32, (H + 7) / 8, views);
    hipLaunchKernelGGL(render_kernel, grd, blk, 0, s, S, W, H, fx, fy, cx, cy, dposes, imgs_dev, depths_dev);
    rc = (int)hipGetLastError();
  }
  if (hipStreamSynchronize(s) != hipSuccess && rc == 0) rc = 1;
  for (void* p : owned) (void)hipFree(p);
  return rc;
}

}  // extern "C"
