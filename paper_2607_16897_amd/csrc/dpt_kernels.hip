// gfx950 kernels of the direct photometric tracker: pyramid, map-point
// selection, inverse-compositional precompute and the Gauss-Newton track.
//
// Built with -ffp-contract=off: every fused multiply-add is written out as
// fmaf, so that the reference precompute and the track evaluate the projection
// and the bilinear sample with identical arithmetic (an identical frame at the
// reference pose then gives residuals of exactly zero).
#include "dpt_internal.h"

namespace dpt {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void transform(const float* T, float X, float Y, float Z, float& x, float& y,
                                          float& z) {
  x = fmaf(T[0], X, fmaf(T[1], Y, fmaf(T[2], Z, T[3])));
  y = fmaf(T[4], X, fmaf(T[5], Y, fmaf(T[6], Z, T[7])));
  z = fmaf(T[8], X, fmaf(T[9], Y, fmaf(T[10], Z, T[11])));
}

// Eq.(1): pinhole projection at one pyramid level.
__device__ __forceinline__ void project(const LevelGeom& g, float x, float y, float z, float& u, float& v) {
  u = fmaf(g.fx, x / z, g.cx);
  v = fmaf(g.fy, y / z, g.cy);
}

// A point is usable when it is in front of the camera and every pattern
// position p satisfies 1 <= p.x < W-2 and 1 <= p.y < H-2 (the bilinear taps and
// their central differences stay inside the level).
__device__ __forceinline__ bool inside(const LevelGeom& g, const Pattern& p, float u, float v) {
  return (u + (float)p.dx_min >= 1.0f) && (u + (float)p.dx_max < (float)(g.W - 2)) &&
         (v + (float)p.dy_min >= 1.0f) && (v + (float)p.dy_max < (float)(g.H - 2));
}

// Bilinear intensity of a uint8 level, pixel centres at integer coordinates.
__device__ __forceinline__ float bilinear(const uint8_t* img, int W, float x, float y) {
  float fx = floorf(x), fy = floorf(y);
  float a = x - fx, c = y - fy;
  const uint8_t* p = img + (int)fy * W + (int)fx;
  float p00 = p[0], p10 = p[1], p01 = p[W], p11 = p[W + 1];
  float top = fmaf(a, p10 - p00, p00);
  float bot = fmaf(a, p11 - p01, p01);
  return fmaf(c, bot - top, top);
}

// Reference-side gradient: central differences / 2 at the four bilinear taps,
// blended with the same bilinear weights.
__device__ __forceinline__ void gradient(const uint8_t* img, int W, float x, float y, float& gx, float& gy) {
  float fx = floorf(x), fy = floorf(y);
  float a = x - fx, c = y - fy;
  const uint8_t* p = img + (int)fy * W + (int)fx;
  float gx00 = 0.5f * ((float)p[1] - (float)p[-1]);
  float gx10 = 0.5f * ((float)p[2] - (float)p[0]);
  float gx01 = 0.5f * ((float)p[W + 1] - (float)p[W - 1]);
  float gx11 = 0.5f * ((float)p[W + 2] - (float)p[W]);
  float gy00 = 0.5f * ((float)p[W] - (float)p[-W]);
  float gy10 = 0.5f * ((float)p[W + 1] - (float)p[1 - W]);
  float gy01 = 0.5f * ((float)p[2 * W] - (float)p[0]);
  float gy11 = 0.5f * ((float)p[2 * W + 1] - (float)p[1]);
  float tx = fmaf(a, gx10 - gx00, gx00), bx = fmaf(a, gx11 - gx01, gx01);
  float ty = fmaf(a, gy10 - gy00, gy00), by = fmaf(a, gy11 - gy01, gy01);
  gx = fmaf(c, bx - tx, tx);
  gy = fmaf(c, by - ty, ty);
}

// ---------------------------------------------------------------- pyramid

// One launch builds every level.  A workgroup owns a TILE x TILE block of
// level 0 (TILE >= 2^(levels-1)), so each level's 2x2 parents stay inside the
// tile; levels alternate between two LDS buffers.
template <int TILE>
__global__ __launch_bounds__(256) void pyramid_kernel(const uint8_t* __restrict__ src, int64_t pitch,
                                                      uint8_t* __restrict__ dst, PyrGeom g, int vec4) {
  __shared__ uint8_t buf0[TILE * TILE];
  __shared__ uint8_t buf1[TILE * TILE / 4];
  const int ox = blockIdx.x * TILE, oy = blockIdx.y * TILE;
  const int W0 = g.W[0], H0 = g.H[0];
  if (vec4) {
    // 4-byte loads: width, pitch and base are multiples of 4
    for (int q = threadIdx.x; q < TILE * TILE / 4; q += blockDim.x) {
      int ly = q / (TILE / 4), lx = (q % (TILE / 4)) * 4;
      int gx = ox + lx, gy = oy + ly;
      uint32_t v = 0;
      if (gy < H0 && gx < W0) {
        v = *reinterpret_cast<const uint32_t*>(src + gy * pitch + gx);
        *reinterpret_cast<uint32_t*>(dst + g.off[0] + (int64_t)gy * W0 + gx) = v;
      }
      *reinterpret_cast<uint32_t*>(buf0 + ly * TILE + lx) = v;
    }
  } else {
    for (int q = threadIdx.x; q < TILE * TILE; q += blockDim.x) {
      int ly = q / TILE, lx = q % TILE;
      int gx = ox + lx, gy = oy + ly;
      uint8_t v = 0;
      if (gy < H0 && gx < W0) {
        v = src[gy * pitch + gx];
        dst[g.off[0] + (int64_t)gy * W0 + gx] = v;
      }
      buf0[q] = v;
    }
  }
  __syncthreads();
  uint8_t* prev = buf0;
  uint8_t* next = buf1;
  for (int l = 1; l < g.levels; ++l) {
    const int T = TILE >> l, Tp = TILE >> (l - 1);
    const int Wl = g.W[l], Hl = g.H[l];
    const int oxl = ox >> l, oyl = oy >> l;
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
      int ly = q / T, lx = q % T;
      int gx = oxl + lx, gy = oyl + ly;
      uint8_t v = 0;
      if (gx < Wl && gy < Hl) {
        const uint8_t* p = prev + (2 * ly) * Tp + 2 * lx;
        int s = (int)p[0] + (int)p[1] + (int)p[Tp] + (int)p[Tp + 1];
        v = (uint8_t)((s + 2) >> 2);
        dst[g.off[l] + (int64_t)gy * Wl + gx] = v;
      }
      next[q] = v;
    }
    __syncthreads();
    uint8_t* t = prev;
    prev = next;
    next = t;
  }
}

hipError_t launch_pyramid(const uint8_t* src, int64_t pitch, uint8_t* dst, const PyrGeom& g, hipStream_t s) {
  int vec4 = ((pitch % 4) == 0 && (reinterpret_cast<uintptr_t>(src) % 4) == 0 && (g.W[0] % 4) == 0 &&
              (reinterpret_cast<uintptr_t>(dst) % 4) == 0)
                 ? 1
                 : 0;
  if (g.levels <= 6) {
    dim3 grid((g.W[0] + 31) / 32, (g.H[0] + 31) / 32);
    hipLaunchKernelGGL(pyramid_kernel<32>, grid, dim3(256), 0, s, src, pitch, dst, g, vec4);
  } else if (g.levels == 7) {
    dim3 grid((g.W[0] + 63) / 64, (g.H[0] + 63) / 64);
    hipLaunchKernelGGL(pyramid_kernel<64>, grid, dim3(256), 0, s, src, pitch, dst, g, vec4);
  } else {
    dim3 grid((g.W[0] + 127) / 128, (g.H[0] + 127) / 128);
    hipLaunchKernelGGL(pyramid_kernel<128>, grid, dim3(256), 0, s, src, pitch, dst, g, vec4);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- block scans / reductions

// Exclusive prefix sum of one int per thread over a 1024-thread workgroup.
// `wsum` is 16 ints of LDS.  Returns the prefix; *total gets the block sum.
__device__ __forceinline__ int block_exclusive_scan(int x, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    int v = wsum[w];
    base += (w < wave) ? v : 0;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

// Sum 32 per-lane values over a wave64 by recursive halving: at each xor step
// a lane keeps half of its values and receives the partner's matching half, so
// 16 + 8 + 4 + 2 + 1 + 1 shuffles replace 32 x 6.  Lane l ends up holding the
// wave total of value (l >> 1).  The order of additions is fixed.
__device__ __forceinline__ float wave_reduce32(float (&a)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int step = 0; step < 5; ++step) {
    const int half = 16 >> step;        // values kept after this step
    const int mask = 32 >> step;        // partner lane distance
    const bool upper = (lane & mask) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      float keep = upper ? a[j + half] : a[j];
      float send = upper ? a[j] : a[j + half];
      float recv = __shfl_xor(send, mask, 64);
      a[j] = keep + recv;
    }
  }
  float v = a[0];
  v += __shfl_xor(v, 1, 64);
  return v;
}

// Workgroup total of 32 per-lane values into out[32] (LDS), fixed order.
// `scratch` is 16 x 32 floats of LDS.
__device__ __forceinline__ void block_reduce32(float (&a)[32], float* scratch, float* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  float v = wave_reduce32(a);
  if ((lane & 1) == 0) scratch[wave * 32 + (lane >> 1)] = v;
  __syncthreads();
  if (threadIdx.x < 32) {
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += scratch[w * 32 + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- point selection

__device__ __forceinline__ int sel_score(const uint8_t* img, int W, int x, int y) {
  const uint8_t* p = img + y * W + x;
  int dx = (int)p[1] - (int)p[-1];
  int dy = (int)p[W] - (int)p[-W];
  return dx * dx + dy * dy;
}

// Top-n candidates by (score desc, index asc), written in ascending index order.
// One 1024-thread workgroup: a 256-bin histogram of score >> 9 finds the coarse
// bucket of the n-th score, a 512-bin histogram of its low bits the exact
// threshold; an ordered compaction then keeps every score above the threshold
// and the first `need` ties in index order.  Scores are at most 2 * 255^2.
constexpr int kSelPPT = 8;

__global__ __launch_bounds__(1024) void select_kernel(const uint8_t* __restrict__ img, int W, int H, int m, int n,
                                                      int32_t* __restrict__ idx, int32_t* __restrict__ count) {
  __shared__ int hist[512];
  __shared__ int wsum[16];
  __shared__ int sh_T, sh_need;
  const int Wc = W - 2 * m, Hc = H - 2 * m;
  const int C = (Wc > 0 && Hc > 0) ? Wc * Hc : 0;
  const int tid = threadIdx.x;
  if (C <= n) {
    if (tid == 0) {
      sh_T = -1;
      sh_need = 0;
    }
  } else {
    for (int b = tid; b < 512; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int c = tid; c < C; c += blockDim.x) {
      int y = m + c / Wc, x = m + c % Wc;
      atomicAdd(&hist[sel_score(img, W, x, y) >> 9], 1);
    }
    __syncthreads();
    __shared__ int sh_B, sh_cum;
    if (tid == 0) {
      int cum = 0, B = 0;
      for (int b = 255; b >= 0; --b) {
        if (cum + hist[b] >= n) {
          B = b;
          break;
        }
        cum += hist[b];
      }
      sh_B = B;
      sh_cum = cum;
    }
    __syncthreads();
    for (int b = tid; b < 512; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const int B = sh_B;
    for (int c = tid; c < C; c += blockDim.x) {
      int y = m + c / Wc, x = m + c % Wc;
      int s = sel_score(img, W, x, y);
      if ((s >> 9) == B) atomicAdd(&hist[s & 511], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int cum = sh_cum, T = B * 512, need = 0;
      for (int f = 511; f >= 0; --f) {
        if (cum + hist[f] >= n) {
          T = B * 512 + f;
          need = n - cum;
          break;
        }
        cum += hist[f];
      }
      sh_T = T;
      sh_need = need;
    }
  }
  __syncthreads();
  const int T = sh_T, need = sh_need;
  int tie_base = 0, out_base = 0;
  for (int base = 0; base < C; base += blockDim.x * kSelPPT) {
    int c0 = base + tid * kSelPPT;
    int sc[kSelPPT];
    int eq_local = 0;
#pragma unroll
    for (int j = 0; j < kSelPPT; ++j) {
      int c = c0 + j;
      sc[j] = -2;
      if (c < C) {
        int y = m + c / Wc, x = m + c % Wc;
        sc[j] = sel_score(img, W, x, y);
      }
      eq_local += (sc[j] == T) ? 1 : 0;
    }
    int eq_total;
    int eq_prefix = block_exclusive_scan(eq_local, wsum, &eq_total) + tie_base;
    bool sel[kSelPPT];
    int sel_local = 0;
#pragma unroll
    for (int j = 0; j < kSelPPT; ++j) {
      bool is_eq = sc[j] == T;
      sel[j] = (sc[j] > T) || (is_eq && eq_prefix < need);
      eq_prefix += is_eq ? 1 : 0;
      sel_local += sel[j] ? 1 : 0;
    }
    int sel_total;
    int pos = block_exclusive_scan(sel_local, wsum, &sel_total) + out_base;
#pragma unroll
    for (int j = 0; j < kSelPPT; ++j) {
      if (sel[j]) {
        int c = c0 + j;
        idx[pos++] = (m + c / Wc) * W + (m + c % Wc);
      }
    }
    tie_base += eq_total;
    out_base += sel_total;
  }
  if (tid == 0) *count = out_base;
}

hipError_t launch_select(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                         int32_t* count, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(1024), 0, s, img, W, H, margin, n, idx, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- IC precompute (Eq.(6))

// One lane per (point, pattern sample) and level: x0 = T_rw P, the point's
// reference validity, the bilinear template intensity I0 and the interpolated
// central-difference gradient.  The Jacobian itself is rebuilt in the track
// from (gx, gy) and x0, so the cache holds 12 bytes per sample.
__global__ __launch_bounds__(256) void precompute_kernel(PrecomputeArgs a) {
  const int K = a.pat.K;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (s >= a.n * K) return;
  const int i = s / K, k = s - i * K;
  float X, Y, Z;
  transform(a.T_rw, a.P[3 * i], a.P[3 * i + 1], a.P[3 * i + 2], X, Y, Z);
  if (l == 0 && k == 0) {
    a.x0[3 * i] = X;
    a.x0[3 * i + 1] = Y;
    a.x0[3 * i + 2] = Z;
  }
  const LevelGeom g = a.lv[l];
  bool ok = Z > a.z_min;
  float u = 0.f, v = 0.f;
  if (ok) {
    project(g, X, Y, Z, u, v);
    ok = inside(g, a.pat, u, v);
  }
  if (k == 0) a.valid[(int64_t)l * a.cap + i] = ok ? 1 : 0;
  float I0 = 0.f, gx = 0.f, gy = 0.f;
  if (ok) {
    const uint8_t* img = a.ref + g.off;
    float px = u + (float)a.pat.dx[k], py = v + (float)a.pat.dy[k];
    I0 = bilinear(img, g.W, px, py);
    gradient(img, g.W, px, py, gx, gy);
  }
  const int64_t o = (int64_t)l * a.cap * K + s;
  a.I0[o] = I0;
  a.gx[o] = gx;
  a.gy[o] = gy;
}

hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  dim3 grid((a.n * a.pat.K + 255) / 256, a.levels);
  hipLaunchKernelGGL(precompute_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- track

// Accumulate this thread's share of one normal-equation pass (Eq.(2), Eq.(5))
// at level l and relative pose T: residual against the cached template, Huber
// weight, IC Jacobian rebuilt from the cached gradient and x0, and the
// 21 + 6 + 3 running sums.  Lane <-> sample s = i*K + k.
template <int KT, bool COST_ONLY>
__device__ __forceinline__ void accumulate(const TrackArgs& a, const Pattern& pat, int l, const float* T,
                                           float (&acc)[32]) {
  const int K = KT ? KT : pat.K;
  const LevelGeom g = a.lv[l];
  const uint8_t* img = a.cur + g.off;
  const int64_t lo = (int64_t)l * a.ref.cap;
  const float* I0 = a.ref.I0 + lo * K;
  const float* GX = a.ref.gx + lo * K;
  const float* GY = a.ref.gy + lo * K;
  const uint8_t* valid = a.ref.valid + lo;
  const float kH = a.huber_k;
  const int nK = a.ref.n * K;
  for (int s = threadIdx.x; s < nK; s += blockDim.x) {
    const int i = s / K, k = s - i * K;
    if (!valid[i]) continue;
    const float X0 = a.ref.x0[3 * i], Y0 = a.ref.x0[3 * i + 1], Z0 = a.ref.x0[3 * i + 2];
    float X, Y, Z;
    transform(T, X0, Y0, Z0, X, Y, Z);
    if (!(Z > a.z_min)) continue;
    float u, v;
    project(g, X, Y, Z, u, v);
    if (!inside(g, pat, u, v)) continue;
    const float Ic = bilinear(img, g.W, u + (float)pat.dx[k], v + (float)pat.dy[k]);
    const float r = I0[s] - Ic;
    const float ar = fabsf(r);
    float w, rho;
    if (kH > 0.f && ar > kH) {
      w = kH / ar;
      rho = kH * (ar - 0.5f * kH);
    } else {
      w = 1.0f;
      rho = 0.5f * r * r;
    }
    acc[kSlotE] += rho;
    acc[kSlotN] += 1.0f;
    if (k == 0) acc[kSlotPts] += 1.0f;
    if (COST_ONLY) continue;
    // J = (gx, gy) * Jw(x0): columns (w1 w2 w3 v1 v2 v3) of a left perturbation
    const float iz = 1.0f / Z0, xp = X0 * iz, yp = Y0 * iz;
    const float gxf = GX[s] * g.fx, gyf = GY[s] * g.fy;
    float J[6];
    J[0] = -fmaf(gxf * xp, yp, fmaf(gyf, yp * yp, gyf));
    J[1] = fmaf(gxf, xp * xp, fmaf(gyf * xp, yp, gxf));
    J[2] = fmaf(gyf, xp, -gxf * yp);
    J[3] = gxf * iz;
    J[4] = gyf * iz;
    J[5] = -fmaf(gxf, xp, gyf * yp) * iz;
    int q = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const float wj = w * J[p];
#pragma unroll
      for (int c = p; c < 6; ++c) {
        acc[q] = fmaf(wj, J[c], acc[q]);
        ++q;
      }
      acc[kSlotB + p] = fmaf(-wj, r, acc[kSlotB + p]);
    }
  }
}

// Index of H(i, j), i <= j, in the row-major upper-triangle order of the sums.
__host__ __device__ constexpr int tri(int i, int j) { return i * 6 - (i * (i - 1)) / 2 + (j - i); }

// Solve H delta = b (6x6 SPD from the 21 upper-triangle sums) by Cholesky in
// FP32 and apply T <- T exp(-delta).  Returns 0, or 1 if a pivot is <= 1e-6 of
// the largest diagonal entry (not positive definite).  Every loop is unrolled
// so the factor lives in registers.
__device__ __forceinline__ int solve_update(const float* tot, float* T, float* max_step) {
  float L[21];  // L(i, j), i >= j, stored at tri(j, i)
  float dmax = 0.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) dmax = fmaxf(dmax, tot[tri(j, j)]);
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    float s = tot[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s = fmaf(-L[tri(k, j)], L[tri(k, j)], s);
    bad |= !(s > 1e-6f * dmax);
    s = fmaxf(s, 1e-30f);
    const float d = sqrtf(s);
    L[tri(j, j)] = d;
    const float inv = 1.0f / d;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      float t = tot[tri(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fmaf(-L[tri(k, i)], L[tri(k, j)], t);
      L[tri(j, i)] = t * inv;
    }
  }
  if (bad) return 1;
  float y[6], d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float s = tot[kSlotB + i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fmaf(-L[tri(k, i)], y[k], s);
    y[i] = s / L[tri(i, i)];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    float s = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s = fmaf(-L[tri(i, k)], d[k], s);
    d[i] = s / L[tri(i, i)];
  }
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) m = fmaxf(m, fabsf(d[j]));
  *max_step = m;
  // exp(xi), xi = -delta = (w, v): R = I + A[w] + B[w]^2, t = (I + B[w] + C[w]^2) v
  const float w0 = -d[0], w1 = -d[1], w2 = -d[2];
  const float vv[3] = {-d[3], -d[4], -d[5]};
  const float th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrtf(th2);
  float A, B, C;
  if (th < 0.05f) {
    A = 1.0f - th2 * (1.0f / 6.0f) * (1.0f - th2 * (1.0f / 20.0f));
    B = 0.5f - th2 * (1.0f / 24.0f) * (1.0f - th2 * (1.0f / 30.0f));
    C = (1.0f / 6.0f) - th2 * (1.0f / 120.0f) * (1.0f - th2 * (1.0f / 42.0f));
  } else {
    const float sn = sinf(th), sh = sinf(0.5f * th);
    A = sn / th;
    B = 2.0f * sh * sh / th2;
    C = (th - sn) / (th2 * th);
  }
  const float W[3][3] = {{0.f, -w2, w1}, {w2, 0.f, -w0}, {-w1, w0, 0.f}};
  float E[3][4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float tv = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float W2 = W[r][0] * W[0][c] + W[r][1] * W[1][c] + W[r][2] * W[2][c];
      const float id = (r == c) ? 1.0f : 0.0f;
      E[r][c] = id + A * W[r][c] + B * W2;
      tv += (id + B * W[r][c] + C * W2) * vv[c];
    }
    E[r][3] = tv;
  }
  float N[12];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      N[4 * r + c] = fmaf(T[4 * r], E[0][c], fmaf(T[4 * r + 1], E[1][c], T[4 * r + 2] * E[2][c]));
    N[4 * r + 3] = fmaf(T[4 * r], E[0][3], fmaf(T[4 * r + 1], E[1][3], fmaf(T[4 * r + 2], E[2][3], T[4 * r + 3])));
  }
#pragma unroll
  for (int j = 0; j < 12; ++j) T[j] = N[j];
  return 0;
}

// Whole coarse-to-fine track of one frame in one 1024-thread workgroup: the
// Gauss-Newton loop needs only workgroup barriers, the 32 sums are reduced in
// a fixed order (bitwise reproducible), and thread 0 solves and updates.
template <int KT>
__global__ __launch_bounds__(kTrackThreads) void track_kernel(TrackArgs a) {
  __shared__ float sh_T[12];
  __shared__ float sh_tot[32];
  __shared__ float sh_red[16 * 32];
  __shared__ int sh_flag;  // 0 continue, 1 level converged, 2 stop
  __shared__ Pattern sh_pat;
  __shared__ int sh_ipl[kMaxLevels];
  if (threadIdx.x < 12) sh_T[threadIdx.x] = a.T_init[threadIdx.x];
  if (threadIdx.x < kMaxLevels) sh_ipl[threadIdx.x] = 0;
  if (threadIdx.x == 0) sh_pat = a.pat;
  __syncthreads();
  int status = 0, iterations = 0;  // authoritative in thread 0
  int64_t samples = 0;
  bool stop = false;  // uniform across the workgroup
  for (int l = a.levels - 1; l >= 0 && !stop; --l) {
    bool converged = false;
    for (int it = 0; it < a.max_iters; ++it) {
      float acc[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) acc[j] = 0.f;
      float T[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
      accumulate<KT, false>(a, sh_pat, l, T, acc);
      block_reduce32(acc, sh_red, sh_tot);
      if (threadIdx.x == 0) {
        samples += (int64_t)sh_tot[kSlotN];
        int flag = 0;
        if ((int)sh_tot[kSlotPts] < a.min_points) {
          flag = 2;
          status = 2;  // too few points
        } else {
          float step;
          if (solve_update(sh_tot, sh_T, &step)) {
            flag = 2;
            status = 3;  // not positive definite
          } else {
            ++iterations;
            ++sh_ipl[l];
            if (step < a.step_eps) flag = 1;
          }
        }
        sh_flag = flag;
      }
      __syncthreads();
      const int flag = sh_flag;
      __syncthreads();
      if (flag == 2) {
        stop = true;
        break;
      }
      if (flag == 1) {
        converged = true;
        break;
      }
    }
    if (threadIdx.x == 0 && !stop && l == 0 && !converged) status = 1;  // iteration cap at level 0
  }
  // final cost-only pass at level 0
  {
    float acc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] = 0.f;
    float T[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
    accumulate<KT, true>(a, sh_pat, 0, T, acc);
    block_reduce32(acc, sh_red, sh_tot);
  }
  if (threadIdx.x == 0) {
    TrackOut* o = a.out;
    for (int j = 0; j < 12; ++j) o->T[j] = sh_T[j];
    o->E = sh_tot[kSlotE];
    o->n = sh_tot[kSlotN];
    o->iterations = iterations;
    for (int j = 0; j < kMaxLevels; ++j) o->iters_per_level[j] = sh_ipl[j];
    o->n_valid_points = (int)sh_tot[kSlotPts];
    o->status = status;
    o->samples = samples + (int64_t)sh_tot[kSlotN];
  }
}

template <int KT>
__global__ __launch_bounds__(kTrackThreads) void normal_eq_kernel(TrackArgs a) {
  __shared__ float sh_red[16 * 32];
  __shared__ float sh_tot[32];
  __shared__ Pattern sh_pat;
  if (threadIdx.x == 0) sh_pat = a.pat;
  __syncthreads();
  float acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.f;
  accumulate<KT, false>(a, sh_pat, a.level, a.T_init, acc);
  block_reduce32(acc, sh_red, sh_tot);
  if (threadIdx.x < 32) a.totals[threadIdx.x] = sh_tot[threadIdx.x];
}

hipError_t launch_track(const TrackArgs& a, hipStream_t s) {
  if (a.pat.K == 8)
    hipLaunchKernelGGL(track_kernel<8>, dim3(1), dim3(kTrackThreads), 0, s, a);
  else
    hipLaunchKernelGGL(track_kernel<0>, dim3(1), dim3(kTrackThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_normal_equations(const TrackArgs& a, hipStream_t s) {
  if (a.pat.K == 8)
    hipLaunchKernelGGL(normal_eq_kernel<8>, dim3(1), dim3(kTrackThreads), 0, s, a);
  else
    hipLaunchKernelGGL(normal_eq_kernel<0>, dim3(1), dim3(kTrackThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace dpt
