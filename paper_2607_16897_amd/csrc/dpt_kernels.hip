// gfx950 kernels of the direct photometric tracker: pyramid, map-point
// selection, inverse-compositional precompute and the Gauss-Newton track.
//
// Built with -ffp-contract=off: every fused multiply-add is written out as
// fmaf, so that the reference precompute and the track evaluate the projection
// and the bilinear sample with identical arithmetic (an identical frame at the
// reference pose then gives residuals of exactly zero).
#include <cstring>
#include <type_traits>

#include "dpt_device.h"

namespace dpt {

// ---------------------------------------------------------------- pyramid

template <int TILE>
__global__ __launch_bounds__(256) void pyramid_kernel(const uint8_t* __restrict__ src, int64_t pitch,
                                                      uint8_t* __restrict__ dst, PyrGeom g, int vec4) {
  pyramid_tile<TILE>(src, pitch, dst, g, vec4);
}

__global__ __launch_bounds__(256) void pyramid64v_kernel(const uint8_t* __restrict__ src, int64_t pitch,
                                                         uint8_t* __restrict__ dst, PyrGeom g) {
  pyramid_tile64v(src, pitch, dst, g);
}

// One thread per block of level 0 (pyramid_block), blocks in row-major order.
template <int LV>
__global__ __launch_bounds__(256) void pyramid_block_kernel(const uint8_t* __restrict__ src, int64_t pitch,
                                                            uint8_t* __restrict__ dst, PyrGeom g) {
  constexpr int B = 1 << (LV - 1);
  const int nbx = g.W[0] / B, t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbx * (g.H[0] / B)) return;
  pyramid_block<LV>(src, pitch, dst, g, t % nbx, t / nbx, true);
}

hipError_t launch_pyramid(const uint8_t* src, int64_t pitch, uint8_t* dst, const PyrGeom& g, hipStream_t s) {
  if (pyramid_block_ok(g, src, pitch, dst)) {
    const int B = 1 << (g.levels - 1), n = (g.W[0] / B) * (g.H[0] / B);
    if (g.levels == 4)
      hipLaunchKernelGGL(pyramid_block_kernel<4>, dim3((n + 255) / 256), dim3(256), 0, s, src, pitch, dst, g);
    else
      hipLaunchKernelGGL(pyramid_block_kernel<3>, dim3((n + 255) / 256), dim3(256), 0, s, src, pitch, dst, g);
    return hipGetLastError();
  }
  int vec4 = ((pitch % 4) == 0 && (reinterpret_cast<uintptr_t>(src) % 4) == 0 && (g.W[0] % 4) == 0 &&
              (reinterpret_cast<uintptr_t>(dst) % 4) == 0)
                 ? 1
                 : 0;
  const bool vec16 = (pitch % 16) == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 && (g.W[0] % 16) == 0 &&
                     (reinterpret_cast<uintptr_t>(dst) % 16) == 0;
  if (vec16 && g.levels <= 7) {
    dim3 grid((g.W[0] + 63) / 64, (g.H[0] + 63) / 64);
    hipLaunchKernelGGL(pyramid64v_kernel, grid, dim3(256), 0, s, src, pitch, dst, g);
  } else if (g.levels <= 6) {
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

// ---------------------------------------------------------------- Gaussian pyramid (Sec. IV-C)

// Level 0 of the floating-point pyramid: the frame's uint8 values as floats.
__global__ __launch_bounds__(256) void gauss_level0_kernel(const uint8_t* __restrict__ src, int64_t pitch,
                                                           float* __restrict__ dst, int W, int H) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x < W && y < H) dst[(int64_t)y * W + x] = (float)src[y * pitch + x];
}

// Level l+1 from level l (w x h): the binomial kernel [1 3 3 1]/8 over samples
// 2y-1 .. 2y+2, clamped to the level, first down the four columns (the
// vertical pass), then across them (the horizontal pass), kept at every second
// sample: level-(l+1) pixel x sits at level-l position 2x + 1/2.
__global__ __launch_bounds__(256) void gauss_down_kernel(const float* __restrict__ src, int w, int h,
                                                         float* __restrict__ dst, int w2, int h2) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= w2 || y >= h2) return;
  const float wt[4] = {0.125f, 0.375f, 0.375f, 0.125f};
  int rows[4], cols[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rows[i] = min(max(2 * y - 1 + i, 0), h - 1) * w;
    cols[i] = min(max(2 * x - 1 + i, 0), w - 1);
  }
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float col = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) col += wt[i] * src[rows[i] + cols[j]];
    acc += wt[j] * col;
  }
  dst[(int64_t)y * w2 + x] = acc;
}

hipError_t launch_pyramid_gauss(const uint8_t* src, int64_t pitch, float* dst, const PyrGeom& g, hipStream_t s) {
  hipLaunchKernelGGL(gauss_level0_kernel, dim3((g.W[0] + 63) / 64, (g.H[0] + 3) / 4), dim3(256), 0, s, src, pitch,
                     dst + g.off[0], g.W[0], g.H[0]);
  for (int l = 1; l < g.levels; ++l)
    hipLaunchKernelGGL(gauss_down_kernel, dim3((g.W[l] + 63) / 64, (g.H[l] + 3) / 4), dim3(256), 0, s,
                       (const float*)(dst + g.off[l - 1]), g.W[l - 1], g.H[l - 1], dst + g.off[l], g.W[l], g.H[l]);
  return hipGetLastError();
}

// ---------------------------------------------------------------- IC precompute (Eq.(6))

// One lane per (point, pattern sample) and level: x0 = T_rw P, the point's
// reference validity, the bilinear template intensity I0 and the interpolated
// central-difference gradient.  The Jacobian itself is rebuilt in the track
// from (gx, gy) and x0, so the cache holds 12 bytes per sample.
__global__ __launch_bounds__(256) void precompute_kernel(PrecomputeArgs one, const PrecomputeArgs* __restrict__ many) {
  const PrecomputeArgs& a = many ? many[blockIdx.z] : one;  // one reference, or reference blockIdx.z of a batch
  const int K = a.pat.K;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (l >= a.levels) return;
  if (s >= a.n * K) return;
  const int i = s / K, k = s - i * K;
  float X, Y, Z;
  transform(a.T_rw, a.P[3 * i], a.P[3 * i + 1], a.P[3 * i + 2], X, Y, Z);
  if (l == 0 && k == 0) a.x0[i] = make_float4(X, Y, Z, 0.0f);
  const LevelGeom g = a.lv[l];
  bool ok = Z > a.z_min;
  float u = 0.f, v = 0.f;
  if (ok) {
    project(g, X, Y, Z, u, v);
    ok = inside(g, a.pat, u, v);
  }
  if (k == 0) a.valid[(int64_t)l * a.cap + i] = ok ? 1 : 0;
  float I0 = 0.f, gx = 0.f, gy = 0.f;
  if (ok) {  // sample k: the cell of the point's projection moved by the pattern offset
    const Cell q = cell_of(u, v);
    const int x = q.iu + (int)a.pat.dx[k], y = q.iv + (int)a.pat.dy[k];
    if (a.reff) {  // floating-point Gaussian pyramid
      I0 = sample_cell(a.reff + g.off, g.W, x, y, q.w);
      gradient_cell(a.reff + g.off, g.W, x, y, q.w, gx, gy);
    } else {
      I0 = sample_cell(a.ref + g.off, g.W, x, y, q.w);
      gradient_cell(a.ref + g.off, g.W, x, y, q.w, gx, gy);
    }
  }
  const int64_t o = (int64_t)l * a.cap * K + s;
  a.I0[o] = I0;
  a.gx[o] = gx;
  a.gy[o] = gy;
  if (a.I0h) {
    a.I0h[o] = __float2half_rn(I0 - 128.0f);
    a.gh[o] = __floats2half2_rn(gx, gy);
  }
}

hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  dim3 grid((a.n * a.pat.K + 255) / 256, a.levels);
  hipLaunchKernelGGL(precompute_kernel, grid, dim3(256), 0, s, a, (const PrecomputeArgs*)nullptr);
  return hipGetLastError();
}

hipError_t launch_precompute_batch(const PrecomputeArgs* d_args, int n_ref, int max_samples, int max_levels,
                                   hipStream_t s) {
  if (n_ref == 0 || max_samples == 0) return hipSuccess;
  PrecomputeArgs none;
  std::memset(&none, 0, sizeof none);
  dim3 grid((max_samples + 255) / 256, max_levels, n_ref);
  hipLaunchKernelGGL(precompute_kernel, grid, dim3(256), 0, s, none, d_args);
  return hipGetLastError();
}

// ---------------------------------------------------------------- fixed-H mode (Sec. IV-C)

// Per-point H contributions at the reference pose (x = x0), reduced per
// workgroup: thread = point i of level blockIdx.y, J_k = gx_k au + gy_k av with
// the warp Jacobian rows (au, av) at x0, so H_i = m00 au^T au + m01 (au^T av +
// av^T au) + m11 av^T av over the point's K cached gradients.  Workgroup
// partial sums go to hpart[l][blockIdx.x][21].
__global__ __launch_bounds__(256) void fixed_h_partial_kernel(PrecomputeArgs one,
                                                             const PrecomputeArgs* __restrict__ many) {
  __shared__ float sh_red[4 * 32];
  __shared__ float sh_tot[32];
  const PrecomputeArgs& a = many ? many[blockIdx.z] : one;
  const int l = blockIdx.y;
  if (l >= a.levels || (int)blockIdx.x * 256 >= a.n) return;  // uniform over the workgroup
  const int K = a.pat.K, i = blockIdx.x * 256 + threadIdx.x;
  float acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.f;
  if (i < a.n && a.valid[(int64_t)l * a.cap + i]) {
    const int64_t o = ((int64_t)l * a.cap + i) * K;
    float m00 = 0.f, m01 = 0.f, m11 = 0.f;
    for (int k = 0; k < K; ++k) {
      const float gx = a.gx[o + k], gy = a.gy[o + k];
      m00 = fmaf(gx, gx, m00);
      m01 = fmaf(gx, gy, m01);
      m11 = fmaf(gy, gy, m11);
    }
    const float4 p = a.x0[i];
    const LevelGeom g = a.lv[l];
    const float iz = 1.0f / p.z, xp = p.x * iz, yp = p.y * iz;
    const float au[6] = {-g.fx * xp * yp, g.fx * fmaf(xp, xp, 1.0f), -g.fx * yp, g.fx * iz, 0.0f, -g.fx * xp * iz};
    const float av[6] = {-g.fy * fmaf(yp, yp, 1.0f), g.fy * xp * yp, g.fy * xp, 0.0f, g.fy * iz, -g.fy * yp * iz};
    int q = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const float ma = fmaf(m00, au[r], m01 * av[r]);
      const float mc = fmaf(m01, au[r], m11 * av[r]);
#pragma unroll
      for (int c = r; c < 6; ++c) acc[q++] = fmaf(ma, au[c], mc * av[c]);
    }
  }
  block_reduce32(acc, sh_red, sh_tot);
  const int pblk = (a.cap + 255) / 256;
  if (threadIdx.x < 21) a.hpart[((int64_t)l * pblk + blockIdx.x) * 21 + threadIdx.x] = sh_tot[threadIdx.x];
}

// Level blockIdx.x: H = the workgroup partials summed in FP64 in workgroup
// order, and its Cholesky factor in FP64 (pivot <= 1e-6 of the largest
// diagonal entry: not positive definite, the FP32 solve's criterion), stored
// rounded to FP32 for the track's substitutions.
__global__ __launch_bounds__(64) void fixed_h_final_kernel(PrecomputeArgs one, const PrecomputeArgs* __restrict__ many) {
  __shared__ double sh_H[21];
  const PrecomputeArgs& a = many ? many[blockIdx.y] : one;
  const int l = blockIdx.x;
  if (l >= a.levels) return;
  const int nblk = (a.n + 255) / 256, pblk = (a.cap + 255) / 256;
  if (threadIdx.x < 21) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += (double)a.hpart[((int64_t)l * pblk + b) * 21 + threadIdx.x];
    sh_H[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  FixedH& f = a.fixed[l];
  double L[21], invd[6], dmax = 0.0;
  for (int j = 0; j < 6; ++j) dmax = fmax(dmax, sh_H[tri(j, j)]);
  int bad = 0;
  for (int j = 0; j < 6; ++j) {
    double d = sh_H[tri(j, j)];
    for (int k = 0; k < j; ++k) d -= L[tri(k, j)] * L[tri(k, j)];
    bad |= !(d > 1e-6 * dmax);
    const double inv = 1.0 / sqrt(fmax(d, 1e-300));
    invd[j] = inv;
    for (int i = j + 1; i < 6; ++i) {
      double t = sh_H[tri(j, i)];
      for (int k = 0; k < j; ++k) t -= L[tri(k, i)] * L[tri(k, j)];
      L[tri(j, i)] = t * inv;
    }
  }
  for (int q = 0; q < 21; ++q) f.H[q] = sh_H[q], f.L[q] = (float)L[q];
  for (int j = 0; j < 6; ++j) f.invd[j] = (float)invd[j];
  f.bad = bad;
}

hipError_t launch_fixed_h(const PrecomputeArgs& a, hipStream_t s) {
  if (a.n > 0)
    hipLaunchKernelGGL(fixed_h_partial_kernel, dim3((a.n + 255) / 256, a.levels), dim3(256), 0, s, a,
                       (const PrecomputeArgs*)nullptr);
  hipLaunchKernelGGL(fixed_h_final_kernel, dim3(a.levels), dim3(64), 0, s, a, (const PrecomputeArgs*)nullptr);
  return hipGetLastError();
}

hipError_t launch_fixed_h_batch(const PrecomputeArgs* d_args, int n_ref, int max_n, int max_levels, hipStream_t s) {
  if (n_ref == 0) return hipSuccess;
  PrecomputeArgs none;
  std::memset(&none, 0, sizeof none);
  if (max_n > 0)
    hipLaunchKernelGGL(fixed_h_partial_kernel, dim3((max_n + 255) / 256, max_levels, n_ref), dim3(256), 0, s, none,
                       d_args);
  hipLaunchKernelGGL(fixed_h_final_kernel, dim3(max_levels, n_ref), dim3(64), 0, s, none, d_args);
  return hipGetLastError();
}

// One thread per selected pixel: P = R_rw^T (z K^-1 [x, y, 1]^T - t_rw) in FP64,
// rounded to FP32.  A pixel without a positive finite depth, and every entry
// past the selection count, becomes a NaN point, which the precompute marks
// invalid at every level.
__global__ __launch_bounds__(256) void backproject_kernel(BackprojectArgs one,
                                                         const BackprojectArgs* __restrict__ many) {
  const BackprojectArgs& a = many ? many[blockIdx.y] : one;  // one map, or map blockIdx.y of a batch
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float nan = __int_as_float(0x7fc00000);
  float out[3] = {nan, nan, nan};
  if (i < *a.count) {
    const int p = a.idx[i];
    const int y = p / a.W, x = p - y * a.W;
    const double z = (double)a.depth[(int64_t)y * a.pitch + x];
    if (z > 0.0 && z < 1e30) {
      const double d[3] = {((double)x - a.cx) / a.fx * z - a.T_rw[3], ((double)y - a.cy) / a.fy * z - a.T_rw[7],
                           z - a.T_rw[11]};
#pragma unroll
      for (int j = 0; j < 3; ++j)
        out[j] = (float)(a.T_rw[j] * d[0] + a.T_rw[4 + j] * d[1] + a.T_rw[8 + j] * d[2]);
    }
  }
  a.P[3 * i] = out[0];
  a.P[3 * i + 1] = out[1];
  a.P[3 * i + 2] = out[2];
}

hipError_t launch_backproject(const BackprojectArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(backproject_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a,
                     (const BackprojectArgs*)nullptr);
  return hipGetLastError();
}

hipError_t launch_backproject_batch(const BackprojectArgs* d_args, int n_maps, int max_n, hipStream_t s) {
  if (n_maps == 0 || max_n == 0) return hipSuccess;
  BackprojectArgs none;
  std::memset(&none, 0, sizeof none);
  hipLaunchKernelGGL(backproject_kernel, dim3((max_n + 255) / 256, n_maps), dim3(256), 0, s, none, d_args);
  return hipGetLastError();
}

// ---------------------------------------------------------------- track

// Accumulate this thread's share of one normal-equation pass (Eq.(2), Eq.(5))
// at one level and relative pose T.  One thread per map point: the K pattern
// samples of a point share its 2x6 warp Jacobian Jw (rows au, av), so with
// J_k = gx_k au + gy_k av the point's contribution is
//   H_i = m00 au^T au + m01 (au^T av + av^T au) + m11 av^T av,  b_i = -(v0 au + v1 av)
// where m = sum_k w_k g_k^T g_k and v = sum_k w_k g_k r_k: five FMAs per sample
// and the 21-term product once per point.  `img` is the current level (uint8
// or float pixels), in LDS or global memory.
template <int KT, bool COST_ONLY, class PIX>
__device__ __forceinline__ void accumulate(const TrackArgs& a, const Pattern& pat, const LevelGeom& g,
                                           const PIX* __restrict__ img, int l, const float* T,
                                           float (&acc)[32]) {
  const int K = KT ? KT : pat.K;
  const int64_t lo = (int64_t)l * a.ref.cap;
  const float* __restrict__ I0 = a.ref.I0 + lo * K;
  const float* __restrict__ GX = a.ref.gx + lo * K;
  const float* __restrict__ GY = a.ref.gy + lo * K;
  const uint8_t* __restrict__ valid = a.ref.valid + lo;
  const float kH = a.huber_k;
  const int n = a.ref.n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (!valid[i]) continue;
    const float4 p = a.ref.x0[i];
    float X, Y, Z;
    transform(T, p.x, p.y, p.z, X, Y, Z);
    if (!(Z > a.z_min)) continue;
    float u, v;
    project(g, X, Y, Z, u, v);
    if (!inside(g, pat, u, v)) continue;
    float i0[KT ? KT : 1], gxs[KT ? KT : 1], gys[KT ? KT : 1];
    if constexpr (KT == 8) {
      const float4* q0 = reinterpret_cast<const float4*>(I0 + (int64_t)i * 8);
      const float4* qx = reinterpret_cast<const float4*>(GX + (int64_t)i * 8);
      const float4* qy = reinterpret_cast<const float4*>(GY + (int64_t)i * 8);
      const float4 a0 = q0[0], a1 = q0[1];
      i0[0] = a0.x, i0[1] = a0.y, i0[2] = a0.z, i0[3] = a0.w, i0[4] = a1.x, i0[5] = a1.y, i0[6] = a1.z, i0[7] = a1.w;
      if (!COST_ONLY) {
        const float4 b0 = qx[0], b1 = qx[1], c0 = qy[0], c1 = qy[1];
        gxs[0] = b0.x, gxs[1] = b0.y, gxs[2] = b0.z, gxs[3] = b0.w, gxs[4] = b1.x, gxs[5] = b1.y, gxs[6] = b1.z,
        gxs[7] = b1.w;
        gys[0] = c0.x, gys[1] = c0.y, gys[2] = c0.z, gys[3] = c0.w, gys[4] = c1.x, gys[5] = c1.y, gys[6] = c1.z,
        gys[7] = c1.w;
      }
    }
    float m00 = 0.f, m01 = 0.f, m11 = 0.f, v0 = 0.f, v1 = 0.f, E = 0.f;
    const Cell q0 = cell_of(u, v);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float Ic = sample_cell(img, g.W, q0.iu + (int)pat.dx[k], q0.iv + (int)pat.dy[k], q0.w);
      const float tmpl = KT ? i0[k] : I0[(int64_t)i * K + k];
      const float r = tmpl - Ic;
      const float ar = fabsf(r);
      const bool hub = (kH > 0.f) & (ar > kH);  // branch-free, so the taps of later samples can issue early
      const float w = hub ? kH / ar : 1.0f;
      const float rho = hub ? kH * (ar - 0.5f * kH) : 0.5f * r * r;
      E += rho;
      if (!COST_ONLY) {
        const float gx = KT ? gxs[k] : GX[(int64_t)i * K + k];
        const float gy = KT ? gys[k] : GY[(int64_t)i * K + k];
        const float wgx = w * gx, wgy = w * gy;
        m00 = fmaf(wgx, gx, m00);
        m01 = fmaf(wgx, gy, m01);
        m11 = fmaf(wgy, gy, m11);
        v0 = fmaf(wgx, r, v0);
        v1 = fmaf(wgy, r, v1);
      }
    }
    acc[kSlotE] += E;
    acc[kSlotN] += (float)K;
    acc[kSlotPts] += 1.0f;
    if (COST_ONLY) continue;
    // warp Jacobian rows at x0 for a left perturbation (w1 w2 w3 v1 v2 v3)
    const float iz = 1.0f / p.z, xp = p.x * iz, yp = p.y * iz;
    const float au[6] = {-g.fx * xp * yp, g.fx * fmaf(xp, xp, 1.0f), -g.fx * yp, g.fx * iz, 0.0f, -g.fx * xp * iz};
    const float av[6] = {-g.fy * fmaf(yp, yp, 1.0f), g.fy * xp * yp, g.fy * xp, 0.0f, g.fy * iz, -g.fy * yp * iz};
    int q = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const float ma = fmaf(m00, au[r], m01 * av[r]);
      const float mc = fmaf(m01, au[r], m11 * av[r]);
#pragma unroll
      for (int c = r; c < 6; ++c) {
        acc[q] = fmaf(ma, au[c], fmaf(mc, av[c], acc[q]));
        ++q;
      }
      acc[kSlotB + r] -= fmaf(au[r], v0, av[r] * v1);
    }
  }
}

// Register-resident variant for K = 8 and at most kCachedPPT points per
// thread: thread t owns points t + j * blockDim.x, whose IC cache is loaded
// once per level and reused by every iteration of that level.
constexpr int kCachedPPT = 4;

__device__ __forceinline__ void load_points(const TrackArgs& a, int l, PointRegs (&pr)[kCachedPPT]) {
#pragma unroll
  for (int j = 0; j < kCachedPPT; ++j) load_point(a, l, threadIdx.x + j * blockDim.x, pr[j]);
}

template <bool COST_ONLY>
__device__ __forceinline__ void accumulate_cached(const TrackArgs& a, const PatRegs& pat, const LevelGeom& g,
                                                  const uint8_t* __restrict__ img, const float* T,
                                                  const PointRegs (&pr)[kCachedPPT], float (&acc)[32]) {
#pragma unroll
  for (int j = 0; j < kCachedPPT; ++j) accumulate_point<COST_ONLY, false>(a, pat, g, img, T, pr[j], acc);
}

// Copy one pyramid level into LDS (used when it fits the workgroup's budget).
__device__ __forceinline__ void stage_level(const uint8_t* __restrict__ src, uint8_t* dst, int bytes) {
  if ((reinterpret_cast<uintptr_t>(src) & 3) == 0) {
    const int words = bytes >> 2;
    const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d4 = reinterpret_cast<uint32_t*>(dst);
    for (int j = threadIdx.x; j < words; j += blockDim.x) d4[j] = s4[j];
    for (int j = (words << 2) + threadIdx.x; j < bytes; j += blockDim.x) dst[j] = src[j];
  } else {
    for (int j = threadIdx.x; j < bytes; j += blockDim.x) dst[j] = src[j];
  }
}

// Whole coarse-to-fine track of one frame per 1024-thread workgroup (workgroup
// b tracks frame b of the batch): the Gauss-Newton loop needs only workgroup
// barriers, the 32 sums are reduced in a fixed order (bitwise reproducible),
// and thread 0 solves and updates.  Levels of at most `lds_bytes` are staged
// in LDS once per level and reused by all iterations of that level.
// PIX = float: the current frame's floating-point Gaussian pyramid (a.curf).
template <int KT, bool CACHED, class PIX = uint8_t>
__global__ __launch_bounds__(kTrackThreads) void track_kernel(TrackArgs a0, const TrackArgs* __restrict__ batch,
                                                              int lds_bytes) {
  extern __shared__ uint8_t dyn_lds[];
  __shared__ TrackArgs sa;
  __shared__ float sh_T[12];
  __shared__ float sh_tot[32];
  __shared__ float sh_red[16 * 32];
  __shared__ int sh_flag;  // 0 continue, 1 level converged, 2 stop
  __shared__ int sh_ipl[kMaxLevels];
  {
    const TrackArgs* src = batch ? batch + blockIdx.x : &a0;
    const int words = (int)(sizeof(TrackArgs) / 4);
    for (int j = threadIdx.x; j < words; j += blockDim.x)
      reinterpret_cast<uint32_t*>(&sa)[j] = reinterpret_cast<const uint32_t*>(src)[j];
  }
  __syncthreads();
  const TrackArgs& a = sa;
  const PatRegs pregs = pattern_regs(a.pat);  // used by the K = 8 register path
  if (threadIdx.x < 12) sh_T[threadIdx.x] = a.T_init[threadIdx.x];
  if (threadIdx.x < kMaxLevels) sh_ipl[threadIdx.x] = 0;
  __syncthreads();
  int status = 0, iterations = 0;  // authoritative in thread 0
  int64_t samples = 0;
  bool stop = false;  // uniform across the workgroup
  constexpr bool FLOAT_PYR = std::is_same<PIX, float>::value;
  static_assert(!(FLOAT_PYR && CACHED), "the register-cached path reads uint8 levels");
  const PIX* cur = FLOAT_PYR ? reinterpret_cast<const PIX*>(a.curf) : reinterpret_cast<const PIX*>(a.cur);
  const PIX* lds_img = reinterpret_cast<const PIX*>(dyn_lds);
  for (int l = a.levels - 1; l >= 0 && !stop; --l) {
    const LevelGeom g = a.lv[l];
    const int bytes = g.W * g.H * (int)sizeof(PIX);
    const bool in_lds = bytes <= lds_bytes;
    if (in_lds) {
      stage_level(reinterpret_cast<const uint8_t*>(cur + g.off), dyn_lds, bytes);
      __syncthreads();
    }
    PointRegs pr[CACHED ? kCachedPPT : 1];
    if constexpr (CACHED) load_points(a, l, pr);
    bool converged = false;
    for (int it = 0; it < a.max_iters; ++it) {
      float acc[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) acc[j] = 0.f;
      float T[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
      if constexpr (CACHED) {
        if (in_lds)
          accumulate_cached<false>(a, pregs, g, dyn_lds, T, pr, acc);
        else
          accumulate_cached<false>(a, pregs, g, a.cur + g.off, T, pr, acc);
      } else {
        if (in_lds)
          accumulate<KT, false>(a, a.pat, g, lds_img, l, T, acc);
        else
          accumulate<KT, false>(a, a.pat, g, cur + g.off, l, T, acc);
      }
      block_reduce32(acc, sh_red, sh_tot);
      if (threadIdx.x == 0) {
        samples += (int64_t)sh_tot[kSlotN];
        int flag = 0;
        if ((int)sh_tot[kSlotPts] < a.min_points) {
          flag = 2;
          status = 2;  // too few points
        } else {
          float step = 0.0f;
          int bad;
          if (a.ref.fixed) {  // fixed-H mode: the level's factor from the precompute
            const FixedH& f = a.ref.fixed[l];
            bad = f.bad;
            if (!bad) solve_fixed(f.L, f.invd, sh_tot + kSlotB, sh_T, &step);
          } else {
            bad = solve_update(sh_tot, sh_T, &step);
          }
          if (bad) {
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
    __syncthreads();  // LDS image is restaged for the next level
  }
  // final cost-only pass at level 0
  {
    float acc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] = 0.f;
    float T[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
    const LevelGeom g = a.lv[0];
    accumulate<KT, true>(a, a.pat, g, cur + g.off, 0, T, acc);
    block_reduce32(acc, sh_red, sh_tot);
  }
  if (threadIdx.x == 0) {
    TrackOut* o = a.out;
    double Tf[12];
    for (int j = 0; j < 12; ++j) Tf[j] = (double)sh_T[j];
    orthonormalize34(Tf);
    for (int j = 0; j < 12; ++j) o->T[j] = sh_T[j], o->Td[j] = Tf[j];
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
  float acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.f;
  const LevelGeom g = a.lv[a.level];
  if (a.curf)
    accumulate<KT, false>(a, a.pat, g, a.curf + g.off, a.level, a.T_init, acc);
  else
    accumulate<KT, false>(a, a.pat, g, a.cur + g.off, a.level, a.T_init, acc);
  block_reduce32(acc, sh_red, sh_tot);
  if (threadIdx.x < 32) a.totals[threadIdx.x] = sh_tot[threadIdx.x];
}

// Largest level (bytes) that a track workgroup stages in LDS.
constexpr int kLdsImageBudget = 96 * 1024;

int track_lds_bytes(const LevelGeom* lv, int levels, int pixel_bytes) {
  int best = 0;
  for (int l = 0; l < levels; ++l) {
    const int b = lv[l].W * lv[l].H * pixel_bytes;
    if (b <= kLdsImageBudget && b > best) best = b;
  }
  return best;
}

template <int KT, bool CACHED, class PIX = uint8_t>
static hipError_t launch_track_k(const TrackArgs& a, const TrackArgs* batch, int n_frames, int lds, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&track_kernel<KT, CACHED, PIX>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsImageBudget);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((track_kernel<KT, CACHED, PIX>), dim3(n_frames), dim3(kTrackThreads), lds, s, a, batch, lds);
  return hipGetLastError();
}

// max_points: the largest map of any frame in the launch (selects the register-cached path)
static hipError_t dispatch_track(const TrackArgs& a, const TrackArgs* batch, int n_frames, int lds, int max_points,
                                 hipStream_t s) {
  if (a.curf) return launch_track_k<0, false, float>(a, batch, n_frames, lds, s);  // Gaussian float pyramid
  if (a.pat.K == 8 && max_points <= kCachedPPT * kTrackThreads)
    return launch_track_k<8, true>(a, batch, n_frames, lds, s);
  if (a.pat.K == 8) return launch_track_k<8, false>(a, batch, n_frames, lds, s);
  return launch_track_k<0, false>(a, batch, n_frames, lds, s);
}

hipError_t launch_track(const TrackArgs& a, hipStream_t s) {
  return dispatch_track(a, nullptr, 1, track_lds_bytes(a.lv, a.levels, a.curf ? 4 : 1), a.ref.n, s);
}

hipError_t launch_track_batch(const TrackArgs& any, const TrackArgs* batch, int n_frames, int lds, int max_points,
                              hipStream_t s) {
  return dispatch_track(any, batch, n_frames, lds, max_points, s);
}

hipError_t launch_normal_equations(const TrackArgs& a, hipStream_t s) {
  if (a.pat.K == 8)
    hipLaunchKernelGGL(normal_eq_kernel<8>, dim3(1), dim3(kTrackThreads), 0, s, a);
  else
    hipLaunchKernelGGL(normal_eq_kernel<0>, dim3(1), dim3(kTrackThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace dpt
