// Device helpers shared by the tracker kernels: projection, sampling,
// workgroup reductions and the 6x6 solve with the SE(3) update.
#pragma once

#include "dpt_internal.h"

namespace dpt {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void transform(const float* T, float X, float Y, float Z, float& x, float& y,
                                          float& z) {
  x = fmaf(T[0], X, fmaf(T[1], Y, fmaf(T[2], Z, T[3])));
  y = fmaf(T[4], X, fmaf(T[5], Y, fmaf(T[6], Z, T[7])));
  z = fmaf(T[8], X, fmaf(T[9], Y, fmaf(T[10], Z, T[11])));
}

// Eq.(1): pinhole projection at one pyramid level, through one reciprocal of
// z (v_rcp_f32, 1 ulp).  Every sampling site (the precompute and every track
// path) projects with this same arithmetic, so a pose equal to the reference's
// reproduces the template's sample positions bit for bit.
__device__ __forceinline__ void project(const LevelGeom& g, float x, float y, float z, float& u, float& v) {
  const float iz = __builtin_amdgcn_rcpf(z);
  u = fmaf(g.fx * x, iz, g.cx);
  v = fmaf(g.fy * y, iz, g.cy);
}

// A point is usable when it is in front of the camera and every pattern
// position p satisfies 1 <= p.x < W-2 and 1 <= p.y < H-2 (the bilinear taps and
// their central differences stay inside the level).
__device__ __forceinline__ bool inside(const LevelGeom& g, const Pattern& p, float u, float v) {
  return (u + (float)p.dx_min >= 1.0f) && (u + (float)p.dx_max < (float)(g.W - 2)) &&
         (v + (float)p.dy_min >= 1.0f) && (v + (float)p.dy_max < (float)(g.H - 2));
}

// The K = 8 pattern held in registers for the whole track: offsets and their
// bounding box as floats (the same values inside() converts on the fly).
struct PatRegs {
  float dx[8], dy[8];
  float dx_min, dx_max, dy_min, dy_max;
};

__device__ __forceinline__ PatRegs pattern_regs(const Pattern& p) {
  PatRegs r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.dx[k] = (float)p.dx[k], r.dy[k] = (float)p.dy[k];
  r.dx_min = (float)p.dx_min, r.dx_max = (float)p.dx_max;
  r.dy_min = (float)p.dy_min, r.dy_max = (float)p.dy_max;
  return r;
}

// inside() on the register pattern, without branches.
__device__ __forceinline__ bool inside(const LevelGeom& g, const PatRegs& p, float u, float v) {
  return (u + p.dx_min >= 1.0f) & (u + p.dx_max < (float)(g.W - 2)) & (v + p.dy_min >= 1.0f) &
         (v + p.dy_max < (float)(g.H - 2));
}

// Bilinear sampling, pixel centres at integer coordinates.  A point projected
// to (u, v) lies in the cell with corner (iu, iv) = floor(u, v) at fractions
// (a, c); the pattern's offsets are whole pixels, so every sample of the point
// is the cell at (iu + dx_k, iv + dy_k) with the same fractions and weights.
// The weights are formed once per point, the same way at every sampling site.
struct Bilin {
  float w00, w10, w01, w11;
};

struct Cell {
  int iu, iv;
  Bilin w;
};

__device__ __forceinline__ Cell cell_of(float u, float v) {
  Cell q;
  const float fu = floorf(u), fv = floorf(v);
  const float a = u - fu, c = v - fv;  // exact: u and floor(u) are close
  q.iu = (int)fu, q.iv = (int)fv;
  q.w.w11 = a * c;
  q.w.w10 = a - q.w.w11;
  q.w.w01 = c - q.w.w11;
  q.w.w00 = (1.0f - a) - q.w.w01;
  return q;
}

// (1-a)(1-c) t00 + a(1-c) t10 + (1-a)c t01 + ac t11.
__device__ __forceinline__ float bilin_mix(const Bilin& w, float t00, float t10, float t01, float t11) {
  return fmaf(w.w11, t11, fmaf(w.w01, t01, fmaf(w.w10, t10, w.w00 * t00)));
}

// Intensity of a level (uint8 or float pixels) in the cell with corner (x, y).
template <class PIX>
__device__ __forceinline__ float sample_cell(const PIX* img, int W, int x, int y, const Bilin& w) {
  const PIX* p = img + y * W + x;
  return bilin_mix(w, (float)p[0], (float)p[1], (float)p[W], (float)p[W + 1]);
}

// Reference-side gradient in the same cell: central differences / 2 at its
// four corners, blended with the same weights.
template <class PIX>
__device__ __forceinline__ void gradient_cell(const PIX* img, int W, int x, int y, const Bilin& w, float& gx,
                                              float& gy) {
  const PIX* p = img + y * W + x;
  const float gx00 = 0.5f * ((float)p[1] - (float)p[-1]);
  const float gx10 = 0.5f * ((float)p[2] - (float)p[0]);
  const float gx01 = 0.5f * ((float)p[W + 1] - (float)p[W - 1]);
  const float gx11 = 0.5f * ((float)p[W + 2] - (float)p[W]);
  const float gy00 = 0.5f * ((float)p[W] - (float)p[-W]);
  const float gy10 = 0.5f * ((float)p[W + 1] - (float)p[1 - W]);
  const float gy01 = 0.5f * ((float)p[2 * W] - (float)p[0]);
  const float gy11 = 0.5f * ((float)p[2 * W + 1] - (float)p[1]);
  gx = bilin_mix(w, gx00, gx10, gx01, gx11);
  gy = bilin_mix(w, gy00, gy10, gy01, gy11);
}

// ---------------------------------------------------------------- pyramid

// One launch builds every level.  A workgroup owns a TILE x TILE block of
// level 0 (TILE >= 2^(levels-1)), so each level's 2x2 parents stay inside the
// tile; levels alternate between two LDS buffers.
// The tile at level-0 origin (ox, oy); write_l0 = false leaves level 0 of dst
// unwritten (a caller that reads level 0 from the source frame itself).
template <int TILE>
__device__ __forceinline__ void pyramid_tile_at(const uint8_t* __restrict__ src, int64_t pitch,
                                                uint8_t* __restrict__ dst, const PyrGeom& g, int vec4, int ox, int oy,
                                                bool write_l0) {
  __shared__ uint8_t buf0[TILE * TILE];
  __shared__ uint8_t buf1[TILE * TILE / 4];
  const int W0 = g.W[0], H0 = g.H[0];
  if (vec4) {
    // 4-byte loads: width, pitch and base are multiples of 4
    for (int q = threadIdx.x; q < TILE * TILE / 4; q += blockDim.x) {
      int ly = q / (TILE / 4), lx = (q % (TILE / 4)) * 4;
      int gx = ox + lx, gy = oy + ly;
      uint32_t v = 0;
      if (gy < H0 && gx < W0) {
        v = *reinterpret_cast<const uint32_t*>(src + gy * pitch + gx);
        if (write_l0) *reinterpret_cast<uint32_t*>(dst + g.off[0] + (int64_t)gy * W0 + gx) = v;
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
        if (write_l0) dst[g.off[0] + (int64_t)gy * W0 + gx] = v;
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

template <int TILE>
__device__ __forceinline__ void pyramid_tile(const uint8_t* __restrict__ src, int64_t pitch,
                                             uint8_t* __restrict__ dst, const PyrGeom& g, int vec4) {
  pyramid_tile_at<TILE>(src, pitch, dst, g, vec4, blockIdx.x * TILE, blockIdx.y * TILE, true);
}

// pyramid_tile for 64x64 tiles of frames whose width, pitch and base address
// are multiples of 16: one 16-byte load and store per thread for level 0 (256
// threads), four level-1 pixels per thread from two 8-byte LDS reads with one
// 4-byte store, then the coarser levels as pyramid_tile.  Up to 7 levels.
__device__ __forceinline__ void pyramid_tile64v_at(const uint8_t* __restrict__ src, int64_t pitch,
                                                   uint8_t* __restrict__ dst, const PyrGeom& g, int ox, int oy,
                                                   bool write_l0) {
  __shared__ __align__(16) uint8_t buf0[64 * 64];
  __shared__ __align__(16) uint8_t buf1[32 * 32];
  const int W0 = g.W[0], H0 = g.H[0];
  {
    const int r = threadIdx.x >> 2, c = (threadIdx.x & 3) * 16;
    const int gx = ox + c, gy = oy + r;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gy < H0 && gx < W0) {  // W0 % 16 == 0: the 16 bytes lie inside the row
      v = *reinterpret_cast<const uint4*>(src + gy * pitch + gx);
      if (write_l0) *reinterpret_cast<uint4*>(dst + g.off[0] + (int64_t)gy * W0 + gx) = v;
    }
    *reinterpret_cast<uint4*>(buf0 + r * 64 + c) = v;
  }
  __syncthreads();
  if (g.levels < 2) return;
  {
    const int r = threadIdx.x >> 3, c = (threadIdx.x & 7) * 4;
    const uint2 a = *reinterpret_cast<const uint2*>(buf0 + (2 * r) * 64 + 2 * c);
    const uint2 b = *reinterpret_cast<const uint2*>(buf0 + (2 * r + 1) * 64 + 2 * c);
    const uint32_t top[2] = {a.x, a.y}, bot[2] = {b.x, b.y};
    uint32_t out = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = top[j >> 1] >> (16 * (j & 1)), u = bot[j >> 1] >> (16 * (j & 1));
      const uint32_t s4 = (t & 0xffu) + ((t >> 8) & 0xffu) + (u & 0xffu) + ((u >> 8) & 0xffu);
      out |= ((s4 + 2u) >> 2) << (8 * j);
    }
    *reinterpret_cast<uint32_t*>(buf1 + r * 32 + c) = out;
    const int W1 = g.W[1], H1 = g.H[1];
    const int gx = (ox >> 1) + c, gy = (oy >> 1) + r;
    if (gy < H1 && gx < W1)  // W1 % 8 == 0 and gx % 4 == 0: all four pixels are inside
      *reinterpret_cast<uint32_t*>(dst + g.off[1] + (int64_t)gy * W1 + gx) = out;
  }
  __syncthreads();
  uint8_t* prev = buf1;
  uint8_t* next = buf0;
  for (int l = 2; l < g.levels; ++l) {
    const int T = 64 >> l, Tp = 64 >> (l - 1);
    const int Wl = g.W[l], Hl = g.H[l];
    const int oxl = ox >> l, oyl = oy >> l;
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
      const int ly = q / T, lx = q % T;
      const int gx = oxl + lx, gy = oyl + ly;
      uint8_t v = 0;
      if (gx < Wl && gy < Hl) {
        const uint8_t* p = prev + (2 * ly) * Tp + 2 * lx;
        const int s4 = (int)p[0] + (int)p[1] + (int)p[Tp] + (int)p[Tp + 1];
        v = (uint8_t)((s4 + 2) >> 2);
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

// Rounded 2x2 box means of two rows of four bytes: bytes 0 and 1 of the
// result hold (t0 + t1 + b0 + b1 + 2) >> 2 and (t2 + t3 + b2 + b3 + 2) >> 2.
// The pair sums travel in two 16-bit lanes (at most 1022 each).
__device__ __forceinline__ uint32_t box_pairs(uint32_t top, uint32_t bot) {
  const uint32_t s = (top & 0x00ff00ffu) + ((top >> 8) & 0x00ff00ffu) + (bot & 0x00ff00ffu) + ((bot >> 8) & 0x00ff00ffu);
  const uint32_t r = ((s + 0x00020002u) >> 2) & 0x00ff00ffu;
  return (r & 0xffu) | ((r >> 8) & 0xff00u);
}

// The pyramid of one B x B block of level 0 (B = 2^(LV-1), LV = 3 or 4
// levels) in one thread's registers: block (bx, by) of a level 0 whose sizes
// are multiples of B, so every level's share of the block is whole and
// (levels' sizes halving exactly) each level is written with one aligned
// store per row.  Needs 8-byte aligned rows of src and dst.
template <int LV>
__device__ __forceinline__ void pyramid_block(const uint8_t* __restrict__ src, int64_t pitch,
                                              uint8_t* __restrict__ dst, const PyrGeom& g, int bx, int by,
                                              bool write_l0) {
  static_assert(LV == 3 || LV == 4, "three or four levels");
  constexpr int B = 1 << (LV - 1);
  const int W0 = g.W[0];
  if constexpr (LV == 4) {
    uint2 r0[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) r0[r] = *reinterpret_cast<const uint2*>(src + (int64_t)(8 * by + r) * pitch + 8 * bx);
    if (write_l0)
#pragma unroll
      for (int r = 0; r < 8; ++r) *reinterpret_cast<uint2*>(dst + g.off[0] + (int64_t)(8 * by + r) * W0 + 8 * bx) = r0[r];
    uint32_t r1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      r1[i] = box_pairs(r0[2 * i].x, r0[2 * i + 1].x) | (box_pairs(r0[2 * i].y, r0[2 * i + 1].y) << 16);
      *reinterpret_cast<uint32_t*>(dst + g.off[1] + (int64_t)(4 * by + i) * g.W[1] + 4 * bx) = r1[i];
    }
    uint32_t r2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      r2[i] = box_pairs(r1[2 * i], r1[2 * i + 1]);
      *reinterpret_cast<uint16_t*>(dst + g.off[2] + (int64_t)(2 * by + i) * g.W[2] + 2 * bx) = (uint16_t)r2[i];
    }
    dst[g.off[3] + (int64_t)by * g.W[3] + bx] = (uint8_t)box_pairs(r2[0], r2[1]);
  } else {
    uint32_t r0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) r0[r] = *reinterpret_cast<const uint32_t*>(src + (int64_t)(4 * by + r) * pitch + 4 * bx);
    if (write_l0)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        *reinterpret_cast<uint32_t*>(dst + g.off[0] + (int64_t)(4 * by + r) * W0 + 4 * bx) = r0[r];
    uint32_t r1[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      r1[i] = box_pairs(r0[2 * i], r0[2 * i + 1]);
      *reinterpret_cast<uint16_t*>(dst + g.off[1] + (int64_t)(2 * by + i) * g.W[1] + 2 * bx) = (uint16_t)r1[i];
    }
    dst[g.off[2] + (int64_t)by * g.W[2] + bx] = (uint8_t)box_pairs(r1[0], r1[1]);
  }
  (void)B;
}

__device__ __forceinline__ void pyramid_tile64v(const uint8_t* __restrict__ src, int64_t pitch,
                                                uint8_t* __restrict__ dst, const PyrGeom& g) {
  pyramid_tile64v_at(src, pitch, dst, g, blockIdx.x * 64, blockIdx.y * 64, true);
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

// Row rotation within 16 lanes (DPP row_ror:K), a VALU operand modifier.
template <int K>
__device__ __forceinline__ float dpp_ror(float v) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v), 0x120 + K, 0xf, 0xf, false));
}

// Sum 32 per-lane values over a wave64.  Two halving steps exchange whole
// half-waves with the gfx950 lane-swap instructions: v_permlane32_swap pairs
// lane L with L ^ 32 and v_permlane16_swap pairs L with L ^ 16, each lane keeping
// half of its values, so 16 + 8 swaps leave 8 values per lane summed over 4
// lanes.  DPP row rotations then sum each over the 16 lanes of a row.  On return
// a[j] of every lane in row r = lane / 16 holds the wave total of value 8 r + j.
// No shuffle through LDS and no data-dependent indexing; fixed addition order.
__device__ __forceinline__ void wave_reduce32(float (&a)[32]) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 16]), false, false);
    a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 8]), false, false);
    a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float v = a[j];
    v += dpp_ror<8>(v);
    v += dpp_ror<4>(v);
    v += dpp_ror<2>(v);
    v += dpp_ror<1>(v);
    a[j] = v;
  }
}

// wave_reduce32 for 16 values: one lane-swap step less.  On return a[j] of
// every lane in row r = lane / 16 holds the wave total of value 4 r + j, j < 4.
__device__ __forceinline__ void wave_reduce16(float (&a)[16]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 8]), false, false);
    a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 4]), false, false);
    a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = a[j];
    v += dpp_ror<8>(v);
    v += dpp_ror<4>(v);
    v += dpp_ror<2>(v);
    v += dpp_ror<1>(v);
    a[j] = v;
  }
}

// Workgroup total of 32 per-lane values into out[32] (LDS), fixed order.
// `scratch` is 16 x 32 floats of LDS.
__device__ __forceinline__ void block_reduce32(float (&a)[32], float* scratch, float* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_reduce32(a);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) scratch[wave * 32 + 8 * (lane >> 4) + j] = a[j];
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += scratch[w * 32 + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// As block_reduce32, with Kahan-compensated summation across the waves.
__device__ __forceinline__ void block_reduce32_kahan(float (&a)[32], float* scratch, float* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_reduce32(a);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) scratch[wave * 32 + 8 * (lane >> 4) + j] = a[j];
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    float s = 0.0f, c = 0.0f;
    for (int w = 0; w < nw; ++w) {
      const float y = scratch[w * 32 + threadIdx.x] - c;
      const float t = s + y;
      c = (t - s) - y;
      s = t;
    }
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Index of H(i, j), i <= j, in the row-major upper-triangle order of the sums.
__host__ __device__ constexpr int tri(int i, int j) { return i * 6 - (i * (i - 1)) / 2 + (j - i); }

// T <- T exp(xi) for the twist xi = (w, v) (rotation part first) of squared
// angle th2 = |w|^2, given the coefficients A = sin(th) / th,
// B = (1 - cos th) / th^2 and C = (th - sin th) / th^3 of the SE(3) exponential:
// R = I + A [w]x + B [w]x^2 and t = (I + B [w]x + C [w]x^2) v.  With
// [w]x^2 = w w^T - th2 I and [w]x v = w x v these are written out entry by
// entry: R = (1 - B th2) I + A [w]x + B w w^T, t = (1 - C th2) v + B (w x v)
// + C (w.v) w.  F = float or double; every product is an explicit FMA.
template <class F>
__device__ __forceinline__ void compose_exp(F* T, F w0, F w1, F w2, F v0, F v1, F v2, F th2, F A, F B, F C) {
  const F Bw0 = B * w0, Bw1 = B * w1, Bw2 = B * w2, Aw0 = A * w0, Aw1 = A * w1, Aw2 = A * w2;
  const F dg = fma(-B, th2, F(1));
  const F E[3][4] = {
      {fma(Bw0, w0, dg), fma(Bw0, w1, -Aw2), fma(Bw0, w2, Aw1), F(0)},
      {fma(Bw0, w1, Aw2), fma(Bw1, w1, dg), fma(Bw1, w2, -Aw0), F(0)},
      {fma(Bw0, w2, -Aw1), fma(Bw1, w2, Aw0), fma(Bw2, w2, dg), F(0)}};
  const F c0 = fma(w1, v2, -(w2 * v1)), c1 = fma(w2, v0, -(w0 * v2)), c2 = fma(w0, v1, -(w1 * v0));
  const F Cwv = C * fma(w0, v0, fma(w1, v1, w2 * v2)), Cv = fma(-C, th2, F(1));
  const F t[3] = {fma(B, c0, fma(Cwv, w0, Cv * v0)), fma(B, c1, fma(Cwv, w1, Cv * v1)),
                  fma(B, c2, fma(Cwv, w2, Cv * v2))};
  F N[12];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) N[4 * r + c] = fma(T[4 * r], E[0][c], fma(T[4 * r + 1], E[1][c], T[4 * r + 2] * E[2][c]));
    N[4 * r + 3] = fma(T[4 * r], t[0], fma(T[4 * r + 1], t[1], fma(T[4 * r + 2], t[2], T[4 * r + 3])));
  }
#pragma unroll
  for (int j = 0; j < 12; ++j) T[j] = N[j];
}

// With H = L L^T given by its factor (L(i, j), i >= j, at tri(j, i), and
// invd = 1 / diag(L)), solve H delta = b by forward and back substitution and
// apply T <- T exp(-delta) in FP32; *max_step = max_j |delta_j|.
__device__ __forceinline__ void substitute_update(const float (&L)[21], const float (&invd)[6], const float (&b)[6],
                                                  float* T, float* max_step);

// Solve H delta = b (6x6 SPD from the 21 upper-triangle sums) by Cholesky in
// FP32 and apply T <- T exp(-delta).  Returns 0, or 1 if a pivot is <= 1e-6 of
// the largest diagonal entry (not positive definite).  Every loop is unrolled
// so the factor lives in registers.
__device__ __forceinline__ int solve_update(const float* tot_lds, float* T, float* max_step) {
  float tot[27];  // one batch of LDS reads, then registers only
#pragma unroll
  for (int q = 0; q < 27; ++q) tot[q] = tot_lds[q];
  float L[21];  // L(i, j), i >= j, stored at tri(j, i)
  float invd[6];
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
    // only 1/L(j, j) is used by the elimination and the substitutions
    const float inv = __builtin_amdgcn_rsqf(fmaxf(s, 1e-30f));
    invd[j] = inv;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      float t = tot[tri(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fmaf(-L[tri(k, i)], L[tri(k, j)], t);
      L[tri(j, i)] = t * inv;
    }
  }
  if (bad) return 1;
  float b[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) b[i] = tot[kSlotB + i];
  substitute_update(L, invd, b, T, max_step);
  return 0;
}

// Fixed-H mode: the factor of the level's constant H comes precomputed
// (Lp[21], invdp[6], as in substitute_update); only the substitutions and the
// update remain.  b: the 6 reduced right-hand-side sums.
__device__ __forceinline__ void solve_fixed(const float* Lp, const float* invdp, const float* bp, float* T,
                                            float* max_step) {
  float L[21], invd[6], b[6];
#pragma unroll
  for (int q = 0; q < 21; ++q) L[q] = Lp[q];
#pragma unroll
  for (int q = 0; q < 6; ++q) invd[q] = invdp[q], b[q] = bp[q];
  substitute_update(L, invd, b, T, max_step);
}

__device__ __forceinline__ void substitute_update(const float (&L)[21], const float (&invd)[6], const float (&b)[6],
                                                  float* T, float* max_step) {
  float y[6], d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fmaf(-L[tri(k, i)], y[k], s);
    y[i] = s * invd[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    float s = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s = fmaf(-L[tri(i, k)], d[k], s);
    d[i] = s * invd[i];
  }
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) m = fmaxf(m, fabsf(d[j]));
  *max_step = m;
  const float w0 = -d[0], w1 = -d[1], w2 = -d[2];
  const float th2 = fmaf(w0, w0, fmaf(w1, w1, w2 * w2));
  float A, B, C;
  if (th2 < 0.0025f) {  // |w| < 0.05
    A = 1.0f - th2 * (1.0f / 6.0f) * (1.0f - th2 * (1.0f / 20.0f));
    B = 0.5f - th2 * (1.0f / 24.0f) * (1.0f - th2 * (1.0f / 30.0f));
    C = (1.0f / 6.0f) - th2 * (1.0f / 120.0f) * (1.0f - th2 * (1.0f / 42.0f));
  } else {
    const float th = sqrtf(th2);
    const float sn = sinf(th), sh = sinf(0.5f * th);
    A = sn / th;
    B = 2.0f * sh * sh / th2;
    C = (th - sn) / (th2 * th);
  }
  compose_exp(T, w0, w1, w2, -d[3], -d[4], -d[5], th2, A, B, C);
}

// FP64 variant of solve_update: Cholesky solve (pivot <= 1e-12 of the largest
// diagonal entry: not positive definite) and T <- T exp(-delta), pose in FP64.
__device__ __forceinline__ int solve_update_d(const float* tot_lds, double* T, double* max_step) {
  float tot[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) tot[q] = tot_lds[q];
  double L[21], invd[6];
  double dmax = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) dmax = fmax(dmax, (double)tot[tri(j, j)]);
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = tot[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s = fma(-L[tri(k, j)], L[tri(k, j)], s);
    bad |= !(s > 1e-12 * dmax);
    s = fmax(s, 1e-300);
    // 1/sqrt(s): hardware estimate, then two Newton steps (each squares the
    // relative error) to full double precision; only 1/L(j, j) is used later
    double inv = __builtin_amdgcn_rsq(s);
    inv = inv * fma(-0.5 * s * inv, inv, 1.5);
    inv = inv * fma(-0.5 * s * inv, inv, 1.5);
    invd[j] = inv;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double t = tot[tri(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fma(-L[tri(k, i)], L[tri(k, j)], t);
      L[tri(j, i)] = t * inv;
    }
  }
  if (bad) return 1;
  double y[6], d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = tot[kSlotB + i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fma(-L[tri(k, i)], y[k], s);
    y[i] = s * invd[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s = fma(-L[tri(i, k)], d[k], s);
    d[i] = s * invd[i];
  }
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) m = fmax(m, fabs(d[j]));
  *max_step = m;
  const double w0 = -d[0], w1 = -d[1], w2 = -d[2];
  const double th2 = fma(w0, w0, fma(w1, w1, w2 * w2));
  double A, B, C;
  if (th2 < 0.0025) {  // |w| < 0.05: series through th^8, truncation below 1e-20
    A = fma(-th2 * (1.0 / 6.0), fma(-th2 * (1.0 / 20.0), fma(-th2 * (1.0 / 42.0), fma(-th2, 1.0 / 72.0, 1.0), 1.0), 1.0),
            1.0);
    B = 0.5 * fma(-th2 * (1.0 / 12.0),
                  fma(-th2 * (1.0 / 30.0), fma(-th2 * (1.0 / 56.0), fma(-th2, 1.0 / 90.0, 1.0), 1.0), 1.0), 1.0);
    C = (1.0 / 6.0) * fma(-th2 * (1.0 / 20.0),
                          fma(-th2 * (1.0 / 42.0), fma(-th2 * (1.0 / 72.0), fma(-th2, 1.0 / 110.0, 1.0), 1.0), 1.0),
                          1.0);
  } else {
    const double th = sqrt(th2);
    const double sn = sin(th), sh = sin(0.5 * th);
    A = sn / th;
    B = 2.0 * sh * sh / th2;
    C = (th - sn) / (th2 * th);
  }
  compose_exp(T, w0, w1, w2, -d[3], -d[4], -d[5], th2, A, B, C);
  return 0;
}

// One map point's IC cache (K = 8) held in registers across the iterations of
// a level: the reference-camera point x0, template intensities and gradients.
struct PointRegs {
  float X0, Y0, Z0;
  float iz, xp, yp;  // 1/Z0, X0/Z0, Y0/Z0 for the warp Jacobian
  float i0_[8], gx_[8], gy_[8];
  bool ok;
  __device__ __forceinline__ float i0(int k) const { return i0_[k]; }
  __device__ __forceinline__ float gx(int k) const { return gx_[k]; }
  __device__ __forceinline__ float gy(int k) const { return gy_[k]; }
};

// Mixed-precision variant: template intensity (minus 128) and gradients in FP16,
// 12 registers per point instead of 24.
struct PointRegsH {
  float X0, Y0, Z0;
  float iz, xp, yp;
  __half i0_[8];
  __half2 g_[8];
  bool ok;
  __device__ __forceinline__ float i0(int k) const { return __half2float(i0_[k]) + 128.0f; }
  __device__ __forceinline__ float gx(int k) const { return __low2float(g_[k]); }
  __device__ __forceinline__ float gy(int k) const { return __high2float(g_[k]); }
};

// Half of a point's 8-sample cache, for kernels that give each point two
// threads: samples 4 sub .. 4 sub + 3 of thread `sub` of the pair.
struct PointRegs4 {
  float X0, Y0, Z0;
  float iz, xp, yp;
  float i0_[4], gx_[4], gy_[4];
  bool ok;
  __device__ __forceinline__ float i0(int k) const { return i0_[k]; }
  __device__ __forceinline__ float gx(int k) const { return gx_[k]; }
  __device__ __forceinline__ float gy(int k) const { return gy_[k]; }
};

struct PointRegsH4 {
  float X0, Y0, Z0;
  float iz, xp, yp;
  __half i0_[4];
  __half2 g_[4];
  bool ok;
  __device__ __forceinline__ float i0(int k) const { return __half2float(i0_[k]) + 128.0f; }
  __device__ __forceinline__ float gx(int k) const { return __low2float(g_[k]); }
  __device__ __forceinline__ float gy(int k) const { return __high2float(g_[k]); }
};

// A load through a generic pointer into device memory, issued as a global
// (not flat) load: a flat load also counts on the LDS counter, so the next
// wait for LDS data would wait for it as well.
// The value moves as a plain word or word vector: HIP's vector structs copy
// through a generic reference, which would turn the load back into a flat one.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  static_assert(sizeof(T) == 1 || sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "word or word vector");
  using W = typename std::conditional<
      sizeof(T) == 1, uint8_t,
      typename std::conditional<sizeof(T) == 4, uint32_t,
                                typename std::conditional<sizeof(T) == 8, uint32_t __attribute__((ext_vector_type(2))),
                                                          uint32_t __attribute__((ext_vector_type(4)))>::type>::type>::type;
  const W w = *(const __attribute__((address_space(1))) W*)p;
  T t;
  __builtin_memcpy(&t, &w, sizeof(T));
  return t;
}

// Load point i's registers for level l.  Branch-free: a point past the map
// (i >= n) reads entry 0 instead, and the geometry of an unusable point is
// selected to finite values (its warp Jacobian multiplies masked zeros); the
// template registers of such a point reach only sums that are selected away.
// The cache arrays hold at least one entry per level, so every read is inside.
__device__ __forceinline__ bool load_geometry(const TrackArgs& a, int l, int i, float4& p, int64_t& e) {
  const int64_t lo = (int64_t)l * a.ref.cap;
  const bool in = i < a.ref.n;
  const int j = in ? i : 0;
  e = lo + j;
  p = gload(a.ref.x0 + j);
  return in & (gload(a.ref.valid + e) != 0);
}

// A point's geometry as loaded (world point, validity byte, inside the map),
// before any use of the loaded words.
struct GeoRaw {
  float x, y, z;
  uint32_t valid;
  bool in;
};

__device__ __forceinline__ void load_geometry_raw(const TrackArgs& a, int l, int i, GeoRaw& r, int64_t& e) {
  const int64_t lo = (int64_t)l * a.ref.cap;
  r.in = i < a.ref.n;
  const int j = r.in ? i : 0;
  e = lo + j;
  const float4 p = gload(a.ref.x0 + j);
  r.x = p.x, r.y = p.y, r.z = p.z;
  r.valid = gload(a.ref.valid + e);
}

template <class PR>
__device__ __forceinline__ void set_geometry(PR& pr, bool ok, const float4& p) {
  pr.ok = ok;
  const float iz = 1.0f / p.z;
  pr.X0 = ok ? p.x : 0.0f;
  pr.Y0 = ok ? p.y : 0.0f;
  pr.Z0 = ok ? p.z : 1.0f;
  pr.iz = ok ? iz : 0.0f;
  pr.xp = ok ? p.x * iz : 0.0f;
  pr.yp = ok ? p.y * iz : 0.0f;
}

// The template registers of cache entry e: all 8 samples, or (PR4 variants)
// the four of thread `sub` of the point's pair.
__device__ __forceinline__ void load_template(const TrackArgs& a, int64_t e, int, PointRegs& pr) {
  const float4* q0 = reinterpret_cast<const float4*>(a.ref.I0 + e * 8);
  const float4* qx = reinterpret_cast<const float4*>(a.ref.gx + e * 8);
  const float4* qy = reinterpret_cast<const float4*>(a.ref.gy + e * 8);
  const float4 a0 = gload(q0), a1 = gload(q0 + 1), b0 = gload(qx), b1 = gload(qx + 1), c0 = gload(qy),
               c1 = gload(qy + 1);
  const float t0[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  const float t1[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  const float t2[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) pr.i0_[k] = t0[k], pr.gx_[k] = t1[k], pr.gy_[k] = t2[k];
}

__device__ __forceinline__ void load_template(const TrackArgs& a, int64_t e, int sub, PointRegs4& pr) {
  const float4 a0 = gload(reinterpret_cast<const float4*>(a.ref.I0 + e * 8) + sub);
  const float4 b0 = gload(reinterpret_cast<const float4*>(a.ref.gx + e * 8) + sub);
  const float4 c0 = gload(reinterpret_cast<const float4*>(a.ref.gy + e * 8) + sub);
  pr.i0_[0] = a0.x, pr.i0_[1] = a0.y, pr.i0_[2] = a0.z, pr.i0_[3] = a0.w;
  pr.gx_[0] = b0.x, pr.gx_[1] = b0.y, pr.gx_[2] = b0.z, pr.gx_[3] = b0.w;
  pr.gy_[0] = c0.x, pr.gy_[1] = c0.y, pr.gy_[2] = c0.z, pr.gy_[3] = c0.w;
}

__device__ __forceinline__ void load_template(const TrackArgs& a, int64_t e, int sub, PointRegsH4& pr) {
  const uint2 h = gload(reinterpret_cast<const uint2*>(a.ref.I0h + e * 8) + sub);
  const uint4 g = gload(reinterpret_cast<const uint4*>(a.ref.gh + e * 8) + sub);
  const uint32_t hw[2] = {h.x, h.y};
  const uint32_t gw[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    pr.i0_[2 * k] = __ushort_as_half((unsigned short)(hw[k] & 0xffffu));
    pr.i0_[2 * k + 1] = __ushort_as_half((unsigned short)(hw[k] >> 16));
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    __half2 v;
    __builtin_memcpy(&v, &gw[k], 4);
    pr.g_[k] = v;
  }
}

__device__ __forceinline__ void load_template(const TrackArgs& a, int64_t e, int, PointRegsH& pr) {
  const uint4 h = gload(reinterpret_cast<const uint4*>(a.ref.I0h + e * 8));
  const uint4* q = reinterpret_cast<const uint4*>(a.ref.gh + e * 8);
  const uint4 g0 = gload(q), g1 = gload(q + 1);
  const uint32_t hw[4] = {h.x, h.y, h.z, h.w};
  const uint32_t gw[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pr.i0_[2 * k] = __ushort_as_half((unsigned short)(hw[k] & 0xffffu));
    pr.i0_[2 * k + 1] = __ushort_as_half((unsigned short)(hw[k] >> 16));
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    __half2 v;
    __builtin_memcpy(&v, &gw[k], 4);
    pr.g_[k] = v;
  }
}

// Point i's registers for level l: one thread per point (sub ignored), or
// thread `sub` (0 or 1) of the point's pair for the PR4 variants.
template <class PR>
__device__ __forceinline__ void load_point(const TrackArgs& a, int l, int i, int sub, PR& pr) {
  float4 p;
  int64_t e;
  const bool ok = load_geometry(a, l, i, p, e);
  set_geometry(pr, ok, p);
  load_template(a, e, sub, pr);
}

template <class PR>
__device__ __forceinline__ void load_point(const TrackArgs& a, int l, int i, PR& pr) {
  load_point(a, l, i, 0, pr);
}

// As load_point, with the geometry left as loaded (r): the cooperative kernel
// issues these loads, then its level tile's copy, and only then waits for them
// (finish_geometry), so both latencies overlap.
template <class PR>
__device__ __forceinline__ void load_point_raw(const TrackArgs& a, int l, int i, int sub, PR& pr, GeoRaw& r) {
  int64_t e;
  load_geometry_raw(a, l, i, r, e);
  load_template(a, e, sub, pr);
}

// The wait for the geometry words happens here (the empty asm reads them), not
// earlier: the compiler may not compute with them before this point.
template <class PR>
__device__ __forceinline__ void finish_geometry(PR& pr, GeoRaw& r) {
  asm volatile("" : "+v"(r.x), "+v"(r.y), "+v"(r.z), "+v"(r.valid) : : "memory");
  set_geometry(pr, r.in & (r.valid != 0), make_float4(r.x, r.y, r.z, 0.0f));
}

// Add one point's normal-equation terms (Eq.(2), Eq.(5)) at relative pose T.
// The K samples share the point's 2x6 warp Jacobian Jw with rows au, av, so with
// J_k = gx_k au + gy_k av:
//   H_i = m00 au^T au + m01 (au^T av + av^T au) + m11 av^T av,   b_i = -(v0 au + v1 av),
// m = sum_k w_k g_k^T g_k, v = sum_k w_k g_k r_k (five FMAs per sample, the
// 21-term product once per point).  Huber weight w = min(1, k/|r|).
// Branch-free: a point that is not usable (reference-invalid, behind the
// camera or a pattern position outside the level) runs the same instructions
// with its taps at the level's first pixels and its sums and counts masked to
// zero, so no exit path has to materialise a zeroed accumulator.
// GLOBAL_IMG: `img` is device global memory (loads compile to global_load);
// otherwise it may be LDS.
// NV = 32: robust mode, the kSlot* layout.  NV = kFixSlots: fixed-H mode, no
// weights (w = 1, cost r^2 / 2) and only b, E and the counts (kFix* layout).
template <bool COST_ONLY, bool GLOBAL_IMG, class PR, int NV = 32>
__device__ __forceinline__ void accumulate_point(const TrackArgs& a, const PatRegs& pat, const LevelGeom& g,
                                                 const uint8_t* __restrict__ img, const float* T,
                                                 const PR& pr, float (&acc)[NV]) {
  constexpr bool FIXED = NV == kFixSlots;
  static_assert(NV == 32 || FIXED, "slot layout");
  constexpr int sE = FIXED ? kFixE : kSlotE, sN = FIXED ? kFixN : kSlotN, sP = FIXED ? kFixPts : kSlotPts;
  const float kH = FIXED ? 0.0f : a.huber_k;
  float X, Y, Z;
  transform(T, pr.X0, pr.Y0, pr.Z0, X, Y, Z);
  float u, v;
  project(g, X, Y, Z, u, v);
  const bool ok = pr.ok & (Z > a.z_min) & inside(g, pat, u, v);
  // An unusable point continues from (0, 0): finite, integer sample positions
  // (zero bilinear fractions) and a tap offset forced to 0.
  u = ok ? u : 0.0f;
  v = ok ? v : 0.0f;
  // Phase 1: all 32 bilinear taps of the point are issued before any is used
  // (one memory round trip per point instead of one per sample).
  const Cell q0 = cell_of(u, v);
  float t00[8], t10[8], t01[8], t11[8];
  const int W = g.W;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int off = ((q0.iv + (int)pat.dy[k]) * W + q0.iu + (int)pat.dx[k]) & -(int)ok;  // masked, not branched
    if constexpr (GLOBAL_IMG) {
      const __attribute__((address_space(1))) uint8_t* p =
          (const __attribute__((address_space(1))) uint8_t*)img + off;
      t00[k] = p[0], t10[k] = p[1], t01[k] = p[W], t11[k] = p[W + 1];
    } else {
      const uint8_t* p = img + off;
      t00[k] = p[0], t10[k] = p[1], t01[k] = p[W], t11[k] = p[W + 1];
    }
  }
  // Phase 2: residuals, Huber weights and the point's sums.  The interpolation
  // repeats the precompute's arithmetic exactly.
  float m00 = 0.f, m01 = 0.f, m11 = 0.f, v0 = 0.f, v1 = 0.f, E = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float Ic = bilin_mix(q0.w, t00[k], t10[k], t01[k], t11[k]);
    const float r = pr.i0(k) - Ic;
    const float ar = fabsf(r);
    const bool hub = (kH > 0.f) & (ar > kH);
    const float w = hub ? kH * __builtin_amdgcn_rcpf(ar) : 1.0f;  // v_rcp_f32, 1 ulp
    const float rho = hub ? kH * (ar - 0.5f * kH) : 0.5f * r * r;
    E += rho;
    if (!COST_ONLY) {
      const float gx = pr.gx(k), gy = pr.gy(k);
      if (FIXED) {
        v0 = fmaf(gx, r, v0);
        v1 = fmaf(gy, r, v1);
      } else {
        const float wgx = w * gx, wgy = w * gy;
        m00 = fmaf(wgx, gx, m00);
        m01 = fmaf(wgx, gy, m01);
        m11 = fmaf(wgy, gy, m11);
        v0 = fmaf(wgx, r, v0);
        v1 = fmaf(wgy, r, v1);
      }
    }
  }
  acc[sE] += ok ? E : 0.0f;
  acc[sN] += ok ? 8.0f : 0.0f;
  acc[sP] += ok ? 1.0f : 0.0f;
  if (COST_ONLY) return;
  v0 = ok ? v0 : 0.0f, v1 = ok ? v1 : 0.0f;
  const float iz = pr.iz, xp = pr.xp, yp = pr.yp;
  const float au[6] = {-g.fx * xp * yp, g.fx * fmaf(xp, xp, 1.0f), -g.fx * yp, g.fx * iz, 0.0f, -g.fx * xp * iz};
  const float av[6] = {-g.fy * fmaf(yp, yp, 1.0f), g.fy * xp * yp, g.fy * xp, 0.0f, g.fy * iz, -g.fy * yp * iz};
  if constexpr (FIXED) {
#pragma unroll
    for (int r = 0; r < 6; ++r) acc[kFixB + r] -= fmaf(au[r], v0, av[r] * v1);
  } else {
    m00 = ok ? m00 : 0.0f, m01 = ok ? m01 : 0.0f, m11 = ok ? m11 : 0.0f;
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

// ---------------------------------------------------------------- LDS-staged accumulation (K = 8)

// The bytes of the current level a workgroup holds in LDS: rows lo..hi
// (inclusive), each W bytes, byte (r, x) of the level at offset
// delta + (r - lo) * W + x.  `bytes` is how many are valid from the start.
struct Tile8 {
  const __attribute__((address_space(3))) uint8_t* lds;
  int lo, hi, delta, bytes;
};

// Byte offset in the level of the pattern's sample k relative to its base
// pixel: dy_k * W + dx_k, the same for every point of the level.
__device__ __forceinline__ void pattern_offsets(const PatRegs& pat, int W, int (&off)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) off[k] = (int)pat.dy[k] * W + (int)pat.dx[k];
}

// The scalar track parameters an iteration reads, copied to registers once
// per launch: the cooperative kernel keeps its TrackArgs in LDS, where a field
// read after a workgroup barrier is an LDS round trip on the iteration's path.
struct IterParams {
  float huber_k, z_min, step_eps;
  int max_iters, min_points;
  __device__ explicit IterParams(const TrackArgs& a)
      : huber_k(a.huber_k), z_min(a.z_min), step_eps(a.step_eps), max_iters(a.max_iters), min_points(a.min_points) {}
};

// accumulate_point for the 8-pixel pattern, with the taps read from the
// workgroup's LDS copy of the level where every point of the wave lies inside
// it (else from global memory, as accumulate_point).  The pattern offsets are
// whole pixels, so all 8 samples share the point's bilinear fractions: the
// weights are formed once per point.  COST_ONLY: only the cost and the counts
// (the final pass).  Otherwise the Gauss-Newton terms and the point count, no
// cost (it is read only after the final pass; the sample count is 8 per point).
//
// NS = 4: the point has two threads, this one (first = false for the second of
// the pair) taking four of its samples with their offsets `off`.  Each adds its
// own samples' normal-equation terms, which sum to the point's (the terms are
// linear in m and v); the first thread counts the point.
template <bool COST_ONLY, class PR, int NV = 32, int NS = 8>
__device__ __forceinline__ void accumulate_point8(const IterParams& a, const PatRegs& pat, const int (&off)[NS],
                                                  const LevelGeom& g, const uint8_t* __restrict__ img,
                                                  const Tile8& tile, const float* T, const PR& pr,
                                                  float (&acc)[NV], bool first = true) {
  constexpr bool FIXED = NV == kFixSlots;
  static_assert(NV == 32 || FIXED, "slot layout");
  constexpr int sE = FIXED ? kFixE : kSlotE, sN = FIXED ? kFixN : kSlotN, sP = FIXED ? kFixPts : kSlotPts;
  const float kH = FIXED ? 0.0f : a.huber_k;
  // Huber weight min(1, k / |r|); without a threshold every weight is 1
  const float kHw = kH > 0.0f ? kH : __builtin_inff();
  float X, Y, Z;
  transform(T, pr.X0, pr.Y0, pr.Z0, X, Y, Z);
  float u, v;
  project(g, X, Y, Z, u, v);
  const bool ok = pr.ok & (Z > a.z_min) & inside(g, pat, u, v);
  u = ok ? u : 0.0f;
  v = ok ? v : 0.0f;
  const Cell q0 = cell_of(u, v);
  const int iu = q0.iu, iv = q0.iv, W = g.W;
  float t00[NS], t10[NS], t01[NS], t11[NS];
  const bool in_tile = !ok | ((iv + (int)pat.dy_min >= tile.lo) & (iv + (int)pat.dy_max + 1 <= tile.hi));
  if (__all(in_tile)) {
    // Every usable point of the wave lies inside the tile.  An unusable one
    // reads from the tile position of a pattern whose top-left sample sits at
    // the tile's first byte: a few rows, inside the allocation whatever the
    // level, and masked below.  All 16 pairs of words are requested before any
    // is used (one LDS round trip per point).
    const uint32_t lb = (uint32_t)(uintptr_t)tile.lds;
    const int base = (int)lb + tile.delta +
                     (ok ? (iv - tile.lo) * W + iu : -((int)pat.dy_min * W + (int)pat.dx_min));
    uint32_t w[NS][4];
    int bt[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      bt[k] = base + off[k];
      const __attribute__((address_space(3))) uint32_t* p =
          (const __attribute__((address_space(3))) uint32_t*)(uintptr_t)(uint32_t)(bt[k] & ~3);
      const __attribute__((address_space(3))) uint32_t* q =
          (const __attribute__((address_space(3))) uint32_t*)(uintptr_t)(uint32_t)((bt[k] + W) & ~3);
      w[k][0] = p[0], w[k][1] = p[1], w[k][2] = q[0], w[k][3] = q[1];
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t top = __builtin_amdgcn_alignbyte(w[k][1], w[k][0], (uint32_t)bt[k]);
      const uint32_t bot = __builtin_amdgcn_alignbyte(w[k][3], w[k][2], (uint32_t)(bt[k] + W));
      t00[k] = (float)(top & 0xffu), t10[k] = (float)((top >> 8) & 0xffu);
      t01[k] = (float)(bot & 0xffu), t11[k] = (float)((bot >> 8) & 0xffu);
    }
  } else {
    const __attribute__((address_space(1))) uint8_t* gimg = (const __attribute__((address_space(1))) uint8_t*)img;
    const int base = iv * W + iu;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int o = ok ? base + off[k] : 0;  // an unusable point reads the level's first pixels
      t00[k] = gimg[o], t10[k] = gimg[o + 1], t01[k] = gimg[o + W], t11[k] = gimg[o + W + 1];
    }
  }
  float m00 = 0.f, m01 = 0.f, m11 = 0.f, v0 = 0.f, v1 = 0.f, E = 0.f;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const float Ic = bilin_mix(q0.w, t00[k], t10[k], t01[k], t11[k]);
    const float r = pr.i0(k) - Ic;
    if constexpr (COST_ONLY) {
      const float ar = fabsf(r);
      const bool hub = (kH > 0.f) & (ar > kH);
      E += hub ? kH * (ar - 0.5f * kH) : 0.5f * r * r;
    } else {
      const float gx = pr.gx(k), gy = pr.gy(k);
      if constexpr (FIXED) {
        v0 = fmaf(gx, r, v0);
        v1 = fmaf(gy, r, v1);
      } else {
        const float w = fminf(1.0f, kHw * __builtin_amdgcn_rcpf(fabsf(r)));
        const float wgx = w * gx, wgy = w * gy;
        m00 = fmaf(wgx, gx, m00);
        m01 = fmaf(wgx, gy, m01);
        m11 = fmaf(wgy, gy, m11);
        v0 = fmaf(wgx, r, v0);
        v1 = fmaf(wgy, r, v1);
      }
    }
  }
  acc[sP] += (ok & first) ? 1.0f : 0.0f;
  if constexpr (COST_ONLY) {
    acc[sE] += ok ? E : 0.0f;
    acc[sN] += ok ? (float)NS : 0.0f;
    return;
  }
  v0 = ok ? v0 : 0.0f, v1 = ok ? v1 : 0.0f;
  const float izr = pr.iz, xp = pr.xp, yp = pr.yp;
  const float au[6] = {-g.fx * xp * yp, g.fx * fmaf(xp, xp, 1.0f), -g.fx * yp, g.fx * izr, 0.0f, -g.fx * xp * izr};
  const float av[6] = {-g.fy * fmaf(yp, yp, 1.0f), g.fy * xp * yp, g.fy * xp, 0.0f, g.fy * izr, -g.fy * yp * izr};
  if constexpr (FIXED) {
#pragma unroll
    for (int r = 0; r < 6; ++r) acc[kFixB + r] -= fmaf(au[r], v0, av[r] * v1);
  } else {
    m00 = ok ? m00 : 0.0f, m01 = ok ? m01 : 0.0f, m11 = ok ? m11 : 0.0f;
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

// ---------------------------------------------------------------- generic-K cooperative accumulation

// Patterns other than the 8-pixel one (p x p patches) and the floating-point
// pyramid: four lanes share a point, lane `sub` of the quad taking samples
// sub, sub + 4, ... < K, so a 49-sample patch costs each lane 13 samples.  The
// quad's partial sums are combined with DPP quad permutations and lane 0 of the
// quad adds the point's normal-equation terms.
struct PointGeo {
  float X0, Y0, Z0;
  float iz, xp, yp;
  int64_t s0;  // cache index of the point's sample 0 at the level
  bool ok;
};

__device__ __forceinline__ void load_point_geo(const TrackArgs& a, int l, int i, PointGeo& pg) {
  float4 p;
  int64_t e;
  const bool ok = load_geometry(a, l, i, p, e);
  set_geometry(pg, ok, p);
  pg.s0 = e * a.pat.K;
}

// DPP quad permutation (quad_perm selector), a VALU operand modifier.
template <int SEL>
__device__ __forceinline__ float dpp_quad(float v) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v), SEL, 0xf, 0xf, false));
}

// Sum over the four lanes of a quad, the same in every lane of it.
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp_quad<0xB1>(v);  // lanes [1, 0, 3, 2]
  v += dpp_quad<0x4E>(v);  // lanes [2, 3, 0, 1]
  return v;
}

// NV = 32: robust mode; NV = kFixSlots: fixed-H mode (no weights, b only), as
// accumulate_point.  PIX: uint8 levels or the floating-point Gaussian pyramid.
template <bool COST_ONLY, class PIX, int NV>
__device__ __forceinline__ void accumulate_point_generic(const TrackArgs& a, const Pattern& pat, const LevelGeom& g,
                                                         const PIX* __restrict__ img, const float* T,
                                                         const PointGeo& pg, int sub, float (&acc)[NV]) {
  constexpr bool FIXED = NV == kFixSlots;
  constexpr int sE = FIXED ? kFixE : kSlotE, sN = FIXED ? kFixN : kSlotN, sP = FIXED ? kFixPts : kSlotPts;
  const float kH = FIXED ? 0.0f : a.huber_k;
  float X, Y, Z;
  transform(T, pg.X0, pg.Y0, pg.Z0, X, Y, Z);
  float u, v;
  project(g, X, Y, Z, u, v);
  const bool ok = pg.ok & (Z > a.z_min) & inside(g, pat, u, v);
  u = ok ? u : 0.0f;
  v = ok ? v : 0.0f;
  const Cell q0 = cell_of(u, v);
  const int K = pat.K, W = g.W;
  const __attribute__((address_space(1))) PIX* gimg = (const __attribute__((address_space(1))) PIX*)img;
  float m00 = 0.f, m01 = 0.f, m11 = 0.f, v0 = 0.f, v1 = 0.f, E = 0.f;
  // Batches of four samples per lane: all their taps and cache entries are
  // issued before any is used.  A slot past the pattern reads sample 0 (always
  // in range) and is weighted by zero.
  constexpr int B = 4;
  for (int k0 = sub; k0 < K; k0 += B * kLanesPerPoint) {
    float t00[B], t10[B], t01[B], t11[B], i0[B], gxs[B], gys[B], msk[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int k = k0 + j * kLanesPerPoint;
      const bool has = k < K;
      const int kk = has ? k : 0;
      msk[j] = has ? 1.0f : 0.0f;
      // an unusable point reads the level's first taps
      const int off = ((q0.iv + (int)pat.dy[kk]) * W + q0.iu + (int)pat.dx[kk]) & -(int)ok;
      t00[j] = gimg[off], t10[j] = gimg[off + 1], t01[j] = gimg[off + W], t11[j] = gimg[off + W + 1];
      i0[j] = gload(a.ref.I0 + pg.s0 + kk);
      if (!COST_ONLY) gxs[j] = gload(a.ref.gx + pg.s0 + kk), gys[j] = gload(a.ref.gy + pg.s0 + kk);
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const float Ic = bilin_mix(q0.w, t00[j], t10[j], t01[j], t11[j]);
      const float r = i0[j] - Ic;
      const float ar = fabsf(r);
      const bool hub = (kH > 0.f) & (ar > kH);
      const float w = (hub ? kH * __builtin_amdgcn_rcpf(ar) : 1.0f) * msk[j];
      const float rho = hub ? kH * (ar - 0.5f * kH) : 0.5f * r * r;
      E = fmaf(msk[j], rho, E);
      if (!COST_ONLY) {
        const float wgx = w * gxs[j], wgy = w * gys[j];
        if (!FIXED) {
          m00 = fmaf(wgx, gxs[j], m00);
          m01 = fmaf(wgx, gys[j], m01);
          m11 = fmaf(wgy, gys[j], m11);
        }
        v0 = fmaf(wgx, r, v0);
        v1 = fmaf(wgy, r, v1);
      }
    }
  }
  const bool use = ok & (sub == 0);
  E = quad_sum(E);
  acc[sE] += use ? E : 0.0f;
  acc[sN] += use ? (float)K : 0.0f;
  acc[sP] += use ? 1.0f : 0.0f;
  if (COST_ONLY) return;
  v0 = quad_sum(v0);
  v1 = quad_sum(v1);
  v0 = use ? v0 : 0.0f, v1 = use ? v1 : 0.0f;
  const float iz = pg.iz, xp = pg.xp, yp = pg.yp;
  const float au[6] = {-g.fx * xp * yp, g.fx * fmaf(xp, xp, 1.0f), -g.fx * yp, g.fx * iz, 0.0f, -g.fx * xp * iz};
  const float av[6] = {-g.fy * fmaf(yp, yp, 1.0f), g.fy * xp * yp, g.fy * xp, 0.0f, g.fy * iz, -g.fy * yp * iz};
  if constexpr (FIXED) {
#pragma unroll
    for (int r = 0; r < 6; ++r) acc[kFixB + r] -= fmaf(au[r], v0, av[r] * v1);
  } else {
    m00 = quad_sum(m00);
    m01 = quad_sum(m01);
    m11 = quad_sum(m11);
    m00 = use ? m00 : 0.0f, m01 = use ? m01 : 0.0f, m11 = use ? m11 : 0.0f;
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

}  // namespace dpt
