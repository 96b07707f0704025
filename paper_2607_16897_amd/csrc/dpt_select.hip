// Map-point selection (stand-in for the map points the indirect pipeline
// provides): the n candidates with the largest integer gradient score
// s = (I[y][x+1] - I[y][x-1])^2 + (I[y+1][x] - I[y-1][x])^2 inside the margin,
// ties to the smaller linear index, written in ascending index order.
//
// Multi-workgroup pipeline over chunks of kSelChunk candidates (candidate c is
// pixel (m + c % Wc, m + c / Wc), so candidate order is index order):
//   A  per-chunk LDS histograms of s >> 9 (s <= 2 * 255^2 < 2^17), summed into a
//      global 256-bin histogram with integer atomics (order-independent)
//   B  one thread finds the coarse bucket of the n-th largest score
//   C  512-bin histogram of the low bits inside that bucket
//   D  one thread finds the exact threshold T and how many ties `need` to keep
//   E  per-chunk counts of scores > T and == T
//   F  one workgroup turns them into per-chunk output offsets and tie bases
//   G  each chunk writes its selected indices with a block-wide prefix sum
#include "dpt_device.h"

namespace dpt {

constexpr int kSelThreads = 256, kSelPPT = 16, kSelChunk = kSelThreads * kSelPPT;

struct SelScratch {  // layout of the int32 scratch buffer
  static constexpr int kHist1 = 0, kHist2 = 256, kParams = 768, kChunks = 776;
};

int64_t select_scratch_ints(int32_t W, int32_t H) {
  const int64_t G = ((int64_t)W * H + kSelChunk - 1) / kSelChunk + 1;
  return SelScratch::kChunks + 4 * G;
}

__device__ __forceinline__ int sel_score(const uint8_t* img, int W, int x, int y) {
  const uint8_t* p = img + y * W + x;
  const int dx = (int)p[1] - (int)p[-1];
  const int dy = (int)p[W] - (int)p[-W];
  return dx * dx + dy * dy;
}

struct SelGeom {
  const uint8_t* img;
  int W, m, Wc, C, n;
};

__device__ __forceinline__ int cand_score(const SelGeom& g, int c) {
  return sel_score(g.img, g.W, g.m + c % g.Wc, g.m + c / g.Wc);
}

__global__ __launch_bounds__(kSelThreads) void sel_hist_coarse(SelGeom g, int* __restrict__ sc) {
  __shared__ int h[256];
  for (int b = threadIdx.x; b < 256; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int c0 = blockIdx.x * kSelChunk;
  for (int q = threadIdx.x; q < kSelChunk; q += blockDim.x) {
    const int c = c0 + q;
    if (c < g.C) atomicAdd(&h[cand_score(g, c) >> 9], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 256; b += blockDim.x)
    if (h[b]) atomicAdd(&sc[SelScratch::kHist1 + b], h[b]);
}

__global__ void sel_find_coarse(SelGeom g, int* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  int* prm = sc + SelScratch::kParams;
  if (g.C <= g.n) {  // take every candidate
    prm[0] = -1, prm[1] = 0, prm[2] = -1, prm[3] = 0;
    return;
  }
  int cum = 0, B = 0;
  for (int b = 255; b >= 0; --b) {
    const int hb = sc[SelScratch::kHist1 + b];
    if (cum + hb >= g.n) {
      B = b;
      break;
    }
    cum += hb;
  }
  prm[0] = B, prm[1] = cum;
}

__global__ __launch_bounds__(kSelThreads) void sel_hist_fine(SelGeom g, int* __restrict__ sc) {
  const int B = sc[SelScratch::kParams];
  if (B < 0) return;
  __shared__ int h[512];
  for (int b = threadIdx.x; b < 512; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int c0 = blockIdx.x * kSelChunk;
  for (int q = threadIdx.x; q < kSelChunk; q += blockDim.x) {
    const int c = c0 + q;
    if (c < g.C) {
      const int s = cand_score(g, c);
      if ((s >> 9) == B) atomicAdd(&h[s & 511], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 512; b += blockDim.x)
    if (h[b]) atomicAdd(&sc[SelScratch::kHist2 + b], h[b]);
}

__global__ void sel_find_fine(SelGeom g, int* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  int* prm = sc + SelScratch::kParams;
  const int B = prm[0];
  if (B < 0) return;
  int cum = prm[1], T = B * 512, need = 0;
  for (int f = 511; f >= 0; --f) {
    const int hf = sc[SelScratch::kHist2 + f];
    if (cum + hf >= g.n) {
      T = B * 512 + f;
      need = g.n - cum;
      break;
    }
    cum += hf;
  }
  prm[2] = T, prm[3] = need;
}

__global__ __launch_bounds__(kSelThreads) void sel_count(SelGeom g, int* __restrict__ sc) {
  __shared__ int s_gt[kSelThreads / 64], s_eq[kSelThreads / 64];
  const int T = sc[SelScratch::kParams + 2];
  const int c0 = blockIdx.x * kSelChunk;
  int gt = 0, eq = 0;
  for (int q = threadIdx.x; q < kSelChunk; q += blockDim.x) {
    const int c = c0 + q;
    if (c < g.C) {
      const int s = cand_score(g, c);
      gt += s > T;
      eq += s == T;
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    gt += __shfl_xor(gt, d, 64);
    eq += __shfl_xor(eq, d, 64);
  }
  if ((threadIdx.x & 63) == 0) s_gt[threadIdx.x >> 6] = gt, s_eq[threadIdx.x >> 6] = eq;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) a += s_gt[w], b += s_eq[w];
    sc[SelScratch::kChunks + 4 * blockIdx.x] = a;
    sc[SelScratch::kChunks + 4 * blockIdx.x + 1] = b;
  }
}

// per-chunk tie base and output offset (chunk order = index order), and the count
__global__ void sel_offsets(int G, int* __restrict__ sc, int32_t* __restrict__ count) {
  if (threadIdx.x != 0) return;
  const int need = sc[SelScratch::kParams + 3];
  int tie = 0, out = 0;
  for (int k = 0; k < G; ++k) {
    int* e = sc + SelScratch::kChunks + 4 * k;
    const int gt = e[0], eq = e[1];
    int take = need - tie;
    take = take < 0 ? 0 : (take > eq ? eq : take);
    e[2] = tie;
    e[3] = out;
    tie += eq;
    out += gt + take;
  }
  *count = out;
}

__global__ __launch_bounds__(kSelThreads) void sel_write(SelGeom g, const int* __restrict__ sc,
                                                         int32_t* __restrict__ idx) {
  __shared__ int wsum[16];
  const int T = sc[SelScratch::kParams + 2], need = sc[SelScratch::kParams + 3];
  const int* e = sc + SelScratch::kChunks + 4 * blockIdx.x;
  const int c0 = blockIdx.x * kSelChunk + threadIdx.x * kSelPPT;
  int s[kSelPPT];
  int eq_local = 0;
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j) {
    const int c = c0 + j;
    s[j] = c < g.C ? cand_score(g, c) : -2;
    eq_local += s[j] == T;
  }
  int tot;
  int tie = block_exclusive_scan(eq_local, wsum, &tot) + e[2];
  bool sel[kSelPPT];
  int sel_local = 0;
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j) {
    const bool is_eq = s[j] == T;
    sel[j] = (s[j] > T) || (is_eq && tie < need);
    tie += is_eq;
    sel_local += sel[j];
  }
  int pos = block_exclusive_scan(sel_local, wsum, &tot) + e[3];
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j)
    if (sel[j]) {
      const int c = c0 + j;
      idx[pos++] = (g.m + c / g.Wc) * g.W + (g.m + c % g.Wc);
    }
}

hipError_t launch_select(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                         int32_t* count, int32_t* scratch, hipStream_t s) {
  SelGeom g;
  g.img = img;
  g.W = W;
  g.m = margin;
  g.Wc = W - 2 * margin;
  const int Hc = H - 2 * margin;
  g.C = (g.Wc > 0 && Hc > 0) ? g.Wc * Hc : 0;
  g.n = n;
  const int G = (g.C + kSelChunk - 1) / kSelChunk;
  hipError_t e = hipMemsetAsync(scratch, 0, sizeof(int32_t) * SelScratch::kChunks, s);
  if (e != hipSuccess) return e;
  if (G == 0) return hipMemsetAsync(count, 0, sizeof(int32_t), s);
  hipLaunchKernelGGL(sel_hist_coarse, dim3(G), dim3(kSelThreads), 0, s, g, scratch);
  hipLaunchKernelGGL(sel_find_coarse, dim3(1), dim3(64), 0, s, g, scratch);
  hipLaunchKernelGGL(sel_hist_fine, dim3(G), dim3(kSelThreads), 0, s, g, scratch);
  hipLaunchKernelGGL(sel_find_fine, dim3(1), dim3(64), 0, s, g, scratch);
  hipLaunchKernelGGL(sel_count, dim3(G), dim3(kSelThreads), 0, s, g, scratch);
  hipLaunchKernelGGL(sel_offsets, dim3(1), dim3(64), 0, s, G, scratch, count);
  hipLaunchKernelGGL(sel_write, dim3(G), dim3(kSelThreads), 0, s, g, scratch, idx);
  return hipGetLastError();
}

}  // namespace dpt
