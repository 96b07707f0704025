// Learned initialiser: a small CNN that proposes the reference-to-current
// twist from the coarsest pyramid pair (60 x 94, two channels), replacing the
// constant-velocity start of the coarse-to-fine Gauss-Newton track.
//
// Network: four 3x3 stride-2 padding-1 convolutions with ReLU (2-16-32-64-64
// channels), global average pool, FC 64-64 ReLU, FC 64-6.  Activations and
// convolution weights are BF16 in NHWC / [co][ky][kx][ci] layouts; the
// forward convolutions are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation) with bias and ReLU fused in
// the epilogue.  Pooling, the FC layers, the loss, the backward pass (FP32
// accumulation from the BF16 operands, split reductions summed in a fixed
// order) and Adam run on the vector units; master weights and Adam moments
// are FP32.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/dptrack.h"
#include "dpt_internal.h"

struct dpt_cnn;

namespace dpt {
namespace cnn {

constexpr int kH0 = 60, kW0 = 94;
constexpr int kC[5] = {2, 16, 32, 64, 64};
constexpr int kHs[5] = {60, 30, 15, 8, 4};
constexpr int kWs[5] = {94, 47, 24, 12, 6};
constexpr int kHidden = 64, kOut = 6;

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- layout
// Flat FP32 parameter vector, tensor order w1 b1 w2 b2 w3 b3 w4 b4 fw1 fb1 fw2 fb2.
// Conv weights are stored [co][ky][kx][ci] internally; the ABI uses [co][ci][ky][kx].
struct Offsets {
  int w[4], b[4], fw1, fb1, fw2, fb2, total;
};

__host__ __device__ inline Offsets offsets() {
  Offsets o{};
  int s = 0;
  for (int l = 0; l < 4; ++l) {
    o.w[l] = s;
    s += kC[l + 1] * kC[l] * 9;
    o.b[l] = s;
    s += kC[l + 1];
  }
  o.fw1 = s;
  s += kHidden * 64;
  o.fb1 = s;
  s += kHidden;
  o.fw2 = s;
  s += kOut * kHidden;
  o.fb2 = s;
  s += kOut;
  o.total = s;
  return o;
}

// ---------------------------------------------------------------- input

// uint8 pairs, planar [B][2][60][94] -> BF16 NHWC [B][60][94][2], (I - 128) / 64 (exact in BF16)
__global__ void input_from_pairs(const uint8_t* __restrict__ pairs, int B, uint16_t* __restrict__ x) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;  // pixel index over B*60*94
  if (p >= B * kH0 * kW0) return;
  const int b = p / (kH0 * kW0), r = p % (kH0 * kW0);
  for (int c = 0; c < 2; ++c)
    x[2 * p + c] = f2bf(((float)pairs[((size_t)b * 2 + c) * kH0 * kW0 + r] - 128.0f) * (1.0f / 64.0f));
}

// coarsest pyramid levels of stream pairs (ref[b], cur[b] device pointers) -> BF16 NHWC
__global__ void input_from_levels(const uint8_t* const* __restrict__ refs, const uint8_t* const* __restrict__ curs,
                                  int B, uint16_t* __restrict__ x) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B * kH0 * kW0) return;
  const int b = p / (kH0 * kW0), r = p % (kH0 * kW0);
  x[2 * p] = f2bf(((float)refs[b][r] - 128.0f) * (1.0f / 64.0f));
  x[2 * p + 1] = f2bf(((float)curs[b][r] - 128.0f) * (1.0f / 64.0f));
}

// ---------------------------------------------------------------- forward convolution (MFMA)

// Implicit GEMM: rows m = output pixels (b, i, j), columns n = output channels,
// k = (ky, kx, ci).  A wave computes 16 rows x CO columns with CO/16 MFMA tiles;
// lane L supplies A[m0 + L%16][k0 + 4(L/16) .. +3] and B[k0 + 4(L/16) .. +3][n0 + L%16]
// and receives D[4(L/16) + j][L%16].
template <int CI, int CO>
__global__ __launch_bounds__(256) void conv_fwd_mfma(const uint16_t* __restrict__ x, int H, int W, int Ho, int Wo,
                                                     int B, const uint16_t* __restrict__ w,
                                                     const float* __restrict__ bias, uint16_t* __restrict__ y) {
  constexpr int K = 9 * CI, KP = (K + 15) / 16 * 16, NT = CO / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int M = B * Ho * Wo;
  const int m0 = (blockIdx.x * 4 + wave) * 16;
  const int m = m0 + (lane & 15);
  const int kq = lane >> 4;
  const bool mvalid = m < M;
  const int b = mvalid ? m / (Ho * Wo) : 0, ij = mvalid ? m % (Ho * Wo) : 0;
  const int i = ij / Wo, j = ij % Wo;
  float4_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KP / 16; ++ks) {
    const int k0 = ks * 16 + 4 * kq;
    short4_t a;
    if constexpr (CI % 4 == 0) {
      const int tap = k0 / CI, c = k0 % CI;
      const int yy = 2 * i + tap / 3 - 1, xx = 2 * j + tap % 3 - 1;
      uint2 v = make_uint2(0u, 0u);
      if (mvalid && yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = *reinterpret_cast<const uint2*>(x + (((size_t)b * H + yy) * W + xx) * CI + c);
      a = short4_t{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
    } else {
      short e[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = k0 + t;
        uint16_t v = 0;
        if (k < K && mvalid) {
          const int tap = k / CI, c = k % CI;
          const int yy = 2 * i + tap / 3 - 1, xx = 2 * j + tap % 3 - 1;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = x[(((size_t)b * H + yy) * W + xx) * CI + c];
        }
        e[t] = (short)v;
      }
      a = short4_t{e[0], e[1], e[2], e[3]};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + (lane & 15);
      short4_t bv;
      if constexpr (CI % 4 == 0) {
        const uint2 v = *reinterpret_cast<const uint2*>(w + (size_t)n * K + k0);
        bv = short4_t{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
      } else {
        short e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = (k0 + q < K) ? (short)w[(size_t)n * K + k0 + q] : (short)0;
        bv = short4_t{e[0], e[1], e[2], e[3]};
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = t * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int mo = m0 + 4 * kq + q;
      if (mo < M) y[(size_t)mo * CO + n] = f2bf(fmaxf(acc[t][q] + bias[n], 0.0f));
    }
  }
}

// ---------------------------------------------------------------- pool + FC (+ loss and its backward)

// One 64-thread workgroup per sample: g = mean(a4), h1 = relu(fw1 g + fb1),
// out = fw2 h1 + fb2.  With targets, also the squared error, dout and the FC /
// pool backward down to dZ4 = dA4 * (a4 > 0); per-sample FC weight gradients go
// to `fcg` [B][fc params] and are summed over the batch in a fixed order later.
__global__ __launch_bounds__(64) void head_kernel(const uint16_t* __restrict__ a4, const float* __restrict__ P,
                                                  const float* __restrict__ targets, int B, float* __restrict__ out,
                                                  float* __restrict__ sqerr, float* __restrict__ fcg,
                                                  float* __restrict__ dz4) {
  const Offsets o = offsets();
  const int b = blockIdx.x, t = threadIdx.x;
  __shared__ float g[64], h1[64], dout[kOut], dz1[64];
  constexpr int HW = 4 * 6;
  const uint16_t* a = a4 + (size_t)b * HW * 64;
  float s = 0.f;
  for (int p = 0; p < HW; ++p) s += bf2f(a[p * 64 + t]);
  g[t] = s * (1.0f / HW);
  __syncthreads();
  float z = P[o.fb1 + t];
  for (int q = 0; q < 64; ++q) z = fmaf(P[o.fw1 + t * 64 + q], g[q], z);
  h1[t] = fmaxf(z, 0.f);
  __syncthreads();
  if (t < kOut) {
    float v = P[o.fb2 + t];
    for (int q = 0; q < kHidden; ++q) v = fmaf(P[o.fw2 + t * kHidden + q], h1[q], v);
    out[b * kOut + t] = v;
    if (targets) {
      const float d = v - targets[b * kOut + t];
      dout[t] = 2.0f * d / (float)(B * kOut);
      sqerr[b * kOut + t] = d * d;
    }
  }
  if (!targets) return;
  __syncthreads();
  // FC gradients of this sample (fixed layout: fw1, fb1, fw2, fb2 relative to o.fw1)
  float* G = fcg + (size_t)b * (o.total - o.fw1);
  for (int q = t; q < kOut * kHidden; q += 64) G[o.fw2 - o.fw1 + q] = dout[q / kHidden] * h1[q % kHidden];
  if (t < kOut) G[o.fb2 - o.fw1 + t] = dout[t];
  float dh = 0.f;
  for (int q = 0; q < kOut; ++q) dh = fmaf(P[o.fw2 + q * kHidden + t], dout[q], dh);
  dz1[t] = h1[t] > 0.f ? dh : 0.f;
  __syncthreads();
  for (int q = 0; q < 64; ++q) G[t * 64 + q] = dz1[t] * g[q];
  G[o.fb1 - o.fw1 + t] = dz1[t];
  float dg = 0.f;
  for (int q = 0; q < kHidden; ++q) dg = fmaf(P[o.fw1 + q * 64 + t], dz1[q], dg);
  dg *= (1.0f / HW);
  for (int p = 0; p < HW; ++p) dz4[((size_t)b * HW + p) * 64 + t] = bf2f(a[p * 64 + t]) > 0.f ? dg : 0.f;
}

// ---------------------------------------------------------------- backward convolution

// dX for one layer, fused with the ReLU mask of the layer below:
// dZprev[b][y][x][c] = (a_prev > 0) * sum_{ky,kx,o} W[o][ky][kx][c] dZ[b][i][j][o],
// with 2i + ky - 1 = y, 2j + kx - 1 = x.  One thread per (b, y, x, c).
template <int CI, int CO>
__global__ void conv_bwd_data(const float* __restrict__ dz, int Ho, int Wo, const uint16_t* __restrict__ w,
                              const uint16_t* __restrict__ aprev, int H, int W, int B, float* __restrict__ dzprev) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)B * H * W * CI) return;
  const int c = id % CI;
  const size_t pix = id / CI;
  const int xx = pix % W, yy = (pix / W) % H, b = pix / ((size_t)W * H);
  if (!(bf2f(aprev[id]) > 0.f)) {
    dzprev[id] = 0.f;
    return;
  }
  float s = 0.f;
  for (int ky = 0; ky < 3; ++ky) {
    const int ty = yy + 1 - ky;
    if (ty < 0 || (ty & 1) || (ty >> 1) >= Ho) continue;
    const int i = ty >> 1;
    for (int kx = 0; kx < 3; ++kx) {
      const int tx = xx + 1 - kx;
      if (tx < 0 || (tx & 1) || (tx >> 1) >= Wo) continue;
      const int j = tx >> 1;
      const float* d = dz + (((size_t)b * Ho + i) * Wo + j) * CO;
      const uint16_t* wk = w + (ky * 3 + kx) * CI + c;
      for (int o = 0; o < CO; ++o) s = fmaf(bf2f(wk[(size_t)o * 9 * CI]), d[o], s);
    }
  }
  dzprev[id] = s;
}

// dW and db, split over the batch: partial[split][co][ky][kx][ci] (then bias [co])
// = sum over samples b in the split and output pixels (i, j) of dZ * x_pad.
template <int CI, int CO>
__global__ void conv_bwd_weight(const float* __restrict__ dz, int Ho, int Wo, const uint16_t* __restrict__ x, int H,
                                int W, int B, int per_split, float* __restrict__ partial) {
  constexpr int NW = CO * 9 * CI, NP = NW + CO;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int split = blockIdx.y;
  if (e >= NP) return;
  const int b0 = split * per_split, b1 = min(B, b0 + per_split);
  float s = 0.f;
  if (e < NW) {
    const int c = e % CI, tap = (e / CI) % 9, o = e / (9 * CI);
    const int ky = tap / 3, kx = tap % 3;
    for (int b = b0; b < b1; ++b)
      for (int i = 0; i < Ho; ++i) {
        const int yy = 2 * i + ky - 1;
        if (yy < 0 || yy >= H) continue;
        for (int j = 0; j < Wo; ++j) {
          const int xx = 2 * j + kx - 1;
          if (xx < 0 || xx >= W) continue;
          s = fmaf(dz[(((size_t)b * Ho + i) * Wo + j) * CO + o], bf2f(x[(((size_t)b * H + yy) * W + xx) * CI + c]), s);
        }
      }
  } else {
    const int o = e - NW;
    for (int b = b0; b < b1; ++b)
      for (int p = 0; p < Ho * Wo; ++p) s += dz[((size_t)b * Ho * Wo + p) * CO + o];
  }
  partial[(size_t)split * NP + e] = s;
}

// grad[off + e] = sum_s partial[s][e], fixed order
__global__ void reduce_splits(const float* __restrict__ partial, int splits, int n, float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int q = 0; q < splits; ++q) s += partial[(size_t)q * n + e];
  grad[e] = s;
}

// sum over batch of the per-sample FC gradients (fixed order), and of the squared errors
__global__ void reduce_batch(const float* __restrict__ v, int B, int n, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += v[(size_t)b * n + e];
  out[e] = s;
}

// ---------------------------------------------------------------- Adam

// Adam (Kingma & Ba 2015) on the FP32 master weights with bias correction c1 =
// 1 - b1^t, c2 = 1 - b2^t; refreshes the BF16 conv weight copies.
__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                            float* __restrict__ V, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                            int conv_end, uint16_t* __restrict__ Pb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float g = G[e];
  const float m = b1 * M[e] + (1.0f - b1) * g;
  const float v = b2 * V[e] + (1.0f - b2) * g * g;
  M[e] = m;
  V[e] = v;
  const float p = P[e] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[e] = p;
  if (e < conv_end) Pb[e] = f2bf(p);
}

__global__ void to_bf16(const float* __restrict__ P, int n, uint16_t* __restrict__ Pb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) Pb[e] = f2bf(P[e]);
}

__global__ void bf16_to_f32(const uint16_t* __restrict__ a, size_t n, float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = bf2f(a[e]);
}

}  // namespace cnn
}  // namespace dpt

// ---------------------------------------------------------------- host

using namespace dpt;
using namespace dpt::cnn;

struct dpt_cnn {
  int32_t max_batch = 0;
  hipStream_t stream = nullptr;
  Offsets o;
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;  // FP32 master, gradient, Adam moments
  uint16_t* Pb = nullptr;                                          // BF16 copy (conv weights used)
  uint16_t* act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float *dz[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // dz[l]: gradient at layer l's output (pre-ReLU)
  float *out = nullptr, *tgt = nullptr, *sqerr = nullptr, *fcg = nullptr, *partial = nullptr, *scal = nullptr;
  uint8_t* pairs = nullptr;
  const uint8_t** d_lv = nullptr;  // [2][max_batch] level pointers
  int step = 0;
  float* h_buf = nullptr;  // pinned
  size_t partial_floats = 0;
  ~dpt_cnn() {
    for (void* p : {(void*)P, (void*)G, (void*)M, (void*)V, (void*)Pb, (void*)out, (void*)tgt, (void*)sqerr,
                    (void*)fcg, (void*)partial, (void*)scal, (void*)pairs, (void*)d_lv})
      if (p) (void)hipFree(p);
    for (int l = 0; l < 5; ++l) {
      if (act[l]) (void)hipFree(act[l]);
      if (dz[l]) (void)hipFree(dz[l]);
    }
    if (h_buf) (void)hipHostFree(h_buf);
  }
};

namespace {

int cfail(int code, const char* msg) { return set_error(code, msg); }

#define CNN_TRY(expr)                                          \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return cfail(DPT_E_HIP, #expr);      \
  } while (0)

constexpr int kSplitsMax = 256;

int splits_for(int l, int B) {
  // samples per split so that each thread loops over a few thousand terms
  const int per_sample = kHs[l + 1] * kWs[l + 1];
  int per = std::max(1, 4096 / per_sample);
  return (B + per - 1) / per;
}

int per_split_for(int l, int B) {
  const int per_sample = kHs[l + 1] * kWs[l + 1];
  return std::max(1, 4096 / per_sample);
}

hipError_t forward(dpt_cnn* c, int B) {
  const int M1 = B * kHs[1] * kWs[1], M2 = B * kHs[2] * kWs[2], M3 = B * kHs[3] * kWs[3], M4 = B * kHs[4] * kWs[4];
  auto grid = [](int M) { return dim3((M + 63) / 64); };
  hipLaunchKernelGGL((conv_fwd_mfma<2, 16>), grid(M1), dim3(256), 0, c->stream, c->act[0], kHs[0], kWs[0], kHs[1],
                     kWs[1], B, c->Pb + c->o.w[0], c->P + c->o.b[0], c->act[1]);
  hipLaunchKernelGGL((conv_fwd_mfma<16, 32>), grid(M2), dim3(256), 0, c->stream, c->act[1], kHs[1], kWs[1], kHs[2],
                     kWs[2], B, c->Pb + c->o.w[1], c->P + c->o.b[1], c->act[2]);
  hipLaunchKernelGGL((conv_fwd_mfma<32, 64>), grid(M3), dim3(256), 0, c->stream, c->act[2], kHs[2], kWs[2], kHs[3],
                     kWs[3], B, c->Pb + c->o.w[2], c->P + c->o.b[2], c->act[3]);
  hipLaunchKernelGGL((conv_fwd_mfma<64, 64>), grid(M4), dim3(256), 0, c->stream, c->act[3], kHs[3], kWs[3], kHs[4],
                     kWs[4], B, c->Pb + c->o.w[3], c->P + c->o.b[3], c->act[4]);
  return hipGetLastError();
}

template <int CI, int CO>
hipError_t bwd_layer(dpt_cnn* c, int l, int B) {
  const int Ho = kHs[l + 1], Wo = kWs[l + 1], H = kHs[l], W = kWs[l];
  const int NP = CO * 9 * CI + CO;
  const int per = per_split_for(l, B), splits = splits_for(l, B);
  hipLaunchKernelGGL((conv_bwd_weight<CI, CO>), dim3((NP + 255) / 256, splits), dim3(256), 0, c->stream, c->dz[l + 1],
                     Ho, Wo, c->act[l], H, W, B, per, c->partial);
  hipLaunchKernelGGL(reduce_splits, dim3((NP + 255) / 256), dim3(256), 0, c->stream, c->partial, splits, NP,
                     c->G + c->o.w[l]);
  if (l > 0) {
    const size_t n = (size_t)B * H * W * CI;
    hipLaunchKernelGGL((conv_bwd_data<CI, CO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->dz[l + 1], Ho, Wo, c->Pb + c->o.w[l], c->act[l], H, W, B, c->dz[l]);
  }
  return hipGetLastError();
}

hipError_t backward(dpt_cnn* c, int B) {
  hipError_t e;
  if ((e = bwd_layer<64, 64>(c, 3, B)) != hipSuccess) return e;
  if ((e = bwd_layer<32, 64>(c, 2, B)) != hipSuccess) return e;
  if ((e = bwd_layer<16, 32>(c, 1, B)) != hipSuccess) return e;
  return bwd_layer<2, 16>(c, 0, B);
}

int load_input(dpt_cnn* c, const uint8_t* pairs, int B, int on_device) {
  const uint8_t* src = pairs;
  if (!on_device) {
    CNN_TRY(hipMemcpyAsync(c->pairs, pairs, (size_t)B * 2 * kH0 * kW0, hipMemcpyHostToDevice, c->stream));
    src = c->pairs;
  }
  const int n = B * kH0 * kW0;
  hipLaunchKernelGGL(input_from_pairs, dim3((n + 255) / 256), dim3(256), 0, c->stream, src, B, c->act[0]);
  CNN_TRY(hipGetLastError());
  return DPT_OK;
}

}  // namespace

extern "C" {

int dpt_cnn_create(int32_t max_batch, void* hip_stream, dpt_cnn** out) {
  if (!out) return cfail(DPT_E_ARG, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 65536) return cfail(DPT_E_ARG, "max_batch outside [1, 65536]");
  dpt_cnn* c = new (std::nothrow) dpt_cnn();
  if (!c) return cfail(DPT_E_OOM, "host allocation failed");
  c->max_batch = max_batch;
  c->stream = (hipStream_t)hip_stream;
  c->o = offsets();
  const size_t n = (size_t)c->o.total, B = (size_t)max_batch;
  bool ok = hipMalloc(&c->P, n * 4) == hipSuccess && hipMalloc(&c->G, n * 4) == hipSuccess &&
            hipMalloc(&c->M, n * 4) == hipSuccess && hipMalloc(&c->V, n * 4) == hipSuccess &&
            hipMalloc(&c->Pb, n * 2) == hipSuccess;
  for (int l = 0; l < 5 && ok; ++l) {
    const size_t e = B * kHs[l] * kWs[l] * kC[l];
    ok = hipMalloc(&c->act[l], e * 2) == hipSuccess && hipMalloc(&c->dz[l], e * 4) == hipSuccess;
  }
  c->partial_floats = (size_t)kSplitsMax * (64 * 9 * 64 + 64);
  size_t maxsplit = 0;
  for (int l = 0; l < 4; ++l)
    maxsplit = std::max(maxsplit, (size_t)splits_for(l, max_batch) * (kC[l + 1] * 9 * kC[l] + kC[l + 1]));
  c->partial_floats = maxsplit;
  ok = ok && hipMalloc(&c->out, B * kOut * 4) == hipSuccess && hipMalloc(&c->tgt, B * kOut * 4) == hipSuccess &&
       hipMalloc(&c->sqerr, B * kOut * 4) == hipSuccess &&
       hipMalloc(&c->fcg, B * (size_t)(c->o.total - c->o.fw1) * 4) == hipSuccess &&
       hipMalloc(&c->partial, c->partial_floats * 4) == hipSuccess && hipMalloc(&c->scal, 64) == hipSuccess &&
       hipMalloc(&c->pairs, B * 2 * kH0 * kW0) == hipSuccess && hipMalloc(&c->d_lv, 2 * B * sizeof(void*)) == hipSuccess &&
       hipHostMalloc(&c->h_buf, std::max(n, B * kOut) * 4 + 64) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    delete c;
    return cfail(DPT_E_OOM, "device allocation failed");
  }
  (void)hipMemsetAsync(c->M, 0, n * 4, c->stream);
  (void)hipMemsetAsync(c->V, 0, n * 4, c->stream);
  (void)hipMemsetAsync(c->P, 0, n * 4, c->stream);
  (void)hipMemsetAsync(c->Pb, 0, n * 2, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return cfail(DPT_E_HIP, "stream synchronize");
  }
  *out = c;
  return DPT_OK;
}

void dpt_cnn_destroy(dpt_cnn* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

int32_t dpt_cnn_num_params(void) { return offsets().total; }

// params: host FP32, tensor order w1 b1 .. fb2, conv weights [co][ci][ky][kx]
int dpt_cnn_set_params(dpt_cnn* c, const float* params) {
  if (!c || !params) return cfail(DPT_E_ARG, "NULL argument");
  const Offsets& o = c->o;
  float* h = c->h_buf;
  std::memcpy(h, params, sizeof(float) * o.total);
  for (int l = 0; l < 4; ++l) {  // [co][ci][ky][kx] -> [co][ky][kx][ci]
    const int CI = kC[l], CO = kC[l + 1];
    for (int co = 0; co < CO; ++co)
      for (int ci = 0; ci < CI; ++ci)
        for (int t = 0; t < 9; ++t) h[o.w[l] + (co * 9 + t) * CI + ci] = params[o.w[l] + (co * CI + ci) * 9 + t];
  }
  CNN_TRY(hipMemcpyAsync(c->P, h, sizeof(float) * o.total, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(to_bf16, dim3((o.total + 255) / 256), dim3(256), 0, c->stream, c->P, o.total, c->Pb);
  CNN_TRY(hipGetLastError());
  CNN_TRY(hipMemsetAsync(c->M, 0, sizeof(float) * o.total, c->stream));
  CNN_TRY(hipMemsetAsync(c->V, 0, sizeof(float) * o.total, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  return DPT_OK;
}

static void to_abi_layout(const Offsets& o, const float* in, float* out) {
  std::memcpy(out, in, sizeof(float) * o.total);
  for (int l = 0; l < 4; ++l) {
    const int CI = kC[l], CO = kC[l + 1];
    for (int co = 0; co < CO; ++co)
      for (int ci = 0; ci < CI; ++ci)
        for (int t = 0; t < 9; ++t) out[o.w[l] + (co * CI + ci) * 9 + t] = in[o.w[l] + (co * 9 + t) * CI + ci];
  }
}

int dpt_cnn_get_params(dpt_cnn* c, float* params) {
  if (!c || !params) return cfail(DPT_E_ARG, "NULL argument");
  CNN_TRY(hipMemcpyAsync(c->h_buf, c->P, sizeof(float) * c->o.total, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  to_abi_layout(c->o, c->h_buf, params);
  return DPT_OK;
}

int dpt_cnn_get_grads(dpt_cnn* c, float* grads) {
  if (!c || !grads) return cfail(DPT_E_ARG, "NULL argument");
  CNN_TRY(hipMemcpyAsync(c->h_buf, c->G, sizeof(float) * c->o.total, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  to_abi_layout(c->o, c->h_buf, grads);
  return DPT_OK;
}

int dpt_cnn_forward(dpt_cnn* c, const uint8_t* pairs, int32_t B, int32_t on_device, float* out_host) {
  if (!c || !pairs || !out_host) return cfail(DPT_E_ARG, "NULL argument");
  if (B < 1 || B > c->max_batch) return cfail(DPT_E_ARG, "batch size");
  int e = load_input(c, pairs, B, on_device);
  if (e != DPT_OK) return e;
  CNN_TRY(forward(c, B));
  hipLaunchKernelGGL(head_kernel, dim3(B), dim3(64), 0, c->stream, c->act[4], c->P, nullptr, B, c->out, nullptr,
                     nullptr, nullptr);
  CNN_TRY(hipGetLastError());
  CNN_TRY(hipMemcpyAsync(out_host, c->out, sizeof(float) * B * kOut, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

// One training step on B pairs: forward, MSE loss against targets (normalised
// twists, B x 6), backward, Adam (lr, beta 0.9 / 0.999, eps 1e-8).  With
// lr == 0 only the gradients are computed (no update).  *loss_out: the loss
// before the update.
int dpt_cnn_train_step(dpt_cnn* c, const uint8_t* pairs, const float* targets, int32_t B, float lr,
                       int32_t on_device, float* loss_out) {
  if (!c || !pairs || !targets || !loss_out) return cfail(DPT_E_ARG, "NULL argument");
  if (B < 1 || B > c->max_batch) return cfail(DPT_E_ARG, "batch size");
  int e = load_input(c, pairs, B, on_device);
  if (e != DPT_OK) return e;
  const float* tg = targets;
  if (!on_device) {
    CNN_TRY(hipMemcpyAsync(c->tgt, targets, sizeof(float) * B * kOut, hipMemcpyHostToDevice, c->stream));
    tg = c->tgt;
  }
  const Offsets& o = c->o;
  CNN_TRY(forward(c, B));
  hipLaunchKernelGGL(head_kernel, dim3(B), dim3(64), 0, c->stream, c->act[4], c->P, tg, B, c->out, c->sqerr, c->fcg,
                     c->dz[4]);
  const int nfc = o.total - o.fw1;
  hipLaunchKernelGGL(reduce_batch, dim3((nfc + 255) / 256), dim3(256), 0, c->stream, c->fcg, B, nfc, c->G + o.fw1);
  hipLaunchKernelGGL(reduce_batch, dim3(1), dim3(64), 0, c->stream, c->sqerr, B, kOut, c->scal);
  CNN_TRY(hipGetLastError());
  CNN_TRY(backward(c, B));
  if (lr > 0.f) {
    c->step += 1;
    const float c1 = 1.0f - std::pow(0.9f, (float)c->step), c2 = 1.0f - std::pow(0.999f, (float)c->step);
    hipLaunchKernelGGL(adam_kernel, dim3((o.total + 255) / 256), dim3(256), 0, c->stream, c->P, c->G, c->M, c->V,
                       o.total, lr, 0.9f, 0.999f, 1e-8f, c1, c2, o.fw1, c->Pb);
    CNN_TRY(hipGetLastError());
  }
  CNN_TRY(hipMemcpyAsync(c->h_buf, c->scal, sizeof(float) * kOut, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  float s = 0.f;
  for (int q = 0; q < kOut; ++q) s += c->h_buf[q];
  *loss_out = s / (float)(B * kOut);
  return DPT_OK;
}

// Test hook: layer activation l (1..4) of the last forward as FP32 NHWC, or
// (l = 5) the network outputs [B][6].
int dpt_cnn_get_activation(dpt_cnn* c, int32_t l, int32_t B, float* host_out) {
  if (!c || !host_out || l < 1 || l > 5 || B < 1 || B > c->max_batch) return cfail(DPT_E_ARG, "argument");
  if (l == 5) {
    CNN_TRY(hipMemcpyAsync(host_out, c->out, sizeof(float) * B * kOut, hipMemcpyDeviceToHost, c->stream));
  } else {
    const size_t n = (size_t)B * kHs[l] * kWs[l] * kC[l];  // dz[l] has exactly this size
    hipLaunchKernelGGL(bf16_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->act[l], n, c->dz[l]);
    CNN_TRY(hipGetLastError());
    CNN_TRY(hipMemcpyAsync(host_out, c->dz[l], sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
  }
  CNN_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

}  // extern "C"

namespace dpt {

// Forward pass on B pairs given as device pointers to coarsest pyramid levels
// (94 x 60, packed rows); writes B x 6 normalised twists to out_host.
int cnn_forward_levels(dpt_cnn* c, const uint8_t* const* refs, const uint8_t* const* curs, int B, float* out_host) {
  if (B < 1 || B > c->max_batch) return cfail(DPT_E_ARG, "batch size");
  std::vector<const uint8_t*> h(2 * (size_t)B);
  for (int b = 0; b < B; ++b) h[b] = refs[b], h[B + b] = curs[b];
  CNN_TRY(hipMemcpyAsync(c->d_lv, h.data(), sizeof(void*) * 2 * B, hipMemcpyHostToDevice, c->stream));
  const int n = B * kH0 * kW0;
  hipLaunchKernelGGL(input_from_levels, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->d_lv, c->d_lv + B, B,
                     c->act[0]);
  CNN_TRY(hipGetLastError());
  CNN_TRY(forward(c, B));
  hipLaunchKernelGGL(head_kernel, dim3(B), dim3(64), 0, c->stream, c->act[4], c->P, nullptr, B, c->out, nullptr,
                     nullptr, nullptr);
  CNN_TRY(hipGetLastError());
  CNN_TRY(hipMemcpyAsync(out_host, c->out, sizeof(float) * B * kOut, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

}  // namespace dpt
