// Learned initialiser: a small CNN that proposes the reference-to-current
// twist from the coarsest pyramid pair (60 x 94, two channels), replacing the
// constant-velocity start of the coarse-to-fine Gauss-Newton track.
//
// Network: four 3x3 stride-2 padding-1 convolutions with ReLU (2-16-32-64-64
// channels), global average pool, FC 64-64 ReLU, FC 64-6.  Activations and
// convolution weights are BF16 in NHWC / [co][ky][kx][ci] layouts; the
// forward convolutions are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation) with bias and ReLU fused in
// the epilogue.  The backward convolutions are implicit GEMMs on the same
// instruction: the data gradient per stride-parity class of the input pixels
// (only the taps that reach a class), the weight gradient as dZ^T Xcol split
// over output pixels, with the bias gradient as a column of ones; gradients
// flowing between layers are stored in BF16, split reductions are summed in a
// fixed order.  Pooling, the FC layers, the loss and Adam run on the vector
// units; master weights and Adam moments are FP32.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/dptrack.h"
#include "dpt_device.h"
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

// ---------------------------------------------------------------- head forward and proposal (device parts)

// The network's outputs are twists scaled to unit range: 5 degrees (in
// radians) for the rotation part, 0.1 m for the translation part.
__constant__ double kTwistScaleDev[6] = {0.08726646259971647, 0.08726646259971647, 0.08726646259971647,
                                         0.1, 0.1, 0.1};

// rel = exp(xi) as 3x4 FP64, xi = the six scaled outputs o6 (rotation first).
__device__ __forceinline__ void propose_twist(const float* o6, double* rel) {
  double xi[6];
  for (int j = 0; j < 6; ++j) xi[j] = (double)o6[j] * kTwistScaleDev[j];
  const double th2 = fma(xi[0], xi[0], fma(xi[1], xi[1], xi[2] * xi[2]));
  double A, Bc, C;
  if (th2 < 1e-8) {  // |w| < 1e-4: series, truncation below 1e-17
    A = 1.0 - th2 * (1.0 / 6.0);
    Bc = 0.5 - th2 * (1.0 / 24.0);
    C = (1.0 / 6.0) - th2 * (1.0 / 120.0);
  } else {
    const double th = sqrt(th2), sn = sin(th), sh = sin(0.5 * th);
    A = sn / th;
    Bc = 2.0 * sh * sh / th2;
    C = (th - sn) / (th2 * th);
  }
  double T[12] = {1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  compose_exp(T, xi[0], xi[1], xi[2], xi[3], xi[4], xi[5], th2, A, Bc, C);
  for (int j = 0; j < 12; ++j) rel[j] = T[j];
}

// The head's forward pass on one sample's layer-4 activations a (4 x 6 x 64,
// LDS or global): g = their mean, h1 = relu(fw1 g + fb1), and for threads
// t < kOut the return value out[t] = fw2 h1 + fb2.  Threads t < 64 do the
// work; every thread of the workgroup calls it (two barriers); g and h1 are
// 64-float LDS vectors.
__device__ __forceinline__ float head_forward(const uint16_t* __restrict__ a, const float* __restrict__ P,
                                              const Offsets& o, float* g, float* h1) {
  constexpr int HW = 4 * 6;
  const int t = threadIdx.x;
  if (t < 64) {
    float s = 0.f;
    for (int p = 0; p < HW; ++p) s += bf2f(a[p * 64 + t]);
    g[t] = s * (1.0f / HW);
  }
  __syncthreads();
  if (t < 64) {
    float z = P[o.fb1 + t];
    for (int q = 0; q < 64; ++q) z = fmaf(P[o.fw1 + t * 64 + q], g[q], z);
    h1[t] = fmaxf(z, 0.f);
  }
  __syncthreads();
  float v = 0.f;
  if (t < kOut) {
    v = P[o.fb2 + t];
    for (int q = 0; q < kHidden; ++q) v = fmaf(P[o.fw2 + t * kHidden + q], h1[q], v);
  }
  return v;
}

// ---------------------------------------------------------------- forward convolutions (fused, MFMA)

// One layer of one sample inside a workgroup, as an implicit GEMM: rows m =
// output pixels (i, j), columns n = output channels, k = (ky, kx, ci), stride
// 2 and one pixel of zero padding; BF16 operands, FP32 accumulation, then bias
// and ReLU, BF16 out.  The sample's activations and the layer's weights are in
// LDS; the waves take the (16-row tile, 16-channel tile) pairs in turn.  Lane L
// supplies A[m0 + L%16][k0 + 4(L/16) .. +3] and B[k0 + 4(L/16) .. +3][n0 + L%16]
// and receives D[4(L/16) + j][L%16].
template <int CI, int CO>
__device__ __forceinline__ void conv_sample(const uint16_t* __restrict__ x, int H, int W, int Ho, int Wo,
                                            const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                            uint16_t* __restrict__ y) {
  constexpr int K = 9 * CI, KP = (K + 15) / 16 * 16, NT = CO / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6, kq = lane >> 4;
  const int M = Ho * Wo, items = (M + 15) / 16 * NT;
  for (int it = wave; it < items; it += nw) {
    const int m0 = it / NT * 16, t = it % NT, n = t * 16 + (lane & 15);
    const int m = m0 + (lane & 15);
    const bool mvalid = m < M;
    const int i = mvalid ? m / Wo : 0, j = mvalid ? m % Wo : 0;
    float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KP / 16; ++ks) {
      const int k0 = ks * 16 + 4 * kq;
      short4_t a, bv;
      if constexpr (CI % 4 == 0) {
        const int tap = k0 / CI, c = k0 % CI;
        const int yy = 2 * i + tap / 3 - 1, xx = 2 * j + tap % 3 - 1;
        uint2 v = make_uint2(0u, 0u);
        if (mvalid && yy >= 0 && yy < H && xx >= 0 && xx < W)
          v = *reinterpret_cast<const uint2*>(x + (yy * W + xx) * CI + c);
        a = short4_t{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
        const uint2 u = *reinterpret_cast<const uint2*>(w + n * K + k0);
        bv = short4_t{(short)(u.x & 0xffff), (short)(u.x >> 16), (short)(u.y & 0xffff), (short)(u.y >> 16)};
      } else {
        short e[4], f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k0 + q;
          uint16_t v = 0;
          if (k < K && mvalid) {
            const int tap = k / CI, c = k % CI;
            const int yy = 2 * i + tap / 3 - 1, xx = 2 * j + tap % 3 - 1;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = x[(yy * W + xx) * CI + c];
          }
          e[q] = (short)v;
          f[q] = k < K ? (short)w[n * K + k] : (short)0;
        }
        a = short4_t{e[0], e[1], e[2], e[3]};
        bv = short4_t{f[0], f[1], f[2], f[3]};
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int mo = m0 + 4 * kq + q;
      if (mo < M) y[mo * CO + n] = f2bf(fmaxf(acc[q] + bias[n], 0.0f));
    }
  }
}

// A layer's BF16 weights ([co][tap][ci], `bytes` a multiple of 16 from a
// 16-byte aligned source) copied into LDS by the workgroup, global memory
// straight into LDS; the caller waits (s_waitcnt 0, then a barrier).
__device__ __forceinline__ void stage_weights(const uint16_t* __restrict__ src, int bytes, uint16_t* lds) {
  const int lane = threadIdx.x & 63, ng = bytes >> 4;
  for (int q0 = (int)(threadIdx.x & ~63u); q0 < ng; q0 += blockDim.x)
    if (q0 + lane < ng)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(src) + 4 * (q0 + lane),
                                       (__attribute__((address_space(3))) void*)(lds + 8 * q0), 16, 0, 0);
}

// LDS of the fused pass (elements): two ping-pong activation buffers and the
// current layer's weights.
constexpr int kFuseA = 15 * 24 * 32 > kH0 * kW0 * 2 ? 15 * 24 * 32 : kH0 * kW0 * 2;  // input, layer 2 out
constexpr int kFuseB = 30 * 47 * 16;                                                  // layer 1 and 3 out
constexpr int kFuseW = 64 * 9 * 64;                                                   // layer 4's weights
static_assert(kHs[1] == 30 && kWs[1] == 47 && kC[1] == 16 && kHs[2] == 15 && kWs[2] == 24 && kC[2] == 32 &&
                  kHs[3] * kWs[3] * kC[3] <= kFuseB && kC[3] * 9 * kC[4] <= kFuseW,
              "fused buffers follow the layer shapes");
constexpr int kFuseThreads = 1024;

// Where the fused pass reads and writes: the input pairs as per-sample level
// pointers (refs, curs) or planar [B][2][60][94] bytes (pairs); act[l]
// (non-null) receives layer l's activations for the backward pass (act[0] the
// BF16 input), act[4] always; out (non-null) the head's outputs, rel
// (non-null) their exponentials.
struct FusedIO {
  const uint8_t* const* refs;
  const uint8_t* const* curs;
  const uint8_t* pairs;
  uint16_t* act[5];
  float* out;
  double* rel;
};

// n BF16 values (a multiple of 8) from LDS to global memory, 16 bytes a thread.
__device__ __forceinline__ void store_act(const uint16_t* __restrict__ src, uint16_t* __restrict__ dst, int n) {
  for (int e = 8 * (int)threadIdx.x; e < n; e += 8 * (int)blockDim.x)
    *reinterpret_cast<uint4*>(dst + e) = *reinterpret_cast<const uint4*>(src + e);
}

// The input and the four convolutions of sample blockIdx.x in one workgroup,
// the activations never leaving LDS (save the copies io asks for) and each
// layer's weights staged in LDS before it runs; then, for inference, the
// head and the proposal.
__global__ __launch_bounds__(kFuseThreads) void conv_net_fused(FusedIO io, const uint16_t* __restrict__ Pb,
                                                               const float* __restrict__ P) {
  __shared__ __align__(16) uint16_t bufA[kFuseA];
  __shared__ float sh_g[64], sh_h1[64], sh_out[kOut];
  __shared__ __align__(16) uint16_t bufB[kFuseB];
  __shared__ __align__(16) uint16_t bufW[kFuseW];
  constexpr int N0 = kH0 * kW0 * 2, N1 = kHs[1] * kWs[1] * kC[1], N2 = kHs[2] * kWs[2] * kC[2],
                N3 = kHs[3] * kWs[3] * kC[3], N4 = kHs[4] * kWs[4] * kC[4];
  static_assert(N0 % 8 == 0 && N1 % 8 == 0 && N2 % 8 == 0 && N3 % 8 == 0 && N4 % 8 == 0, "16-byte copies");
  const int b = blockIdx.x;
  const Offsets o = offsets();
  stage_weights(Pb + o.w[0], kC[1] * 9 * kC[0] * 2, bufW);
  const uint8_t* ref = io.pairs ? io.pairs + (size_t)(2 * b) * kH0 * kW0 : io.refs[b];
  const uint8_t* cur = io.pairs ? io.pairs + (size_t)(2 * b + 1) * kH0 * kW0 : io.curs[b];
  for (int r = threadIdx.x; r < kH0 * kW0; r += blockDim.x) {  // (I - 128) / 64, exact in BF16
    bufA[2 * r] = f2bf(((float)ref[r] - 128.0f) * (1.0f / 64.0f));
    bufA[2 * r + 1] = f2bf(((float)cur[r] - 128.0f) * (1.0f / 64.0f));
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (io.act[0]) store_act(bufA, io.act[0] + (size_t)b * N0, N0);
  conv_sample<2, 16>(bufA, kHs[0], kWs[0], kHs[1], kWs[1], bufW, P + o.b[0], bufB);
  __syncthreads();
  stage_weights(Pb + o.w[1], kC[2] * 9 * kC[1] * 2, bufW);
  if (io.act[1]) store_act(bufB, io.act[1] + (size_t)b * N1, N1);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  conv_sample<16, 32>(bufB, kHs[1], kWs[1], kHs[2], kWs[2], bufW, P + o.b[1], bufA);
  __syncthreads();
  stage_weights(Pb + o.w[2], kC[3] * 9 * kC[2] * 2, bufW);
  if (io.act[2]) store_act(bufA, io.act[2] + (size_t)b * N2, N2);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  conv_sample<32, 64>(bufA, kHs[2], kWs[2], kHs[3], kWs[3], bufW, P + o.b[2], bufB);
  __syncthreads();
  stage_weights(Pb + o.w[3], kC[4] * 9 * kC[3] * 2, bufW);
  if (io.act[3]) store_act(bufB, io.act[3] + (size_t)b * N3, N3);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  conv_sample<64, 64>(bufB, kHs[3], kWs[3], kHs[4], kWs[4], bufW, P + o.b[3], bufA);
  __syncthreads();
  store_act(bufA, io.act[4] + (size_t)b * N4, N4);
  if (!io.out) return;
  // the head (head_kernel's arithmetic) and the proposal's exponential
  const float v = head_forward(bufA, P, o, sh_g, sh_h1);
  if (threadIdx.x < kOut) {
    io.out[b * kOut + threadIdx.x] = v;
    sh_out[threadIdx.x] = v;
  }
  __syncthreads();
  if (io.rel && threadIdx.x == 0) propose_twist(sh_out, io.rel + 12 * b);
}

// The fused pass over B samples on stream s.
hipError_t launch_fused(const FusedIO& io, int B, const uint16_t* Pb, const float* P, hipStream_t s) {
  hipLaunchKernelGGL(conv_net_fused, dim3(B), dim3(kFuseThreads), 0, s, io, Pb, P);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pool + FC (+ loss and its backward)

// One 64-thread workgroup per sample: g = mean(a4), h1 = relu(fw1 g + fb1),
// out = fw2 h1 + fb2.  With targets, also the squared error, dout and the FC /
// pool backward down to dZ4 = dA4 * (a4 > 0); per-sample FC weight gradients go
// to `fcg` [B][fc params] and are summed over the batch in a fixed order later.
__global__ __launch_bounds__(64) void head_kernel(const uint16_t* __restrict__ a4, const float* __restrict__ P,
                                                  const float* __restrict__ targets, int B, float* __restrict__ out,
                                                  float* __restrict__ sqerr, float* __restrict__ fcg,
                                                  uint16_t* __restrict__ dz4) {
  const Offsets o = offsets();
  const int b = blockIdx.x, t = threadIdx.x;
  __shared__ float g[64], h1[64], dout[kOut], dz1[64];
  constexpr int HW = 4 * 6;
  const uint16_t* a = a4 + (size_t)b * HW * 64;
  const float v = head_forward(a, P, o, g, h1);
  if (t < kOut) {
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
  const uint16_t dgb = f2bf(dg);
  for (int p = 0; p < HW; ++p) dz4[((size_t)b * HW + p) * 64 + t] = bf2f(a[p * 64 + t]) > 0.f ? dgb : (uint16_t)0;
}

// ---------------------------------------------------------------- backward convolution

__device__ __forceinline__ short4_t bf16x4(uint2 v) {
  return short4_t{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
}

// Data gradient of layer L >= 1, fused with the ReLU mask of its input:
// dZprev[b][y][x][c] = (a_prev > 0) * sum over taps (ky, kx) and channels o of
// W[o][ky][kx][c] dZ[b][i][j][o], where 2i + ky - 1 = y and 2j + kx - 1 = x.
// Stride 2 makes the reaching taps depend only on the parities of (y, x): an
// even row is reached by ky = 1 alone, an odd one by ky = 0 and 2 (columns
// likewise), so the rows of the implicit GEMM are the input pixels of one
// parity class (blockIdx.y) and k = (reaching tap, o).  wT: the layer's BF16
// weights as [tap][ci][co].  A wave computes 16 pixels x CI channels.
template <int L>
__global__ __launch_bounds__(256) void conv_bwd_data_mfma(const uint16_t* __restrict__ dz,
                                                          const uint16_t* __restrict__ wT,
                                                          const uint16_t* __restrict__ aprev, int B,
                                                          uint16_t* __restrict__ dzprev) {
  constexpr int CI = kC[L], CO = kC[L + 1], H = kHs[L], W = kWs[L], Ho = kHs[L + 1], Wo = kWs[L + 1];
  constexpr int NT = CI / 16;
  static_assert(CI % 16 == 0 && CO % 16 == 0, "16-channel tiles");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
  const int py = blockIdx.y >> 1, px = blockIdx.y & 1;
  const int Hc = (H - py + 1) / 2, Wc = (W - px + 1) / 2;
  const int M = B * Hc * Wc;
  const int m0 = (blockIdx.x * 4 + wave) * 16;
  if (m0 >= M) return;
  const int m = m0 + (lane & 15);
  const bool mvalid = m < M;
  const int b = mvalid ? m / (Hc * Wc) : 0, r = mvalid ? m % (Hc * Wc) : 0;
  const int y = 2 * (r / Wc) + py, x = 2 * (r % Wc) + px;
  float4_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int ta = 0; ta < (py ? 2 : 1); ++ta)
    for (int tb = 0; tb < (px ? 2 : 1); ++tb) {
      const int ky = py ? 2 * ta : 1, kx = px ? 2 * tb : 1, tap = ky * 3 + kx;
      const int i = (y + 1 - ky) >> 1, j = (x + 1 - kx) >> 1;  // y + 1 - ky >= 0 and even
      const bool ok = mvalid && i < Ho && j < Wo;
      // a row the tap does not reach reads pixel 0 and discards it
      const uint16_t* drow = dz + (ok ? (((size_t)b * Ho + i) * Wo + j) * CO : 0);
#pragma unroll
      for (int o0 = 0; o0 < CO; o0 += 16) {
        const int k0 = o0 + 4 * q;
        uint2 dv = *reinterpret_cast<const uint2*>(drow + k0);
        if (!ok) dv = make_uint2(0u, 0u);
        const short4_t av = bf16x4(dv);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int n = t * 16 + (lane & 15);
          const short4_t bv = bf16x4(*reinterpret_cast<const uint2*>(wT + ((size_t)tap * CI + n) * CO + k0));
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
  // D[4q + j][lane % 16]: pixel row m0 + 4q + j, channel t * 16 + lane % 16
#pragma unroll
  for (int jq = 0; jq < 4; ++jq) {
    const int mo = m0 + 4 * q + jq;
    if (mo >= M) continue;
    const int bo = mo / (Hc * Wc), ro = mo % (Hc * Wc);
    const int yo = 2 * (ro / Wc) + py, xo = 2 * (ro % Wc) + px;
    const size_t base = (((size_t)bo * H + yo) * W + xo) * CI;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const size_t id = base + t * 16 + (lane & 15);
      dzprev[id] = bf2f(aprev[id]) > 0.f ? f2bf(acc[t][jq]) : (uint16_t)0;
    }
  }
}

// Weight and bias gradient of layer L over the output pixels p = (b, i, j) of
// split blockIdx.y: partial[split][o][n] = sum_p dZ[p][o] Xcol[p][n], where
// Xcol[p][tap * CI + c] = X[b][2i + ky - 1][2j + kx - 1][c] (zero outside the
// image) and column n = 9 CI is all ones (the bias); columns up to the next
// multiple of 16 are zero.  One wave per 16 x 16 output tile (blockIdx.x * 4 +
// wave over CO / 16 x NPAD / 16 tiles), 16 pixels per MFMA step.
template <int L>
__global__ __launch_bounds__(256) void conv_bwd_weight_mfma(const uint16_t* __restrict__ dz,
                                                            const uint16_t* __restrict__ x, int P, int per_split,
                                                            float* __restrict__ partial) {
  constexpr int CI = kC[L], CO = kC[L + 1], H = kHs[L], W = kWs[L], Ho = kHs[L + 1], Wo = kWs[L + 1];
  constexpr int NPAD = (9 * CI + 1 + 15) / 16 * 16, MT = CO / 16, NT = NPAD / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= MT * NT) return;
  const int mt = tile / NT, nt = tile % NT, split = blockIdx.y;
  const int p0 = split * per_split, p1 = min(P, p0 + per_split);
  const int o = mt * 16 + (lane & 15), n = nt * 16 + (lane & 15);
  const bool real = n < 9 * CI, ones = n == 9 * CI;
  const int tap = real ? n / CI : 0, c = real ? n % CI : 0, ky = tap / 3, kx = tap % 3;
  // the lane's four rows of the step at pb: dZ and the im2col column
  auto operands = [&](int pb, short (&a)[4], short (&bb)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int p = pb + 4 * q + t;
      uint16_t av = 0, bv = 0;
      if (p < p1) {
        av = dz[(size_t)p * CO + o];
        if (ones) {
          bv = 0x3f80;  // 1.0
        } else if (real) {
          const int b = p / (Ho * Wo), ij = p % (Ho * Wo);
          const int yy = 2 * (ij / Wo) + ky - 1, xx = 2 * (ij % Wo) + kx - 1;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W) bv = x[(((size_t)b * H + yy) * W + xx) * CI + c];
        }
      }
      a[t] = (short)av;
      bb[t] = (short)bv;
    }
  };
  float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
  short a[4], bb[4];
  operands(p0, a, bb);
  for (int pb = p0; pb < p1; pb += 16) {  // the next step's loads in flight during this step's product
    short a2[4], b2[4];
    operands(pb + 16, a2, b2);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(short4_t{a[0], a[1], a[2], a[3]},
                                                     short4_t{bb[0], bb[1], bb[2], bb[3]}, acc, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = a2[t], bb[t] = b2[t];
  }
  float* out = partial + (size_t)split * CO * NPAD;
#pragma unroll
  for (int jq = 0; jq < 4; ++jq) out[(size_t)(mt * 16 + 4 * q + jq) * NPAD + n] = acc[jq];
}

// sum_k v[k * n + e] for the n elements e of a block's share, in a fixed
// order: the PARTS threads of an element (threads el, el + 256 / PARTS, ...)
// sum k = part, part + PARTS, ... in order, and the parts meet in a fixed
// pairwise tree in LDS.  The result goes to out(e, sum) (part 0's thread).
template <int PARTS, class Out>
__device__ __forceinline__ void sum_slices(const float* __restrict__ v, int K, int n, Out out) {
  constexpr int EPB = 256 / PARTS;  // elements per block
  __shared__ float sh[256];
  const int el = (int)threadIdx.x % EPB, part = (int)threadIdx.x / EPB;
  const int e = (int)blockIdx.x * EPB + el;
  float s = 0.f;
  if (e < n)
    for (int k = part; k < K; k += PARTS) s += v[(size_t)k * n + e];
  sh[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int w = PARTS / 2; w > 0; w >>= 1) {
    if (part < w) sh[threadIdx.x] += sh[threadIdx.x + w * EPB];
    __syncthreads();
  }
  if (part == 0 && e < n) out(e, sh[el]);
}

// Threads per element for a sum over K slices: about sixteen slices each.
inline int parts_for(int K) { return K > 1024 ? 256 : K > 256 ? 64 : K > 64 ? 16 : K > 16 ? 4 : 1; }

// Sum of the splits of conv_bwd_weight_mfma into the gradient vector: weights
// at w_off + o * 9 CI + n ([co][ky][kx][ci]), bias at b_off + o.
template <int L, int PARTS>
__global__ __launch_bounds__(256) void reduce_wgrad(const float* __restrict__ partial, int splits,
                                                    float* __restrict__ gw, float* __restrict__ gb) {
  constexpr int CI = kC[L], CO = kC[L + 1], NPAD = (9 * CI + 1 + 15) / 16 * 16;
  sum_slices<PARTS>(partial, splits, CO * NPAD, [&](int e, float s) {
    const int o = e / NPAD, n = e % NPAD;
    if (n < 9 * CI)
      gw[o * 9 * CI + n] = s;
    else if (n == 9 * CI)
      gb[o] = s;
  });
}

// Sum over the batch of the per-sample FC gradients, and of the squared errors.
template <int PARTS>
__global__ __launch_bounds__(256) void reduce_batch(const float* __restrict__ v, int B, int n,
                                                    float* __restrict__ out) {
  sum_slices<PARTS>(v, B, n, [&](int e, float s) { out[e] = s; });
}

// ---------------------------------------------------------------- Adam

// Adam (Kingma & Ba 2015) on the FP32 master weights with bias correction c1 =
// 1 - b1^t, c2 = 1 - b2^t; refreshes the BF16 conv weight copies.
// BF16 copies of parameter e: Pb[e]; a convolution weight ([co][ky][kx][ci])
// also into PbT as [tap][ci][co], the operand layout of the data gradient.
__device__ __forceinline__ void store_bf16_param(int e, float p, uint16_t* __restrict__ Pb,
                                                 uint16_t* __restrict__ PbT) {
  const uint16_t h = f2bf(p);
  Pb[e] = h;
  const Offsets o = offsets();
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int CI = kC[l], CO = kC[l + 1], r = e - o.w[l];
    if (r >= 0 && r < CO * 9 * CI) {
      const int co = r / (9 * CI), tap = (r / CI) % 9, ci = r % CI;
      PbT[o.w[l] + (tap * CI + ci) * CO + co] = h;
    }
  }
}

__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                            float* __restrict__ V, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                            int conv_end, uint16_t* __restrict__ Pb, uint16_t* __restrict__ PbT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float g = G[e];
  const float m = b1 * M[e] + (1.0f - b1) * g;
  const float v = b2 * V[e] + (1.0f - b2) * g * g;
  M[e] = m;
  V[e] = v;
  const float p = P[e] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[e] = p;
  if (e < conv_end) store_bf16_param(e, p, Pb, PbT);
}

__global__ void to_bf16(const float* __restrict__ P, int n, uint16_t* __restrict__ Pb, uint16_t* __restrict__ PbT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) store_bf16_param(e, P[e], Pb, PbT);
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
  uint16_t* PbT = nullptr;                                         // BF16 conv weights as [tap][ci][co]
  uint16_t* act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // dz[l]: gradient at layer l's output (pre-ReLU), BF16 NHWC; sized for FP32
  // so that the activation test hook can stage an FP32 copy there
  uint16_t* dz[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float *out = nullptr, *tgt = nullptr, *sqerr = nullptr, *fcg = nullptr, *partial = nullptr, *scal = nullptr;
  uint8_t* pairs = nullptr;
  const uint8_t** d_lv = nullptr;  // [2][max_batch] level pointers
  int step = 0;
  float* h_buf = nullptr;  // pinned
  size_t partial_floats = 0;
  ~dpt_cnn() {
    for (void* p : {(void*)P, (void*)G, (void*)M, (void*)V, (void*)Pb, (void*)PbT, (void*)out, (void*)tgt, (void*)sqerr,
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

// Output pixels per split of the weight gradient, per layer: 8-16 MFMA steps
// per wave and a few thousand waves, so the loads of many waves overlap (the
// first and last layers have the fewest tiles, so the shortest splits).
constexpr int kPixPerSplit[4] = {128, 256, 256, 128};

int splits_for(int l, int B) { return (B * kHs[l + 1] * kWs[l + 1] + kPixPerSplit[l] - 1) / kPixPerSplit[l]; }

// Launch of a sum over K slices with the PARTS that parts_for(K) picks.
template <template <int> class Kernel, class... Args>
void launch_sum(int K, int n, hipStream_t s, Args... args) {
  switch (parts_for(K)) {
    case 256: hipLaunchKernelGGL(Kernel<256>::fn, dim3(n), dim3(256), 0, s, args...); break;
    case 64: hipLaunchKernelGGL(Kernel<64>::fn, dim3((n + 3) / 4), dim3(256), 0, s, args...); break;
    case 16: hipLaunchKernelGGL(Kernel<16>::fn, dim3((n + 15) / 16), dim3(256), 0, s, args...); break;
    case 4: hipLaunchKernelGGL(Kernel<4>::fn, dim3((n + 63) / 64), dim3(256), 0, s, args...); break;
    default: hipLaunchKernelGGL(Kernel<1>::fn, dim3((n + 255) / 256), dim3(256), 0, s, args...); break;
  }
}

template <int L>
struct WgradSum {
  template <int PARTS>
  struct K {
    static constexpr auto fn = reduce_wgrad<L, PARTS>;
  };
};
template <int PARTS>
struct BatchSum {
  static constexpr auto fn = reduce_batch<PARTS>;
};

constexpr int npad(int l) { return (9 * kC[l] + 1 + 15) / 16 * 16; }

template <int L>
hipError_t bwd_layer(dpt_cnn* c, int B) {
  constexpr int CO = kC[L + 1];
  const int P = B * kHs[L + 1] * kWs[L + 1], splits = splits_for(L, B);
  const int tiles = (CO / 16) * (npad(L) / 16);
  hipLaunchKernelGGL((conv_bwd_weight_mfma<L>), dim3((tiles + 3) / 4, splits), dim3(256), 0, c->stream, c->dz[L + 1],
                     c->act[L], P, kPixPerSplit[L], c->partial);
  launch_sum<WgradSum<L>::template K>(splits, CO * npad(L), c->stream, (const float*)c->partial, splits,
                                      c->G + c->o.w[L], c->G + c->o.b[L]);
  if constexpr (L > 0) {
    int rows = 0;  // the largest parity class
    for (int cls = 0; cls < 4; ++cls)
      rows = std::max(rows, B * ((kHs[L] - (cls >> 1) + 1) / 2) * ((kWs[L] - (cls & 1) + 1) / 2));
    hipLaunchKernelGGL((conv_bwd_data_mfma<L>), dim3((rows + 63) / 64, 4), dim3(256), 0, c->stream, c->dz[L + 1],
                       c->PbT + c->o.w[L], c->act[L], B, c->dz[L]);
  }
  return hipGetLastError();
}

hipError_t backward(dpt_cnn* c, int B) {
  hipError_t e;
  if ((e = bwd_layer<3>(c, B)) != hipSuccess) return e;
  if ((e = bwd_layer<2>(c, B)) != hipSuccess) return e;
  if ((e = bwd_layer<1>(c, B)) != hipSuccess) return e;
  return bwd_layer<0>(c, B);
}

// The forward pass of B planar pairs (host or device) through the fused
// kernel, every layer's activations kept for the backward pass; with head,
// the head's outputs to c->out as well.
int forward_pairs(dpt_cnn* c, const uint8_t* pairs, int B, int on_device, bool head) {
  const uint8_t* src = pairs;
  if (!on_device) {
    CNN_TRY(hipMemcpyAsync(c->pairs, pairs, (size_t)B * 2 * kH0 * kW0, hipMemcpyHostToDevice, c->stream));
    src = c->pairs;
  }
  FusedIO io{};
  io.pairs = src;
  for (int l = 0; l < 5; ++l) io.act[l] = c->act[l];
  io.out = head ? c->out : nullptr;
  CNN_TRY(launch_fused(io, B, c->Pb, c->P, c->stream));
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
            hipMalloc(&c->Pb, n * 2) == hipSuccess && hipMalloc(&c->PbT, n * 2) == hipSuccess;
  for (int l = 0; l < 5 && ok; ++l) {
    const size_t e = B * kHs[l] * kWs[l] * kC[l];
    ok = hipMalloc(&c->act[l], e * 2) == hipSuccess && hipMalloc(&c->dz[l], e * 4) == hipSuccess;
  }
  size_t maxsplit = 0;
  for (int l = 0; l < 4; ++l)
    maxsplit = std::max(maxsplit, (size_t)splits_for(l, max_batch) * kC[l + 1] * npad(l));
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
  (void)hipMemsetAsync(c->PbT, 0, n * 2, c->stream);
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
  hipLaunchKernelGGL(to_bf16, dim3((o.total + 255) / 256), dim3(256), 0, c->stream, c->P, o.total, c->Pb, c->PbT);
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
  int e = forward_pairs(c, pairs, B, on_device, true);
  if (e != DPT_OK) return e;
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
  int e = forward_pairs(c, pairs, B, on_device, false);
  if (e != DPT_OK) return e;
  const float* tg = targets;
  if (!on_device) {
    CNN_TRY(hipMemcpyAsync(c->tgt, targets, sizeof(float) * B * kOut, hipMemcpyHostToDevice, c->stream));
    tg = c->tgt;
  }
  const Offsets& o = c->o;
  hipLaunchKernelGGL(head_kernel, dim3(B), dim3(64), 0, c->stream, c->act[4], c->P, tg, B, c->out, c->sqerr, c->fcg,
                     c->dz[4]);
  const int nfc = o.total - o.fw1;
  launch_sum<BatchSum>(B, nfc, c->stream, (const float*)c->fcg, B, nfc, c->G + o.fw1);
  launch_sum<BatchSum>(B, kOut, c->stream, (const float*)c->sqerr, B, (int)kOut, c->scal);
  CNN_TRY(hipGetLastError());
  CNN_TRY(backward(c, B));
  if (lr > 0.f) {
    c->step += 1;
    const float c1 = 1.0f - std::pow(0.9f, (float)c->step), c2 = 1.0f - std::pow(0.999f, (float)c->step);
    hipLaunchKernelGGL(adam_kernel, dim3((o.total + 255) / 256), dim3(256), 0, c->stream, c->P, c->G, c->M, c->V,
                       o.total, lr, 0.9f, 0.999f, 1e-8f, c1, c2, o.fw1, c->Pb, c->PbT);
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
    float* tmp = reinterpret_cast<float*>(c->dz[l]);
    hipLaunchKernelGGL(bf16_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->act[l], n, tmp);
    CNN_TRY(hipGetLastError());
    CNN_TRY(hipMemcpyAsync(host_out, tmp, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
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
  FusedIO io{};
  io.refs = c->d_lv, io.curs = c->d_lv + B, io.act[4] = c->act[4], io.out = c->out;
  CNN_TRY(launch_fused(io, B, c->Pb, c->P, c->stream));
  CNN_TRY(hipMemcpyAsync(out_host, c->out, sizeof(float) * B * kOut, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int cnn_propose(dpt_cnn* c, const uint8_t* const* d_lv, int B, hipStream_t s, double* rel) {
  if (B < 1 || B > c->max_batch) return cfail(DPT_E_ARG, "batch size");
  FusedIO io{};
  io.refs = d_lv, io.curs = d_lv + B, io.act[4] = c->act[4], io.out = c->out, io.rel = rel;
  CNN_TRY(launch_fused(io, B, c->Pb, c->P, s));
  return DPT_OK;
}

}  // namespace dpt
