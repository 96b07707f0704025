// Map-point selection (stand-in for the map points the indirect pipeline
// provides): the n candidates with the largest integer gradient score
// s = (I[y][x+1] - I[y][x-1])^2 + (I[y+1][x] - I[y-1][x])^2 inside the margin,
// ties to the smaller linear index, written in ascending index order.
//
// Multi-workgroup pipeline over chunks of kSelChunk candidates (candidate c is
// pixel (m + c % Wc, m + c / Wc), so candidate order is index order):
//   A  per-chunk LDS histograms of s >> 9 (s <= 2 * 255^2 < 2^17), summed into a
//      global 256-bin histogram with integer atomics (order-independent)
//   B  every workgroup finds the coarse bucket of the n-th largest score with
//      one wave, then the 512-bin histogram of the low bits inside it
//   C  every workgroup finds the exact threshold T and how many ties `need` to
//      keep, then its chunk's counts of scores > T and == T
//   D  every workgroup scans the chunk counts before it for its output offset
//      and tie base, then writes its selected indices with a block-wide prefix
//      sum; the last chunk writes the count
#include <cstdint>
#include <cstring>
#include <mutex>

#include "dpt_device.h"

namespace dpt {

constexpr int kSelThreads = 256, kSelPPT = 16, kSelChunk = kSelThreads * kSelPPT;

struct SelScratch {  // layout of the int32 scratch buffer (histograms and kDone zero between runs)
  static constexpr int kHist1 = 0, kHist2 = 256, kDone = 768, kChunks = 772;
};

int64_t select_scratch_ints(int32_t W, int32_t H) {
  const int64_t G = ((int64_t)W * H + kSelChunk - 1) / kSelChunk + 1;
  return SelScratch::kChunks + 2 * G;
}

__device__ __forceinline__ int sel_score(const uint8_t* img, int pitch, int x, int y) {
  const uint8_t* p = img + (int64_t)y * pitch + x;
  const int dx = (int)p[1] - (int)p[-1];
  const int dy = (int)p[pitch] - (int)p[-pitch];
  return dx * dx + dy * dy;
}


// Row and column of candidate c: the float quotient (c < 2^24 is exact, and
// the product's error is far below one row) corrected by at most one row.
__device__ __forceinline__ void cand_xy(const SelGeom& g, int c, int* x, int* y) {
  int r = (int)((float)c * g.inv_wc);
  int q = c - r * g.Wc;
  if (q < 0) {
    --r;
    q += g.Wc;
  } else if (q >= g.Wc) {
    ++r;
    q -= g.Wc;
  }
  *x = q;
  *y = r;
}

__device__ __forceinline__ int cand_score(const SelGeom& g, int c) {
  int x, y;
  cand_xy(g, c, &x, &y);
  return sel_score(g.img, g.pitch, g.m + x, g.m + y);
}

// Four candidates of a row at once from 4-byte loads: possible when the
// candidate rows start 4-byte aligned (image and pitch multiples of 4, margin
// a multiple of 4 and at least 4, so the words left and right of a group stay
// in the row) and every row holds a multiple of 4 candidates (a group never
// spans two rows, and the candidate total is a multiple of 4).
__device__ __forceinline__ bool sel_vec4(const SelGeom& g) {
  return ((uintptr_t)g.img & 3) == 0 && (g.pitch & 3) == 0 && (g.m & 3) == 0 && g.m >= 4 && (g.Wc & 3) == 0;
}

__device__ __forceinline__ int byte_of(uint32_t w, int i) { return (int)((w >> (8 * i)) & 255u); }

// Scores of candidates c .. c + 3 (c a multiple of 4, sel_vec4): five aligned
// words, the row above and below the four pixels and the row from one pixel
// left of them to one right.
__device__ __forceinline__ int4 cand_score4(const SelGeom& g, int c) {
  int x, y;
  cand_xy(g, c, &x, &y);
  const uint8_t* p = g.img + (int64_t)(g.m + y) * g.pitch + (g.m + x);
  const uint32_t lw = *reinterpret_cast<const uint32_t*>(p - 4), mw = *reinterpret_cast<const uint32_t*>(p),
                 rw = *reinterpret_cast<const uint32_t*>(p + 4);
  const uint32_t up = *reinterpret_cast<const uint32_t*>(p - g.pitch),
                 dn = *reinterpret_cast<const uint32_t*>(p + g.pitch);
  const int left[4] = {byte_of(lw, 3), byte_of(mw, 0), byte_of(mw, 1), byte_of(mw, 2)};
  const int right[4] = {byte_of(mw, 1), byte_of(mw, 2), byte_of(mw, 3), byte_of(rw, 0)};
  int sc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int dx = right[k] - left[k], dy = byte_of(dn, k) - byte_of(up, k);
    sc[k] = dx * dx + dy * dy;
  }
  return make_int4(sc[0], sc[1], sc[2], sc[3]);
}

// f(q, score) for every candidate c0 + q < C of the chunk at c0, the
// workgroup's threads on consecutive candidates (or groups of four).
template <class F>
__device__ __forceinline__ void for_chunk_scores(const SelGeom& g, int c0, F&& f) {
  if (sel_vec4(g)) {
    for (int q = 4 * (int)threadIdx.x; q < kSelChunk; q += 4 * (int)blockDim.x) {
      if (c0 + q >= g.C) break;
      const int4 v = cand_score4(g, c0 + q);
      f(q, v.x), f(q + 1, v.y), f(q + 2, v.z), f(q + 3, v.w);
    }
  } else {
    for (int q = threadIdx.x; q < kSelChunk; q += blockDim.x) {
      if (c0 + q >= g.C) break;
      f(q, cand_score(g, c0 + q));
    }
  }
}

// The selection of one image (`one`), or of image blockIdx.y of a batch (`many`
// non-null): every kernel below runs over (chunks, images) and a workgroup past
// its image's chunk count returns at once.
__device__ __forceinline__ SelJob sel_job(const SelJob& one, const SelJob* many) {
  return many ? many[blockIdx.y] : one;
}

__global__ __launch_bounds__(kSelThreads) void sel_clear(SelJob one, const SelJob* many) {
  const SelJob j = sel_job(one, many);
  for (int b = threadIdx.x; b < SelScratch::kChunks; b += blockDim.x) j.sc[b] = 0;
  if (j.G == 0 && threadIdx.x == 0) *j.count = 0;  // no candidates: nothing selected
}

__global__ __launch_bounds__(kSelThreads) void sel_hist_coarse(SelJob one, const SelJob* many) {
  const SelJob j = sel_job(one, many);
  if ((int)blockIdx.x >= j.G) return;
  const SelGeom& g = j.g;
  int* __restrict__ sc = j.sc;
  __shared__ int h[256];
  for (int b = threadIdx.x; b < 256; b += blockDim.x) h[b] = 0;
  __syncthreads();
  // bin 0 (scores below 512, most of a frame) is not counted: it is the
  // candidate total minus the other bins, which spares its atomics
  for_chunk_scores(g, blockIdx.x * kSelChunk, [&](int, int sv) {
    const int b = sv >> 9;
    if (b) atomicAdd(&h[b], 1);
  });
  __syncthreads();
  for (int b = threadIdx.x + 1; b < 256; b += blockDim.x)
    if (h[b]) atomicAdd(&sc[SelScratch::kHist1 + b], h[b]);
}

// One wave: the largest bin b with sum_{b' >= b} h[b'] >= n over NB bins
// (NB / 64 per lane), given `above` candidates already counted in higher bins.
// total >= 0: bin 0 is not stored and holds total minus the other bins.
// Returns b (or -1 if the total is short of n) and the count above b.
template <int NB>
__device__ __forceinline__ int2 wave_find_bin(const int* __restrict__ h, int n, int above, int total = -1) {
  constexpr int PB = NB / 64;
  const int lane = threadIdx.x & 63;
  int v[PB], t = 0;
#pragma unroll
  for (int j = 0; j < PB; ++j) t += (v[j] = h[lane * PB + j]);
  if (total >= 0) {
    int rest = t;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) rest += __shfl_xor(rest, d, 64);
    if (lane == 0) {
      v[0] = total - rest;
      t += v[0];
    }
  }
  // suffix sum over the lanes above this one
  int suf = t;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_down(suf, d, 64);
    if (lane + d < 64) suf += y;
  }
  int cum = above + suf - t;  // candidates in bins above this lane's
  int found = -1, cum_at = 0;
  if (cum < n && cum + t >= n) {
#pragma unroll
    for (int j = PB - 1; j >= 0; --j) {
      if (found < 0 && cum + v[j] >= n) found = lane * PB + j, cum_at = cum;
      if (found < 0) cum += v[j];
    }
  }
  const unsigned long long hit = __ballot(found >= 0);
  if (hit == 0) return make_int2(-1, 0);
  const int src = __ffsll((long long)hit) - 1;
  return make_int2(__shfl(found, src, 64), __shfl(cum_at, src, 64));
}

// Coarse bucket B and the count above it (B = -1: take every candidate).
__device__ __forceinline__ int2 coarse_bucket(const SelGeom& g, const int* sc) {
  if (g.C <= g.n) return make_int2(-1, 0);
  return wave_find_bin<256>(sc + SelScratch::kHist1, g.n, 0, g.C);
}

__global__ __launch_bounds__(kSelThreads) void sel_hist_fine(SelJob one, const SelJob* many) {
  const SelJob j = sel_job(one, many);
  if ((int)blockIdx.x >= j.G) return;
  const SelGeom& g = j.g;
  int* __restrict__ sc = j.sc;
  __shared__ int h[512];
  __shared__ int sB;
  if (threadIdx.x < 64) {
    const int2 r = coarse_bucket(g, sc);
    if (threadIdx.x == 0) sB = r.x;
  }
  for (int b = threadIdx.x; b < 512; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int B = sB;
  if (B < 0) return;
  for_chunk_scores(g, blockIdx.x * kSelChunk, [&](int, int sv) {
    if ((sv >> 9) == B) atomicAdd(&h[sv & 511], 1);
  });
  __syncthreads();
  for (int b = threadIdx.x; b < 512; b += blockDim.x)
    if (h[b]) atomicAdd(&sc[SelScratch::kHist2 + b], h[b]);
}

// Threshold T and the number of ties at T to keep (T = -1: take everything).
__device__ __forceinline__ int2 threshold(const SelGeom& g, const int* sc) {
  const int2 cb = coarse_bucket(g, sc);
  if (cb.x < 0) return make_int2(-1, 0);
  const int2 f = wave_find_bin<512>(sc + SelScratch::kHist2, g.n, cb.y);
  return make_int2(cb.x * 512 + f.x, g.n - f.y);
}

__global__ __launch_bounds__(kSelThreads) void sel_count(SelJob one, const SelJob* many) {
  const SelJob j = sel_job(one, many);
  if ((int)blockIdx.x >= j.G) return;
  const SelGeom& g = j.g;
  int* __restrict__ sc = j.sc;
  __shared__ int s_gt[kSelThreads / 64], s_eq[kSelThreads / 64];
  __shared__ int sT;
  if (threadIdx.x < 64) {
    const int2 r = threshold(g, sc);
    if (threadIdx.x == 0) sT = r.x;
  }
  __syncthreads();
  const int T = sT;
  int gt = 0, eq = 0;
  for_chunk_scores(g, blockIdx.x * kSelChunk, [&](int, int sv) {
    gt += sv > T;
    eq += sv == T;
  });
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
    sc[SelScratch::kChunks + 2 * blockIdx.x] = a;
    sc[SelScratch::kChunks + 2 * blockIdx.x + 1] = b;
  }
}

// Sum over the chunks before this one of (gt + kept ties) and of eq, where a
// chunk keeps clamp(need - ties before it, 0, eq) of its ties.  Each of the
// 256 threads reduces a strided share of the earlier chunks: the ties before
// chunk k are an exclusive prefix of eq, so the kept ties before this chunk
// total min(need, ties before it).
__device__ __forceinline__ int2 chunk_base(const int* sc, int G, int need, int* red) {
  int gt = 0, eq = 0;
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    if (k < (int)blockIdx.x) {
      gt += sc[SelScratch::kChunks + 2 * k];
      eq += sc[SelScratch::kChunks + 2 * k + 1];
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    gt += __shfl_xor(gt, d, 64);
    eq += __shfl_xor(eq, d, 64);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = gt, red[4 + (threadIdx.x >> 6)] = eq;
  __syncthreads();
  int a = 0, b = 0;
  for (int w = 0; w < kSelThreads / 64; ++w) a += red[w], b += red[4 + w];
  const int kept = need < b ? need : b;  // need >= 0
  return make_int2(a + kept, b);        // output offset, tie base
}

__global__ __launch_bounds__(kSelThreads) void sel_write(SelJob one, const SelJob* many) {
  const SelJob j = sel_job(one, many);
  if ((int)blockIdx.x >= j.G) return;
  const SelGeom& g = j.g;
  int* __restrict__ sc = j.sc;
  const int G = j.G;
  int32_t* __restrict__ idx = j.idx;
  int32_t* __restrict__ count = j.count;
  __shared__ int wsum[16];
  __shared__ int red[8];
  __shared__ int sT, sNeed, sLast;
  __shared__ int4 s_score[kSelChunk / 4];  // the chunk's scores, candidate order
  if (threadIdx.x < 64) {
    const int2 r = threshold(g, sc);
    if (threadIdx.x == 0) sT = r.x, sNeed = r.y;
  }
  // scores computed with consecutive threads on consecutive candidates (the
  // image reads coalesce), then each thread takes kSelPPT consecutive ones
  {
    int* sv = reinterpret_cast<int*>(s_score);
    const int cb = blockIdx.x * kSelChunk;
    for (int q = threadIdx.x; q < kSelChunk; q += blockDim.x)
      if (cb + q >= g.C) sv[q] = -2;  // past the last candidate
    for_chunk_scores(g, cb, [&](int q, int v) { sv[q] = v; });
  }
  __syncthreads();
  const int T = sT, need = sNeed;
  const int2 base = chunk_base(sc, G, need, red);
  const int c0 = blockIdx.x * kSelChunk + threadIdx.x * kSelPPT;
  int s[kSelPPT];
  int eq_local = 0;
#pragma unroll
  for (int j = 0; j < kSelPPT / 4; ++j) {
    const int4 v = s_score[threadIdx.x * (kSelPPT / 4) + j];
    s[4 * j] = v.x, s[4 * j + 1] = v.y, s[4 * j + 2] = v.z, s[4 * j + 3] = v.w;
  }
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j) eq_local += s[j] == T;
  int tot;
  int tie = block_exclusive_scan(eq_local, wsum, &tot) + base.y;
  bool sel[kSelPPT];
  int sel_local = 0;
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j) {
    const bool is_eq = s[j] == T;
    sel[j] = (s[j] > T) || (is_eq && tie < need);
    tie += is_eq;
    sel_local += sel[j];
  }
  int pos = block_exclusive_scan(sel_local, wsum, &tot) + base.x;
#pragma unroll
  for (int j = 0; j < kSelPPT; ++j)
    if (sel[j]) {
      int x, y;
      cand_xy(g, c0 + j, &x, &y);
      idx[pos++] = (g.m + y) * g.W + (g.m + x);
    }
  if (blockIdx.x == G - 1 && threadIdx.x == 0) *count = base.x + tot;
  // the last workgroup of the image to finish leaves the histograms cleared for
  // the next selection: every other one used the values it read from them
  // before its count went up (no fence: nothing written here is read in this
  // launch, and a release fence would write back the whole L2)
  __syncthreads();
  if (threadIdx.x == 0) sLast = atomicAdd(&sc[SelScratch::kDone], 1) == G - 1;
  __syncthreads();
  if (sLast) {
    for (int b = threadIdx.x; b < SelScratch::kDone; b += blockDim.x) sc[b] = 0;
    if (threadIdx.x == 0) sc[SelScratch::kDone] = 0;
  }
}

SelJob make_sel_job(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                    int32_t* count, int32_t* scratch) {
  SelJob j;
  j.g.img = img;
  j.g.W = W;
  j.g.m = margin;
  j.g.Wc = W - 2 * margin;
  const int Hc = H - 2 * margin;
  j.g.C = (j.g.Wc > 0 && Hc > 0) ? j.g.Wc * Hc : 0;
  j.g.n = n;
  j.g.inv_wc = j.g.Wc > 0 ? 1.0f / (float)j.g.Wc : 0.0f;
  j.g.pitch = W;
  j.g.pad = 0;
  j.sc = scratch;
  j.idx = idx;
  j.count = count;
  j.G = (j.g.C + kSelChunk - 1) / kSelChunk;
  j.pad = 0;
  return j;
}

// The pipeline for one image (many == nullptr) or for n_img images whose
// chunk counts are at most G_max.  The write pass leaves the histograms
// cleared, so sel_clear runs only where an image has no candidates (its count
// must still be written); the scratch starts zeroed (select_scratch_init).
static hipError_t run_select(const SelJob& one, const SelJob* many, int n_img, int G_max, bool any_empty,
                             hipStream_t s) {
  const dim3 grid(G_max > 0 ? G_max : 1, n_img);
  if (any_empty) hipLaunchKernelGGL(sel_clear, dim3(1, n_img), dim3(kSelThreads), 0, s, one, many);
  if (G_max > 0) {
    hipLaunchKernelGGL(sel_hist_coarse, grid, dim3(kSelThreads), 0, s, one, many);
    hipLaunchKernelGGL(sel_hist_fine, grid, dim3(kSelThreads), 0, s, one, many);
    hipLaunchKernelGGL(sel_count, grid, dim3(kSelThreads), 0, s, one, many);
    hipLaunchKernelGGL(sel_write, grid, dim3(kSelThreads), 0, s, one, many);
  }
  return hipGetLastError();
}

hipError_t launch_select(const uint8_t* img, int32_t W, int32_t H, int32_t margin, int32_t n, int32_t* idx,
                         int32_t* count, int32_t* scratch, hipStream_t s) {
  const SelJob j = make_sel_job(img, W, H, margin, n, idx, count, scratch);
  return run_select(j, nullptr, 1, j.G, j.G == 0, s);
}

hipError_t launch_select_batch(const SelJob* d_jobs, int n_img, int G_max, bool any_empty, hipStream_t s) {
  SelJob none;
  std::memset(&none, 0, sizeof none);
  return run_select(none, d_jobs, n_img, G_max, any_empty, s);
}

// ---------------------------------------------------------------- selection without allocation

// Histograms, completion counter and per-chunk counts of one selection of an
// image of up to kNoAllocSelectPixels pixels, for callers that cannot allocate.
// Every device holds its own copy for the life of the process; all calls on a
// device share it (calls that overlap on one device race).
constexpr int64_t kNoAllocSelectInts = SelScratch::kChunks + 2 * ((kNoAllocSelectPixels + kSelChunk - 1) / kSelChunk + 1);
static __device__ __align__(256) int32_t g_select_scratch[kNoAllocSelectInts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};  // device address of g_select_scratch, per device

// The device address of the current device's copy of g_select_scratch, looked
// up once per device (the array's name in host code is not that address).
hipError_t select_scratch_ptr(int32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_select_scratch))) != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

hipError_t launch_select_noalloc(const uint8_t* img, int32_t W, int32_t H, int64_t pitch, int32_t margin, int32_t n,
                                 int32_t* idx, int32_t* count, hipStream_t s) {
  if ((int64_t)W * H > kNoAllocSelectPixels || pitch < W || pitch > INT32_MAX) return hipErrorInvalidValue;
  int32_t* sc = nullptr;
  hipError_t e = select_scratch_ptr(&sc);
  if (e != hipSuccess) return e;
  SelJob j = make_sel_job(img, W, H, margin, n, idx, count, sc);
  j.g.pitch = (int32_t)pitch;
  // the histograms and the completion counter start at zero: cleared by a
  // kernel (no memset node, so the call can also be captured into a graph);
  // sel_clear also writes the count of an image without candidates
  hipLaunchKernelGGL(sel_clear, dim3(1, 1), dim3(kSelThreads), 0, s, j, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return run_select(j, nullptr, 1, j.G, false, s);
}

}  // namespace dpt
