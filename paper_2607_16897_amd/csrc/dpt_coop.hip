// Cooperative multi-workgroup track: every camera stream's map is split into
// chunks of CH points, one workgroup per chunk, one thread per point, and all
// chunks of all streams run in one cooperative (co-resident) launch that
// covers every level and iteration of the frame.
//
// Per Gauss-Newton iteration the chunks of a stream exchange their 32 partial
// sums through a double-buffered global array.  Each partial is one 64-bit
// word holding an epoch tag above the float's bits, so a reader knows from the
// word alone whether it is current: a chunk publishes its partials and polls
// the stream's words until every chunk's carry the tag, with no counter, no
// fence and no second read.  Every word is stored twice: a group-scope copy,
// which stays in the L2 of the chunk's XCD, and a device-scope copy, written
// through to memory.  A stream's chunks share one XCD (the work list places
// them so), where a device-scope poll finds the first copy in the shared L2 in
// about half the round trip of the second; every eighth poll reads the second
// copies instead, so a chunk that the dispatcher placed on another XCD is still
// seen.  Every chunk then sums the partials in one fixed order
// and every thread solves the 6x6 system itself: all threads of all chunks of
// a stream compute bitwise-identical poses, so one exchange per iteration
// suffices and the result is reproducible.  Waits are bounded: a chunk that
// polls longer than `spin_limit` times gives up and reports a timeout instead
// of hanging.
#include <climits>
#include <cstring>
#include <type_traits>

#include "dpt_device.h"

namespace dpt {

// Chunk words read per round trip while polling (one load each in flight).
constexpr int kPollBatch = 8;

// Polls of the L2 copies between two polls of the device-scope copies, minus one.
constexpr int kSlowPollMask = 7;

// Publish one partial word: the group-scope store (kept in the XCD's L2, no
// write-through) to `fast`, the device-scope one to `slow`.
__device__ __forceinline__ void publish_word(__attribute__((address_space(1))) uint64_t* fast,
                                             __attribute__((address_space(1))) uint64_t* slow, uint64_t w) {
  asm volatile("global_store_dwordx2 %0, %1, off sc0" : : "v"(fast), "v"(w) : "memory");
  __hip_atomic_store(slow, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The value lane (lane ^ D) holds, D = 16 or 32, moved within the register
// file (v_permlane16_swap / v_permlane32_swap exchange the rows, or the
// halves, of two registers) instead of through the LDS crossbar.
template <int D>
__device__ __forceinline__ uint32_t lane_xor_u(uint32_t u) {
  static_assert(D == 16 || D == 32, "row or half swap");
  if constexpr (D == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  }
}

template <int D>
__device__ __forceinline__ float lane_xor(float x) {
  return __uint_as_float(lane_xor_u<D>(__float_as_uint(x)));
}

// Row rotation within 16 lanes (DPP row_ror:K) of an integer.
template <int K>
__device__ __forceinline__ int dpp_ror_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xf, 0xf, false);
}

// The wave's minimum of lo and maximum of hi, in every lane: DPP rotations
// within each 16-lane row, then the row and half-wave swaps, with no LDS
// round trip between the steps.  All 64 lanes active.
__device__ __forceinline__ void wave_min_max(int& lo, int& hi) {
  lo = min(lo, dpp_ror_i<8>(lo)), hi = max(hi, dpp_ror_i<8>(hi));
  lo = min(lo, dpp_ror_i<4>(lo)), hi = max(hi, dpp_ror_i<4>(hi));
  lo = min(lo, dpp_ror_i<2>(lo)), hi = max(hi, dpp_ror_i<2>(hi));
  lo = min(lo, dpp_ror_i<1>(lo)), hi = max(hi, dpp_ror_i<1>(hi));
  lo = min(lo, (int)lane_xor_u<16>((uint32_t)lo)), hi = max(hi, (int)lane_xor_u<16>((uint32_t)hi));
  lo = min(lo, (int)lane_xor_u<32>((uint32_t)lo)), hi = max(hi, (int)lane_xor_u<32>((uint32_t)hi));
}

// Wave 0 only.  Publish this chunk's column sums (`mine`, lanes < NV) under
// `tag`, wait until all nch chunks of the stream published theirs, and return
// the stream totals (lanes < NV).  False on timeout.  A chunk's words are 32
// apart whatever NV is.  The wave's 64 / NV lane groups poll consecutive
// ranges of the chunks (group q the q-th range, lane v word v), so a poll
// round has 64 loads in flight, and the group sums meet in a fixed tree, the
// same in every chunk of the stream.
template <bool KAHAN, int NV>
__device__ __forceinline__ bool exchange_partials(uint64_t* partials, int chunk, int nch, uint32_t tag, float mine,
                                                  int spin_limit, float* total, int* polls = nullptr) {
  constexpr int G = 64 / NV;
  static_assert(G == 2 || G == 4, "32 or 16 values per chunk");
  static_assert(!(KAHAN && G != 2), "compensated sums use 32 values");
  const int lane = threadIdx.x & 63, q = lane / NV, v = lane % NV;
  // global-memory pointers: global loads and stores, which unlike flat ones
  // leave the LDS counter alone and skip the aperture check
  using gptr = __attribute__((address_space(1))) uint64_t*;
  gptr buf = (gptr)(partials + (size_t)(tag & 1u) * nch * 32);
  gptr slow = (gptr)(partials + (size_t)(2 + (tag & 1u)) * nch * 32);
  const uint64_t hi = (uint64_t)tag << 32;
  if (lane < NV) publish_word(&buf[chunk * 32 + lane], &slow[chunk * 32 + lane], hi | __float_as_uint(mine));
  const int per = (nch + G - 1) / G, cb = q * per, ce = cb + per < nch ? cb + per : nch;
  for (int t = 0; t < spin_limit; ++t) {
    const gptr rb = (t & kSlowPollMask) == kSlowPollMask ? slow : buf;
    float s = 0.0f, comp = 0.0f;
    int ok = 1;
    for (int c0 = cb; c0 < ce; c0 += kPollBatch) {
      // a batch of loads in flight, then the checks, with no branch between
      // the loads: past its range's end a lane re-reads the range's last
      // chunk and leaves the word out
      uint64_t w[kPollBatch];
#pragma unroll
      for (int j = 0; j < kPollBatch; ++j)
        w[j] = __hip_atomic_load(&rb[min(c0 + j, ce - 1) * 32 + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int j = 0; j < kPollBatch; ++j) {
        const bool in = c0 + j < ce;
        ok &= !in | ((uint32_t)(w[j] >> 32) == tag);
        const float x = __uint_as_float((uint32_t)w[j]);
        if (KAHAN) {
          const float y = x - comp;
          const float u = s + y;
          const float cn = (u - s) - y;
          s = in ? u : s;
          comp = in ? cn : comp;
        } else {
          const float u = s + x;
          s = in ? u : s;
        }
      }
    }
    if (__all(ok)) {
      if constexpr (G == 4) s += lane_xor<16>(s);  // (g0 + g1), (g2 + g3)
      if constexpr (KAHAN) {  // the two compensated sums: (s0 - c0) + (s1 - c1)
        const float ps = lane_xor<32>(s), pc = lane_xor<32>(comp);
        const float lo_s = q == 0 ? s : ps, lo_c = q == 0 ? comp : pc;
        const float hi_s = q == 0 ? ps : s, hi_c = q == 0 ? pc : comp;
        const float y = hi_s - (lo_c + hi_c);
        s = lo_s + y;
      } else {
        s += lane_xor<32>(s);
      }
      *total = s;
      if (kCycleProfile && polls) *polls = t + 1;
      return true;
    }
    // no sleep between rounds: a round is already a memory round trip, and
    // the next one starts as soon as this one has shown a word missing
  }
  return false;
}

// Polling by the whole workgroup, for streams of more than kPollBatch chunks:
// thread t reads value t % 32 of chunks c = t / 32 (mod blockDim / 32 groups),
// four loads in flight, and sums them in chunk order; the groups' sums meet in
// LDS (sh_grp, blockDim floats) and are added in group order, a fixed order
// shared by every chunk of the stream.  All threads; false on timeout.
template <bool KAHAN, int NV>
__device__ __forceinline__ bool exchange_wide(const uint64_t* partials, int nch, uint32_t tag, int spin_limit,
                                              float* sh_grp, float* sh_tot) {
  const int t = threadIdx.x, v = t & 31, q = t >> 5, G = blockDim.x >> 5;
  // global-memory pointers, no branch between a batch's loads and no sleep
  // between rounds, as in exchange_partials: past the last chunk a lane
  // re-reads it and drops the word
  using gptr = const __attribute__((address_space(1))) uint64_t*;
  const gptr buf = (gptr)(partials + (size_t)(tag & 1u) * nch * 32);
  const gptr slow = (gptr)(partials + (size_t)(2 + (tag & 1u)) * nch * 32);
  float s = 0.0f, comp = 0.0f;
  bool ok = true;
  if (v < NV) {
    ok = false;
    for (int it = 0; it < spin_limit && !ok; ++it) {
      const gptr rb = (it & kSlowPollMask) == kSlowPollMask ? slow : buf;
      s = 0.0f, comp = 0.0f;
      ok = true;
      for (int c0 = q; c0 < nch; c0 += 4 * G) {
        uint64_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          w[j] = __hip_atomic_load(&rb[min(c0 + j * G, nch - 1) * 32 + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool in = c0 + j * G < nch;
          ok &= !in | ((uint32_t)(w[j] >> 32) == tag);
          const float x = __uint_as_float((uint32_t)w[j]);
          if (KAHAN) {
            const float y = x - comp;
            const float u = s + y;
            const float cn = (u - s) - y;
            s = in ? u : s;
            comp = in ? cn : comp;
          } else {
            const float u = s + x;
            s = in ? u : s;
          }
        }
      }
    }
    sh_grp[q * NV + v] = s;
  }
  const int bad = __syncthreads_or(!ok);
  if (t < NV) {
    float tot = 0.0f, c2 = 0.0f;
    for (int g = 0; g < G; ++g) {
      const float x = sh_grp[g * NV + t];
      if (KAHAN) {
        const float y = x - c2;
        const float u = tot + y;
        c2 = (u - tot) - y;
        tot = u;
      } else {
        tot += x;
      }
    }
    sh_tot[t] = tot;
  }
  return bad == 0;
}

// Block sum of acc[NV] (after each thread accumulated its point), exchanged
// across the stream's chunks; the totals land in sh_tot and, in every thread,
// in tot.  Returns false on timeout (same value in every thread).  NV = 32 or
// 16.  WIDE: streams of more than kPollBatch chunks are polled by the whole
// workgroup (exchange_wide, sh_grp: blockDim floats of LDS); otherwise wave 0
// polls alone.  NW: the workgroup's waves (blockDim / 64).
template <bool KAHAN, int NV, bool WIDE, int NW>
__device__ __forceinline__ bool stream_total(float (&acc)[NV], float* sh_red, float* sh_tot, int* sh_ok,
                                             uint64_t* partials, int chunk, int nch, uint32_t tag,
                                             int spin_limit, float* sh_grp, float (&tot)[NV],
                                             uint64_t* t_bar = nullptr, int* polls = nullptr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int PER_ROW = NV / 4;  // values per 16-lane row after the wave reduction
  if constexpr (NV == 32)
    wave_reduce32(acc);
  else
    wave_reduce16(acc);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int j = 0; j < PER_ROW; ++j) sh_red[wave * NV + PER_ROW * (lane >> 4) + j] = acc[j];
  }
  __syncthreads();
  if (kCycleProfile && t_bar) *t_bar = clock64();
  if (wave == 0) {
    float s = 0.0f, comp = 0.0f;
    if (lane < NV) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {  // all NW reads in flight at once, then the sum in wave order
        const float x = sh_red[w * NV + lane];
        if (KAHAN) {
          const float y = x - comp;
          const float u = s + y;
          comp = (u - s) - y;
          s = u;
        } else {
          s += x;
        }
      }
    }
    if (WIDE && nch > kPollBatch) {  // publish; the whole workgroup polls below
      if (lane < NV)
        publish_word((__attribute__((address_space(1))) uint64_t*)&partials[(size_t)(tag & 1u) * nch * 32 + chunk * 32 + lane],
                     (__attribute__((address_space(1))) uint64_t*)&partials[(size_t)(2 + (tag & 1u)) * nch * 32 +
                                                                           chunk * 32 + lane],
                     ((uint64_t)tag << 32) | __float_as_uint(s));
    } else {
      float tot = s;
      bool ok = true;
      if (nch > 1) ok = exchange_partials<KAHAN, NV>(partials, chunk, nch, tag, s, spin_limit, &tot, polls);
      if (lane < NV) sh_tot[lane] = tot;
      if (lane == 0) *sh_ok = ok ? 1 : 0;
    }
  }
  bool ok;
  if (WIDE && nch > kPollBatch) {
    ok = exchange_wide<KAHAN, NV>(partials, nch, tag, spin_limit, sh_grp, sh_tot);
    __syncthreads();
  } else {
    __syncthreads();
    ok = *sh_ok != 0;
  }
  // every total requested with the verdict, before any test of either: left to
  // itself the compiler reads each behind the branch that first needs it, one
  // LDS round trip per test on the iteration's path
#pragma unroll
  for (int j = 0; j < NV; ++j) tot[j] = sh_tot[j];
  asm volatile("" ::: "memory");
  return ok;
}

// 3x4 rigid transforms (row-major [R | t]) in FP64, one output element per
// thread t < 12: out = A B, and out = A^-1 = [R^T | -R^T t].
__device__ __forceinline__ double compose34_elem(const double* A, const double* B, int t) {
  const int r = t >> 2, c = t & 3;
  double v = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c];
  return c == 3 ? v + A[4 * r + 3] : v;
}

__device__ __forceinline__ double invert34_elem(const double* A, int t) {
  const int r = t >> 2, c = t & 3;
  if (c < 3) return A[4 * c + r];
  return -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
}

// Constant-velocity start P1 P0^-1 P1 from the pose history (h0 = P0, h1 = P1
// in LDS), taken relative to the reference (P T_rw^-1), into T0.  Block-wide.
__device__ __forceinline__ void const_velocity_start(double* T0, const double* rw, const double* h0,
                                                     const double* h1, double* m1, double* m2) {
  const int t = threadIdx.x;
  if (t < 12) m1[t] = invert34_elem(h0, t);
  if (t >= 16 && t < 28) m2[t - 16] = invert34_elem(rw, t - 16);
  __syncthreads();
  double v = 0.0;
  if (t < 12) v = compose34_elem(h1, m1, t);  // P1 P0^-1
  __syncthreads();
  if (t < 12) m1[t] = v;
  __syncthreads();
  if (t < 12) v = compose34_elem(m1, h1, t);  // (P1 P0^-1) P1
  __syncthreads();
  if (t < 12) m1[t] = v;
  __syncthreads();
  if (t < 12) T0[t] = compose34_elem(m1, m2, t);  // relative to the reference
  __syncthreads();
  if (t == 0) orthonormalize34(T0);
  __syncthreads();
}

// Start pose relative to the reference for this launch: the given one, one
// in device memory (a learned proposal), or the constant-velocity prediction
// from the stream's pose history.  Block-wide;
// the result, the reference pose and the history land in LDS.
__device__ __forceinline__ void start_pose(const StartSlot* __restrict__ st, const double* __restrict__ hist,
                                           double* T0, double* rw, double* h0, double* h1, double* m1, double* m2,
                                           const uint8_t** l0, int64_t* l0_stride) {
  const int t = threadIdx.x;
  __shared__ int sh_mode;
  if (t < 12) {
    // kStartDevice: the proposal an earlier launch on this stream wrote
    T0[t] = st->mode > 1.5 ? st->dev_rel[t] : st->T_rel[t];
    rw[t] = st->T_rw[t];
    h0[t] = hist[t];
    h1[t] = hist[12 + t];
  }
  if (t == 0) sh_mode = st->mode > 1.5 ? kStartDevice : st->mode > 0.5 ? kStartConstVelocity : kStartGiven;
  if (t == 32) *l0 = st->l0, *l0_stride = st->l0_stride;
  __syncthreads();
  if (sh_mode == kStartConstVelocity) const_velocity_start(T0, rw, h0, h1, m1, m2);
}

// ---------------------------------------------------------------- cycle split (DPT_CYCLE_PROFILE builds)

#ifdef DPT_CYCLE_PROFILE
constexpr int kCycFields = DPT_CYCLE_FIELDS;
__device__ uint64_t g_cycles[kCycleSlots * kCycFields];
#endif

// Where this workgroup runs: XCC id << 32 | HW_ID (CU, SIMD, shader engine).
__device__ __forceinline__ uint64_t hw_place() {
#ifdef DPT_CYCLE_PROFILE
  uint32_t xcc, hw;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
  return ((uint64_t)xcc << 32) | hw;
#else
  return 0;
#endif
}

// Thread 0's phase sums of one launch into the slot's totals.
__device__ __forceinline__ void cycles_flush(const uint64_t (&cy)[4], uint64_t iters, uint64_t t_start,
                                             uint64_t rt_start, uint64_t polls, const uint64_t (&fr)[5]) {
#ifdef DPT_CYCLE_PROFILE
  if (threadIdx.x != 0 || blockIdx.x >= (unsigned)kCycleSlots) return;
  uint64_t* o = g_cycles + (size_t)blockIdx.x * kCycFields;
  for (int k = 0; k < 4; ++k) atomicAdd((unsigned long long*)&o[k], (unsigned long long)cy[k]);
  atomicAdd((unsigned long long*)&o[DPT_CYCLE_ITERATIONS], (unsigned long long)iters);
  atomicAdd((unsigned long long*)&o[DPT_CYCLE_LAUNCHES], 1ull);
  atomicAdd((unsigned long long*)&o[DPT_CYCLE_KERNEL], (unsigned long long)(clock64() - t_start));
  atomicAdd((unsigned long long*)&o[DPT_CYCLE_REALTIME], (unsigned long long)(wall_clock64() - rt_start));
  atomicAdd((unsigned long long*)&o[DPT_CYCLE_POLLS], (unsigned long long)polls);
  for (int k = 0; k < 5; ++k) atomicAdd((unsigned long long*)&o[DPT_CYCLE_FRAME_START + k], (unsigned long long)fr[k]);
  o[DPT_CYCLE_PLACE] = hw_place();
#else
  (void)cy, (void)iters, (void)t_start, (void)rt_start, (void)polls, (void)fr;
#endif
}

hipError_t read_cycle_profile(uint64_t* host, int n_slots, bool reset) {
#ifdef DPT_CYCLE_PROFILE
  if (n_slots < 1 || n_slots > kCycleSlots) return hipErrorInvalidValue;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyFromSymbol(host, HIP_SYMBOL(g_cycles), sizeof(uint64_t) * kCycFields * n_slots)) != hipSuccess)
    return e;
  if (reset) {
    static uint64_t zeros[kCycleSlots * kCycFields] = {};
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_cycles), zeros, sizeof zeros)) != hipSuccess) return e;
  }
  return hipDeviceSynchronize();
#else
  (void)host, (void)n_slots, (void)reset;
  return hipErrorNotSupported;
#endif
}

// ---------------------------------------------------------------- LDS tiles of the current level

// Bytes of a level a workgroup of the 8-pixel kernels stages in LDS: levels of
// up to this size whole, larger ones as the band of rows its points' taps span.
// Launches of many workgroups (two per compute unit, 160 KB of LDS each) take
// the small tile: with the kernel's own ~2 KB a workgroup stays within 64 KB.
// A launch small enough to run one workgroup per compute unit (the plain-launch
// path) takes the large one, which holds a 752x480 frame's second level whole
// and ~190 rows of its first.
constexpr int kTileBytesSmall = 60 * 1024;
constexpr int kTileBytesLarge = 144 * 1024;
constexpr int kTilePad = 16;  // the last pair of words read past the last byte
// Rows kept around the band at the level's start pose: the pose moves during the
// level's iterations.  Points whose taps leave the band are read from global
// memory (their whole wave).
constexpr int kBandMargin = 4;

// Stage level g of the current frame (img = its first byte) in the workgroup's
// LDS tile: the whole level if it fits, else the rows the taps of the usable
// points span at pose T, widened by kBandMargin and cut to the tile's size.
// Copies the 16-byte granules that overlap those rows (each holds at least one
// byte of them, so none crosses into a page the level does not touch).
// Block-wide (NW waves); the caller has finished every read of the previous
// tile.  The points' geometry arrives as loaded (raw) and is completed into pr
// here: before the band is computed from it, or, for a whole level, after the
// copy is issued, so the copy's latency and the point loads' overlap.
template <int NW, class PR>
__device__ __forceinline__ Tile8 stage_tile(const IterParams& a, const PatRegs& pat, const LevelGeom& g,
                                            const uint8_t* img, const float* T, PR& pr, GeoRaw& raw,
                                            uint8_t* tile_mem, int tile_bytes, int* sh_band) {
  const int W = g.W, H = g.H;
  const int rows_fit = (tile_bytes - 32) / W;
  int lo = 0, hi = H - 1;
  if (rows_fit < H) {
    finish_geometry(pr, raw);
    float X, Y, Z;
    transform(T, pr.X0, pr.Y0, pr.Z0, X, Y, Z);
    const float iz = __builtin_amdgcn_rcpf(Z);
    const float u = fmaf(g.fx * X, iz, g.cx), v = fmaf(g.fy * Y, iz, g.cy);
    const bool ok = pr.ok & (Z > a.z_min) & inside(g, pat, u, v);
    const int iv = (int)floorf(ok ? v : 0.0f);
    int rlo = ok ? iv + (int)pat.dy_min : INT_MAX, rhi = ok ? iv + (int)pat.dy_max + 1 : INT_MIN;
    wave_min_max(rlo, rhi);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh_band[2 * wave] = rlo, sh_band[2 * wave + 1] = rhi;
    __syncthreads();
    rlo = INT_MAX, rhi = INT_MIN;
#pragma unroll
    for (int w = 0; w < NW; ++w) rlo = min(rlo, sh_band[2 * w]), rhi = max(rhi, sh_band[2 * w + 1]);
    if (rlo <= rhi) {
      lo = max(0, rlo - kBandMargin);
      hi = min(H - 1, rhi + kBandMargin);
    }
    if (hi - lo + 1 > rows_fit) hi = lo + rows_fit - 1;  // the rows below are read from global memory
  }
  const uintptr_t sa = reinterpret_cast<uintptr_t>(img + (int64_t)lo * W), s0 = sa & ~(uintptr_t)15;
  const int delta = (int)(sa - s0);
  const int ng = (delta + (hi - lo + 1) * W + 15) >> 4;
  // Global memory straight into LDS (global_load_lds_dwordx4): each wave moves
  // 64 consecutive granules per instruction, every load in flight at once and
  // no registers held.  The caller waits for all of them (s_waitcnt 0, then a
  // workgroup barrier) before the tile is read.
  const int lane = threadIdx.x & 63;
  for (int q0 = (int)(threadIdx.x & ~63u); q0 < ng; q0 += blockDim.x) {
    const int q = q0 + lane;
    if (q < ng)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(s0 + 16 * (uintptr_t)q),
                                       (__attribute__((address_space(3))) void*)(tile_mem + 16 * q0), 16, 0, 0);
  }
  if (rows_fit >= H) finish_geometry(pr, raw);
  Tile8 t;
  t.lds = (const __attribute__((address_space(3))) uint8_t*)(tile_mem);
  t.lo = lo, t.hi = hi, t.delta = delta, t.bytes = ng * 16;
  return t;
}

// The pattern offsets of this thread's samples: all 8, or (NS = 4) the half
// `sub` of a point's pair takes.
template <int NS>
__device__ __forceinline__ void lane_offsets(const PatRegs& pat, int W, int sub, int (&off)[NS]) {
  int all[8];
  pattern_offsets(pat, W, all);
#pragma unroll
  for (int k = 0; k < NS; ++k) off[k] = NS == 8 ? all[k] : (sub ? all[NS + k] : all[k]);
}

// A tile that holds no row: every usable point reads global memory.
__device__ __forceinline__ Tile8 no_tile(uint8_t* tile_mem) {
  Tile8 t;
  t.lds = (const __attribute__((address_space(3))) uint8_t*)(tile_mem);
  t.lo = 1, t.hi = 0, t.delta = 0, t.bytes = 16;
  return t;
}

// MIXED: FP16 reference cache, Kahan-compensated FP32 sums across waves and
// chunks, FP64 solve, exponential and pose state.
// FIXED: fixed-H mode (FP32): unweighted residuals, only b, the cost and the
// counts are reduced and exchanged (16 slots), and each level's constant H
// comes factored from the precompute.
// GENERIC: any pattern K (four lanes per point, CH / 4 points per chunk) on
// uint8 levels or (PIX = float) the floating-point Gaussian pyramid.
//
// LPP = 2 (8-pixel pattern only): two threads per point, four samples each;
// a chunk of CH threads holds CH / 2 points.
template <int CH, bool MIXED, bool FIXED, bool GENERIC = false, class PIX = uint8_t, bool WIN = false, int LPP = 1>
__global__ __launch_bounds__(CH, 2) void coop_track_kernel(const CoopStream* __restrict__ streams,
                                                           const int2* __restrict__ work,
                                                           const StartSlot* __restrict__ start,
                                                           TrackOut* __restrict__ out_ring, int slot, int n_out,
                                                           int n_frames, uint32_t seq0, uint32_t tag_base,
                                                           int spin_limit, int tile_bytes) {
  static_assert(!(MIXED && FIXED), "the fixed-H mode computes in FP32");
  static_assert(!(MIXED && GENERIC) && (GENERIC || std::is_same<PIX, uint8_t>::value), "variant");
  static_assert(LPP == 1 || (LPP == 2 && !GENERIC), "two threads per point: the 8-pixel kernels");
  using PR8 = typename std::conditional<MIXED, PointRegsH, PointRegs>::type;
  using PR4 = typename std::conditional<MIXED, PointRegsH4, PointRegs4>::type;
  using PR = typename std::conditional<GENERIC, PointGeo, typename std::conditional<LPP == 2, PR4, PR8>::type>::type;
  constexpr bool FLOAT_PYR = std::is_same<PIX, float>::value;
  constexpr int TPP = GENERIC ? kLanesPerPoint : LPP;  // threads per point
  constexpr int PPC = CH / TPP;                        // points per chunk
  constexpr int NS = 8 / LPP;                          // samples per thread (8-pixel kernels)
  constexpr int NV = FIXED ? kFixSlots : 32;
  constexpr int sE = FIXED ? kFixE : kSlotE, sN = FIXED ? kFixN : kSlotN, sP = FIXED ? kFixPts : kSlotPts;
  __shared__ CoopStream ss;
  __shared__ float sh_fac[FIXED ? 2 : 1][28];  // fixed H: factor of the level (L, invd, bad), by level parity
  __shared__ double sh_T0[12], sh_rw[12], sh_h0[12], sh_h1[12], sh_m1[12], sh_m2[12];
  __shared__ float sh_tot[32];
  __shared__ float sh_red[(CH / 64) * 32];
  __shared__ float sh_grp[GENERIC ? CH : 1];  // the whole-workgroup exchange of many-chunk streams
  __shared__ int sh_ok;
  __shared__ int sh_band[2 * (CH / 64)];
  extern __shared__ __align__(16) uint8_t sh_tile[];  // tile_bytes + kTilePad for the 8-pixel kernels, else none
  __shared__ const uint8_t* sh_l0;
  __shared__ int64_t sh_l0_stride;
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding slot of the XCD-aware work list
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(streams + w.x);
    for (int j = threadIdx.x; j < (int)(sizeof(CoopStream) / 4); j += blockDim.x)
      reinterpret_cast<uint32_t*>(&ss)[j] = src[j];
  }
  __syncthreads();
  if (start[w.x].bank) {  // the stream's second reference bank, and its window pyramids
    for (int j = threadIdx.x; j < (int)(sizeof(RefCache) / 4); j += blockDim.x)
      reinterpret_cast<uint32_t*>(&ss.a.ref)[j] = reinterpret_cast<const uint32_t*>(&ss.ref_alt)[j];
    if (threadIdx.x == 0) ss.win = ss.win_alt;
    __syncthreads();
  }
  start_pose(start + w.x, ss.hist, sh_T0, sh_rw, sh_h0, sh_h1, sh_m1, sh_m2, &sh_l0, &sh_l0_stride);
  const TrackArgs& a = ss.a;
  const IterParams ip(a);
  const PatRegs pregs = pattern_regs(a.pat);
  const int chunk = w.y, nch = ss.n_chunks;
  const int i = chunk * PPC + (int)threadIdx.x / TPP;
  const int sub = (int)threadIdx.x % TPP;
  const int nf = WIN ? n_frames : 1;
  uint32_t tag = tag_base;
  uint64_t cy[4] = {0, 0, 0, 0}, cy_iters = 0, cy_t0 = 0, cy_rt0 = 0, cy_polls = 0;
  uint64_t cy_fr[5] = {0, 0, 0, 0, 0};  // frame start, level starts, final pass, frames, frame end
  if constexpr (kCycleProfile) cy_t0 = clock64(), cy_rt0 = wall_clock64();
  // WIN: the frames of the launch in order, each from the constant-velocity
  // prediction of the history the previous one extended.  Every chunk keeps its
  // own copy of the history in LDS: the poses are bitwise identical in all
  // chunks of a stream, so no exchange is needed between frames.
  for (int f = 0; f < nf; ++f) {
    uint64_t cf0 = 0;
    if constexpr (kCycleProfile) cf0 = clock64();
    if (WIN && f > 0) const_velocity_start(sh_T0, sh_rw, sh_h0, sh_h1, sh_m1, sh_m2);
    const PIX* cur = WIN        ? reinterpret_cast<const PIX*>(ss.win + f * ss.win_stride)
                     : FLOAT_PYR ? reinterpret_cast<const PIX*>(a.curf)
                                 : reinterpret_cast<const PIX*>(a.cur);
    // level 0 of the frame: from the source frames themselves when the window
    // pyramids were built without it
    const PIX* cur0 = WIN && sh_l0 ? reinterpret_cast<const PIX*>(sh_l0 + f * sh_l0_stride) : cur + a.lv[0].off;
    // pose state, identical in every thread of every chunk of the stream
    float T[12];
    double Td[MIXED ? 12 : 1];
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      T[j] = (float)sh_T0[j];
      if (MIXED) Td[j] = sh_T0[j];
    }
    int status = 0, iterations = 0;
    int ipl[kMaxLevels];
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) ipl[j] = 0;
    int64_t samples = 0;
    bool stop = false, timed_out = false;
    PR pr;
    // the level-0 tile and point registers, reused by the final pass when the
    // levels ran down to 0
    Tile8 tile0 = no_tile(sh_tile);
    bool at0 = false;
    if constexpr (kCycleProfile) cy_fr[0] += clock64() - cf0, ++cy_fr[3];
    for (int l = a.levels - 1; l >= 0 && !stop; --l) {
      uint64_t cl0 = 0;
      if constexpr (kCycleProfile) cl0 = clock64();
      const LevelGeom g = a.lv[l];
      const PIX* img = WIN && l == 0 ? cur0 : cur + g.off;
      Tile8 tile;
      int offs[NS];
      if constexpr (GENERIC) {
        load_point_geo(a, l, i, pr);
      } else {
        GeoRaw raw;
        load_point_raw(a, l, i, sub, pr, raw);
        lane_offsets<NS>(pregs, g.W, sub, offs);
        tile = stage_tile<CH / 64>(ip, pregs, g, reinterpret_cast<const uint8_t*>(img), T, pr, raw, sh_tile, tile_bytes,
                                   sh_band);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (l == 0) tile0 = tile, at0 = true;
      }
      if constexpr (FIXED) {
        // read by every thread after the next exchange's barrier; the other
        // parity's copy may still be in use by a previous level's solve
        const FixedH& fh = a.ref.fixed[l];
        if (threadIdx.x < 21) sh_fac[l & 1][threadIdx.x] = fh.L[threadIdx.x];
        if (threadIdx.x >= 32 && threadIdx.x < 38) sh_fac[l & 1][21 + threadIdx.x - 32] = fh.invd[threadIdx.x - 32];
        if (threadIdx.x == 40) sh_fac[l & 1][27] = fh.bad ? 1.0f : 0.0f;
      }
      bool converged = false;
      const int it0 = iterations;
      if constexpr (kCycleProfile) cy_fr[1] += clock64() - cl0;
      for (int it = 0; it < ip.max_iters; ++it) {
        uint64_t c0 = 0, c1 = 0, c2 = 0;
        if constexpr (kCycleProfile) c0 = clock64();
        float acc[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = 0.f;
        if constexpr (GENERIC)
          accumulate_point_generic<false, PIX, NV>(a, a.pat, g, img, T, pr, sub, acc);
        else
          accumulate_point8<false, PR, NV, NS>(ip, pregs, offs, g, reinterpret_cast<const uint8_t*>(img), tile, T,
                                               pr, acc, sub == 0);
        if constexpr (kCycleProfile) c1 = clock64();
        int polls = 0;
        float tot[NV];
        if (!stream_total<MIXED, NV, GENERIC, CH / 64>(acc, sh_red, sh_tot, &sh_ok, ss.partials, chunk, nch, tag,
                                                       spin_limit, sh_grp, tot, &c2, &polls)) {
          timed_out = stop = true;
          break;
        }
        uint64_t c3 = 0;
        if constexpr (kCycleProfile) c3 = clock64();
        ++tag;
        // the 8-pixel kernels count samples as 8 per point outside the final pass
        samples += GENERIC ? (int64_t)(int)tot[sN] : 8 * (int64_t)(int)tot[sP];  // counts < 2^24: exact
        if ((int)tot[sP] < ip.min_points) {
          status = 2;  // too few points
          stop = true;
          break;
        }
        int bad;
        double step;
        if (FIXED) {
          const float* fac = sh_fac[FIXED ? (l & 1) : 0];
          bad = fac[27] != 0.0f;
          float stepf = 0.0f;
          if (!bad) solve_fixed(fac, fac + 21, tot + kFixB, T, &stepf);
          step = stepf;
        } else if (MIXED) {
          bad = solve_update_d(tot, Td, &step);
          if (!bad)
#pragma unroll
            for (int j = 0; j < 12; ++j) T[j] = (float)Td[j];
        } else {
          float stepf;
          bad = solve_update(tot, T, &stepf);
          step = stepf;
        }
        if constexpr (kCycleProfile) {
          const uint64_t c4 = clock64();
          cy[0] += c1 - c0, cy[1] += c2 - c1, cy[2] += c3 - c2, cy[3] += c4 - c3, ++cy_iters, cy_polls += polls;
        }
        if (bad) {
          status = 3;  // not positive definite
          stop = true;
          break;
        }
        ++iterations;
        if (step < (double)ip.step_eps) {
          converged = true;
          break;
        }
      }
#pragma unroll
      for (int j = 0; j < kMaxLevels; ++j) ipl[j] = j == l ? iterations - it0 : ipl[j];
      if (!stop && l == 0 && !converged) status = 1;  // iteration cap at level 0
    }
    uint64_t cp0 = 0;
    if constexpr (kCycleProfile) cp0 = clock64();
    if (!timed_out) {  // final cost-only pass at level 0
      float acc[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) acc[j] = 0.f;
      const LevelGeom g = a.lv[0];
      if constexpr (GENERIC) {
        load_point_geo(a, 0, i, pr);
        accumulate_point_generic<true, PIX, NV>(a, a.pat, g, WIN ? cur0 : cur + g.off, T, pr, sub, acc);
      } else {
        if (!at0) {  // the levels stopped above 0: level 0's registers, taps from global memory
          if constexpr (LPP == 2)
            load_point(a, 0, i, sub, pr);
          else
            load_point(a, 0, i, pr);
        }
        int offs[NS];
        lane_offsets<NS>(pregs, g.W, sub, offs);
        accumulate_point8<true, PR, NV, NS>(ip, pregs, offs, g, WIN ? cur0 : cur + g.off, tile0, T, pr, acc, sub == 0);
      }
      float tot[NV];
      if (!stream_total<MIXED, NV, GENERIC, CH / 64>(acc, sh_red, sh_tot, &sh_ok, ss.partials, chunk, nch, tag,
                                                     spin_limit, sh_grp, tot))
        timed_out = true;
      ++tag;
    }
    if constexpr (kCycleProfile) cy_fr[2] += clock64() - cp0;
    if constexpr (!WIN) {
      if (chunk == 0 && threadIdx.x == 0) {
        TrackOut* o = out_ring + (size_t)slot * n_out + w.x;
        double Tf[12];
        for (int j = 0; j < 12; ++j) Tf[j] = MIXED ? Td[j] : (double)T[j];
        orthonormalize34(Tf);
        for (int j = 0; j < 12; ++j) {
          o->T[j] = T[j];
          o->Td[j] = Tf[j];
        }
        // the pose history gains this track's estimate T_cw = T_rel T_rw (every
        // chunk read the history at its start, before its first exchange)
        for (int j = 0; j < 12; ++j) {
          ss.hist[j] = sh_h1[j];
          ss.hist[12 + j] = compose34_elem(Tf, sh_rw, j);
        }
        o->E = sh_tot[sE];
        o->n = sh_tot[sN];
        o->iterations = iterations;
        for (int j = 0; j < kMaxLevels; ++j) o->iters_per_level[j] = ipl[j];
        o->n_valid_points = (int)sh_tot[sP];
        o->status = timed_out ? kStatusTimeout : status;
        o->samples = samples + (int64_t)sh_tot[sN];
        // the fields reach the host before the sequence number: a system-scope
        // release (no acquire, so the L2 keeps the reference data it holds)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        o->seq = seq0;
      }
      if constexpr (kCycleProfile) cycles_flush(cy, cy_iters, cy_t0, cy_rt0, cy_polls, cy_fr);
      return;
    }
    uint64_t ct0 = 0;
    if constexpr (kCycleProfile) ct0 = clock64();
    if (threadIdx.x == 0) {
      double Tf[12];
      for (int j = 0; j < 12; ++j) Tf[j] = MIXED ? Td[j] : (double)T[j];
      orthonormalize34(Tf);
      for (int j = 0; j < 12; ++j) sh_m1[j] = Tf[j];
      if (chunk == 0) {
        TrackOut* o = out_ring + (size_t)((slot + f) % kRing) * n_out + w.x;
        for (int j = 0; j < 12; ++j) {
          o->T[j] = T[j];
          o->Td[j] = Tf[j];
        }
        o->E = sh_tot[sE];
        o->n = sh_tot[sN];
        o->iterations = iterations;
        for (int j = 0; j < kMaxLevels; ++j) o->iters_per_level[j] = ipl[j];
        o->n_valid_points = (int)sh_tot[sP];
        o->status = timed_out ? kStatusTimeout : status;
        o->samples = samples + (int64_t)sh_tot[sN];
        // a chunk gave up: so do the frames after this one
        if (timed_out)
          for (int q = f + 1; q < nf; ++q) out_ring[(size_t)((slot + q) % kRing) * n_out + w.x].status = kStatusTimeout;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // the fields reach the host before the sequence numbers
        o->seq = seq0 + f;
        if (timed_out)
          for (int q = f + 1; q < nf; ++q) out_ring[(size_t)((slot + q) % kRing) * n_out + w.x].seq = seq0 + q;
      }
    }
    __syncthreads();
    // the history gains this frame's estimate T_cw = T_rel T_rw
    if (threadIdx.x < 12) {
      const double v = compose34_elem(sh_m1, sh_rw, threadIdx.x);
      sh_h0[threadIdx.x] = sh_h1[threadIdx.x];
      sh_h1[threadIdx.x] = v;
    }
    __syncthreads();
    if constexpr (kCycleProfile) cy_fr[4] += clock64() - ct0;
    if (timed_out) break;
  }
  // the stream's history for the next launch (every chunk read it at its start,
  // before its first exchange)
  if (WIN && chunk == 0 && threadIdx.x < 12) {
    ss.hist[threadIdx.x] = sh_h0[threadIdx.x];
    ss.hist[12 + threadIdx.x] = sh_h1[threadIdx.x];
  }
  if constexpr (kCycleProfile) cycles_flush(cy, cy_iters, cy_t0, cy_rt0, cy_polls, cy_fr);
}

// The kernel of a variant (kCoop* bits); WIN: the window form.  Null for a
// combination that does not exist (a generic variant at another chunk size,
// window tracking of the floating-point pyramid).
template <int CH, bool WIN>
static const void* coop_fn(int variant) {
  if (variant & kCoopGeneric) {
    if (CH != kGenericThreads) return nullptr;
    constexpr int G = kGenericThreads;
    switch (variant & (kCoopFixedH | kCoopFloatPyr)) {
      case 0: return reinterpret_cast<const void*>(&coop_track_kernel<G, false, false, true, uint8_t, WIN>);
      case kCoopFixedH: return reinterpret_cast<const void*>(&coop_track_kernel<G, false, true, true, uint8_t, WIN>);
      case kCoopFloatPyr:
        return WIN ? nullptr : reinterpret_cast<const void*>(&coop_track_kernel<G, false, false, true, float>);
      default: return WIN ? nullptr : reinterpret_cast<const void*>(&coop_track_kernel<G, false, true, true, float>);
    }
  }
  if (variant & kCoopPairs) {
    if (CH == 64) return nullptr;  // a pair chunk holds 64 or 128 points
    switch (variant & ~kCoopPairs) {
      case kCoopFP32:
        return reinterpret_cast<const void*>(&coop_track_kernel<CH, false, false, false, uint8_t, WIN, 2>);
      case kCoopMixed:
        return reinterpret_cast<const void*>(&coop_track_kernel<CH, true, false, false, uint8_t, WIN, 2>);
      case kCoopFixedH:
        return reinterpret_cast<const void*>(&coop_track_kernel<CH, false, true, false, uint8_t, WIN, 2>);
      default: return nullptr;
    }
  }
  switch (variant) {
    case kCoopFP32: return reinterpret_cast<const void*>(&coop_track_kernel<CH, false, false, false, uint8_t, WIN>);
    case kCoopMixed: return reinterpret_cast<const void*>(&coop_track_kernel<CH, true, false, false, uint8_t, WIN>);
    case kCoopFixedH: return reinterpret_cast<const void*>(&coop_track_kernel<CH, false, true, false, uint8_t, WIN>);
    default: return nullptr;
  }
}

// Co-resident workgroups per CU: the least over every variant at this chunk size.
template <int CH>
static int coop_blocks_per_cu() {
  static int nb = -1;
  if (nb < 0) {
    const int vs[] = {kCoopFP32,
                      kCoopMixed,
                      kCoopFixedH,
                      kCoopPairs,
                      kCoopPairs | kCoopMixed,
                      kCoopPairs | kCoopFixedH,
                      kCoopGeneric,
                      kCoopGeneric | kCoopFixedH,
                      kCoopGeneric | kCoopFloatPyr,
                      kCoopGeneric | kCoopFixedH | kCoopFloatPyr};
    int best = 1 << 30;
    for (int v : vs)
      for (const void* f : {coop_fn<CH, false>(v), coop_fn<CH, true>(v)}) {
        if (!f) continue;
        int k = 0;
        const size_t dyn = (v & kCoopGeneric) ? 0 : kTileBytesSmall + kTilePad;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, f, CH, dyn) != hipSuccess) {
          (void)hipGetLastError();
          k = 0;
        }
        best = std::min(best, k);
      }
    nb = best;
  }
  return nb;
}

int coop_max_blocks(int chunk) {
  static int cu_count[64] = {};  // per device, queried once
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 0;
  }
  int cus = cu_count[dev];
  if (cus == 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    cu_count[dev] = cus;
  }
  switch (chunk) {
    case 64: return coop_blocks_per_cu<64>() * cus;
    case 128: return coop_blocks_per_cu<128>() * cus;
    case 256: return coop_blocks_per_cu<256>() * cus;
    default: return 0;
  }
}

// The chunks of a stream wait for each other, so all workgroups of the grid
// must be resident together.  A grid of at most a quarter of the device's
// co-resident capacity is launched as an ordinary kernel: it is resident as
// soon as the device has that much room, which leaves room for three more such
// launches running concurrently on other streams, and it avoids the
// cooperative launch's extra per-launch cost (about 15 us here).  Larger grids
// use the cooperative launch, which guarantees co-residency.  Either way every
// wait is bounded by spin_limit, so a chunk that cannot be scheduled turns
// into a reported timeout, not a hang.
template <int CH>
static hipError_t coop_launch_k(const CoopStream* d_streams, const int2* d_work, int n_work, const StartSlot* start,
                                TrackOut* out_ring, int slot, int n_out, int n_frames, uint32_t seq0, uint32_t tag_base,
                                int variant, int spin_limit, hipStream_t s) {
  const void* fn = n_frames > 0 ? coop_fn<CH, true>(variant) : coop_fn<CH, false>(variant);
  if (!fn) return hipErrorInvalidValue;
  const bool plain = 4 * n_work <= coop_max_blocks(CH);
  // the 8-pixel kernels' level tile: large where the launch is small enough for
  // one workgroup per compute unit, else small (two per compute unit)
  int tile_bytes = (variant & kCoopGeneric) ? 0 : plain ? kTileBytesLarge : kTileBytesSmall;
  const size_t dyn = tile_bytes ? (size_t)tile_bytes + kTilePad : 0;
  if (dyn > 64 * 1024) {
    static bool raised[2][32] = {};  // per window form and variant: the attribute is set once
    bool& r = raised[n_frames > 0][variant & 31];
    if (!r) {
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
      if (e != hipSuccess) return e;
      r = true;
    }
  }
  void* args[] = {(void*)&d_streams, (void*)&d_work,   (void*)&start,    (void*)&out_ring,   (void*)&slot,
                  (void*)&n_out,     (void*)&n_frames, (void*)&seq0,     (void*)&tag_base,   (void*)&spin_limit,
                  (void*)&tile_bytes};
  if (plain) return hipLaunchKernel(fn, dim3(n_work), dim3(CH), args, dyn, s);
  return hipLaunchCooperativeKernel(fn, dim3(n_work), dim3(CH), args, dyn, s);
}

hipError_t launch_coop_track(const CoopStream* d_streams, const int2* d_work, int n_work, const StartSlot* start,
                             TrackOut* out_ring, int slot, int n_out, int n_frames, uint32_t seq0, uint32_t tag_base,
                             int chunk, int variant, int spin_limit, hipStream_t s) {
  if (slot < 0 || slot >= kRing || n_frames < 0 || n_frames > kRing) return hipErrorInvalidValue;
  switch (chunk) {
    case 64:
      return coop_launch_k<64>(d_streams, d_work, n_work, start, out_ring, slot, n_out, n_frames, seq0, tag_base,
                               variant, spin_limit, s);
    case 128:
      return coop_launch_k<128>(d_streams, d_work, n_work, start, out_ring, slot, n_out, n_frames, seq0, tag_base,
                                variant, spin_limit, s);
    case 256:
      return coop_launch_k<256>(d_streams, d_work, n_work, start, out_ring, slot, n_out, n_frames, seq0, tag_base,
                                variant, spin_limit, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- engine (host)

hipError_t CoopEngine::init(int n_streams, const int* max_points, int chunk_, int ppc_, bool xcd, hipStream_t s) {
  release();
  n = n_streams;
  chunk = chunk_;
  ppc = ppc_;
  xcd_pack = xcd;
  stream = s;
  h_streams.assign(n, CoopStream{});
  max_chunks.resize(n);
  partial_words = 0;
  for (int k = 0; k < n; ++k) {
    max_chunks[k] = (max_points[k] + ppc - 1) / ppc;
    partial_words += (size_t)4 * max_chunks[k] * 32;  // two parities, each an L2 and a device-scope copy
  }
  if (partial_words == 0) partial_words = 64;
  hipError_t e;
  if ((e = hipMalloc(&d_streams, sizeof(CoopStream) * n)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_partials, sizeof(uint64_t) * partial_words)) != hipSuccess) return e;
  if ((e = hipMemset(d_partials, 0, sizeof(uint64_t) * partial_words)) != hipSuccess) return e;
  tag_base = 1;
  // coherent (uncached on the device) pinned host memory: the kernel reads the
  // start slots and writes the results over the host link
  const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
  if ((e = hipHostMalloc((void**)&h_start, sizeof(StartSlot) * kRing * n, fl)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&h_out, sizeof(TrackOut) * kRing * n, fl)) != hipSuccess) return e;
  if ((e = hipHostGetDevicePointer((void**)&dv_start, h_start, 0)) != hipSuccess) return e;
  if ((e = hipHostGetDevicePointer((void**)&dv_out, h_out, 0)) != hipSuccess) return e;
  memset(h_start, 0, sizeof(StartSlot) * kRing * n);
  memset(h_out, 0, sizeof(TrackOut) * kRing * n);
  size_t off = 0;
  for (int k = 0; k < n; ++k) {
    h_streams[k].partials = d_partials + off;
    off += (size_t)4 * max_chunks[k] * 32;
  }
  dirty = true;
  return hipSuccess;
}

void CoopEngine::release() {
  for (void* p : {(void*)d_streams, (void*)d_work, (void*)d_partials})
    if (p) (void)hipFree(p);
  if (h_start) (void)hipHostFree(h_start);
  if (h_out) (void)hipHostFree(h_out);
  d_streams = nullptr, d_work = nullptr, d_partials = nullptr;
  h_start = nullptr, h_out = nullptr, dv_start = nullptr, dv_out = nullptr;
  work_cap = 0;
  partial_words = 0;
}

void CoopEngine::set_stream(int k, const TrackArgs& a, const RefCache& alt, double* hist, const uint8_t* win,
                            const uint8_t* win_alt, int64_t win_stride) {
  CoopStream& c = h_streams[k];
  c.a = a;
  c.a.out = nullptr;  // results go to the launch's slot of h_out
  c.ref_alt = alt;
  c.hist = hist;
  c.win = win;
  c.win_alt = win_alt;
  c.win_stride = win_stride;
  const int n = std::max(a.ref.n, alt.n);  // the chunks cover the larger bank; the other leaves some idle
  c.n_chunks = n > 0 ? (n + ppc - 1) / ppc : 1;
  dirty = true;
}

// Work list: chunk slots of every stream.  With xcd_pack, the chunks of a stream
// go to block indices of one residue mod 8 (workgroups are dealt to the eight
// XCDs round robin), so a stream's partial sums stay within one XCD's L2;
// streams are assigned to XCDs largest first, each to the least loaded one.
hipError_t CoopEngine::upload() {
  h_work.clear();
  if (xcd_pack) {
    std::vector<std::vector<int2>> lists(8);
    std::vector<int> order(n), load(8, 0);
    for (int k = 0; k < n; ++k) order[k] = k;
    std::sort(order.begin(), order.end(),
              [&](int p, int q) { return h_streams[p].n_chunks > h_streams[q].n_chunks; });
    for (int k : order) {
      int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (int c = 0; c < h_streams[k].n_chunks; ++c) lists[x].push_back(make_int2(k, c));
      load[x] += h_streams[k].n_chunks;
    }
    size_t depth = 0;
    for (auto& L : lists) depth = std::max(depth, L.size());
    for (size_t j = 0; j < depth; ++j)
      for (int x = 0; x < 8; ++x) h_work.push_back(j < lists[x].size() ? lists[x][j] : make_int2(-1, 0));
    while (!h_work.empty() && h_work.back().x < 0) h_work.pop_back();
  } else {
    for (int k = 0; k < n; ++k)
      for (int c = 0; c < h_streams[k].n_chunks; ++c) h_work.push_back(make_int2(k, c));
  }
  hipError_t e;
  if ((int)h_work.size() > work_cap) {
    if (d_work) (void)hipFree(d_work);
    d_work = nullptr;
    work_cap = (int)h_work.size();
    if ((e = hipMalloc(&d_work, sizeof(int2) * work_cap)) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(d_work, h_work.data(), sizeof(int2) * h_work.size(), hipMemcpyHostToDevice, stream)) !=
      hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(d_streams, h_streams.data(), sizeof(CoopStream) * n, hipMemcpyHostToDevice, stream)) !=
      hipSuccess)
    return e;
  // the pageable sources above are consumed before the call returns only after a sync
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  dirty = false;
  return hipSuccess;
}

int CoopEngine::grid() const { return (int)h_work.size(); }

hipError_t CoopEngine::launch(int spin_limit, int slot, int n_frames) {
  hipError_t e;
  if (slot < 0 || slot >= kRing || n_frames < 0 || n_frames > kRing) return hipErrorInvalidValue;
  if (dirty && (e = upload()) != hipSuccess) return e;
  // tags used by this launch: at most levels * max_iters + 1 epochs per stream and frame
  uint32_t span = 1;
  for (const CoopStream& c : h_streams) span = std::max(span, (uint32_t)(c.a.levels * c.a.max_iters + 1));
  span *= (uint32_t)std::max(n_frames, 1);
  if (tag_base > 0xFFFFFFFFu - span) {  // wrap: restart the tags on cleared words
    if ((e = clear_partials()) != hipSuccess) return e;
  }
  const int nf = std::max(n_frames, 1);
  if (seq_next > 0xFFFFFFFFu - (uint32_t)nf) seq_next = 1;  // 0 never marks a result
  const uint32_t seq0 = seq_next;
  seq_next += (uint32_t)nf;
  for (int f = 0; f < nf; ++f) slot_seq[(slot + f) % kRing] = seq0 + (uint32_t)f;
  e = launch_coop_track(d_streams, d_work, grid(), dv_start + (size_t)slot * n, dv_out, slot, n, n_frames, seq0,
                        tag_base, chunk, variant, spin_limit, stream);
  tag_base += span;
  return e;
}

bool CoopEngine::done(int slot) const {
  const TrackOut* o = h_out + (size_t)slot * n;
  for (int k = 0; k < n; ++k)
    if (__atomic_load_n(&o[k].seq, __ATOMIC_ACQUIRE) != slot_seq[slot]) return false;
  return true;
}

hipError_t CoopEngine::clear_partials() {
  tag_base = 1;
  return hipMemsetAsync(d_partials, 0, sizeof(uint64_t) * partial_words, stream);
}

// ---------------------------------------------------------------- pose history

struct HistoryArgs {
  double T[24];  // two 3x4 poses: older, newer
};

__global__ void set_history_kernel(double* hist, HistoryArgs h) {
  if (threadIdx.x < 24) hist[threadIdx.x] = h.T[threadIdx.x];
}

// Histories of n streams: vals[s] = (older 3x4, newer 3x4) into hists[s].
__global__ void set_history_batch_kernel(double* const* hists, const double* vals, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 24 * n) return;
  hists[e / 24][e % 24] = vals[e];
}

hipError_t launch_set_history_batch(double* const* d_hists, const double* d_vals, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(set_history_batch_kernel, dim3((24 * n + 255) / 256), dim3(256), 0, s, d_hists, d_vals, n);
  return hipGetLastError();
}

hipError_t launch_set_history(double* hist, const double* T0, const double* T1, hipStream_t s) {
  HistoryArgs h;
  for (int j = 0; j < 12; ++j) h.T[j] = T0[j], h.T[12 + j] = T1[j];
  hipLaunchKernelGGL(set_history_kernel, dim3(1), dim3(32), 0, s, hist, h);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batched pyramid

template <int TILE>
__global__ __launch_bounds__(256) void pyramid_batch_kernel(const PyrJob* __restrict__ jobs) {
  const PyrJob& j = jobs[blockIdx.z];
  if ((int)blockIdx.x * TILE >= j.g.W[0] || (int)blockIdx.y * TILE >= j.g.H[0]) return;
  if (TILE == 64 && j.vec16)
    pyramid_tile64v(j.src, j.pitch, j.dst, j.g);
  else
    pyramid_tile<TILE>(j.src, j.pitch, j.dst, j.g, j.vec4);
}

// As pyramid_batch_kernel, with job z's source and pitch taken from the kernel
// arguments (no table upload per call) and the vector paths chosen here.
template <int TILE>
__global__ __launch_bounds__(256) void pyramid_batch_args_kernel(const PyrJob* __restrict__ jobs, PyrSrcArgs srcs) {
  const int z = blockIdx.z;
  const PyrJob& j = jobs[z];
  if ((int)blockIdx.x * TILE >= j.g.W[0] || (int)blockIdx.y * TILE >= j.g.H[0]) return;
  const uint8_t* src = srcs.src[z];
  const int64_t pitch = srcs.pitch[z];
  const uintptr_t sa = reinterpret_cast<uintptr_t>(src), da = reinterpret_cast<uintptr_t>(j.dst);
  const int W0 = j.g.W[0];
  if (TILE == 64 && (pitch % 16) == 0 && (sa % 16) == 0 && (W0 % 16) == 0 && (da % 16) == 0)
    pyramid_tile64v(src, pitch, j.dst, j.g);
  else
    pyramid_tile<TILE>(src, pitch, j.dst, j.g,
                       ((pitch % 4) == 0 && (sa % 4) == 0 && (W0 % 4) == 0 && (da % 4) == 0) ? 1 : 0);
}

// pyramid_block over a batch: blockIdx.y = image, one thread per block.
template <int LV>
__global__ __launch_bounds__(256) void pyramid_batch_block_kernel(const PyrJob* __restrict__ jobs, PyrSrcArgs srcs) {
  constexpr int B = 1 << (LV - 1);
  const int z = blockIdx.y;
  const PyrJob& j = jobs[z];
  const int nbx = j.g.W[0] / B, t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbx * (j.g.H[0] / B)) return;
  pyramid_block<LV>(srcs.src[z], srcs.pitch[z], j.dst, j.g, t % nbx, t / nbx, true);
}

hipError_t launch_pyramid_batch_args(const PyrJob* d_static, const PyrSrcArgs& srcs, int n_jobs, int max_w,
                                     int max_h, int levels, bool block, hipStream_t s) {
  if (n_jobs > kPyrArgJobs) return hipErrorInvalidValue;
  if (block) {  // every image passed pyramid_block_ok
    const int B = 1 << (levels - 1), n = (max_w / B) * (max_h / B);
    if (levels == 4)
      hipLaunchKernelGGL(pyramid_batch_block_kernel<4>, dim3((n + 255) / 256, n_jobs), dim3(256), 0, s, d_static, srcs);
    else
      hipLaunchKernelGGL(pyramid_batch_block_kernel<3>, dim3((n + 255) / 256, n_jobs), dim3(256), 0, s, d_static, srcs);
    return hipGetLastError();
  }
  if (levels <= 7)
    hipLaunchKernelGGL(pyramid_batch_args_kernel<64>, dim3((max_w + 63) / 64, (max_h + 63) / 64, n_jobs), dim3(256),
                       0, s, d_static, srcs);
  else
    hipLaunchKernelGGL(pyramid_batch_args_kernel<128>, dim3((max_w + 127) / 128, (max_h + 127) / 128, n_jobs),
                       dim3(256), 0, s, d_static, srcs);
  return hipGetLastError();
}

// Window pyramids: blockIdx.z = stream * n_frames + frame; a workgroup builds
// kWinTiles consecutive tiles of a tile row.
constexpr int kWinTiles = 4;
template <int TILE>
__global__ __launch_bounds__(256) void pyramid_window_kernel(const WinJob* __restrict__ jobs, PyrWinSrc srcs,
                                                             int n_frames) {
  const int z = blockIdx.z, js = z / n_frames, f = z - js * n_frames;
  const WinJob& j = jobs[js];
  const int oy = blockIdx.y * TILE;
  if (oy >= j.g.H[0]) return;
  const uint8_t* src = srcs.src[js] + f * srcs.stride[js];
  uint8_t* dst = j.dst + f * j.dst_stride;
  const int64_t pitch = srcs.pitch[js];
  const bool write_l0 = srcs.write_l0[js] != 0;
  const uintptr_t sa = reinterpret_cast<uintptr_t>(src), da = reinterpret_cast<uintptr_t>(dst);
  const int W0 = j.g.W[0];
  const bool v16 = TILE == 64 && (pitch % 16) == 0 && (sa % 16) == 0 && (W0 % 16) == 0 && (da % 16) == 0;
  const int v4 = ((pitch % 4) == 0 && (sa % 4) == 0 && (W0 % 4) == 0 && (da % 4) == 0) ? 1 : 0;
  for (int t = 0; t < kWinTiles; ++t) {  // the tile's LDS is free again when the previous call returns
    const int ox = ((int)blockIdx.x * kWinTiles + t) * TILE;
    if (ox >= W0) break;
    if (v16)
      pyramid_tile64v_at(src, pitch, dst, j.g, ox, oy, write_l0);
    else
      pyramid_tile_at<TILE>(src, pitch, dst, j.g, v4, ox, oy, write_l0);
  }
}

// pyramid_block over the frames of a window: blockIdx.y = stream * n_frames + frame.
template <int LV>
__global__ __launch_bounds__(256) void pyramid_window_block_kernel(const WinJob* __restrict__ jobs, PyrWinSrc srcs,
                                                                   int n_frames) {
  constexpr int B = 1 << (LV - 1);
  const int z = blockIdx.y, js = z / n_frames, f = z - js * n_frames;
  const WinJob& j = jobs[js];
  const int nbx = j.g.W[0] / B, t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbx * (j.g.H[0] / B)) return;
  pyramid_block<LV>(srcs.src[js] + f * srcs.stride[js], srcs.pitch[js], j.dst + f * j.dst_stride, j.g, t % nbx, t / nbx,
                    srcs.write_l0[js] != 0);
}

hipError_t launch_pyramid_window(const WinJob* d_jobs, const PyrWinSrc& srcs, int n_streams, int n_frames, int max_w,
                                 int max_h, int levels, bool block, hipStream_t s) {
  if (n_streams < 1 || n_streams > kPyrArgJobs || n_frames < 1 || (int64_t)n_streams * n_frames > 65535)
    return hipErrorInvalidValue;
  if (block) {  // every stream passed pyramid_block_ok for every frame
    const int B = 1 << (levels - 1), n = (max_w / B) * (max_h / B);
    if (levels == 4)
      hipLaunchKernelGGL(pyramid_window_block_kernel<4>, dim3((n + 255) / 256, n_streams * n_frames), dim3(256), 0, s,
                         d_jobs, srcs, n_frames);
    else
      hipLaunchKernelGGL(pyramid_window_block_kernel<3>, dim3((n + 255) / 256, n_streams * n_frames), dim3(256), 0, s,
                         d_jobs, srcs, n_frames);
    return hipGetLastError();
  }
  constexpr int T64 = 64 * kWinTiles, T128 = 128 * kWinTiles;
  if (levels <= 7)
    hipLaunchKernelGGL(pyramid_window_kernel<64>, dim3((max_w + T64 - 1) / T64, (max_h + 63) / 64, n_streams * n_frames),
                       dim3(256), 0, s, d_jobs, srcs, n_frames);
  else
    hipLaunchKernelGGL(pyramid_window_kernel<128>,
                       dim3((max_w + T128 - 1) / T128, (max_h + 127) / 128, n_streams * n_frames), dim3(256), 0, s,
                       d_jobs, srcs, n_frames);
  return hipGetLastError();
}

hipError_t launch_pyramid_batch(const PyrJob* d_jobs, int n_jobs, int max_w, int max_h, int levels, hipStream_t s) {
  if (levels <= 7)
    hipLaunchKernelGGL(pyramid_batch_kernel<64>, dim3((max_w + 63) / 64, (max_h + 63) / 64, n_jobs), dim3(256), 0, s,
                       d_jobs);
  else
    hipLaunchKernelGGL(pyramid_batch_kernel<128>, dim3((max_w + 127) / 128, (max_h + 127) / 128, n_jobs), dim3(256),
                       0, s, d_jobs);
  return hipGetLastError();
}

}  // namespace dpt
