// Cooperative multi-workgroup track: every camera stream's map is split into
// chunks of CH points, one workgroup per chunk, one thread per point, and all
// chunks of all streams run in one cooperative (co-resident) launch that
// covers every level and iteration of the frame.
//
// Per Gauss-Newton iteration the chunks of a stream exchange their 32 partial
// sums through a double-buffered global array and a stream-local arrival
// counter.  Each chunk then sums the partials in chunk order and solves the
// 6x6 system itself: all chunks of a stream compute bitwise-identical poses,
// so one barrier per iteration suffices and the result is reproducible.
// Waits are bounded: a chunk that waits longer than `spin_limit` polls gives up
// and reports a timeout instead of hanging.
#include <type_traits>

#include "dpt_device.h"

namespace dpt {

constexpr int kStatusTimeout = 4;

// Publish this chunk's sums for `epoch`, wait for the other chunks of the stream
// and replace sh_tot with the stream total (fixed chunk order).  Returns false
// on timeout.
template <bool KAHAN>
__device__ __forceinline__ bool stream_sync_sum(float* partials, int* sync, int chunk, int nch, int epoch,
                                                float* sh_tot, int spin_limit, int* sh_ok) {
  float* buf = partials + (size_t)(epoch & 1) * nch * 32;
  const int tid = threadIdx.x;
  if (tid < 32) buf[chunk * 32 + tid] = sh_tot[tid];
  if (tid < 64) __threadfence();  // wave 0: make its partial stores visible device-wide
  if (tid == 0) {
    atomicAdd(&sync[0], 1);
    const int target = (epoch + 1) * nch;
    int ok = 0;
    for (int t = 0; t < spin_limit; ++t) {
      if (__hip_atomic_load(&sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *sh_ok = ok;
  }
  if (tid < 64) __threadfence();  // acquire the other chunks' partials
  __syncthreads();
  const bool ok = *sh_ok != 0;
  if (ok && tid < 32) {
    float s = 0.0f, comp = 0.0f;
    for (int c = 0; c < nch; ++c) {
      const float x = __builtin_nontemporal_load(&buf[c * 32 + tid]);
      if (KAHAN) {  // compensated sum over the chunks
        const float y = x - comp;
        const float t = s + y;
        comp = (t - s) - y;
        s = t;
      } else {
        s += x;
      }
    }
    sh_tot[tid] = s;
  }
  __syncthreads();
  return ok;
}

// MIXED: FP16 reference cache, Kahan-compensated FP32 sums across waves and
// chunks, FP64 solve, exponential and pose state.
template <int CH, bool MIXED>
__global__ __launch_bounds__(CH, 2) void coop_track_kernel(const CoopStream* __restrict__ streams,
                                                           const int2* __restrict__ work,
                                                           const double* __restrict__ T_init, int spin_limit) {
  using PR = typename std::conditional<MIXED, PointRegsH, PointRegs>::type;
  __shared__ CoopStream ss;
  __shared__ float sh_T[12];
  __shared__ double sh_Td[12];
  __shared__ float sh_tot[32];
  __shared__ float sh_red[(CH / 64) * 32];
  __shared__ int sh_flag, sh_ok;
  __shared__ int sh_ipl[kMaxLevels];
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding slot of the XCD-aware work list
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(streams + w.x);
    for (int j = threadIdx.x; j < (int)(sizeof(CoopStream) / 4); j += blockDim.x)
      reinterpret_cast<uint32_t*>(&ss)[j] = src[j];
  }
  if (threadIdx.x < 12) {
    sh_Td[threadIdx.x] = T_init[w.x * 12 + threadIdx.x];
    sh_T[threadIdx.x] = (float)T_init[w.x * 12 + threadIdx.x];
  }
  if (threadIdx.x < kMaxLevels) sh_ipl[threadIdx.x] = 0;
  __syncthreads();
  const TrackArgs& a = ss.a;
  const int chunk = w.y, nch = ss.n_chunks;
  const int i = chunk * CH + threadIdx.x;
  int status = 0, iterations = 0, epoch = 0;  // status / iterations authoritative in thread 0
  int64_t samples = 0;
  bool stop = false, timed_out = false;
  PR pr;
  for (int l = a.levels - 1; l >= 0 && !stop; --l) {
    const LevelGeom g = a.lv[l];
    const uint8_t* img = a.cur + g.off;
    load_point(a, l, i, pr);
    bool converged = false;
    for (int it = 0; it < a.max_iters; ++it) {
      float acc[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) acc[j] = 0.f;
      float T[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
      accumulate_point<false>(a, a.pat, g, img, T, pr, acc);
      if (MIXED)
        block_reduce32_kahan(acc, sh_red, sh_tot);
      else
        block_reduce32(acc, sh_red, sh_tot);
      if (!stream_sync_sum<MIXED>(ss.partials, ss.sync, chunk, nch, epoch, sh_tot, spin_limit, &sh_ok)) {
        timed_out = stop = true;
        break;
      }
      ++epoch;
      if (threadIdx.x == 0) {
        samples += (int64_t)sh_tot[kSlotN];
        int flag = 0;
        if ((int)sh_tot[kSlotPts] < a.min_points) {
          flag = 2;
          status = 2;  // too few points
        } else {
          int bad;
          double step;
          if (MIXED) {
            bad = solve_update_d(sh_tot, sh_Td, &step);
            if (!bad)
              for (int j = 0; j < 12; ++j) sh_T[j] = (float)sh_Td[j];
          } else {
            float stepf;
            bad = solve_update(sh_tot, sh_T, &stepf);
            step = stepf;
          }
          if (bad) {
            flag = 2;
            status = 3;  // not positive definite
          } else {
            ++iterations;
            ++sh_ipl[l];
            if (step < (double)a.step_eps) flag = 1;
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
  if (!timed_out) {  // final cost-only pass at level 0
    float acc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] = 0.f;
    float T[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) T[j] = sh_T[j];
    const LevelGeom g = a.lv[0];
    load_point(a, 0, i, pr);
    accumulate_point<true>(a, a.pat, g, a.cur + g.off, T, pr, acc);
    if (MIXED)
      block_reduce32_kahan(acc, sh_red, sh_tot);
    else
      block_reduce32(acc, sh_red, sh_tot);
    if (!stream_sync_sum<MIXED>(ss.partials, ss.sync, chunk, nch, epoch, sh_tot, spin_limit, &sh_ok))
      timed_out = true;
  }
  if (chunk == 0 && threadIdx.x == 0) {
    TrackOut* o = a.out;
    for (int j = 0; j < 12; ++j) {
      o->T[j] = sh_T[j];
      o->Td[j] = MIXED ? sh_Td[j] : (double)sh_T[j];
    }
    o->E = sh_tot[kSlotE];
    o->n = sh_tot[kSlotN];
    o->iterations = iterations;
    for (int j = 0; j < kMaxLevels; ++j) o->iters_per_level[j] = sh_ipl[j];
    o->n_valid_points = (int)sh_tot[kSlotPts];
    o->status = timed_out ? kStatusTimeout : status;
    o->samples = samples + (int64_t)sh_tot[kSlotN];
  }
  // the last chunk of the stream to leave resets the counters for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&ss.sync[1], 1) == nch - 1) {
      atomicExch(&ss.sync[0], 0);
      atomicExch(&ss.sync[1], 0);
    }
  }
}

template <int CH>
static int coop_blocks_per_cu() {
  static int nb = -1;
  if (nb < 0) {
    int v = 0, v2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, coop_track_kernel<CH, false>, CH, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&v2, coop_track_kernel<CH, true>, CH, 0) != hipSuccess) {
      (void)hipGetLastError();
      v = v2 = 0;
    }
    nb = std::min(v, v2);
  }
  return nb;
}

int coop_max_blocks(int chunk) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  switch (chunk) {
    case 64: return coop_blocks_per_cu<64>() * cus;
    case 128: return coop_blocks_per_cu<128>() * cus;
    case 256: return coop_blocks_per_cu<256>() * cus;
    default: return 0;
  }
}

template <int CH>
static hipError_t coop_launch_k(const CoopStream* d_streams, const int2* d_work, int n_work, const double* d_T,
                                bool mixed, int spin_limit, hipStream_t s) {
  void* args[] = {(void*)&d_streams, (void*)&d_work, (void*)&d_T, (void*)&spin_limit};
  const void* fn = mixed ? reinterpret_cast<const void*>(&coop_track_kernel<CH, true>)
                         : reinterpret_cast<const void*>(&coop_track_kernel<CH, false>);
  return hipLaunchCooperativeKernel(fn, dim3(n_work), dim3(CH), args, 0, s);
}

hipError_t launch_coop_track(const CoopStream* d_streams, const int2* d_work, int n_work, const double* d_T,
                             int chunk, bool mixed, int spin_limit, hipStream_t s) {
  switch (chunk) {
    case 64: return coop_launch_k<64>(d_streams, d_work, n_work, d_T, mixed, spin_limit, s);
    case 128: return coop_launch_k<128>(d_streams, d_work, n_work, d_T, mixed, spin_limit, s);
    case 256: return coop_launch_k<256>(d_streams, d_work, n_work, d_T, mixed, spin_limit, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- engine (host)

hipError_t CoopEngine::init(int n_streams, const int* max_points, int chunk_, bool xcd, hipStream_t s) {
  release();
  n = n_streams;
  chunk = chunk_;
  xcd_pack = xcd;
  stream = s;
  h_streams.assign(n, CoopStream{});
  max_chunks.resize(n);
  size_t partial_floats = 0;
  for (int k = 0; k < n; ++k) {
    max_chunks[k] = (max_points[k] + chunk - 1) / chunk;
    partial_floats += (size_t)2 * max_chunks[k] * 32;
  }
  hipError_t e;
  if ((e = hipMalloc(&d_streams, sizeof(CoopStream) * n)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_partials, sizeof(float) * (partial_floats ? partial_floats : 32))) != hipSuccess) return e;
  if ((e = hipMalloc(&d_sync, sizeof(int) * 2 * n)) != hipSuccess) return e;
  if ((e = hipMemset(d_sync, 0, sizeof(int) * 2 * n)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_T, sizeof(double) * 12 * n)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&h_T, sizeof(double) * 12 * n)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_out, sizeof(TrackOut) * n)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&h_out, sizeof(TrackOut) * n)) != hipSuccess) return e;
  size_t off = 0;
  for (int k = 0; k < n; ++k) {
    h_streams[k].partials = d_partials + off;
    h_streams[k].sync = d_sync + 2 * k;
    off += (size_t)2 * max_chunks[k] * 32;
  }
  dirty = true;
  return hipSuccess;
}

void CoopEngine::release() {
  for (void* p : {(void*)d_streams, (void*)d_work, (void*)d_partials, (void*)d_sync, (void*)d_T, (void*)d_out})
    if (p) (void)hipFree(p);
  if (h_T) (void)hipHostFree(h_T);
  if (h_out) (void)hipHostFree(h_out);
  d_streams = nullptr, d_work = nullptr, d_partials = nullptr, d_sync = nullptr, d_T = nullptr, d_out = nullptr;
  h_T = nullptr, h_out = nullptr;
  work_cap = 0;
}

void CoopEngine::set_stream(int k, const TrackArgs& a) {
  CoopStream& c = h_streams[k];
  c.a = a;
  c.a.out = d_out + k;
  c.n_chunks = a.ref.n > 0 ? (a.ref.n + chunk - 1) / chunk : 1;
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

hipError_t CoopEngine::launch(int spin_limit) {
  hipError_t e;
  if (dirty && (e = upload()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_T, h_T, sizeof(double) * 12 * n, hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((e = launch_coop_track(d_streams, d_work, grid(), d_T, chunk, mixed, spin_limit, stream)) != hipSuccess)
    return e;
  return hipMemcpyAsync(h_out, d_out, sizeof(TrackOut) * n, hipMemcpyDeviceToHost, stream);
}

hipError_t CoopEngine::reset_sync() { return hipMemsetAsync(d_sync, 0, sizeof(int) * 2 * n, stream); }

// ---------------------------------------------------------------- batched pyramid

template <int TILE>
__global__ __launch_bounds__(256) void pyramid_batch_kernel(const PyrJob* __restrict__ jobs) {
  const PyrJob& j = jobs[blockIdx.z];
  if ((int)blockIdx.x * TILE >= j.g.W[0] || (int)blockIdx.y * TILE >= j.g.H[0]) return;
  pyramid_tile<TILE>(j.src, j.pitch, j.dst, j.g, j.vec4);
}

hipError_t launch_pyramid_batch(const PyrJob* d_jobs, int n_jobs, int max_w, int max_h, int levels, hipStream_t s) {
  if (levels <= 6)
    hipLaunchKernelGGL(pyramid_batch_kernel<32>, dim3((max_w + 31) / 32, (max_h + 31) / 32, n_jobs), dim3(256), 0, s,
                       d_jobs);
  else if (levels == 7)
    hipLaunchKernelGGL(pyramid_batch_kernel<64>, dim3((max_w + 63) / 64, (max_h + 63) / 64, n_jobs), dim3(256), 0, s,
                       d_jobs);
  else
    hipLaunchKernelGGL(pyramid_batch_kernel<128>, dim3((max_w + 127) / 128, (max_h + 127) / 128, n_jobs), dim3(256),
                       0, s, d_jobs);
  return hipGetLastError();
}

}  // namespace dpt
