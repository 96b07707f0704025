// C-ABI host library of the direct photometric tracker (include/dptrack.h).
// Owns device memory per context, validates arguments, marshals launch
// arguments and turns HIP failures into negative return codes with a message.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <thread>

#include "../../include/dptrack.h"
#include "dpt_internal.h"

using namespace dpt;

namespace {

// The calling thread's last error message, in a fixed buffer: recording an
// error allocates nothing.
struct ErrMsg {
  char text[512] = {0};
  void clear() { text[0] = 0; }
  const char* c_str() const { return text; }
};
thread_local ErrMsg g_err;

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err.text, sizeof g_err.text, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DPT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Rigid-transform helpers on row-major 4x4 doubles (host, FP64).
void compose(const double* A, const double* B, double* C) {
  double T[16];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 4; ++c) {
      double s = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c];
      if (c == 3) s += A[4 * r + 3];
      T[4 * r + c] = s;
    }
  }
  T[12] = T[13] = T[14] = 0.0;
  T[15] = 1.0;
  std::memcpy(C, T, sizeof T);
}

void invert(const double* A, double* B) {
  double T[16];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[4 * r + c] = A[4 * c + r];
    T[4 * r + 3] = -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
  }
  T[12] = T[13] = T[14] = 0.0;
  T[15] = 1.0;
  std::memcpy(B, T, sizeof T);
}

bool finite16(const double* T) {
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  return true;
}

int check_camera(const dpt_camera* c) {
  if (!c) return fail(DPT_E_ARG, "camera is NULL");
  if (c->width < 16 || c->height < 16 || c->width > 8192 || c->height > 8192)
    return fail(DPT_E_ARG, "camera size %dx%d outside [16, 8192]", c->width, c->height);
  if (!(c->fx > 0) || !(c->fy > 0) || !std::isfinite(c->cx) || !std::isfinite(c->cy))
    return fail(DPT_E_ARG, "invalid intrinsics");
  return DPT_OK;
}

int check_params(const dpt_params* p, const dpt_camera* c) {
  if (!p) return fail(DPT_E_ARG, "params is NULL");
  if (p->levels < 1 || p->levels > kMaxLevels) return fail(DPT_E_ARG, "levels %d outside [1, 8]", p->levels);
  if ((c->width >> (p->levels - 1)) < 8 || (c->height >> (p->levels - 1)) < 8)
    return fail(DPT_E_ARG, "coarsest level smaller than 8 pixels");
  if (p->max_iters < 1 || p->max_iters > 100) return fail(DPT_E_ARG, "max_iters %d outside [1, 100]", p->max_iters);
  if (p->n_pattern < 1 || p->n_pattern > kMaxPattern) return fail(DPT_E_ARG, "n_pattern %d outside [1, 128]", p->n_pattern);
  for (int k = 0; k < 2 * p->n_pattern; ++k)
    if (p->pattern[k] < -16 || p->pattern[k] > 16) return fail(DPT_E_ARG, "pattern offset %d outside [-16, 16]", p->pattern[k]);
  if (!std::isfinite(p->huber_k) || !(p->step_eps >= 0) || !(p->z_min >= 0)) return fail(DPT_E_ARG, "invalid thresholds");
  if (p->min_points < 0) return fail(DPT_E_ARG, "min_points < 0");
  if (p->precision != DPT_PREC_FP32 && p->precision != DPT_PREC_MIXED) return fail(DPT_E_ARG, "precision %d", p->precision);
  if (p->precision == DPT_PREC_MIXED && p->n_pattern != 8) return fail(DPT_E_ARG, "mixed precision needs K = 8");
  if (p->flags & ~(DPT_FLAG_FIXED_H | DPT_FLAG_GAUSS_F32)) return fail(DPT_E_ARG, "unknown flags 0x%x", p->flags);
  if ((p->flags & DPT_FLAG_FIXED_H) && p->precision != DPT_PREC_FP32)
    return fail(DPT_E_ARG, "the fixed-H mode computes in FP32");
  if ((p->flags & DPT_FLAG_GAUSS_F32) && p->precision != DPT_PREC_FP32)
    return fail(DPT_E_ARG, "the Gaussian float pyramid runs in FP32");
  return DPT_OK;
}

Pattern make_pattern(const dpt_params* p) {
  Pattern pt;
  std::memset(&pt, 0, sizeof pt);
  pt.K = p->n_pattern;
  pt.dx_min = pt.dy_min = 1 << 20;
  pt.dx_max = pt.dy_max = -(1 << 20);
  for (int k = 0; k < p->n_pattern; ++k) {
    int dx = p->pattern[2 * k], dy = p->pattern[2 * k + 1];
    pt.dx[k] = (int8_t)dx;
    pt.dy[k] = (int8_t)dy;
    pt.dx_min = dx < pt.dx_min ? dx : pt.dx_min;
    pt.dx_max = dx > pt.dx_max ? dx : pt.dx_max;
    pt.dy_min = dy < pt.dy_min ? dy : pt.dy_min;
    pt.dy_max = dy > pt.dy_max ? dy : pt.dy_max;
  }
  return pt;
}

}  // namespace

int dpt::set_error(int code, const char* msg) {
  snprintf(g_err.text, sizeof g_err.text, "%s", msg);
  return code;
}

namespace dpt {

// Launch timing with HIP events: a ring of (start, end) pairs recorded on the
// stream around each launch; a pair is drained into the totals once its end
// event has completed.
struct ProfRing {
  static constexpr int kN = 128;  // pairs recorded and not yet read back
  hipEvent_t ev[kN][2] = {};
  bool created = false;
  // Only every `every`-th launch is bracketed: each event record is a marker
  // the queue processes between kernels (several microseconds), so timing
  // every launch would slow the stream it measures.
  int every = 1;
  int64_t tick = 0;
  int next = 0, n_pending = 0;  // pending pairs: the n_pending slots before `next`
  double total_ms = 0.0;
  int64_t count = 0;
  float last_ms = -1.0f;

  hipError_t create() {
    if (created) return hipSuccess;
    for (auto& p : ev)
      for (hipEvent_t& e : p) {
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
      }
    created = true;
    return hipSuccess;
  }
  void destroy() {
    for (auto& p : ev)
      for (hipEvent_t& e : p)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    created = false;
  }
  hipError_t drain_one() {
    const int s = (next - n_pending + kN) % kN;
    hipError_t e = hipEventSynchronize(ev[s][1]);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, ev[s][0], ev[s][1])) != hipSuccess) return e;
    total_ms += ms;
    ++count;
    last_ms = ms;
    --n_pending;
    return hipSuccess;
  }
  hipError_t begin(hipStream_t st, int* slot) {
    *slot = -1;
    if (tick++ % every != 0) return hipSuccess;
    if (n_pending == kN) {
      const hipError_t e = drain_one();
      if (e != hipSuccess) return e;
    }
    *slot = next;
    next = (next + 1) % kN;
    return hipEventRecord(ev[*slot][0], st);
  }
  hipError_t end(hipStream_t st, int slot) {
    if (slot < 0) return hipSuccess;
    ++n_pending;
    return hipEventRecord(ev[slot][1], st);
  }
  hipError_t drain() {
    while (n_pending) {
      const hipError_t e = drain_one();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  void reset(int every_ = 1) {
    every = every_ > 0 ? every_ : 1;
    tick = 0;
    total_ms = 0.0;
    count = 0;
    last_ms = -1.0f;
  }
};

// n 4-byte words from host-mapped memory to device memory.
__global__ void copy_host_words(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// A per-call argument table uploaded through pinned memory: two alternating
// (host, device) buffers, a buffer's host side rewritten only after its
// previous upload has run, so calls never wait for the stream otherwise.
template <class T>
struct StagedTable {
  static_assert(sizeof(T) % 4 == 0, "copied in 4-byte words");
  T* h[2] = {nullptr, nullptr};
  const T* hd[2] = {nullptr, nullptr};  // the host buffers' device addresses
  T* d[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int cap = 0, next = 0;

  hipError_t init(int n) {
    cap = n;
    hipError_t e;
    // mapped and coherent: the upload is a kernel reading them over the host link
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    for (int i = 0; i < 2; ++i) {
      if ((e = hipHostMalloc((void**)&h[i], sizeof(T) * n, fl)) != hipSuccess) return e;
      if ((e = hipHostGetDevicePointer((void**)&hd[i], h[i], 0)) != hipSuccess) return e;
      if ((e = hipMalloc((void**)&d[i], sizeof(T) * n)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  void release() {
    for (int i = 0; i < 2; ++i) {
      if (h[i]) (void)hipHostFree(h[i]);
      if (d[i]) (void)hipFree(d[i]);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      h[i] = d[i] = nullptr;
      ev[i] = nullptr;
    }
  }
  // Host buffer to fill for the next upload (waits only for that buffer's previous upload).
  hipError_t acquire(T** host, int* which) {
    *which = next;
    next ^= 1;
    *host = h[*which];
    return hipEventSynchronize(ev[*which]);
  }
  // A kernel on stream s copies the first n entries to the device (a launch
  // in the stream's order, where a copy command would cost an engine switch).
  hipError_t upload(int which, int n, hipStream_t s, const T** dev) {
    const int words = (int)(sizeof(T) / 4) * n;
    if (words > 0) {
      hipLaunchKernelGGL(copy_host_words, dim3(std::min((words + 255) / 256, 64)), dim3(256), 0, s,
                         reinterpret_cast<uint32_t*>(d[which]), reinterpret_cast<const uint32_t*>(hd[which]), words);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    *dev = d[which];
    return hipEventRecord(ev[which], s);
  }
};

// The reference state that a reference update writes and the tracks read:
// one bank.  With a reference stream a context holds two and alternates.
struct RefBank {
  uint8_t* pyr_ref = nullptr;
  float* pyrf_ref = nullptr;
  float4* x0 = nullptr;
  uint8_t* valid = nullptr;
  float *I0 = nullptr, *gx = nullptr, *gy = nullptr;
  __half* I0h = nullptr;
  __half2* gh = nullptr;
  float* pts = nullptr;
  FixedH* d_fixed = nullptr;
  float* d_hpart = nullptr;
};

}  // namespace dpt

struct dpt_ctx {
  dpt_camera cam;
  dpt_params prm;
  int32_t cap = 0;  // max points
  hipStream_t stream = nullptr;
  LevelGeom lv[kMaxLevels];
  PyrGeom pg;
  int64_t pyr_bytes = 0;
  uint8_t* pyr[2] = {nullptr, nullptr};
  float* pyrf[2] = {nullptr, nullptr};  // DPT_FLAG_GAUSS_F32: the floating-point Gaussian pyramids
  bool have_pyr[2] = {false, false};
  uint8_t* staging = nullptr;  // level-0 upload buffer for host images
  float4* x0 = nullptr;
  uint8_t* valid = nullptr;
  float *I0 = nullptr, *gx = nullptr, *gy = nullptr;
  __half* I0h = nullptr;  // mixed precision cache
  __half2* gh = nullptr;
  float* pts = nullptr;  // device copy of the world points
  int32_t n_points = 0;
  bool have_ref = false;
  double T_rw[16];
  int32_t* sel_idx = nullptr;
  int32_t* sel_count = nullptr;
  int32_t* sel_scratch = nullptr;
  TrackOut* d_out = nullptr;
  TrackOut* h_out = nullptr;  // pinned
  float* h_pts = nullptr;        // pinned staging of host map points
  hipEvent_t ev_pts = nullptr;   // the last upload out of h_pts
  int32_t* h_sel = nullptr;      // pinned: selection count, then the indices
  float* depth_stage = nullptr;  // device copy of a host depth map (allocated on first use)
  float* d_tot = nullptr;
  float* h_tot = nullptr;  // pinned
  FixedH* d_fixed = nullptr;  // fixed-H mode: [levels]
  float* d_hpart = nullptr;   // fixed-H mode: [levels][ceil(cap / 256)][21]
  Pattern pat;
  bool prof = false;
  ProfRing prof_pyr, prof_trk;  // pyramid and track launch timings
  int32_t launch_mode = DPT_LAUNCH_AUTO, chunk = 256;
  int32_t spin_limit = kSpinLimit;
  CoopEngine eng;
  bool eng_ready = false;
  double* d_hist = nullptr;  // pose history: the last two T_cw, 2 x 3x4 FP64 (device)
  double* d_prop = nullptr;  // learned start proposal relative to the reference, 3x4 FP64 (device)
  // the coarsest reference and current levels, for the proposal: one table
  // per reference bank, each uploaded the first time that bank is read
  const uint8_t** d_cnn_lv = nullptr;
  bool cnn_lv_ok[2] = {false, false};
  bool have_prop = false;
  std::vector<std::pair<int, dpt_result*>> pending;  // tracks in flight: (ring slot, caller's result)
  int slot_next = 0;
  // window tracking: box pyramids of up to win_cap consecutive frames, one
  // buffer per reference bank (the second one with a reference stream): a
  // window's pyramids go to the buffer of the bank its track reads
  uint8_t* win = nullptr;
  uint8_t* win_b1 = nullptr;
  int64_t win_stride = 0;  // bytes per frame pyramid, a multiple of 256
  int32_t win_cap = 0;
  uint8_t* win_staging = nullptr;  // level 0 of host frames, win_cap frames of W x H
  WinJob* d_winjob = nullptr;      // the window pyramid jobs (device) into win, and into win_b1
  WinJob* d_winjob_b1 = nullptr;
  // reference stream (dpt_set_reference_stream): reference updates run there,
  // into the bank the tracks in flight do not read; the fields above hold the
  // bank last written (committed once have_ref is set)
  hipStream_t rstream = nullptr;
  RefBank alt;                 // the other bank
  RefBank phys[2];             // the banks' buffers by identity (bank 0: allocated at creation)
  int32_t bank = 0;            // which of phys[] the fields hold
  int32_t bank_n[2] = {0, 0};  // points committed to each bank
  hipEvent_t ev_read[2] = {nullptr, nullptr};  // context stream: past the last track that read bank b
  hipEvent_t ev_ready = nullptr;               // reference stream: the last committed update done
  bool update_open = false;    // a reference update has started writing the fields' bank
  bool commit_pending = false;  // committed, the context's stream not yet ordered after it
  bool batch_owned = false;     // a batch stream: the batch orders its updates and tracks
  // tween-window schedule (host state)
  dpt_tween_policy tween{};
  bool tween_policy = false, tween_anchored = false, tween_needs_anchor = false;
  int32_t tween_direct = 0;
  double tween_hist[2][16];  // the last two accepted or anchored T_cw, older first

  ~dpt_ctx() {
    prof_pyr.destroy();
    prof_trk.destroy();
    if (d_hist) (void)hipFree(d_hist);
    if (d_prop) (void)hipFree(d_prop);
    if (d_cnn_lv) (void)hipFree(d_cnn_lv);
    for (void* p : {(void*)alt.pyr_ref, (void*)alt.pyrf_ref, (void*)alt.x0, (void*)alt.valid, (void*)alt.I0,
                    (void*)alt.gx, (void*)alt.gy, (void*)alt.I0h, (void*)alt.gh, (void*)alt.pts, (void*)alt.d_fixed,
                    (void*)alt.d_hpart})
      if (p) (void)hipFree(p);
    for (hipEvent_t e : {ev_read[0], ev_read[1], ev_ready})
      if (e) (void)hipEventDestroy(e);
    if (ev_pts) (void)hipEventDestroy(ev_pts);
    if (h_pts) (void)hipHostFree(h_pts);
    if (h_sel) (void)hipHostFree(h_sel);
    if (depth_stage) (void)hipFree(depth_stage);
    for (void* p : {(void*)pyr[0], (void*)pyr[1], (void*)staging, (void*)x0, (void*)valid, (void*)I0, (void*)gx,
                    (void*)gy, (void*)I0h, (void*)gh, (void*)pts, (void*)sel_idx, (void*)sel_count, (void*)sel_scratch, (void*)d_out,
                    (void*)d_tot, (void*)d_fixed, (void*)d_hpart, (void*)pyrf[0], (void*)pyrf[1], (void*)win,
                    (void*)win_staging, (void*)d_winjob, (void*)win_b1, (void*)d_winjob_b1})
      if (p) (void)hipFree(p);
    if (h_out) (void)hipHostFree(h_out);
    if (h_tot) (void)hipHostFree(h_tot);
  }
};

namespace {

int dev_alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(DPT_E_OOM, "hipMalloc of %zu bytes failed", bytes);
  }
  return DPT_OK;
}

void fill_track_args(const dpt_ctx* c, TrackArgs& a) {
  std::memset(&a, 0, sizeof a);
  a.cur = c->pyr[DPT_SLOT_CUR];
  a.curf = c->pyrf[DPT_SLOT_CUR];
  for (int l = 0; l < kMaxLevels; ++l) a.lv[l] = c->lv[l];
  a.levels = c->prm.levels;
  a.max_iters = c->prm.max_iters;
  a.min_points = c->prm.min_points;
  const bool fixed = (c->prm.flags & DPT_FLAG_FIXED_H) != 0;
  a.huber_k = fixed ? 0.0f : c->prm.huber_k;  // the fixed-H mode has no weights
  a.step_eps = c->prm.step_eps;
  a.z_min = c->prm.z_min;
  a.pat = c->pat;
  a.ref.x0 = c->x0;
  a.ref.valid = c->valid;
  a.ref.I0 = c->I0;
  a.ref.gx = c->gx;
  a.ref.gy = c->gy;
  a.ref.I0h = c->I0h;
  a.ref.gh = c->gh;
  a.ref.fixed = fixed ? c->d_fixed : nullptr;
  a.ref.n = c->n_points;
  a.ref.cap = c->cap;
  a.out = c->d_out;
  a.totals = c->d_tot;
}

RefBank fields_bank(const dpt_ctx* c) {
  RefBank b;
  b.pyr_ref = c->pyr[DPT_SLOT_REF];
  b.pyrf_ref = c->pyrf[DPT_SLOT_REF];
  b.x0 = c->x0, b.valid = c->valid, b.I0 = c->I0, b.gx = c->gx, b.gy = c->gy, b.I0h = c->I0h, b.gh = c->gh;
  b.pts = c->pts, b.d_fixed = c->d_fixed, b.d_hpart = c->d_hpart;
  return b;
}

void set_fields(dpt_ctx* c, const RefBank& b) {
  c->pyr[DPT_SLOT_REF] = b.pyr_ref;
  c->pyrf[DPT_SLOT_REF] = b.pyrf_ref;
  c->x0 = b.x0, c->valid = b.valid, c->I0 = b.I0, c->gx = b.gx, c->gy = b.gy, c->I0h = b.I0h, c->gh = b.gh;
  c->pts = b.pts, c->d_fixed = b.d_fixed, c->d_hpart = b.d_hpart;
}

// The reference cache of bank b as the cooperative engine's descriptor holds it.
RefCache refcache_of(const dpt_ctx* c, int b) {
  const RefBank& k = c->phys[b].x0 ? c->phys[b] : c->phys[0];
  const bool fixed = (c->prm.flags & DPT_FLAG_FIXED_H) != 0;
  RefCache r;
  std::memset(&r, 0, sizeof r);
  r.x0 = k.x0, r.valid = k.valid, r.I0 = k.I0, r.gx = k.gx, r.gy = k.gy, r.I0h = k.I0h, r.gh = k.gh;
  r.fixed = fixed ? k.d_fixed : nullptr;
  r.n = c->phys[b].x0 ? c->bank_n[b] : c->bank_n[0];
  r.cap = c->cap;
  return r;
}

// The stream reference updates run on.
hipStream_t ref_stream(const dpt_ctx* c) { return c->rstream ? c->rstream : c->stream; }

// Before the context's stream reads the reference (a track, a test hook):
// after an update committed on the reference stream, mark the end of the
// other bank's readers and order the context's stream after the update.
int consume_commit(dpt_ctx* c) {
  if (!c->commit_pending) return DPT_OK;
  HIP_TRY(hipEventRecord(c->ev_read[c->bank ^ 1], c->stream));
  HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_ready, 0));
  c->commit_pending = false;
  return DPT_OK;
}

// A reference update starts (a reference pyramid build).  With a reference
// stream the fields switch to the bank the tracks do not read, and the
// reference stream waits for the tracks that read that bank last.
int open_update(dpt_ctx* c) {
  if (!c->rstream || c->update_open) return DPT_OK;
  int e = consume_commit(c);  // an update without tracks since the last one: its readers are ordered here
  if (e != DPT_OK) return e;
  const RefBank cur = fields_bank(c);
  set_fields(c, c->alt);
  c->alt = cur;
  c->bank ^= 1;
  HIP_TRY(hipStreamWaitEvent(c->rstream, c->ev_read[c->bank], 0));
  c->update_open = true;
  return DPT_OK;
}

void rel_pose_f32(const dpt_ctx* c, const double* T_cw, float* out12) {
  double Tinv[16], Trel[16];
  invert(c->T_rw, Tinv);
  compose(T_cw, Tinv, Trel);
  orthonormalize34(Trel);
  for (int j = 0; j < 12; ++j) out12[j] = (float)Trel[j];
}

void rel_pose_f32(const dpt_ctx* c, const double* T_cw, double* out12) {
  double Tinv[16], Trel[16];
  invert(c->T_rw, Tinv);
  compose(T_cw, Tinv, Trel);
  for (int j = 0; j < 12; ++j) out12[j] = Trel[j];
  orthonormalize34(out12);
}

}  // namespace

extern "C" {

const char* dpt_last_error(void) { return g_err.c_str(); }

int dpt_create(const dpt_camera* cam, const dpt_params* prm, int32_t max_points, void* hip_stream, dpt_ctx** out) {
  g_err.clear();
  if (!out) return fail(DPT_E_ARG, "out is NULL");
  *out = nullptr;
  int e;
  if ((e = check_camera(cam)) != DPT_OK) return e;
  if ((e = check_params(prm, cam)) != DPT_OK) return e;
  if (max_points < 1 || max_points > 65536) return fail(DPT_E_ARG, "max_points %d outside [1, 65536]", max_points);
  dpt_ctx* c = new (std::nothrow) dpt_ctx();
  if (!c) return fail(DPT_E_OOM, "host allocation failed");
  c->cam = *cam;
  c->prm = *prm;
  c->cap = max_points;
  c->stream = (hipStream_t)hip_stream;
  c->pat = make_pattern(prm);
  std::memset(c->lv, 0, sizeof c->lv);
  std::memset(&c->pg, 0, sizeof c->pg);
  c->pg.levels = prm->levels;
  int64_t off = 0;
  for (int l = 0; l < prm->levels; ++l) {
    const double s = std::ldexp(1.0, l);
    LevelGeom& g = c->lv[l];
    g.W = cam->width >> l;
    g.H = cam->height >> l;
    g.off = off;
    g.fx = (float)(cam->fx / s);
    g.fy = (float)(cam->fy / s);
    g.cx = (float)((cam->cx + 0.5) / s - 0.5);
    g.cy = (float)((cam->cy + 0.5) / s - 0.5);
    c->pg.W[l] = g.W;
    c->pg.H[l] = g.H;
    c->pg.off[l] = off;
    off += (int64_t)g.W * g.H;
  }
  c->pyr_bytes = off;
  const size_t K = (size_t)prm->n_pattern, L = (size_t)prm->levels, cap = (size_t)max_points;
  if ((e = dev_alloc((void**)&c->pyr[0], (size_t)off)) || (e = dev_alloc((void**)&c->pyr[1], (size_t)off)) ||
      (e = dev_alloc((void**)&c->staging, (size_t)cam->width * cam->height)) ||
      (e = dev_alloc((void**)&c->x0, cap * sizeof(float4))) || (e = dev_alloc((void**)&c->valid, L * cap)) ||
      (e = dev_alloc((void**)&c->I0, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->gx, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->gy, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->pts, cap * 3 * sizeof(float))) ||
      (e = dev_alloc((void**)&c->sel_idx, (size_t)cam->width * cam->height * sizeof(int32_t))) ||
      (e = dev_alloc((void**)&c->sel_count, sizeof(int32_t))) ||
      (e = dev_alloc((void**)&c->sel_scratch, sizeof(int32_t) * select_scratch_ints(cam->width, cam->height))) || (e = dev_alloc((void**)&c->d_out, sizeof(TrackOut))) ||
      (e = dev_alloc((void**)&c->d_tot, kRedSlots * sizeof(float)))) {
    delete c;
    return e;
  }
  // the selection passes leave their histograms cleared for the next run: start cleared
  if (hipMemset(c->sel_scratch, 0, sizeof(int32_t) * select_scratch_ints(cam->width, cam->height)) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(DPT_E_HIP, "selection scratch initialisation failed");
  }
  if ((prm->flags & DPT_FLAG_GAUSS_F32) && ((e = dev_alloc((void**)&c->pyrf[0], (size_t)off * sizeof(float))) ||
                                            (e = dev_alloc((void**)&c->pyrf[1], (size_t)off * sizeof(float))))) {
    delete c;
    return e;
  }
  if ((prm->flags & DPT_FLAG_FIXED_H) &&
      ((e = dev_alloc((void**)&c->d_fixed, L * sizeof(FixedH))) ||
       (e = dev_alloc((void**)&c->d_hpart, L * ((cap + 255) / 256) * 21 * sizeof(float))))) {
    delete c;
    return e;
  }
  if (prm->precision == DPT_PREC_MIXED &&
      ((e = dev_alloc((void**)&c->I0h, L * cap * K * sizeof(__half))) ||
       (e = dev_alloc((void**)&c->gh, L * cap * K * sizeof(__half2))))) {
    delete c;
    return e;
  }
  if (hipHostMalloc((void**)&c->h_out, sizeof(TrackOut)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_tot, kRedSlots * sizeof(float)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_pts, cap * 3 * sizeof(float)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_sel, (cap + 1) * sizeof(int32_t)) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_pts, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(DPT_E_OOM, "pinned host allocation failed");
  }
  if ((e = dev_alloc((void**)&c->d_hist, 24 * sizeof(double)))) {
    delete c;
    return e;
  }
  c->phys[0] = fields_bank(c);
  static const double kIdentity[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  if (launch_set_history(c->d_hist, kIdentity, kIdentity, c->stream) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(DPT_E_HIP, "pose history initialisation failed");
  }
  *out = c;
  return DPT_OK;
}

void dpt_destroy(dpt_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->rstream) (void)hipStreamSynchronize(ctx->rstream);
  delete ctx;
}

int dpt_build_pyramid(dpt_ctx* c, int32_t slot, const uint8_t* img, int64_t pitch, int32_t img_on_device) {
  g_err.clear();
  if (!c || !img) return fail(DPT_E_ARG, "NULL argument");
  if (img_on_device != 0 && img_on_device != 1) return fail(DPT_E_ARG, "img_on_device %d is neither 0 nor 1", img_on_device);
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (pitch < c->cam.width) return fail(DPT_E_ARG, "pitch %lld < width %d", (long long)pitch, c->cam.width);
  if (slot == DPT_SLOT_REF) {
    const int e = open_update(c);
    if (e != DPT_OK) return e;
  }
  // a reference pyramid belongs to the reference stream (the context's own without one)
  const hipStream_t st = slot == DPT_SLOT_REF ? ref_stream(c) : c->stream;
  const uint8_t* src = img;
  int64_t sp = pitch;
  uint8_t* stage = c->staging;
  if (!img_on_device) {
    HIP_TRY(hipMemcpy2DAsync(stage, c->cam.width, img, pitch, c->cam.width, c->cam.height, hipMemcpyHostToDevice, st));
    src = stage;
    sp = c->cam.width;
  }
  int ps = -1;
  const bool prof = c->prof && st == c->stream;  // the profile ring times the context's stream
  if (prof) HIP_TRY(c->prof_pyr.begin(c->stream, &ps));
  HIP_TRY(launch_pyramid(src, sp, c->pyr[slot], c->pg, st));
  if (c->pyrf[slot]) HIP_TRY(launch_pyramid_gauss(src, sp, c->pyrf[slot], c->pg, st));
  if (prof) HIP_TRY(c->prof_pyr.end(c->stream, ps));
  c->have_pyr[slot] = true;
  if (slot == DPT_SLOT_REF) c->have_ref = false;
  if (!img_on_device) HIP_TRY(hipStreamSynchronize(st));  // the host buffer is only borrowed
  return DPT_OK;
}

int dpt_get_pyramid(dpt_ctx* c, int32_t slot, int32_t level, uint8_t* host_dst) {
  g_err.clear();
  if (!c || !host_dst) return fail(DPT_E_ARG, "NULL argument");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_pyr[slot]) return fail(DPT_E_STATE, "slot %d has no pyramid", slot);
  if (slot == DPT_SLOT_REF && c->rstream) HIP_TRY(hipStreamSynchronize(c->rstream));  // built on the reference stream
  const LevelGeom& g = c->lv[level];
  HIP_TRY(hipMemcpyAsync(host_dst, c->pyr[slot] + g.off, (size_t)g.W * g.H, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int dpt_get_pyramid_f32(dpt_ctx* c, int32_t slot, int32_t level, float* host_dst) {
  g_err.clear();
  if (!c || !host_dst) return fail(DPT_E_ARG, "NULL argument");
  if (!(c->prm.flags & DPT_FLAG_GAUSS_F32)) return fail(DPT_E_STATE, "the context has no Gaussian float pyramid");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_pyr[slot]) return fail(DPT_E_STATE, "slot %d has no pyramid", slot);
  if (slot == DPT_SLOT_REF && c->rstream) HIP_TRY(hipStreamSynchronize(c->rstream));
  const LevelGeom& g = c->lv[level];
  HIP_TRY(hipMemcpyAsync(host_dst, c->pyrf[slot] + g.off, (size_t)g.W * g.H * sizeof(float), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int dpt_select_points_noalloc(const uint8_t* img, int32_t width, int32_t height, int64_t pitch, int32_t n,
                              int32_t margin, int32_t* idx, int32_t* count, void* hip_stream) {
  g_err.clear();
  if (!img || !idx || !count) return fail(DPT_E_ARG, "NULL argument");
  if (width < 3 || height < 3) return fail(DPT_E_ARG, "image %dx%d", width, height);
  if ((int64_t)width * height > kNoAllocSelectPixels)
    return fail(DPT_E_ARG, "image %dx%d exceeds the %lld pixels of the static scratch", width, height,
                (long long)kNoAllocSelectPixels);
  if (pitch < width || pitch > INT32_MAX) return fail(DPT_E_ARG, "pitch %lld", (long long)pitch);
  if (n < 1 || (int64_t)n > (int64_t)width * height) return fail(DPT_E_ARG, "n %d", n);
  if (margin < 1 || 2 * margin >= width || 2 * margin >= height) return fail(DPT_E_ARG, "margin %d", margin);
  HIP_TRY(launch_select_noalloc(img, width, height, pitch, margin, n, idx, count,
                                static_cast<hipStream_t>(hip_stream)));
  return DPT_OK;
}

int dpt_select_points(dpt_ctx* c, int32_t n, int32_t margin, int32_t* host_idx, int32_t* n_out) {
  g_err.clear();
  if (!c || !host_idx || !n_out) return fail(DPT_E_ARG, "NULL argument");
  if (n < 1 || (int64_t)n > (int64_t)c->cam.width * c->cam.height) return fail(DPT_E_ARG, "n %d", n);
  if (margin < 1 || 2 * margin >= c->cam.width || 2 * margin >= c->cam.height) return fail(DPT_E_ARG, "margin %d", margin);
  if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "no reference pyramid");
  const hipStream_t rs = ref_stream(c);  // the reference pyramid belongs to the reference stream
  HIP_TRY(launch_select(c->pyr[DPT_SLOT_REF], c->cam.width, c->cam.height, margin, n, c->sel_idx, c->sel_count,
                        c->sel_scratch, rs));
  // count and the first min(n, cap) indices come back with one synchronisation
  const int32_t first = n < c->cap ? n : c->cap;
  HIP_TRY(hipMemcpyAsync(c->h_sel, c->sel_count, sizeof(int32_t), hipMemcpyDeviceToHost, rs));
  HIP_TRY(hipMemcpyAsync(c->h_sel + 1, c->sel_idx, (size_t)first * sizeof(int32_t), hipMemcpyDeviceToHost, rs));
  HIP_TRY(hipStreamSynchronize(rs));
  const int32_t cnt = c->h_sel[0];
  if (cnt < 0 || cnt > n) return fail(DPT_E_HIP, "selection returned %d of %d", cnt, n);
  std::memcpy(host_idx, c->h_sel + 1, (size_t)std::min(cnt, first) * sizeof(int32_t));
  if (cnt > first) {  // more points than the map holds (selection only): copy the rest directly
    HIP_TRY(hipMemcpy(host_idx + first, c->sel_idx + first, (size_t)(cnt - first) * sizeof(int32_t),
                      hipMemcpyDeviceToHost));
  }
  *n_out = cnt;
  return DPT_OK;
}

}  // extern "C"

namespace {

// Arguments of the IC precompute of n device points P at T_rw for context c.
PrecomputeArgs precompute_args(const dpt_ctx* c, const float* P, int32_t n, const double T_rw[16]) {
  PrecomputeArgs a;
  std::memset(&a, 0, sizeof a);
  a.ref = c->pyr[DPT_SLOT_REF];
  a.reff = c->pyrf[DPT_SLOT_REF];
  for (int l = 0; l < kMaxLevels; ++l) a.lv[l] = c->lv[l];
  a.levels = c->prm.levels;
  a.z_min = c->prm.z_min;
  a.pat = c->pat;
  a.P = P;
  for (int j = 0; j < 12; ++j) a.T_rw[j] = (float)T_rw[j];
  a.x0 = c->x0;
  a.valid = c->valid;
  a.I0 = c->I0;
  a.gx = c->gx;
  a.gy = c->gy;
  a.I0h = c->I0h;
  a.gh = c->gh;
  a.fixed = c->d_fixed;
  a.hpart = c->d_hpart;
  a.n = n;
  a.cap = c->cap;
  return a;
}

int commit_reference(dpt_ctx* c, int32_t n, const double T_rw[16], bool record = true) {
  std::memcpy(c->T_rw, T_rw, sizeof c->T_rw);
  c->n_points = n;
  c->have_ref = true;
  c->bank_n[c->bank] = n;
  if (c->rstream && !c->batch_owned) {
    if (record) HIP_TRY(hipEventRecord(c->ev_ready, c->rstream));
    c->commit_pending = true;
    c->update_open = false;
  }
  return DPT_OK;
}

// With a reference stream, a reference update starts with a new reference
// pyramid (which selects the bank it writes).
int check_update_open(const dpt_ctx* c) {
  if (c->rstream && !c->update_open)
    return fail(DPT_E_STATE, "with a reference stream, a reference update starts with dpt_build_pyramid(DPT_SLOT_REF)");
  return DPT_OK;
}

// IC precompute of the reference cache from n device points P at T_rw.
int precompute_reference(dpt_ctx* c, const float* P, int32_t n, const double T_rw[16]) {
  const PrecomputeArgs a = precompute_args(c, P, n, T_rw);
  HIP_TRY(launch_precompute(a, ref_stream(c)));
  if (c->prm.flags & DPT_FLAG_FIXED_H) HIP_TRY(launch_fixed_h(a, ref_stream(c)));
  return commit_reference(c, n, T_rw);
}

}  // namespace

extern "C" {

int dpt_set_reference_points(dpt_ctx* c, const float* xyz, int32_t n, const double T_rw[16], int32_t on_device) {
  g_err.clear();
  if (on_device != 0 && on_device != 1) return fail(DPT_E_ARG, "xyz_on_device %d is neither 0 nor 1", on_device);
  if (!c || !T_rw || (n > 0 && !xyz)) return fail(DPT_E_ARG, "NULL argument");
  if (n < 0 || n > c->cap) return fail(DPT_E_ARG, "n %d outside [0, %d]", n, c->cap);
  if (!finite16(T_rw)) return fail(DPT_E_ARG, "T_rw not finite");
  if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "no reference pyramid");
  int e = check_update_open(c);
  if (e != DPT_OK) return e;
  const float* P = xyz;
  if (n > 0 && !on_device) {
    // staged through pinned memory: the caller's buffer is free on return and
    // the upload does not block; the staging buffer is reused only after the
    // previous upload out of it has run
    HIP_TRY(hipEventSynchronize(c->ev_pts));
    std::memcpy(c->h_pts, xyz, (size_t)n * 3 * sizeof(float));
    HIP_TRY(hipMemcpyAsync(c->pts, c->h_pts, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, ref_stream(c)));
    HIP_TRY(hipEventRecord(c->ev_pts, ref_stream(c)));
    P = c->pts;
  }
  return precompute_reference(c, P, n, T_rw);
}

int dpt_set_reference_from_depth(dpt_ctx* c, int32_t n, int32_t margin, const float* depth, int64_t depth_pitch,
                                 int32_t depth_on_device, const double T_rw[16]) {
  g_err.clear();
  if (depth_on_device != 0 && depth_on_device != 1)
    return fail(DPT_E_ARG, "depth_on_device %d is neither 0 nor 1", depth_on_device);
  if (!c || !depth || !T_rw) return fail(DPT_E_ARG, "NULL argument");
  if (n < 1 || n > c->cap) return fail(DPT_E_ARG, "n %d outside [1, %d]", n, c->cap);
  if (margin < 1 || 2 * margin >= c->cam.width || 2 * margin >= c->cam.height) return fail(DPT_E_ARG, "margin %d", margin);
  if (depth_pitch < c->cam.width) return fail(DPT_E_ARG, "depth pitch %lld < width %d", (long long)depth_pitch, c->cam.width);
  if (!finite16(T_rw)) return fail(DPT_E_ARG, "T_rw not finite");
  if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "no reference pyramid");
  int e = check_update_open(c);
  if (e != DPT_OK) return e;
  const hipStream_t rs = ref_stream(c);
  const float* D = depth;
  int64_t pitch = depth_pitch;
  if (!depth_on_device) {
    if (!c->depth_stage) {
      const int e2 = dev_alloc((void**)&c->depth_stage, (size_t)c->cam.width * c->cam.height * sizeof(float));
      if (e2) return e2;
    }
    HIP_TRY(hipMemcpy2DAsync(c->depth_stage, c->cam.width * sizeof(float), depth, depth_pitch * sizeof(float),
                             c->cam.width * sizeof(float), c->cam.height, hipMemcpyHostToDevice, rs));
    HIP_TRY(hipStreamSynchronize(rs));  // pageable source
    D = c->depth_stage;
    pitch = c->cam.width;
  }
  HIP_TRY(launch_select(c->pyr[DPT_SLOT_REF], c->cam.width, c->cam.height, margin, n, c->sel_idx, c->sel_count,
                        c->sel_scratch, rs));
  BackprojectArgs b;
  b.idx = c->sel_idx;
  b.count = c->sel_count;
  b.depth = D;
  b.pitch = pitch;
  b.W = c->cam.width;
  b.n = n;
  b.fx = c->cam.fx, b.fy = c->cam.fy, b.cx = c->cam.cx, b.cy = c->cam.cy;
  for (int j = 0; j < 12; ++j) b.T_rw[j] = T_rw[j];
  b.P = c->pts;
  HIP_TRY(launch_backproject(b, rs));
  return precompute_reference(c, c->pts, n, T_rw);
}

}  // extern "C"

namespace {

int synchronize(dpt_ctx* c);
int alloc_window_bank(dpt_ctx* c, int n_frames, uint8_t** win, WinJob** job);

// Allocate the second reference bank of a context (the buffers a reference
// update writes: reference pyramid, cache, points, fixed-H state).
int alloc_alt_bank(dpt_ctx* c) {
  if (c->phys[1].x0) return DPT_OK;
  const size_t L = (size_t)c->prm.levels, cap = (size_t)c->cap, K = (size_t)c->prm.n_pattern;
  RefBank& b = c->phys[1];
  int e;
  if ((e = dev_alloc((void**)&b.pyr_ref, (size_t)c->pyr_bytes)) || (e = dev_alloc((void**)&b.x0, cap * sizeof(float4))) ||
      (e = dev_alloc((void**)&b.valid, L * cap)) || (e = dev_alloc((void**)&b.I0, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&b.gx, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&b.gy, L * cap * K * sizeof(float))) || (e = dev_alloc((void**)&b.pts, cap * 3 * sizeof(float))))
    return e;
  if (c->pyrf[DPT_SLOT_REF] && (e = dev_alloc((void**)&b.pyrf_ref, (size_t)c->pyr_bytes * sizeof(float)))) return e;
  if (c->d_fixed && ((e = dev_alloc((void**)&b.d_fixed, L * sizeof(FixedH))) ||
                     (e = dev_alloc((void**)&b.d_hpart, L * ((cap + 255) / 256) * 21 * sizeof(float)))))
    return e;
  if (c->I0h && ((e = dev_alloc((void**)&b.I0h, L * cap * K * sizeof(__half))) ||
                 (e = dev_alloc((void**)&b.gh, L * cap * K * sizeof(__half2)))))
    return e;
  if (c->win_cap > 0 && (e = alloc_window_bank(c, c->win_cap, &c->win_b1, &c->d_winjob_b1)) != DPT_OK) return e;
  for (hipEvent_t* ev : {&c->ev_read[0], &c->ev_read[1], &c->ev_ready})
    if (!*ev) HIP_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  return DPT_OK;
}

}  // namespace

extern "C" {

int dpt_stream_create(void** out) {
  g_err.clear();
  if (!out) return fail(DPT_E_ARG, "NULL argument");
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  *out = s;
  return DPT_OK;
}

int dpt_stream_destroy(void* s) {
  g_err.clear();
  if (!s) return DPT_OK;
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(s)));
  HIP_TRY(hipStreamDestroy(static_cast<hipStream_t>(s)));
  return DPT_OK;
}

int dpt_set_reference_stream(dpt_ctx* c, void* hip_stream) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  if (c->update_open) return fail(DPT_E_STATE, "a reference update is open: finish it first");
  hipStream_t rs = static_cast<hipStream_t>(hip_stream);
  if (rs == c->stream) rs = nullptr;  // the context's own stream: no separate reference stream
  // everything in flight on either stream finishes first
  int e;
  if (!c->pending.empty() && (e = synchronize(c)) != DPT_OK) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->rstream) HIP_TRY(hipStreamSynchronize(c->rstream));
  c->commit_pending = false;
  if (rs) {
    const bool fresh = !c->phys[1].x0;
    if ((e = alloc_alt_bank(c)) != DPT_OK) return e;
    if (fresh) {  // the fields hold bank 0: the other one is bank 1
      c->alt = c->phys[1];
      c->bank_n[1] = 0;
    }
    if (c->eng_ready) c->eng.dirty = true;  // the descriptors gain the second bank
  }
  c->rstream = rs;
  return DPT_OK;
}

}  // extern "C"

extern "C" {

int dpt_tween_set_policy(dpt_ctx* c, const dpt_tween_policy* p) {
  g_err.clear();
  if (!c || !p) return fail(DPT_E_ARG, "NULL argument");
  if (!(p->max_cost >= 0.0f) || !std::isfinite(p->max_baseline) || p->max_direct < 0)
    return fail(DPT_E_ARG, "invalid tween thresholds");
  if (p->n_points < 1 || p->n_points > c->cap) return fail(DPT_E_ARG, "n_points %d outside [1, %d]", p->n_points, c->cap);
  if (p->margin < 1 || 2 * p->margin >= c->cam.width || 2 * p->margin >= c->cam.height)
    return fail(DPT_E_ARG, "margin %d", p->margin);
  c->tween = *p;
  c->tween_policy = true;
  return DPT_OK;
}

int dpt_tween_anchor(dpt_ctx* c, const uint8_t* img, int64_t pitch, int32_t img_on_device, const float* depth,
                     int64_t depth_pitch, int32_t depth_on_device, const double T_cw[16]) {
  g_err.clear();
  if (!c || !img || !depth || !T_cw) return fail(DPT_E_ARG, "NULL argument");
  if (!c->tween_policy) return fail(DPT_E_STATE, "no tween policy");
  if (!finite16(T_cw)) return fail(DPT_E_ARG, "T_cw not finite");
  int e;
  if (!c->pending.empty() && (e = dpt_synchronize(c)) != DPT_OK) return e;
  if ((e = dpt_build_pyramid(c, DPT_SLOT_REF, img, pitch, img_on_device)) != DPT_OK) return e;
  if ((e = dpt_set_reference_from_depth(c, c->tween.n_points, c->tween.margin, depth, depth_pitch, depth_on_device,
                                        T_cw)) != DPT_OK)
    return e;
  double T[16];
  std::memcpy(T, T_cw, sizeof T);
  orthonormalize34(T);
  std::memcpy(c->tween_hist[0], c->tween_anchored ? c->tween_hist[1] : T, sizeof T);
  std::memcpy(c->tween_hist[1], T, sizeof T);
  if ((e = dpt_set_pose_history(c, c->tween_hist[0], c->tween_hist[1])) != DPT_OK) return e;
  c->tween_anchored = true;
  c->tween_needs_anchor = false;
  c->tween_direct = 0;
  return DPT_OK;
}

int dpt_tween_frame(dpt_ctx* c, const uint8_t* img, int64_t pitch, int32_t img_on_device, dpt_tween_result* out) {
  g_err.clear();
  if (!c || !img || !out) return fail(DPT_E_ARG, "NULL argument");
  if (!c->tween_policy || !c->tween_anchored) return fail(DPT_E_STATE, "the tween schedule has no reference yet");
  if (c->tween_needs_anchor) return fail(DPT_E_STATE, "the last tween frame went to the indirect pipeline: anchor first");
  std::memset(out, 0, sizeof *out);
  if (c->tween_direct >= c->tween.max_direct) {
    out->decision = DPT_TWEEN_INDIRECT_MAX_FRAMES;
    out->direct_since_ref = c->tween_direct;
    c->tween_needs_anchor = true;
    return DPT_OK;
  }
  int e;
  if ((e = dpt_build_pyramid(c, DPT_SLOT_CUR, img, pitch, img_on_device)) != DPT_OK) return e;
  // constant velocity: T1 T0^-1 T1 (rigid inverse), back on SO(3)
  double inv0[16], m[16], start[16];
  invert(c->tween_hist[0], inv0);
  compose(c->tween_hist[1], inv0, m);
  compose(m, c->tween_hist[1], start);
  orthonormalize34(start);
  if ((e = dpt_track_frame(c, start, &out->track)) != DPT_OK) return e;
  out->tracked = 1;
  const double* T = out->track.T_cw;
  // camera centres -R^T t of the estimate and of the reference
  double ce[3], cr[3];
  for (int j = 0; j < 3; ++j) {
    ce[j] = -(T[j] * T[3] + T[4 + j] * T[7] + T[8 + j] * T[11]);
    cr[j] = -(c->T_rw[j] * c->T_rw[3] + c->T_rw[4 + j] * c->T_rw[7] + c->T_rw[8 + j] * c->T_rw[11]);
  }
  out->baseline = std::sqrt((ce[0] - cr[0]) * (ce[0] - cr[0]) + (ce[1] - cr[1]) * (ce[1] - cr[1]) +
                            (ce[2] - cr[2]) * (ce[2] - cr[2]));
  const int st = out->track.status;
  if (st != DPT_TRACK_OK && st != DPT_TRACK_MAX_ITERS)
    out->decision = DPT_TWEEN_INDIRECT_FAILED;
  else if (!(out->track.final_cost <= (double)c->tween.max_cost))
    out->decision = DPT_TWEEN_INDIRECT_COST;
  else if (c->tween.max_baseline > 0.0f && out->baseline > (double)c->tween.max_baseline)
    out->decision = DPT_TWEEN_INDIRECT_BASELINE;
  else
    out->decision = DPT_TWEEN_DIRECT;
  if (out->decision == DPT_TWEEN_DIRECT) {
    ++c->tween_direct;
    std::memcpy(c->tween_hist[0], c->tween_hist[1], sizeof c->tween_hist[0]);
    std::memcpy(c->tween_hist[1], T, sizeof c->tween_hist[1]);
  } else {
    c->tween_needs_anchor = true;
  }
  out->direct_since_ref = c->tween_direct;
  return DPT_OK;
}

}  // extern "C"

namespace {

// Patterns other than the 8-pixel one, and the floating-point pyramid, run on
// the generic cooperative variant (four lanes per point, fixed 256-thread chunks).
bool generic_track(const dpt_params& p) { return p.n_pattern != 8 || (p.flags & DPT_FLAG_GAUSS_F32); }

// Two threads per point: the pair launch mode, for the 8-pixel kernels.
bool pair_track(const dpt_params& p, int mode) { return mode == DPT_LAUNCH_COOP_PAIRS && !generic_track(p); }

int coop_variant(const dpt_params& p, int mode) {
  const int pairs = pair_track(p, mode) ? kCoopPairs : 0;
  if (p.precision == DPT_PREC_MIXED) return kCoopMixed | pairs;
  int v = (p.flags & DPT_FLAG_FIXED_H) ? kCoopFixedH : kCoopFP32;
  if (generic_track(p)) v |= kCoopGeneric | ((p.flags & DPT_FLAG_GAUSS_F32) ? kCoopFloatPyr : 0);
  return v | pairs;
}

// Threads and points per chunk of a cooperative launch (`chunk` as configured).
int coop_threads(const dpt_params& p, int chunk, int mode) {
  return generic_track(p) ? kGenericThreads : pair_track(p, mode) ? 2 * chunk : chunk;
}
int coop_ppc(const dpt_params& p, int chunk) {
  return generic_track(p) ? kGenericThreads / kLanesPerPoint : chunk;
}

// Whether this frame runs on the cooperative chunked kernel.
bool use_coop(dpt_ctx* c) {
  if (c->prm.precision == DPT_PREC_MIXED) return true;  // only the cooperative kernel has the mixed variant
  if (c->launch_mode == DPT_LAUNCH_WORKGROUP) return false;
  const int ppc = coop_ppc(c->prm, c->chunk);
  const int nch = c->n_points > 0 ? (c->n_points + ppc - 1) / ppc : 1;
  return nch <= coop_max_blocks(coop_threads(c->prm, c->chunk, c->launch_mode)) / 8;  // the XCD-packed grid may hold up to 8x padding
}

// The context's single-stream cooperative engine, built on first use and
// refreshed when the map changed size.
int ensure_engine(dpt_ctx* c) {
  const int threads = coop_threads(c->prm, c->chunk, c->launch_mode), ppc = coop_ppc(c->prm, c->chunk);
  const int nmax = std::max(c->n_points, std::max(c->bank_n[0], c->bank_n[1]));
  const int nch = nmax > 0 ? (nmax + ppc - 1) / ppc : 1;
  if (8 * nch > coop_max_blocks(threads))
    return fail(DPT_E_ARG, "%d points exceed the cooperative capacity at %d points per chunk", c->n_points, ppc);
  if (!c->eng_ready) {
    HIP_TRY(c->eng.init(1, &c->cap, threads, ppc, true, c->stream));
    c->eng.variant = coop_variant(c->prm, c->launch_mode);
    c->eng_ready = true;
  }
  const RefCache r0 = refcache_of(c, 0), r1 = refcache_of(c, 1);
  if (c->eng.dirty || c->eng.h_streams[0].a.ref.n != r0.n || c->eng.h_streams[0].ref_alt.n != r1.n ||
      c->eng.h_streams[0].ref_alt.x0 != r1.x0 || c->eng.h_streams[0].win != c->win ||
      c->eng.h_streams[0].win_alt != c->win_b1) {
    TrackArgs a;
    fill_track_args(c, a);
    a.ref = r0;
    c->eng.set_stream(0, a, r1, c->d_hist, c->win, c->win_b1, c->win_stride);
  }
  if (c->eng.dirty) HIP_TRY(c->eng.upload());
  return DPT_OK;
}

// Start slot of one stream for the context's current reference.
void fill_start(const dpt_ctx* c, int mode, const double* T_cw_init, StartSlot* st, const double* dev_rel = nullptr) {
  std::memset(st, 0, sizeof *st);
  st->mode = mode;
  if (mode == kStartGiven) rel_pose_f32(c, T_cw_init, st->T_rel);
  st->dev_rel = dev_rel;
  st->bank = c->bank;  // the committed reference (the fields' bank)
  for (int j = 0; j < 12; ++j) st->T_rw[j] = c->T_rw[j];
}

// Result of a finished track: T_cw = T_rel T_rw, with the reference pose the
// track ran against (row-major, its first 12 entries).
void fill_result(const dpt_ctx* c, const TrackOut& o, const double* T_rw, dpt_result* out) {
  double Trel[16], Trw[16];
  for (int j = 0; j < 12; ++j) {
    Trel[j] = o.Td[j];
    Trw[j] = T_rw[j];
  }
  Trel[12] = Trel[13] = Trel[14] = 0.0;
  Trel[15] = 1.0;
  Trw[12] = Trw[13] = Trw[14] = 0.0;
  Trw[15] = 1.0;
  std::memset(out, 0, sizeof *out);
  compose(Trel, Trw, out->T_cw);
  out->final_cost = o.n > 0 ? (double)o.E / (double)o.n : 0.0;
  out->iterations = o.iterations;
  for (int l = 0; l < kMaxLevels; ++l) out->iters_per_level[l] = o.iters_per_level[l];
  out->n_valid_points = o.n_valid_points;
  out->status = o.status;
  out->samples = o.samples;
}

// Enqueue one cooperative track; its result is filled at the next synchronize().
int enqueue_coop(dpt_ctx* c, int mode, const double* T_cw_init, dpt_result* out) {
  if ((int)c->pending.size() >= kRing)
    return fail(DPT_E_STATE, "%d tracks in flight: synchronise first", kRing);
  const int e = ensure_engine(c);
  if (e != DPT_OK) return e;
  const int slot = c->slot_next;
  c->slot_next = (slot + 1) % kRing;
  fill_start(c, mode, T_cw_init, c->eng.start(slot), c->d_prop);
  int ps = -1;
  if (c->prof) HIP_TRY(c->prof_trk.begin(c->stream, &ps));
  HIP_TRY(c->eng.launch(c->spin_limit, slot));
  if (c->prof) HIP_TRY(c->prof_trk.end(c->stream, ps));
  c->pending.emplace_back(slot, out);
  return DPT_OK;
}

// After a failed wait: let the stream run out (every wait inside the kernels is
// bounded, so it does unless the device itself failed), fill the results of
// the tracks that finished, mark the others TIMEOUT, and forget them all, so no
// entry of the pending list outlives the caller's result buffers and no kernel
// still reads the caller's frames.  Leaves the failure's message in place.
void abandon(dpt_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  (void)hipGetLastError();
  for (const auto& p : c->pending) {
    if (p.first < 0 || !p.second) continue;
    if (c->eng.done(p.first)) {
      fill_result(c, c->eng.out(p.first)[0], c->eng.start(p.first)[0].T_rw, p.second);
    } else {
      std::memset(p.second, 0, sizeof *p.second);
      p.second->status = kStatusTimeout;
    }
  }
  c->pending.clear();
}

// Wait for the stream and fill the results of every track in flight.
int synchronize(dpt_ctx* c) {
  const hipError_t es = hipStreamSynchronize(c->stream);
  if (es != hipSuccess) {
    const int r = fail(DPT_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
    abandon(c);
    return r;
  }
  bool timeout = false;
  for (const auto& p : c->pending) {
    if (p.first < 0) continue;  // ran synchronously, result already filled
    const TrackOut& o = c->eng.out(p.first)[0];
    timeout |= o.status == kStatusTimeout;
    if (p.second) fill_result(c, o, c->eng.start(p.first)[0].T_rw, p.second);
  }
  c->pending.clear();
  if (c->prof) {
    HIP_TRY(c->prof_pyr.drain());
    HIP_TRY(c->prof_trk.drain());
  }
  if (timeout) {
    (void)c->eng.clear_partials();
    (void)hipStreamSynchronize(c->stream);
    return fail(DPT_E_HIP, "cooperative track: chunk synchronisation timed out");
  }
  return DPT_OK;
}

// Wait until `done()` holds: the results of a launch in flight arrive through
// host-mapped memory, each stream's last written after a system-scope fence.
// Gives up if the stream has run dry without them, or after a minute.
template <class Done>
int wait_results(hipStream_t stream, Done done) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int64_t k = 0; !done(); ++k) {
    if ((k & 1023) == 1023) {
      const hipError_t q = hipStreamQuery(stream);
      if (q == hipSuccess && !done()) return fail(DPT_E_HIP, "the stream finished without a track's results");
      if (q != hipSuccess && q != hipErrorNotReady) return fail(DPT_E_HIP, "stream: %s", hipGetErrorString(q));
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
        return fail(DPT_E_HIP, "no track results after 60 s");
      std::this_thread::yield();
    }
  }
  return DPT_OK;
}

// The oldest n tracks in flight: wait for their results only, fill them, and
// leave the later ones running.  A timeout among them falls back to synchronize().
int collect(dpt_ctx* c, int n) {
  if (n < 0 || n > (int)c->pending.size())
    return fail(DPT_E_ARG, "%d results asked, %d tracks in flight", n, (int)c->pending.size());
  bool timeout = false;
  for (int i = 0; i < n; ++i) {
    const int slot = c->pending[i].first;
    if (slot < 0) continue;
    const int e = wait_results(c->stream, [&] { return c->eng.done(slot); });
    if (e != DPT_OK) {
      abandon(c);
      return e;
    }
    const TrackOut& o = c->eng.out(slot)[0];
    timeout |= o.status == kStatusTimeout;
  }
  if (timeout) return synchronize(c);
  for (int i = 0; i < n; ++i) {
    const auto& p = c->pending[i];
    if (p.first >= 0 && p.second) fill_result(c, c->eng.out(p.first)[0], c->eng.start(p.first)[0].T_rw, p.second);
  }
  c->pending.erase(c->pending.begin(), c->pending.begin() + n);
  return DPT_OK;
}

// One-workgroup track (any pattern), synchronous.
int track_workgroup(dpt_ctx* c, const double T_cw_init[16], dpt_result* out) {
  TrackArgs a;
  fill_track_args(c, a);
  rel_pose_f32(c, T_cw_init, a.T_init);
  int ps = -1;
  if (c->prof) HIP_TRY(c->prof_trk.begin(c->stream, &ps));
  HIP_TRY(launch_track(a, c->stream));
  if (c->prof) HIP_TRY(c->prof_trk.end(c->stream, ps));
  HIP_TRY(hipMemcpyAsync(c->h_out, c->d_out, sizeof(TrackOut), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->prof) {
    HIP_TRY(c->prof_pyr.drain());
    HIP_TRY(c->prof_trk.drain());
  }
  fill_result(c, *c->h_out, c->T_rw, out);
  return DPT_OK;
}

// Every track passes here: the reference must be committed, and the
// context's stream is ordered after an update on the reference stream.
int check_track_state(dpt_ctx* c) {
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  if (!c->have_pyr[DPT_SLOT_CUR]) return fail(DPT_E_STATE, "no current pyramid");
  return consume_commit(c);
}

// Window pyramids for n_frames frames (grown on demand; nothing may be in
// flight).  *grown tells the caller that the engines must see the new buffer.
// One bank's window pyramid buffer of n_frames frames and its job.
int alloc_window_bank(dpt_ctx* c, int n_frames, uint8_t** win, WinJob** job) {
  const int64_t stride = (c->pyr_bytes + 255) / 256 * 256;
  int e;
  if ((e = dev_alloc((void**)win, (size_t)stride * n_frames)) != DPT_OK) return e;
  if (!*job && (e = dev_alloc((void**)job, sizeof(WinJob))) != DPT_OK) return e;
  WinJob j;
  std::memset(&j, 0, sizeof j);
  j.dst = *win;
  j.dst_stride = stride;
  j.g = c->pg;
  HIP_TRY(hipMemcpy(*job, &j, sizeof j, hipMemcpyHostToDevice));
  c->win_stride = stride;
  return DPT_OK;
}

// Window pyramids for n_frames frames, for each bank in use (grown on demand;
// nothing may be in flight).  *grown tells the caller that the engines must
// see the new buffers.
int ensure_window(dpt_ctx* c, int n_frames, bool* grown) {
  *grown = false;
  if (n_frames <= c->win_cap) return DPT_OK;
  for (void** p : {(void**)&c->win, (void**)&c->win_b1, (void**)&c->win_staging}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  c->win_cap = 0;
  int e;
  if ((e = alloc_window_bank(c, n_frames, &c->win, &c->d_winjob)) != DPT_OK) return e;
  if (c->phys[1].x0 && (e = alloc_window_bank(c, n_frames, &c->win_b1, &c->d_winjob_b1)) != DPT_OK) return e;
  c->win_cap = n_frames;
  *grown = true;
  return DPT_OK;
}

// The window pyramid buffer and job of the bank the fields hold.
uint8_t* bank_win(const dpt_ctx* c) { return c->bank ? c->win_b1 : c->win; }
WinJob* bank_winjob(const dpt_ctx* c) { return c->bank ? c->d_winjob_b1 : c->d_winjob; }

// Level 0 of n_frames host frames into the context's device staging.
int stage_window(dpt_ctx* c, const uint8_t* frames, int64_t pitch, int64_t frame_stride, int n_frames,
                 hipStream_t s) {
  const int W = c->cam.width, H = c->cam.height;
  int e;
  if (!c->win_staging && (e = dev_alloc((void**)&c->win_staging, (size_t)W * H * c->win_cap)) != DPT_OK) return e;
  for (int f = 0; f < n_frames; ++f)
    HIP_TRY(hipMemcpy2DAsync(c->win_staging + (size_t)f * W * H, W, frames + f * frame_stride, pitch, W, H,
                             hipMemcpyHostToDevice, s));
  return DPT_OK;
}

int check_window_args(const dpt_ctx* c, const uint8_t* frames, int64_t pitch, int64_t frame_stride, int n_frames,
                      int on_device, int init_mode) {
  if (!frames) return fail(DPT_E_ARG, "frames is NULL");
  if (on_device != 0 && on_device != 1) return fail(DPT_E_ARG, "frames_on_device %d is neither 0 nor 1", on_device);
  if (n_frames < 1 || n_frames > DPT_MAX_WINDOW)
    return fail(DPT_E_ARG, "n_frames %d outside [1, %d]", n_frames, DPT_MAX_WINDOW);
  if (init_mode != DPT_INIT_GIVEN && init_mode != DPT_INIT_CONST_VELOCITY)
    return fail(DPT_E_ARG, "init_mode %d", init_mode);
  if (pitch < c->cam.width) return fail(DPT_E_ARG, "pitch %lld < width %d", (long long)pitch, c->cam.width);
  if (n_frames > 1 && frame_stride < pitch * (c->cam.height - 1) + c->cam.width)
    return fail(DPT_E_ARG, "frame_stride %lld smaller than one frame", (long long)frame_stride);
  if (c->prm.flags & DPT_FLAG_GAUSS_F32)
    return fail(DPT_E_ARG, "window tracking reads box pyramids (DPT_FLAG_GAUSS_F32 is set)");
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  return DPT_OK;
}

}  // namespace

extern "C" {

int dpt_track_frame(dpt_ctx* c, const double T_cw_init[16], dpt_result* out) {
  g_err.clear();
  if (!c || !T_cw_init || !out) return fail(DPT_E_ARG, "NULL argument");
  if (!finite16(T_cw_init)) return fail(DPT_E_ARG, "T_cw_init not finite");
  int e = check_track_state(c);
  if (e != DPT_OK) return e;
  if (use_coop(c)) {
    if ((e = enqueue_coop(c, kStartGiven, T_cw_init, out)) != DPT_OK) return e;
    return synchronize(c);
  }
  if (!c->pending.empty() && (e = synchronize(c)) != DPT_OK) return e;
  return track_workgroup(c, T_cw_init, out);
}

int dpt_track_enqueue(dpt_ctx* c, int32_t init_mode, const double T_cw_init[16], dpt_result* out) {
  g_err.clear();
  if (!c || !out) return fail(DPT_E_ARG, "NULL argument");
  if (init_mode != DPT_INIT_GIVEN && init_mode != DPT_INIT_CONST_VELOCITY && init_mode != DPT_INIT_PROPOSED)
    return fail(DPT_E_ARG, "init_mode %d", init_mode);
  if (init_mode == DPT_INIT_GIVEN && (!T_cw_init || !finite16(T_cw_init)))
    return fail(DPT_E_ARG, "T_cw_init missing or not finite");
  if (init_mode == DPT_INIT_PROPOSED && !c->have_prop)
    return fail(DPT_E_STATE, "no learned proposal: call dpt_cnn_propose first");
  int e = check_track_state(c);
  if (e != DPT_OK) return e;
  if (!use_coop(c)) {
    if (init_mode != DPT_INIT_GIVEN)
      return fail(DPT_E_ARG, "a constant-velocity or proposed start needs the cooperative track (launch mode AUTO or COOP)");
    const int e2 = dpt_track_frame(c, T_cw_init, out);
    if (e2 == DPT_OK) c->pending.emplace_back(-1, nullptr);  // in order with the tracks in flight, already done
    return e2;
  }
  const int mode = init_mode == DPT_INIT_GIVEN ? kStartGiven
                   : init_mode == DPT_INIT_PROPOSED ? kStartDevice
                                                    : kStartConstVelocity;
  return enqueue_coop(c, mode, T_cw_init, out);
}

int dpt_synchronize(dpt_ctx* c) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  return synchronize(c);
}

int dpt_collect(dpt_ctx* c, int32_t n) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  return collect(c, n);
}

int dpt_tracks_in_flight(dpt_ctx* c) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  return (int)c->pending.size();
}

int dpt_set_pose_history(dpt_ctx* c, const double T_older[16], const double T_newer[16]) {
  g_err.clear();
  if (!c || !T_older || !T_newer) return fail(DPT_E_ARG, "NULL argument");
  if (!finite16(T_older) || !finite16(T_newer)) return fail(DPT_E_ARG, "pose not finite");
  HIP_TRY(launch_set_history(c->d_hist, T_older, T_newer, c->stream));
  return DPT_OK;
}

int dpt_track_window_enqueue(dpt_ctx* c, const uint8_t* frames, int64_t pitch, int64_t frame_stride,
                             int32_t n_frames, int32_t frames_on_device, int32_t init_mode, const double T_cw_init[16],
                             dpt_result* out) {
  g_err.clear();
  if (!c || !out) return fail(DPT_E_ARG, "NULL argument");
  int e = check_window_args(c, frames, pitch, frame_stride, n_frames, frames_on_device, init_mode);
  if (e != DPT_OK) return e;
  if (init_mode == DPT_INIT_GIVEN && (!T_cw_init || !finite16(T_cw_init)))
    return fail(DPT_E_ARG, "T_cw_init missing or not finite");
  if (!use_coop(c)) return fail(DPT_E_ARG, "window tracking needs the cooperative track (launch mode AUTO or COOP)");
  if ((int)c->pending.size() + n_frames > kRing)
    return fail(DPT_E_STATE, "%d tracks in flight and %d more exceed %d: synchronise first", (int)c->pending.size(),
                n_frames, kRing);
  if (n_frames > c->win_cap) {  // the buffers in use by tracks in flight are replaced
    if (!c->pending.empty() && (e = synchronize(c)) != DPT_OK) return e;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->rstream) HIP_TRY(hipStreamSynchronize(c->rstream));
    bool grown = false;
    if ((e = ensure_window(c, n_frames, &grown)) != DPT_OK) return e;
    if (grown && c->eng_ready) c->eng.dirty = true;
  }
  if ((e = ensure_engine(c)) != DPT_OK) return e;
  // The first window after a reference update committed on the reference
  // stream builds its pyramids there too, behind the update (whose wait covers
  // the tracks that last read this bank's window buffer), beside the previous
  // window's track; the context's stream then waits for both.
  const bool on_ref = c->rstream && c->commit_pending && frames_on_device;
  const hipStream_t ps_stream = on_ref ? c->rstream : c->stream;
  if (!on_ref && (e = consume_commit(c)) != DPT_OK) return e;
  const uint8_t* src = frames;
  int64_t sp = pitch, sst = frame_stride;
  if (!frames_on_device) {
    if ((e = stage_window(c, frames, pitch, frame_stride, n_frames, c->stream)) != DPT_OK) return e;
    src = c->win_staging;
    sp = c->cam.width;
    sst = (int64_t)c->cam.width * c->cam.height;
  }
  // frames with rows W bytes apart serve as level 0 themselves: the pyramid
  // launch then writes the coarser levels only
  const bool l0_direct = sp == c->cam.width;
  PyrWinSrc srcs;
  std::memset(&srcs, 0, sizeof srcs);
  srcs.src[0] = src;
  srcs.pitch[0] = sp;
  srcs.stride[0] = sst;
  srcs.write_l0[0] = l0_direct ? 0 : 1;
  int ps = -1;
  const bool prof_pyr = c->prof && !on_ref;  // the profile ring times the context's stream
  if (prof_pyr) HIP_TRY(c->prof_pyr.begin(c->stream, &ps));
  const bool block = sst % 8 == 0 && c->win_stride % 8 == 0 && pyramid_block_ok(c->pg, src, sp, bank_win(c));
  HIP_TRY(launch_pyramid_window(bank_winjob(c), srcs, 1, n_frames, c->cam.width, c->cam.height, c->prm.levels,
                                block, ps_stream));
  if (prof_pyr) HIP_TRY(c->prof_pyr.end(c->stream, ps));
  if (on_ref) {  // the update's event now also covers the window's pyramids
    HIP_TRY(hipEventRecord(c->ev_ready, c->rstream));
    if ((e = consume_commit(c)) != DPT_OK) return e;
  }
  const int slot = c->slot_next;
  for (int f = 0; f < n_frames; ++f) {
    const int mode = f == 0 && init_mode == DPT_INIT_GIVEN ? kStartGiven : kStartConstVelocity;
    fill_start(c, mode, T_cw_init, c->eng.start((slot + f) % kRing));
  }
  if (l0_direct) {
    StartSlot* st = c->eng.start(slot);
    st->l0 = src;
    st->l0_stride = sst;
  }
  if (c->prof) HIP_TRY(c->prof_trk.begin(c->stream, &ps));
  HIP_TRY(c->eng.launch(c->spin_limit, slot, n_frames));
  if (c->prof) HIP_TRY(c->prof_trk.end(c->stream, ps));
  for (int f = 0; f < n_frames; ++f) c->pending.emplace_back((slot + f) % kRing, out + f);
  c->slot_next = (slot + n_frames) % kRing;
  if (!frames_on_device) HIP_TRY(hipStreamSynchronize(c->stream));  // the host frames are only borrowed
  return DPT_OK;
}

int dpt_cycle_profile(int64_t* out, int32_t n_slots, int32_t reset) {
  g_err.clear();
  if (!out) return fail(DPT_E_ARG, "NULL argument");
  if (n_slots < 1 || n_slots > kCycleSlots) return fail(DPT_E_ARG, "n_slots %d", n_slots);
  if (!kCycleProfile) return fail(DPT_E_STATE, "library built without DPT_CYCLE_PROFILE");
  HIP_TRY(read_cycle_profile(reinterpret_cast<uint64_t*>(out), n_slots, reset != 0));
  return DPT_OK;
}

int dpt_set_spin_limit(dpt_ctx* c, int32_t polls) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  if (polls < 0) return fail(DPT_E_ARG, "polls %d < 0", polls);
  c->spin_limit = polls;
  return DPT_OK;
}

int dpt_set_launch_config(dpt_ctx* c, int32_t mode, int32_t chunk) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  if (mode < DPT_LAUNCH_AUTO || mode > DPT_LAUNCH_COOP_PAIRS) return fail(DPT_E_ARG, "mode %d", mode);
  if (chunk != 64 && chunk != 128 && chunk != 256) return fail(DPT_E_ARG, "chunk %d not in {64, 128, 256}", chunk);
  if (mode == DPT_LAUNCH_COOP_PAIRS && chunk == 256)
    return fail(DPT_E_ARG, "chunk %d: two threads per point take 64 or 128 points per chunk", chunk);
  if (mode == DPT_LAUNCH_WORKGROUP && c->prm.precision == DPT_PREC_MIXED)
    return fail(DPT_E_ARG, "mixed precision runs on the cooperative launch only");
  if ((chunk != c->chunk || pair_track(c->prm, mode) != pair_track(c->prm, c->launch_mode)) && c->eng_ready) {
    const int e = synchronize(c);
    if (e != DPT_OK) return e;
    c->eng.release();
    c->eng_ready = false;
  }
  c->launch_mode = mode;
  c->chunk = chunk;
  return DPT_OK;
}

int dpt_get_reference_cache(dpt_ctx* c, int32_t level, uint8_t* valid, float* I0, float* gx, float* gy, float* x0) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  {
    const int e0 = consume_commit(c);  // ordered after a reference update in flight
    if (e0 != DPT_OK) return e0;
  }
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  const size_t n = (size_t)c->n_points, K = (size_t)c->prm.n_pattern, cap = (size_t)c->cap;
  const size_t lo = (size_t)level * cap;
  if (n) {
    if (valid) HIP_TRY(hipMemcpyAsync(valid, c->valid + lo, n, hipMemcpyDeviceToHost, c->stream));
    if (I0) HIP_TRY(hipMemcpyAsync(I0, c->I0 + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (gx) HIP_TRY(hipMemcpyAsync(gx, c->gx + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (gy) HIP_TRY(hipMemcpyAsync(gy, c->gy + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (x0) HIP_TRY(hipMemcpy2DAsync(x0, 12, c->x0, sizeof(float4), 12, n, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int dpt_normal_equations(dpt_ctx* c, int32_t level, const double T_rel[16], float* H21, float* b6, double* E,
                         int64_t* n, int32_t* npts) {
  g_err.clear();
  if (!c || !T_rel || !H21 || !b6 || !E || !n || !npts) return fail(DPT_E_ARG, "NULL argument");
  {
    const int e0 = consume_commit(c);  // ordered after a reference update in flight
    if (e0 != DPT_OK) return e0;
  }
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!finite16(T_rel)) return fail(DPT_E_ARG, "T_rel not finite");
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  if (!c->have_pyr[DPT_SLOT_CUR]) return fail(DPT_E_STATE, "no current pyramid");
  TrackArgs a;
  fill_track_args(c, a);
  for (int j = 0; j < 12; ++j) a.T_init[j] = (float)T_rel[j];
  a.level = level;
  HIP_TRY(launch_normal_equations(a, c->stream));
  HIP_TRY(hipMemcpyAsync(c->h_tot, c->d_tot, kRedSlots * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->prm.flags & DPT_FLAG_FIXED_H) {  // H is the level's precomputed one
    FixedH f;
    HIP_TRY(hipMemcpy(&f, c->d_fixed + level, sizeof f, hipMemcpyDeviceToHost));
    for (int j = 0; j < 21; ++j) H21[j] = (float)f.H[j];
  } else {
    for (int j = 0; j < 21; ++j) H21[j] = c->h_tot[j];
  }
  for (int j = 0; j < 6; ++j) b6[j] = c->h_tot[kSlotB + j];
  *E = c->h_tot[kSlotE];
  *n = (int64_t)c->h_tot[kSlotN];
  *npts = (int32_t)c->h_tot[kSlotPts];
  return DPT_OK;
}

int dpt_get_fixed_hessian(dpt_ctx* c, int32_t level, double* H36, int32_t* not_pd) {
  g_err.clear();
  if (!c || !H36 || !not_pd) return fail(DPT_E_ARG, "NULL argument");
  {
    const int e0 = consume_commit(c);  // ordered after a reference update in flight
    if (e0 != DPT_OK) return e0;
  }
  if (!(c->prm.flags & DPT_FLAG_FIXED_H)) return fail(DPT_E_STATE, "the context is not in the fixed-H mode");
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  HIP_TRY(hipStreamSynchronize(c->stream));  // the factor is written on the context's (or reference) stream
  FixedH f;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&f, c->d_fixed + level, sizeof f, hipMemcpyDeviceToHost));
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) H36[6 * i + j] = H36[6 * j + i] = f.H[i * 6 - (i * (i - 1)) / 2 + (j - i)];
  *not_pd = f.bad;
  return DPT_OK;
}

int dpt_set_profiling(dpt_ctx* c, int32_t enable) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  if (enable < 0) return fail(DPT_E_ARG, "enable %d < 0", enable);
  int e = synchronize(c);
  if (e != DPT_OK) return e;
  if (enable) {
    HIP_TRY(c->prof_pyr.create());
    HIP_TRY(c->prof_trk.create());
  }
  c->prof_pyr.reset(enable);
  c->prof_trk.reset(enable);
  c->prof = enable != 0;
  return DPT_OK;
}

int dpt_last_kernel_ms(dpt_ctx* c, float* pyramid_ms, float* track_ms) {
  g_err.clear();
  if (!c || !pyramid_ms || !track_ms) return fail(DPT_E_ARG, "NULL argument");
  const int e = synchronize(c);
  if (e != DPT_OK) return e;
  *pyramid_ms = c->prof_pyr.last_ms;
  *track_ms = c->prof_trk.last_ms;
  return DPT_OK;
}

int dpt_get_profile(dpt_ctx* c, double* pyramid_ms, int64_t* n_pyramid, double* track_ms, int64_t* n_track) {
  g_err.clear();
  if (!c || !pyramid_ms || !n_pyramid || !track_ms || !n_track) return fail(DPT_E_ARG, "NULL argument");
  const int e = synchronize(c);
  if (e != DPT_OK) return e;
  *pyramid_ms = c->prof_pyr.total_ms;
  *n_pyramid = c->prof_pyr.count;
  *track_ms = c->prof_trk.total_ms;
  *n_track = c->prof_trk.count;
  return DPT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched streams

struct dpt_batch {
  int32_t n = 0;
  hipStream_t stream = nullptr;
  std::vector<dpt_ctx*> ctx;
  // reference stream (dpt_batch_set_reference_stream): every stream's reference
  // banks switch together; the events order the batch's two streams
  hipStream_t rstream = nullptr;
  hipEvent_t ev_read[2] = {nullptr, nullptr};  // batch stream: past the last track that read bank b
  hipEvent_t ev_ready = nullptr;               // reference stream: the last update done
  int32_t bank = 0;
  bool update_open = false, commit_pending = false;
  int32_t launch_mode = DPT_LAUNCH_AUTO, chunk = 256;
  int32_t spin_limit = kSpinLimit;
  // cooperative groups of streams (each fits one co-resident launch)
  std::vector<CoopEngine*> groups;
  std::vector<std::vector<int>> group_streams;
  bool groups_dirty = true;
  // pyramid jobs
  PyrJob* d_jobs = nullptr;  // two tables of n jobs, used alternately
  PyrJob* h_jobs = nullptr;  // pinned, two tables
  hipEvent_t ev_jobs[2] = {nullptr, nullptr};  // each table's last upload
  int jobs_next = 0;
  // destinations and geometry (n <= kPyrArgJobs) per slot (the reference in
  // bank 0, current frames), then the reference in bank 1 (reference stream)
  PyrJob* d_static[3] = {nullptr, nullptr, nullptr};
  // one-workgroup-per-stream launch
  TrackArgs* d_args = nullptr;
  TrackArgs* h_args = nullptr;  // pinned
  TrackOut* d_outs = nullptr;
  TrackOut* h_outs = nullptr;  // pinned
  bool prof = false;
  ProfRing prof_pyr, prof_trk;
  std::vector<std::pair<int, dpt_result*>> pending;  // tracks in flight: (ring slot, caller's n results)
  int slot_next = 0;
  // batched reference updates and pose histories
  StagedTable<SelJob> sel_jobs;
  StagedTable<BackprojectArgs> bp_args;
  StagedTable<PrecomputeArgs> pre_args;
  StagedTable<double> hist_vals;  // 24 per stream
  double** d_hist_ptrs = nullptr;  // device array of the streams' history pointers
  WinJob* d_winjobs[2] = {nullptr, nullptr};  // the streams' window pyramid jobs per bank (device)
  bool winjobs_ok[2] = {false, false};         // each table matches the streams' current buffers
  double* d_prop = nullptr;        // learned start proposals, n x 3x4 FP64 (device)
  const uint8_t** d_cnn_lv = nullptr;  // the streams' coarsest reference then current levels, per bank
  bool cnn_lv_ok[2] = {false, false};
  bool have_prop = false;

  void clear_groups() {
    for (CoopEngine* g : groups) delete g;
    groups.clear();
    group_streams.clear();
    groups_dirty = true;
  }
  ~dpt_batch() {
    (void)hipStreamSynchronize(stream);
    if (rstream) (void)hipStreamSynchronize(rstream);
    for (hipEvent_t e : {ev_read[0], ev_read[1], ev_ready})
      if (e) (void)hipEventDestroy(e);
    clear_groups();
    for (dpt_ctx* c : ctx) delete c;
    prof_pyr.destroy();
    prof_trk.destroy();
    sel_jobs.release();
    bp_args.release();
    pre_args.release();
    hist_vals.release();
    if (d_hist_ptrs) (void)hipFree(d_hist_ptrs);
    for (WinJob* t : d_winjobs)
      if (t) (void)hipFree(t);
    if (d_prop) (void)hipFree(d_prop);
    if (d_cnn_lv) (void)hipFree(d_cnn_lv);
    for (hipEvent_t e : ev_jobs)
      if (e) (void)hipEventDestroy(e);
    if (d_jobs) (void)hipFree(d_jobs);
    for (PyrJob* p : d_static)
      if (p) (void)hipFree(p);
    if (d_args) (void)hipFree(d_args);
    if (d_outs) (void)hipFree(d_outs);
    if (h_jobs) (void)hipHostFree(h_jobs);
    if (h_args) (void)hipHostFree(h_args);
    if (h_outs) (void)hipHostFree(h_outs);
  }
};

namespace {

// The batch's counterparts of open_update / consume_commit: every stream's
// fields switch bank together at a reference pyramid build, the update closes
// (one event on the reference stream) when the last reference is set or at
// the next track, and the batch stream is ordered after it before tracking.
int batch_consume(dpt_batch* b) {
  if (!b->commit_pending) return DPT_OK;
  HIP_TRY(hipEventRecord(b->ev_read[b->bank ^ 1], b->stream));
  HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_ready, 0));
  b->commit_pending = false;
  return DPT_OK;
}

int batch_close_update(dpt_batch* b) {
  if (!b->update_open) return DPT_OK;
  HIP_TRY(hipEventRecord(b->ev_ready, b->rstream));
  b->update_open = false;
  b->commit_pending = true;
  for (dpt_ctx* c : b->ctx) c->update_open = false;
  return DPT_OK;
}

int batch_open_update(dpt_batch* b) {
  if (!b->rstream || b->update_open) return DPT_OK;
  int e = batch_consume(b);
  if (e != DPT_OK) return e;
  for (dpt_ctx* c : b->ctx) {
    const RefBank cur = fields_bank(c);
    set_fields(c, c->alt);
    c->alt = cur;
    c->bank ^= 1;
    c->update_open = true;
  }
  b->bank ^= 1;
  HIP_TRY(hipStreamWaitEvent(b->rstream, b->ev_read[b->bank], 0));
  b->update_open = true;
  return DPT_OK;
}

hipStream_t batch_ref_stream(const dpt_batch* b) { return b->rstream ? b->rstream : b->stream; }

// The streams' window pyramid jobs into the buffers of `bank`, rebuilt after
// the buffers changed (nothing in flight reads the table then).
int batch_winjobs(dpt_batch* b, int bank, WinJob** out) {
  if (!b->winjobs_ok[bank]) {
    if (!b->d_winjobs[bank] && hipMalloc(&b->d_winjobs[bank], sizeof(WinJob) * b->n) != hipSuccess) {
      (void)hipGetLastError();
      b->d_winjobs[bank] = nullptr;
      return fail(DPT_E_OOM, "window job table allocation failed");
    }
    for (int s = 0; s < b->n; ++s) {
      const WinJob* j = bank ? b->ctx[s]->d_winjob_b1 : b->ctx[s]->d_winjob;
      if (!j) return fail(DPT_E_STATE, "stream %d has no window buffer for bank %d", s, bank);
      HIP_TRY(hipMemcpy(b->d_winjobs[bank] + s, j, sizeof(WinJob), hipMemcpyDeviceToDevice));
    }
    b->winjobs_ok[bank] = true;
  }
  *out = b->d_winjobs[bank];
  return DPT_OK;
}

int batch_chunks(const dpt_batch* b, int s) {
  const dpt_ctx* c = b->ctx[s];
  const int n = std::max(c->n_points, std::max(c->bank_n[0], c->bank_n[1]));  // the chunks cover both banks
  const int ppc = coop_ppc(b->ctx[0]->prm, b->chunk);
  return n > 0 ? (n + ppc - 1) / ppc : 1;
}

// Grid of the XCD-packed work list (CoopEngine::upload) of streams with these
// chunk counts, given largest first: each stream goes to the least-loaded of
// the eight XCDs, block j of XCD x is grid slot 8 j + x, trailing padding cut.
int packed_grid(const std::vector<int>& chunks_desc) {
  int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int c : chunks_desc) *std::min_element(load, load + 8) += c;
  const int depth = *std::max_element(load, load + 8);
  if (depth == 0) return 0;
  int last = 0;
  for (int x = 0; x < 8; ++x)
    if (load[x] == depth) last = x;
  return 8 * (depth - 1) + last + 1;
}

// Partition streams into groups that each fit one cooperative launch: streams
// largest first, a group closed when its packed grid would exceed the
// co-resident capacity.
int build_groups(dpt_batch* b) {
  b->clear_groups();
  const int cap = coop_max_blocks(coop_threads(b->ctx[0]->prm, b->chunk, b->launch_mode));
  std::vector<int> order(b->n);
  for (int s = 0; s < b->n; ++s) order[s] = s;
  std::sort(order.begin(), order.end(), [&](int p, int q) { return batch_chunks(b, p) > batch_chunks(b, q); });
  std::vector<int> cur, cur_chunks;
  auto flush = [&]() -> int {
    if (cur.empty()) return DPT_OK;
    std::sort(cur.begin(), cur.end());
    CoopEngine* g = new (std::nothrow) CoopEngine();
    if (!g) return fail(DPT_E_OOM, "host allocation failed");
    std::vector<int> maxp(cur.size());
    for (size_t k = 0; k < cur.size(); ++k) maxp[k] = b->ctx[cur[k]]->cap;
    hipError_t e = g->init((int)cur.size(), maxp.data(), coop_threads(b->ctx[0]->prm, b->chunk, b->launch_mode),
                           coop_ppc(b->ctx[0]->prm, b->chunk), true, b->stream);
    if (e != hipSuccess) {
      delete g;
      return fail(DPT_E_HIP, "cooperative group init: %s", hipGetErrorString(e));
    }
    g->variant = coop_variant(b->ctx[0]->prm, b->launch_mode);
    for (size_t k = 0; k < cur.size(); ++k) {
      TrackArgs a;
      fill_track_args(b->ctx[cur[k]], a);
      a.ref = refcache_of(b->ctx[cur[k]], 0);
      g->set_stream((int)k, a, refcache_of(b->ctx[cur[k]], 1), b->ctx[cur[k]]->d_hist, b->ctx[cur[k]]->win,
                    b->ctx[cur[k]]->win_b1,
                    b->ctx[cur[k]]->win_stride);
    }
    b->groups.push_back(g);
    b->group_streams.push_back(cur);
    cur.clear();
    cur_chunks.clear();
    return DPT_OK;
  };
  for (int s : order) {
    const int c = batch_chunks(b, s);
    if (packed_grid({c}) > cap)
      return fail(DPT_E_ARG, "stream %d: %d chunks exceed the co-resident capacity %d", s, c, cap);
    cur_chunks.push_back(c);
    if (cur.size() > 0 && packed_grid(cur_chunks) > cap) {
      cur_chunks.pop_back();
      int e = flush();
      if (e != DPT_OK) return e;
      cur_chunks.push_back(c);
    }
    cur.push_back(s);
  }
  int e = flush();
  if (e != DPT_OK) return e;
  b->groups_dirty = false;
  return DPT_OK;
}

bool batch_use_coop(const dpt_batch* b) {
  if (b->ctx[0]->prm.precision == DPT_PREC_MIXED) return true;
  return b->launch_mode != DPT_LAUNCH_WORKGROUP &&
         coop_max_blocks(coop_threads(b->ctx[0]->prm, b->chunk, b->launch_mode)) > 0;
}

// abandon() for a batch: every group's results of every launch in flight.
void batch_abandon(dpt_batch* b) {
  (void)hipStreamSynchronize(b->stream);
  (void)hipGetLastError();
  for (const auto& p : b->pending) {
    if (p.first < 0 || !p.second) continue;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const std::vector<int>& ss = b->group_streams[gi];
      const bool fin = b->groups[gi]->done(p.first);
      const TrackOut* o = b->groups[gi]->out(p.first);
      const StartSlot* st = b->groups[gi]->start(p.first);
      for (size_t k = 0; k < ss.size(); ++k) {
        dpt_result* r = &p.second[ss[k]];
        if (fin) {
          fill_result(b->ctx[ss[k]], o[k], st[k].T_rw, r);
        } else {
          std::memset(r, 0, sizeof *r);
          r->status = kStatusTimeout;
        }
      }
    }
  }
  b->pending.clear();
}

// Wait for the stream and fill the results of every batched track in flight.
int batch_synchronize(dpt_batch* b) {
  const hipError_t es = hipStreamSynchronize(b->stream);
  if (es != hipSuccess) {
    const int r = fail(DPT_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
    batch_abandon(b);
    return r;
  }
  bool timeout = false;
  for (const auto& p : b->pending) {
    if (p.first < 0) continue;  // ran synchronously, results already filled
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const std::vector<int>& ss = b->group_streams[gi];
      const TrackOut* o = b->groups[gi]->out(p.first);
      const StartSlot* st = b->groups[gi]->start(p.first);
      for (size_t k = 0; k < ss.size(); ++k) {
        timeout |= o[k].status == kStatusTimeout;
        if (p.second) fill_result(b->ctx[ss[k]], o[k], st[k].T_rw, &p.second[ss[k]]);
      }
    }
  }
  b->pending.clear();
  if (b->prof) {
    HIP_TRY(b->prof_pyr.drain());
    HIP_TRY(b->prof_trk.drain());
  }
  if (timeout) {
    for (CoopEngine* g : b->groups) (void)g->clear_partials();
    (void)hipStreamSynchronize(b->stream);
    return fail(DPT_E_HIP, "cooperative batch track: chunk synchronisation timed out");
  }
  return DPT_OK;
}

// A reference committed to a bank since the launch descriptors were written:
// refresh them in place, or regroup when a stream now needs more chunks.
void refresh_groups(dpt_batch* b) {
  for (size_t gi = 0; gi < b->groups.size() && !b->groups_dirty; ++gi) {
    CoopEngine* g = b->groups[gi];
    const std::vector<int>& ss = b->group_streams[gi];
    for (size_t k = 0; k < ss.size(); ++k) {
      const dpt_ctx* c = b->ctx[ss[k]];
      const RefCache r0 = refcache_of(c, 0), r1 = refcache_of(c, 1);
      const CoopStream& hs = g->h_streams[k];
      if (hs.a.ref.n == r0.n && hs.ref_alt.n == r1.n && hs.ref_alt.x0 == r1.x0 && hs.win == c->win &&
          hs.win_alt == c->win_b1)
        continue;
      if (batch_chunks(b, ss[k]) > hs.n_chunks) {
        b->groups_dirty = true;
        break;
      }
      TrackArgs a;
      fill_track_args(c, a);
      a.ref = r0;
      g->set_stream((int)k, a, r1, c->d_hist, c->win, c->win_b1, c->win_stride);
    }
  }
}

// Enqueue one cooperative track of every stream.  modes[s] is kStartGiven
// (start from T_cw_init[s]), kStartConstVelocity or kStartDevice (the proposal
// in d_prop).
int batch_enqueue_coop(dpt_batch* b, const int* modes, const double* T_cw_init, dpt_result* out) {
  refresh_groups(b);
  if (b->groups_dirty) {  // regrouping frees the rings: finish and fill what is in flight first
    int e = b->pending.empty() ? DPT_OK : batch_synchronize(b);
    if (e != DPT_OK) return e;
    if ((e = build_groups(b)) != DPT_OK) return e;
  }
  if ((int)b->pending.size() >= kRing) return fail(DPT_E_STATE, "%d batched tracks in flight: synchronise first", kRing);
  for (CoopEngine* g : b->groups)
    if (g->dirty) HIP_TRY(g->upload());
  const int slot = b->slot_next;
  b->slot_next = (slot + 1) % kRing;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const std::vector<int>& ss = b->group_streams[gi];
    StartSlot* st = b->groups[gi]->start(slot);
    for (size_t k = 0; k < ss.size(); ++k)
      fill_start(b->ctx[ss[k]], modes[ss[k]], T_cw_init ? T_cw_init + 16 * ss[k] : nullptr, &st[k],
                 b->d_prop ? b->d_prop + 12 * ss[k] : nullptr);
  }
  int ps = -1;
  if (b->prof) HIP_TRY(b->prof_trk.begin(b->stream, &ps));
  for (CoopEngine* g : b->groups) HIP_TRY(g->launch(b->spin_limit, slot));
  if (b->prof) HIP_TRY(b->prof_trk.end(b->stream, ps));
  b->pending.emplace_back(slot, out);
  return DPT_OK;
}

// As collect(), for the oldest n batched track launches (each of all streams).
int batch_collect(dpt_batch* b, int n) {
  if (n < 0 || n > (int)b->pending.size())
    return fail(DPT_E_ARG, "%d results asked, %d batched tracks in flight", n, (int)b->pending.size());
  bool timeout = false;
  for (int i = 0; i < n; ++i) {
    const int slot = b->pending[i].first;
    if (slot < 0) continue;
    for (CoopEngine* g : b->groups) {
      const int e = wait_results(b->stream, [&] { return g->done(slot); });
      if (e != DPT_OK) {
        batch_abandon(b);
        return e;
      }
      const TrackOut* o = g->out(slot);
      for (int k = 0; k < g->n; ++k) timeout |= o[k].status == kStatusTimeout;
    }
  }
  if (timeout) return batch_synchronize(b);
  for (int i = 0; i < n; ++i) {
    const auto& p = b->pending[i];
    if (p.first < 0) continue;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const std::vector<int>& ss = b->group_streams[gi];
      const TrackOut* o = b->groups[gi]->out(p.first);
      const StartSlot* st = b->groups[gi]->start(p.first);
      for (size_t k = 0; k < ss.size(); ++k)
        if (p.second) fill_result(b->ctx[ss[k]], o[k], st[k].T_rw, &p.second[ss[k]]);
    }
  }
  b->pending.erase(b->pending.begin(), b->pending.begin() + n);
  return DPT_OK;
}

int batch_check_state(dpt_batch* b) {
  for (int s = 0; s < b->n; ++s) {
    if (!b->ctx[s]->have_ref) return fail(DPT_E_STATE, "stream %d has no reference points", s);
    if (!b->ctx[s]->have_pyr[DPT_SLOT_CUR]) return fail(DPT_E_STATE, "stream %d has no current pyramid", s);
  }
  int e = batch_close_update(b);
  return e != DPT_OK ? e : batch_consume(b);
}

// One workgroup per stream, synchronous.
int batch_track_workgroup(dpt_batch* b, const double* T_cw_init, dpt_result* out) {
  int lds = 0, max_points = 0;
  for (int s = 0; s < b->n; ++s) {
    dpt_ctx* c = b->ctx[s];
    TrackArgs& a = b->h_args[s];
    fill_track_args(c, a);
    rel_pose_f32(c, T_cw_init + 16 * s, a.T_init);
    a.out = b->d_outs + s;
    lds = std::max(lds, track_lds_bytes(c->lv, c->prm.levels, c->pyrf[0] ? 4 : 1));
    max_points = std::max(max_points, c->n_points);
  }
  HIP_TRY(hipMemcpyAsync(b->d_args, b->h_args, sizeof(TrackArgs) * b->n, hipMemcpyHostToDevice, b->stream));
  int ps = -1;
  if (b->prof) HIP_TRY(b->prof_trk.begin(b->stream, &ps));
  HIP_TRY(launch_track_batch(b->h_args[0], b->d_args, b->n, lds, max_points, b->stream));
  if (b->prof) HIP_TRY(b->prof_trk.end(b->stream, ps));
  HIP_TRY(hipMemcpyAsync(b->h_outs, b->d_outs, sizeof(TrackOut) * b->n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (b->prof) {
    HIP_TRY(b->prof_pyr.drain());
    HIP_TRY(b->prof_trk.drain());
  }
  for (int s = 0; s < b->n; ++s) fill_result(b->ctx[s], b->h_outs[s], b->ctx[s]->T_rw, &out[s]);
  return DPT_OK;
}

}  // namespace

extern "C" {

int dpt_batch_create(int32_t n_streams, const dpt_camera* cams, const dpt_params* prm, const int32_t* max_points,
                     void* hip_stream, dpt_batch** out) {
  g_err.clear();
  if (!out || !cams || !prm || !max_points) return fail(DPT_E_ARG, "NULL argument");
  *out = nullptr;
  if (n_streams < 1 || n_streams > 4096) return fail(DPT_E_ARG, "n_streams %d outside [1, 4096]", n_streams);
  dpt_batch* b = new (std::nothrow) dpt_batch();
  if (!b) return fail(DPT_E_OOM, "host allocation failed");
  b->n = n_streams;
  b->stream = (hipStream_t)hip_stream;
  for (int s = 0; s < n_streams; ++s) {
    dpt_ctx* c = nullptr;
    int e = dpt_create(&cams[s], prm, max_points[s], hip_stream, &c);
    if (e != DPT_OK) {
      delete b;
      return e;
    }
    b->ctx.push_back(c);
  }
  if (hipMalloc(&b->d_jobs, 2 * sizeof(PyrJob) * n_streams) != hipSuccess ||
      hipMalloc(&b->d_args, sizeof(TrackArgs) * n_streams) != hipSuccess ||
      hipMalloc(&b->d_outs, sizeof(TrackOut) * n_streams) != hipSuccess ||
      hipHostMalloc(&b->h_jobs, 2 * sizeof(PyrJob) * n_streams) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_jobs[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_jobs[1], hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(&b->h_args, sizeof(TrackArgs) * n_streams) != hipSuccess ||
      hipHostMalloc(&b->h_outs, sizeof(TrackOut) * n_streams) != hipSuccess ||
      b->sel_jobs.init(n_streams) != hipSuccess || b->bp_args.init(n_streams) != hipSuccess ||
      b->pre_args.init(n_streams) != hipSuccess || b->hist_vals.init(24 * n_streams) != hipSuccess ||
      hipMalloc(&b->d_hist_ptrs, sizeof(double*) * n_streams) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return fail(DPT_E_OOM, "batch allocation failed");
  }
  if (n_streams <= kPyrArgJobs) {  // the static pyramid tables: sources go in the kernel arguments
    std::vector<PyrJob> t(n_streams);
    for (int slot = 0; slot < 2; ++slot) {
      for (int s = 0; s < n_streams; ++s) {
        std::memset(&t[s], 0, sizeof t[s]);
        t[s].dst = b->ctx[s]->pyr[slot];
        t[s].g = b->ctx[s]->pg;
      }
      if (hipMalloc(&b->d_static[slot], sizeof(PyrJob) * n_streams) != hipSuccess ||
          hipMemcpy(b->d_static[slot], t.data(), sizeof(PyrJob) * n_streams, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(DPT_E_OOM, "batch allocation failed");
      }
    }
  }
  {
    std::vector<double*> hp(n_streams);
    for (int s = 0; s < n_streams; ++s) hp[s] = b->ctx[s]->d_hist;
    if (hipMemcpy(b->d_hist_ptrs, hp.data(), sizeof(double*) * n_streams, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      delete b;
      return fail(DPT_E_HIP, "batch history table upload failed");
    }
  }
  *out = b;
  return DPT_OK;
}

void dpt_batch_destroy(dpt_batch* b) { delete b; }

int dpt_batch_set_reference_stream(dpt_batch* b, void* hip_stream) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  if (b->update_open) return fail(DPT_E_STATE, "a reference update is open: finish it first");
  hipStream_t rs = static_cast<hipStream_t>(hip_stream);
  if (rs == b->stream) rs = nullptr;
  int e;
  if (!b->pending.empty() && (e = batch_synchronize(b)) != DPT_OK) return e;
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (b->rstream) HIP_TRY(hipStreamSynchronize(b->rstream));
  b->commit_pending = false;
  if (rs) {
    for (hipEvent_t* ev : {&b->ev_read[0], &b->ev_read[1], &b->ev_ready})
      if (!*ev) HIP_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    for (dpt_ctx* c : b->ctx) {
      if (c->bank != b->bank) return fail(DPT_E_STATE, "stream banks out of step");
      const bool fresh = !c->phys[1].x0;
      if ((e = alloc_alt_bank(c)) != DPT_OK) return e;
      if (fresh) c->alt = c->phys[1], c->bank_n[1] = 0;
    }
    b->winjobs_ok[1] = false;  // the streams' bank-1 window buffers may be new
    if (b->d_static[DPT_SLOT_REF] && !b->d_static[2]) {  // the second bank's reference pyramid table
      std::vector<PyrJob> t(b->n);
      for (int s = 0; s < b->n; ++s) {
        std::memset(&t[s], 0, sizeof t[s]);
        t[s].dst = b->ctx[s]->phys[1].pyr_ref;
        t[s].g = b->ctx[s]->pg;
      }
      if ((e = dev_alloc((void**)&b->d_static[2], sizeof(PyrJob) * b->n)) != DPT_OK) return e;
      HIP_TRY(hipMemcpy(b->d_static[2], t.data(), sizeof(PyrJob) * b->n, hipMemcpyHostToDevice));
    }
    b->groups_dirty = true;  // the launch descriptors gain the second banks
  }
  for (dpt_ctx* c : b->ctx) c->rstream = rs, c->batch_owned = true, c->commit_pending = false;
  b->rstream = rs;
  return DPT_OK;
}

int dpt_batch_build_pyramids(dpt_batch* b, int32_t slot, const uint8_t* const* imgs, const int64_t* pitches,
                             int32_t on_device) {
  g_err.clear();
  if (on_device != 0 && on_device != 1) return fail(DPT_E_ARG, "on_device %d is neither 0 nor 1", on_device);
  if (!b || !imgs || !pitches) return fail(DPT_E_ARG, "NULL argument");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (slot == DPT_SLOT_REF) {
    const int e0 = batch_open_update(b);
    if (e0 != DPT_OK) return e0;
  }
  // reference pyramids belong to the reference stream (the batch's own without one)
  const hipStream_t st = slot == DPT_SLOT_REF ? batch_ref_stream(b) : b->stream;
  const bool prof = b->prof && st == b->stream;
  // the static table of the bank the fields now hold (the reference's switches with it)
  const PyrJob* d_static = slot == DPT_SLOT_REF && b->bank == 1 ? b->d_static[2] : b->d_static[slot];
  if (d_static && !b->ctx[0]->pyrf[slot]) {  // sources by value: no table upload
    PyrSrcArgs srcs;
    std::memset(&srcs, 0, sizeof srcs);
    int max_w = 0, max_h = 0;
    for (int s = 0; s < b->n; ++s) {
      dpt_ctx* c = b->ctx[s];
      if (!imgs[s]) return fail(DPT_E_ARG, "image %d is NULL", s);
      if (pitches[s] < c->cam.width) return fail(DPT_E_ARG, "stream %d: pitch < width", s);
      srcs.src[s] = imgs[s];
      srcs.pitch[s] = pitches[s];
      if (!on_device) {
        HIP_TRY(hipMemcpy2DAsync(c->staging, c->cam.width, imgs[s], pitches[s], c->cam.width, c->cam.height,
                                 hipMemcpyHostToDevice, st));
        srcs.src[s] = c->staging;
        srcs.pitch[s] = c->cam.width;
      }
      max_w = std::max(max_w, c->cam.width);
      max_h = std::max(max_h, c->cam.height);
    }
    bool block = true;
    for (int s = 0; s < b->n; ++s)
      block = block && pyramid_block_ok(b->ctx[s]->pg, srcs.src[s], srcs.pitch[s], b->ctx[s]->pyr[slot]);
    int ps = -1;
    if (prof) HIP_TRY(b->prof_pyr.begin(b->stream, &ps));
    HIP_TRY(launch_pyramid_batch_args(d_static, srcs, b->n, max_w, max_h, b->ctx[0]->prm.levels, block,
                                      st));
    if (prof) HIP_TRY(b->prof_pyr.end(b->stream, ps));
    if (!on_device) HIP_TRY(hipStreamSynchronize(st));  // the host images are only borrowed
    for (int s = 0; s < b->n; ++s) {
      b->ctx[s]->have_pyr[slot] = true;
      if (slot == DPT_SLOT_REF) b->ctx[s]->have_ref = false;
    }
    return DPT_OK;
  }
  // alternate job tables: the one written now was uploaded two calls ago
  const int jt = b->jobs_next;
  b->jobs_next ^= 1;
  HIP_TRY(hipEventSynchronize(b->ev_jobs[jt]));
  PyrJob* h_jobs = b->h_jobs + (size_t)jt * b->n;
  PyrJob* d_jobs = b->d_jobs + (size_t)jt * b->n;
  int max_w = 0, max_h = 0;
  for (int s = 0; s < b->n; ++s) {
    dpt_ctx* c = b->ctx[s];
    if (!imgs[s]) return fail(DPT_E_ARG, "image %d is NULL", s);
    if (pitches[s] < c->cam.width) return fail(DPT_E_ARG, "stream %d: pitch < width", s);
    const uint8_t* src = imgs[s];
    int64_t sp = pitches[s];
    if (!on_device) {
      HIP_TRY(hipMemcpy2DAsync(c->staging, c->cam.width, imgs[s], pitches[s], c->cam.width, c->cam.height,
                               hipMemcpyHostToDevice, st));
      src = c->staging;
      sp = c->cam.width;
    }
    PyrJob& j = h_jobs[s];
    j.src = src;
    j.pitch = sp;
    j.dst = c->pyr[slot];
    j.g = c->pg;
    j.vec4 = ((sp % 4) == 0 && (reinterpret_cast<uintptr_t>(src) % 4) == 0 && (c->pg.W[0] % 4) == 0) ? 1 : 0;
    j.vec16 = ((sp % 16) == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 && (c->pg.W[0] % 16) == 0 &&
               (reinterpret_cast<uintptr_t>(c->pyr[slot]) % 16) == 0)
                  ? 1
                  : 0;
    max_w = std::max(max_w, c->cam.width);
    max_h = std::max(max_h, c->cam.height);
  }
  HIP_TRY(hipMemcpyAsync(d_jobs, h_jobs, sizeof(PyrJob) * b->n, hipMemcpyHostToDevice, st));
  int ps = -1;
  if (prof) HIP_TRY(b->prof_pyr.begin(b->stream, &ps));
  HIP_TRY(launch_pyramid_batch(d_jobs, b->n, max_w, max_h, b->ctx[0]->prm.levels, st));
  for (int s = 0; s < b->n; ++s)
    if (b->ctx[s]->pyrf[slot])
      HIP_TRY(launch_pyramid_gauss(h_jobs[s].src, h_jobs[s].pitch, b->ctx[s]->pyrf[slot], b->ctx[s]->pg, st));
  // after the launches that read the table: the tables alternate between the two streams' builds
  HIP_TRY(hipEventRecord(b->ev_jobs[jt], st));
  if (prof) HIP_TRY(b->prof_pyr.end(b->stream, ps));
  if (!on_device) HIP_TRY(hipStreamSynchronize(st));  // the host images are only borrowed
  for (int s = 0; s < b->n; ++s) {
    b->ctx[s]->have_pyr[slot] = true;
    if (slot == DPT_SLOT_REF) b->ctx[s]->have_ref = false;
  }
  return DPT_OK;
}

int dpt_batch_select_points(dpt_batch* b, int32_t s, int32_t n, int32_t margin, int32_t* host_idx, int32_t* n_out) {
  g_err.clear();
  if (!b || s < 0 || s >= b->n) return fail(DPT_E_ARG, "stream index");
  return dpt_select_points(b->ctx[s], n, margin, host_idx, n_out);
}

int dpt_batch_set_reference_points(dpt_batch* b, int32_t s, const float* xyz, int32_t n, const double T_rw[16],
                                   int32_t on_device) {
  g_err.clear();
  if (!b || s < 0 || s >= b->n) return fail(DPT_E_ARG, "stream index");
  const int before = b->ctx[s]->n_points;
  int e = dpt_set_reference_points(b->ctx[s], xyz, n, T_rw, on_device);
  if (e == DPT_OK && before != n) b->groups_dirty = true;
  return e;
}

int dpt_batch_set_reference_from_depth(dpt_batch* b, int32_t s, int32_t n, int32_t margin, const float* depth,
                                       int64_t depth_pitch, int32_t depth_on_device, const double T_rw[16]) {
  g_err.clear();
  if (!b || s < 0 || s >= b->n) return fail(DPT_E_ARG, "stream %d", s);
  const int before = b->ctx[s]->n_points;
  int e = dpt_set_reference_from_depth(b->ctx[s], n, margin, depth, depth_pitch, depth_on_device, T_rw);
  if (e == DPT_OK && before != n) b->groups_dirty = true;
  return e;
}

int dpt_batch_set_reference_from_depth_all(dpt_batch* b, const int32_t* n_points, int32_t margin,
                                           const float* const* depths, const int64_t* depth_pitches,
                                           const double* T_rw) {
  g_err.clear();
  if (!b || !n_points || !depths || !depth_pitches || !T_rw) return fail(DPT_E_ARG, "NULL argument");
  for (int s = 0; s < b->n; ++s) {
    const dpt_ctx* c = b->ctx[s];
    if (n_points[s] < 1 || n_points[s] > c->cap) return fail(DPT_E_ARG, "stream %d: n %d outside [1, %d]", s, n_points[s], c->cap);
    if (margin < 1 || 2 * margin >= c->cam.width || 2 * margin >= c->cam.height) return fail(DPT_E_ARG, "margin %d", margin);
    if (!depths[s]) return fail(DPT_E_ARG, "depth %d is NULL", s);
    if (depth_pitches[s] < c->cam.width) return fail(DPT_E_ARG, "stream %d: depth pitch < width", s);
    if (!finite16(T_rw + 16 * s)) return fail(DPT_E_ARG, "T_rw %d not finite", s);
    if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "stream %d has no reference pyramid", s);
    if (b->rstream && !c->update_open)
      return fail(DPT_E_STATE, "with a reference stream, a reference update starts with dpt_batch_build_pyramids(DPT_SLOT_REF)");
  }
  const hipStream_t rs = batch_ref_stream(b);
  SelJob* hs;
  BackprojectArgs* hb;
  PrecomputeArgs* hp;
  int ws, wb, wp;
  HIP_TRY(b->sel_jobs.acquire(&hs, &ws));
  HIP_TRY(b->bp_args.acquire(&hb, &wb));
  HIP_TRY(b->pre_args.acquire(&hp, &wp));
  int G_max = 0, max_n = 0, max_samples = 0, max_levels = 0;
  bool any_empty = false;
  for (int s = 0; s < b->n; ++s) {
    dpt_ctx* c = b->ctx[s];
    const int n = n_points[s];
    hs[s] = make_sel_job(c->pyr[DPT_SLOT_REF], c->cam.width, c->cam.height, margin, n, c->sel_idx, c->sel_count,
                         c->sel_scratch);
    BackprojectArgs& bp = hb[s];
    bp.idx = c->sel_idx;
    bp.count = c->sel_count;
    bp.depth = depths[s];
    bp.pitch = depth_pitches[s];
    bp.W = c->cam.width;
    bp.n = n;
    bp.fx = c->cam.fx, bp.fy = c->cam.fy, bp.cx = c->cam.cx, bp.cy = c->cam.cy;
    for (int j = 0; j < 12; ++j) bp.T_rw[j] = T_rw[16 * s + j];
    bp.P = c->pts;
    hp[s] = precompute_args(c, c->pts, n, T_rw + 16 * s);
    G_max = std::max(G_max, hs[s].G);
    any_empty |= hs[s].G == 0;
    max_n = std::max(max_n, n);
    max_samples = std::max(max_samples, n * c->prm.n_pattern);
    max_levels = std::max(max_levels, c->prm.levels);
  }
  const SelJob* ds;
  const BackprojectArgs* db;
  const PrecomputeArgs* dp;
  HIP_TRY(b->sel_jobs.upload(ws, b->n, rs, &ds));
  HIP_TRY(b->bp_args.upload(wb, b->n, rs, &db));
  HIP_TRY(b->pre_args.upload(wp, b->n, rs, &dp));
  HIP_TRY(launch_select_batch(ds, b->n, G_max, any_empty, rs));
  HIP_TRY(launch_backproject_batch(db, b->n, max_n, rs));
  HIP_TRY(launch_precompute_batch(dp, b->n, max_samples, max_levels, rs));
  if (b->ctx[0]->prm.flags & DPT_FLAG_FIXED_H) HIP_TRY(launch_fixed_h_batch(dp, b->n, max_n, max_levels, rs));
  for (int s = 0; s < b->n; ++s) {
    if (b->ctx[s]->n_points != n_points[s]) b->groups_dirty = true;
    const int e = commit_reference(b->ctx[s], n_points[s], T_rw + 16 * s);
    if (e != DPT_OK) return e;
  }
  return batch_close_update(b);
}

int dpt_batch_set_pose_history_all(dpt_batch* b, const double* T_older, const double* T_newer) {
  g_err.clear();
  if (!b || !T_older || !T_newer) return fail(DPT_E_ARG, "NULL argument");
  for (int s = 0; s < b->n; ++s)
    if (!finite16(T_older + 16 * s) || !finite16(T_newer + 16 * s)) return fail(DPT_E_ARG, "pose %d not finite", s);
  double* h;
  int w;
  HIP_TRY(b->hist_vals.acquire(&h, &w));
  for (int s = 0; s < b->n; ++s)
    for (int j = 0; j < 12; ++j) {
      h[24 * s + j] = T_older[16 * s + j];
      h[24 * s + 12 + j] = T_newer[16 * s + j];
    }
  const double* d;
  HIP_TRY(b->hist_vals.upload(w, 24 * b->n, b->stream, &d));
  HIP_TRY(launch_set_history_batch(b->d_hist_ptrs, d, b->n, b->stream));
  return DPT_OK;
}

int dpt_batch_track(dpt_batch* b, const double* T_cw_init, dpt_result* out) {
  g_err.clear();
  if (!b || !T_cw_init || !out) return fail(DPT_E_ARG, "NULL argument");
  for (int s = 0; s < b->n; ++s)
    if (!finite16(T_cw_init + 16 * s)) return fail(DPT_E_ARG, "T_cw_init %d not finite", s);
  int e = batch_check_state(b);
  if (e != DPT_OK) return e;
  if (batch_use_coop(b)) {
    std::vector<int> modes(b->n, kStartGiven);
    if ((e = batch_enqueue_coop(b, modes.data(), T_cw_init, out)) != DPT_OK) return e;
    return batch_synchronize(b);
  }
  if (!b->pending.empty() && (e = batch_synchronize(b)) != DPT_OK) return e;
  return batch_track_workgroup(b, T_cw_init, out);
}

int dpt_batch_track_enqueue(dpt_batch* b, int32_t init_mode, const double* T_cw_init, dpt_result* out) {
  g_err.clear();
  if (!b || !out) return fail(DPT_E_ARG, "NULL argument");
  if (init_mode != DPT_INIT_GIVEN && init_mode != DPT_INIT_CONST_VELOCITY && init_mode != DPT_INIT_PROPOSED)
    return fail(DPT_E_ARG, "init_mode %d", init_mode);
  if (init_mode == DPT_INIT_GIVEN) {
    if (!T_cw_init) return fail(DPT_E_ARG, "T_cw_init is NULL");
    for (int s = 0; s < b->n; ++s)
      if (!finite16(T_cw_init + 16 * s)) return fail(DPT_E_ARG, "T_cw_init %d not finite", s);
  }
  if (init_mode == DPT_INIT_PROPOSED && !b->have_prop)
    return fail(DPT_E_STATE, "no learned proposal: call dpt_cnn_propose_batch first");
  int e = batch_check_state(b);
  if (e != DPT_OK) return e;
  if (!batch_use_coop(b)) {
    if (init_mode != DPT_INIT_GIVEN)
      return fail(DPT_E_ARG, "a constant-velocity or proposed start needs the cooperative track (launch mode AUTO or COOP)");
    const int e2 = dpt_batch_track(b, T_cw_init, out);
    if (e2 == DPT_OK) b->pending.emplace_back(-1, nullptr);  // in order with the tracks in flight, already done
    return e2;
  }
  std::vector<int> modes(b->n, init_mode == DPT_INIT_GIVEN ? kStartGiven
                               : init_mode == DPT_INIT_PROPOSED ? kStartDevice
                                                                : kStartConstVelocity);
  return batch_enqueue_coop(b, modes.data(), T_cw_init, out);
}

int dpt_batch_synchronize(dpt_batch* b) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  return batch_synchronize(b);
}

int dpt_batch_collect(dpt_batch* b, int32_t n) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  return batch_collect(b, n);
}

int dpt_batch_tracks_in_flight(dpt_batch* b) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  return (int)b->pending.size();
}

int dpt_batch_track_window_enqueue(dpt_batch* b, const uint8_t* const* frames, const int64_t* pitches,
                                   const int64_t* frame_strides, int32_t n_frames, int32_t frames_on_device,
                                   int32_t init_mode, const double* T_cw_init, dpt_result* out) {
  g_err.clear();
  if (!b || !frames || !pitches || !frame_strides || !out) return fail(DPT_E_ARG, "NULL argument");
  int e;
  for (int s = 0; s < b->n; ++s)
    if ((e = check_window_args(b->ctx[s], frames[s], pitches[s], frame_strides[s], n_frames, frames_on_device,
                               init_mode)) != DPT_OK)
      return e;
  if (init_mode == DPT_INIT_GIVEN) {
    if (!T_cw_init) return fail(DPT_E_ARG, "T_cw_init is NULL");
    for (int s = 0; s < b->n; ++s)
      if (!finite16(T_cw_init + 16 * s)) return fail(DPT_E_ARG, "T_cw_init %d not finite", s);
  }
  if (!batch_use_coop(b)) return fail(DPT_E_ARG, "window tracking needs the cooperative track (launch mode AUTO or COOP)");
  if ((e = batch_close_update(b)) != DPT_OK) return e;
  if ((int)b->pending.size() + n_frames > kRing)
    return fail(DPT_E_STATE, "%d batched tracks in flight and %d more exceed %d: synchronise first",
                (int)b->pending.size(), n_frames, kRing);
  bool need = false;
  for (int s = 0; s < b->n; ++s) need |= n_frames > b->ctx[s]->win_cap;
  if (need) {  // new buffers: finish what is in flight, then regroup with them
    if ((e = batch_synchronize(b)) != DPT_OK) return e;
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->rstream) HIP_TRY(hipStreamSynchronize(b->rstream));
    for (int s = 0; s < b->n; ++s) {
      bool grown = false;
      if ((e = ensure_window(b->ctx[s], n_frames, &grown)) != DPT_OK) return e;
    }
    b->winjobs_ok[0] = b->winjobs_ok[1] = false;
    b->clear_groups();
  }
  // as for a context: the first window after a committed update builds its
  // pyramids on the reference stream, behind the update
  const bool on_ref = b->rstream && b->commit_pending && frames_on_device;
  const hipStream_t pst = on_ref ? b->rstream : b->stream;
  if (!on_ref && (e = batch_consume(b)) != DPT_OK) return e;
  WinJob* winjobs = nullptr;
  if ((e = batch_winjobs(b, b->bank, &winjobs)) != DPT_OK) return e;
  refresh_groups(b);
  if (b->groups_dirty) {  // regrouping frees the rings: finish and fill what is in flight first
    if (!b->pending.empty() && (e = batch_synchronize(b)) != DPT_OK) return e;
    if ((e = build_groups(b)) != DPT_OK) return e;
  }
  for (CoopEngine* g : b->groups)
    if (g->dirty) HIP_TRY(g->upload());
  // the frames as the pyramid launch and the track read them (host frames
  // through each stream's staging); rows W bytes apart serve as level 0
  std::vector<const uint8_t*> src(b->n);
  std::vector<int64_t> sp(b->n), sst(b->n);
  for (int s = 0; s < b->n; ++s) {
    dpt_ctx* c = b->ctx[s];
    src[s] = frames[s], sp[s] = pitches[s], sst[s] = frame_strides[s];
    if (!frames_on_device) {
      if ((e = stage_window(c, frames[s], pitches[s], frame_strides[s], n_frames, b->stream)) != DPT_OK) return e;
      src[s] = c->win_staging, sp[s] = c->cam.width, sst[s] = (int64_t)c->cam.width * c->cam.height;
    }
  }
  // pyramids of every stream's frames, up to kPyrArgJobs streams per launch
  int ps = -1;
  const bool prof_pyr = b->prof && !on_ref;  // the profile ring times the batch's stream
  if (prof_pyr) HIP_TRY(b->prof_pyr.begin(b->stream, &ps));
  for (int s0 = 0; s0 < b->n; s0 += kPyrArgJobs) {
    const int m = std::min(kPyrArgJobs, b->n - s0);
    PyrWinSrc srcs;
    std::memset(&srcs, 0, sizeof srcs);
    int max_w = 0, max_h = 0;
    bool block = true;
    for (int k = 0; k < m; ++k) {
      dpt_ctx* c = b->ctx[s0 + k];
      srcs.src[k] = src[s0 + k];
      srcs.pitch[k] = sp[s0 + k];
      srcs.stride[k] = sst[s0 + k];
      srcs.write_l0[k] = sp[s0 + k] == c->cam.width ? 0 : 1;
      max_w = std::max(max_w, c->cam.width);
      max_h = std::max(max_h, c->cam.height);
      // every frame's source rows and window pyramid aligned like the first's
      block = block && sst[s0 + k] % 8 == 0 && c->win_stride % 8 == 0 &&
              pyramid_block_ok(c->pg, src[s0 + k], sp[s0 + k], bank_win(c));
    }
    HIP_TRY(launch_pyramid_window(winjobs + s0, srcs, m, n_frames, max_w, max_h, b->ctx[0]->prm.levels, block, pst));
  }
  if (prof_pyr) HIP_TRY(b->prof_pyr.end(b->stream, ps));
  if (on_ref) {  // the update's event now also covers the windows' pyramids
    HIP_TRY(hipEventRecord(b->ev_ready, b->rstream));
    if ((e = batch_consume(b)) != DPT_OK) return e;
  }
  const int slot = b->slot_next;
  for (int f = 0; f < n_frames; ++f) {
    const int mode = f == 0 && init_mode == DPT_INIT_GIVEN ? kStartGiven : kStartConstVelocity;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const std::vector<int>& ss = b->group_streams[gi];
      StartSlot* st = b->groups[gi]->start((slot + f) % kRing);
      for (size_t k = 0; k < ss.size(); ++k) {
        fill_start(b->ctx[ss[k]], mode, T_cw_init ? T_cw_init + 16 * ss[k] : nullptr, &st[k]);
        if (f == 0 && sp[ss[k]] == b->ctx[ss[k]]->cam.width) st[k].l0 = src[ss[k]], st[k].l0_stride = sst[ss[k]];
      }
    }
  }
  if (b->prof) HIP_TRY(b->prof_trk.begin(b->stream, &ps));
  for (CoopEngine* g : b->groups) HIP_TRY(g->launch(b->spin_limit, slot, n_frames));
  if (b->prof) HIP_TRY(b->prof_trk.end(b->stream, ps));
  for (int f = 0; f < n_frames; ++f) b->pending.emplace_back((slot + f) % kRing, out + (size_t)f * b->n);
  b->slot_next = (slot + n_frames) % kRing;
  if (!frames_on_device) HIP_TRY(hipStreamSynchronize(b->stream));  // the host frames are only borrowed
  return DPT_OK;
}

int dpt_batch_set_pose_history(dpt_batch* b, int32_t s, const double T_older[16], const double T_newer[16]) {
  g_err.clear();
  if (!b || s < 0 || s >= b->n) return fail(DPT_E_ARG, "stream %d", s);
  return dpt_set_pose_history(b->ctx[s], T_older, T_newer);
}

int dpt_batch_set_spin_limit(dpt_batch* b, int32_t polls) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  if (polls < 0) return fail(DPT_E_ARG, "polls %d < 0", polls);
  b->spin_limit = polls;
  return DPT_OK;
}

int dpt_batch_set_launch_config(dpt_batch* b, int32_t mode, int32_t chunk) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  if (mode < DPT_LAUNCH_AUTO || mode > DPT_LAUNCH_COOP_PAIRS) return fail(DPT_E_ARG, "mode %d", mode);
  if (chunk != 64 && chunk != 128 && chunk != 256) return fail(DPT_E_ARG, "chunk %d not in {64, 128, 256}", chunk);
  if (mode == DPT_LAUNCH_COOP_PAIRS && chunk == 256)
    return fail(DPT_E_ARG, "chunk %d: two threads per point take 64 or 128 points per chunk", chunk);
  if (mode == DPT_LAUNCH_WORKGROUP && b->ctx[0]->prm.precision == DPT_PREC_MIXED)
    return fail(DPT_E_ARG, "mixed precision runs on the cooperative launch only");
  const int e = batch_synchronize(b);
  if (e != DPT_OK) return e;
  if (chunk != b->chunk || pair_track(b->ctx[0]->prm, mode) != pair_track(b->ctx[0]->prm, b->launch_mode))
    b->clear_groups();
  b->launch_mode = mode;
  b->chunk = chunk;
  return DPT_OK;
}

int dpt_batch_set_profiling(dpt_batch* b, int32_t enable) {
  g_err.clear();
  if (!b) return fail(DPT_E_ARG, "NULL batch");
  if (enable < 0) return fail(DPT_E_ARG, "enable %d < 0", enable);
  int e = batch_synchronize(b);
  if (e != DPT_OK) return e;
  if (enable) {
    HIP_TRY(b->prof_pyr.create());
    HIP_TRY(b->prof_trk.create());
  }
  b->prof_pyr.reset(enable);
  b->prof_trk.reset(enable);
  b->prof = enable != 0;
  return DPT_OK;
}

int dpt_batch_last_kernel_ms(dpt_batch* b, float* pyramid_ms, float* track_ms) {
  g_err.clear();
  if (!b || !pyramid_ms || !track_ms) return fail(DPT_E_ARG, "NULL argument");
  const int e = batch_synchronize(b);
  if (e != DPT_OK) return e;
  *pyramid_ms = b->prof_pyr.last_ms;
  *track_ms = b->prof_trk.last_ms;
  return DPT_OK;
}

int dpt_batch_get_profile(dpt_batch* b, double* pyramid_ms, int64_t* n_pyramid, double* track_ms, int64_t* n_track) {
  g_err.clear();
  if (!b || !pyramid_ms || !n_pyramid || !track_ms || !n_track) return fail(DPT_E_ARG, "NULL argument");
  const int e = batch_synchronize(b);
  if (e != DPT_OK) return e;
  *pyramid_ms = b->prof_pyr.total_ms;
  *n_pyramid = b->prof_pyr.count;
  *track_ms = b->prof_trk.total_ms;
  *n_track = b->prof_trk.count;
  return DPT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ learned initialiser (tracker side)

namespace {

// exp of a twist (omega, v) as a 4x4 rigid transform (FP64), for the CNN's start pose
void twist_exp(const double* xi, double* T) {
  const double* w = xi;
  const double* v = xi + 3;
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = std::sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = std::sin(th) / th;
    B = (1.0 - std::cos(th)) / th2;
    C = (th - std::sin(th)) / (th2 * th);
  }
  const double W[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
  for (int r = 0; r < 3; ++r) {
    double tv = 0;
    for (int c = 0; c < 3; ++c) {
      const double W2 = W[r][0] * W[0][c] + W[r][1] * W[1][c] + W[r][2] * W[2][c];
      const double id = r == c ? 1.0 : 0.0;
      T[4 * r + c] = id + A * W[r][c] + B * W2;
      tv += (id + B * W[r][c] + C * W2) * v[c];
    }
    T[4 * r + 3] = tv;
  }
  T[12] = T[13] = T[14] = 0.0;
  T[15] = 1.0;
}

constexpr double kTwistScale[6] = {0.08726646259971647, 0.08726646259971647, 0.08726646259971647, 0.1, 0.1, 0.1};

int predict_streams(dpt_cnn* cnn, dpt_ctx* const* ctxs, int n, double* T_out) {
  std::vector<const uint8_t*> refs(n), curs(n);
  for (int s = 0; s < n; ++s) {
    dpt_ctx* c = ctxs[s];
    const int L = c->prm.levels - 1;
    if (c->lv[L].W != 94 || c->lv[L].H != 60) return fail(DPT_E_ARG, "stream %d: coarsest level is not 94 x 60", s);
    if (!c->have_pyr[DPT_SLOT_REF] || !c->have_pyr[DPT_SLOT_CUR] || !c->have_ref)
      return fail(DPT_E_STATE, "stream %d: pyramids or reference missing", s);
    const int e0 = consume_commit(c);
    if (e0 != DPT_OK) return e0;
    refs[s] = c->pyr[DPT_SLOT_REF] + c->lv[L].off;
    curs[s] = c->pyr[DPT_SLOT_CUR] + c->lv[L].off;
  }
  std::vector<float> out(6 * (size_t)n);
  int e = cnn_forward_levels(cnn, refs.data(), curs.data(), n, out.data());
  if (e != DPT_OK) return e;
  for (int s = 0; s < n; ++s) {
    double xi[6], Trel[16];
    for (int j = 0; j < 6; ++j) xi[j] = (double)out[6 * s + j] * kTwistScale[j];
    twist_exp(xi, Trel);
    compose(Trel, ctxs[s]->T_rw, T_out + 16 * s);
  }
  return DPT_OK;
}

// Enqueue the learned proposal of n streams on stream s: the forward pass on
// their coarsest reference and current levels, then each start relative to
// its reference into prop (n x 3x4 FP64, device).  The level pointer table is
// uploaded at the first call (the pyramids never move).
int propose_streams(dpt_cnn* cnn, dpt_ctx* const* ctxs, int n, hipStream_t s, const uint8_t*** d_lv, bool* lv_ok,
                    double** prop) {
  std::vector<const uint8_t*> h(2 * (size_t)n);
  const int bank = ctxs[0]->bank;  // a batch's streams switch banks together
  for (int k = 0; k < n; ++k) {
    dpt_ctx* c = ctxs[k];
    const int L = c->prm.levels - 1;
    if (c->lv[L].W != 94 || c->lv[L].H != 60) return fail(DPT_E_ARG, "stream %d: coarsest level is not 94 x 60", k);
    if (!c->have_pyr[DPT_SLOT_REF] || !c->have_pyr[DPT_SLOT_CUR] || !c->have_ref)
      return fail(DPT_E_STATE, "stream %d: pyramids or reference missing", k);
    const int e0 = consume_commit(c);
    if (e0 != DPT_OK) return e0;
    if (c->bank != bank) return fail(DPT_E_STATE, "stream banks out of step");
    h[k] = c->pyr[DPT_SLOT_REF] + c->lv[L].off;
    h[n + k] = c->pyr[DPT_SLOT_CUR] + c->lv[L].off;
  }
  if (!*d_lv) HIP_TRY(hipMalloc((void**)d_lv, sizeof(void*) * 4 * n));
  const uint8_t** tab = *d_lv + (size_t)bank * 2 * n;
  if (!lv_ok[bank]) {  // the bank's buffers are fixed for the context's life: one upload
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy((void*)tab, h.data(), sizeof(void*) * 2 * n, hipMemcpyHostToDevice));
    lv_ok[bank] = true;
  }
  if (!*prop) HIP_TRY(hipMalloc((void**)prop, sizeof(double) * 12 * n));
  return cnn_propose(cnn, tab, n, s, *prop);
}

}  // namespace

extern "C" {

int dpt_cnn_propose(dpt_cnn* cnn, dpt_ctx* c) {
  g_err.clear();
  if (!cnn || !c) return fail(DPT_E_ARG, "NULL argument");
  const int e = propose_streams(cnn, &c, 1, c->stream, &c->d_cnn_lv, c->cnn_lv_ok, &c->d_prop);
  if (e == DPT_OK) c->have_prop = true;
  return e;
}

int dpt_cnn_propose_batch(dpt_cnn* cnn, dpt_batch* b) {
  g_err.clear();
  if (!cnn || !b) return fail(DPT_E_ARG, "NULL argument");
  {
    int e0 = batch_close_update(b);
    if (e0 != DPT_OK || (e0 = batch_consume(b)) != DPT_OK) return e0;
  }
  const int e = propose_streams(cnn, b->ctx.data(), b->n, b->stream, &b->d_cnn_lv, b->cnn_lv_ok, &b->d_prop);
  if (e == DPT_OK) b->have_prop = true;
  return e;
}

int dpt_cnn_predict(dpt_cnn* cnn, dpt_ctx* c, double T_cw_out[16]) {
  g_err.clear();
  if (!cnn || !c || !T_cw_out) return fail(DPT_E_ARG, "NULL argument");
  return predict_streams(cnn, &c, 1, T_cw_out);
}

int dpt_cnn_predict_batch(dpt_cnn* cnn, dpt_batch* b, double* T_cw_out) {
  g_err.clear();
  if (!cnn || !b || !T_cw_out) return fail(DPT_E_ARG, "NULL argument");
  {
    int e0 = batch_close_update(b);
    if (e0 != DPT_OK || (e0 = batch_consume(b)) != DPT_OK) return e0;
  }
  return predict_streams(cnn, b->ctx.data(), b->n, T_cw_out);
}

}  // extern "C"

extern "C" int dpt_batch_get_level(dpt_batch* b, int32_t slot, int32_t level, uint8_t* dst, int32_t dst_on_device) {
  if (dst_on_device != 0 && dst_on_device != 1) return fail(DPT_E_ARG, "dst_on_device %d is neither 0 nor 1", dst_on_device);
  g_err.clear();
  if (!b || !dst) return fail(DPT_E_ARG, "NULL argument");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (level < 0 || level >= b->ctx[0]->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  const LevelGeom& g0 = b->ctx[0]->lv[level];
  const size_t bytes = (size_t)g0.W * g0.H;
  for (int s = 0; s < b->n; ++s) {
    const dpt_ctx* c = b->ctx[s];
    if (c->lv[level].W != g0.W || c->lv[level].H != g0.H) return fail(DPT_E_ARG, "level sizes differ across streams");
    if (!c->have_pyr[slot]) return fail(DPT_E_STATE, "stream %d has no pyramid in slot %d", s, slot);
  }
  if (slot == DPT_SLOT_REF && b->rstream) HIP_TRY(hipStreamSynchronize(b->rstream));  // built on the reference stream
  for (int s = 0; s < b->n; ++s)
    HIP_TRY(hipMemcpyAsync(dst + s * bytes, b->ctx[s]->pyr[slot] + g0.off, bytes,
                           dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return DPT_OK;
}
