// C-ABI host library of the direct photometric tracker (include/dptrack.h).
// Owns device memory per context, validates arguments, marshals launch
// arguments and turns HIP failures into negative return codes with a message.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/dptrack.h"
#include "dpt_internal.h"

using namespace dpt;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
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
  if (p->precision != DPT_PREC_FP32) return fail(DPT_E_ARG, "precision %d not available in this entry point", p->precision);
  if (p->flags != 0) return fail(DPT_E_ARG, "unknown flags 0x%x", p->flags);
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

struct dpt_ctx {
  dpt_camera cam;
  dpt_params prm;
  int32_t cap = 0;  // max points
  hipStream_t stream = nullptr;
  LevelGeom lv[kMaxLevels];
  PyrGeom pg;
  int64_t pyr_bytes = 0;
  uint8_t* pyr[2] = {nullptr, nullptr};
  bool have_pyr[2] = {false, false};
  uint8_t* staging = nullptr;  // level-0 upload buffer for host images
  float* x0 = nullptr;
  uint8_t* valid = nullptr;
  float *I0 = nullptr, *gx = nullptr, *gy = nullptr;
  float* pts = nullptr;  // device copy of the world points
  int32_t n_points = 0;
  bool have_ref = false;
  double T_rw[16];
  int32_t* sel_idx = nullptr;
  int32_t* sel_count = nullptr;
  TrackOut* d_out = nullptr;
  TrackOut* h_out = nullptr;  // pinned
  float* d_tot = nullptr;
  float* h_tot = nullptr;  // pinned
  Pattern pat;

  ~dpt_ctx() {
    for (void* p : {(void*)pyr[0], (void*)pyr[1], (void*)staging, (void*)x0, (void*)valid, (void*)I0, (void*)gx,
                    (void*)gy, (void*)pts, (void*)sel_idx, (void*)sel_count, (void*)d_out, (void*)d_tot})
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
  for (int l = 0; l < kMaxLevels; ++l) a.lv[l] = c->lv[l];
  a.levels = c->prm.levels;
  a.max_iters = c->prm.max_iters;
  a.min_points = c->prm.min_points;
  a.huber_k = c->prm.huber_k;
  a.step_eps = c->prm.step_eps;
  a.z_min = c->prm.z_min;
  a.pat = c->pat;
  a.ref.x0 = c->x0;
  a.ref.valid = c->valid;
  a.ref.I0 = c->I0;
  a.ref.gx = c->gx;
  a.ref.gy = c->gy;
  a.ref.n = c->n_points;
  a.ref.cap = c->cap;
  a.out = c->d_out;
  a.totals = c->d_tot;
}

void rel_pose_f32(const dpt_ctx* c, const double* T_cw, float* out12) {
  double Tinv[16], Trel[16];
  invert(c->T_rw, Tinv);
  compose(T_cw, Tinv, Trel);
  for (int j = 0; j < 12; ++j) out12[j] = (float)Trel[j];
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
      (e = dev_alloc((void**)&c->x0, cap * 3 * sizeof(float))) || (e = dev_alloc((void**)&c->valid, L * cap)) ||
      (e = dev_alloc((void**)&c->I0, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->gx, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->gy, L * cap * K * sizeof(float))) ||
      (e = dev_alloc((void**)&c->pts, cap * 3 * sizeof(float))) ||
      (e = dev_alloc((void**)&c->sel_idx, (size_t)cam->width * cam->height * sizeof(int32_t))) ||
      (e = dev_alloc((void**)&c->sel_count, sizeof(int32_t))) || (e = dev_alloc((void**)&c->d_out, sizeof(TrackOut))) ||
      (e = dev_alloc((void**)&c->d_tot, kRedSlots * sizeof(float)))) {
    delete c;
    return e;
  }
  if (hipHostMalloc((void**)&c->h_out, sizeof(TrackOut)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_tot, kRedSlots * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(DPT_E_OOM, "pinned host allocation failed");
  }
  *out = c;
  return DPT_OK;
}

void dpt_destroy(dpt_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

int dpt_build_pyramid(dpt_ctx* c, int32_t slot, const uint8_t* img, int64_t pitch, int32_t img_on_device) {
  g_err.clear();
  if (!c || !img) return fail(DPT_E_ARG, "NULL argument");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (pitch < c->cam.width) return fail(DPT_E_ARG, "pitch %lld < width %d", (long long)pitch, c->cam.width);
  const uint8_t* src = img;
  int64_t sp = pitch;
  if (!img_on_device) {
    HIP_TRY(hipMemcpy2DAsync(c->staging, c->cam.width, img, pitch, c->cam.width, c->cam.height,
                             hipMemcpyHostToDevice, c->stream));
    src = c->staging;
    sp = c->cam.width;
  }
  HIP_TRY(launch_pyramid(src, sp, c->pyr[slot], c->pg, c->stream));
  c->have_pyr[slot] = true;
  if (slot == DPT_SLOT_REF) c->have_ref = false;
  if (!img_on_device) HIP_TRY(hipStreamSynchronize(c->stream));  // the host buffer is only borrowed
  return DPT_OK;
}

int dpt_get_pyramid(dpt_ctx* c, int32_t slot, int32_t level, uint8_t* host_dst) {
  g_err.clear();
  if (!c || !host_dst) return fail(DPT_E_ARG, "NULL argument");
  if (slot != DPT_SLOT_REF && slot != DPT_SLOT_CUR) return fail(DPT_E_ARG, "slot %d", slot);
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_pyr[slot]) return fail(DPT_E_STATE, "slot %d has no pyramid", slot);
  const LevelGeom& g = c->lv[level];
  HIP_TRY(hipMemcpyAsync(host_dst, c->pyr[slot] + g.off, (size_t)g.W * g.H, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int dpt_select_points(dpt_ctx* c, int32_t n, int32_t margin, int32_t* host_idx, int32_t* n_out) {
  g_err.clear();
  if (!c || !host_idx || !n_out) return fail(DPT_E_ARG, "NULL argument");
  if (n < 1 || (int64_t)n > (int64_t)c->cam.width * c->cam.height) return fail(DPT_E_ARG, "n %d", n);
  if (margin < 1 || 2 * margin >= c->cam.width || 2 * margin >= c->cam.height) return fail(DPT_E_ARG, "margin %d", margin);
  if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "no reference pyramid");
  HIP_TRY(launch_select(c->pyr[DPT_SLOT_REF], c->cam.width, c->cam.height, margin, n, c->sel_idx, c->sel_count,
                        c->stream));
  int32_t cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, c->sel_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (cnt < 0 || cnt > n) return fail(DPT_E_HIP, "selection returned %d of %d", cnt, n);
  if (cnt) {
    HIP_TRY(hipMemcpyAsync(host_idx, c->sel_idx, (size_t)cnt * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  *n_out = cnt;
  return DPT_OK;
}

int dpt_set_reference_points(dpt_ctx* c, const float* xyz, int32_t n, const double T_rw[16], int32_t on_device) {
  g_err.clear();
  if (!c || !T_rw || (n > 0 && !xyz)) return fail(DPT_E_ARG, "NULL argument");
  if (n < 0 || n > c->cap) return fail(DPT_E_ARG, "n %d outside [0, %d]", n, c->cap);
  if (!finite16(T_rw)) return fail(DPT_E_ARG, "T_rw not finite");
  if (!c->have_pyr[DPT_SLOT_REF]) return fail(DPT_E_STATE, "no reference pyramid");
  const float* P = xyz;
  if (n > 0 && !on_device) {
    HIP_TRY(hipMemcpyAsync(c->pts, xyz, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    P = c->pts;
  }
  PrecomputeArgs a;
  std::memset(&a, 0, sizeof a);
  a.ref = c->pyr[DPT_SLOT_REF];
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
  a.n = n;
  a.cap = c->cap;
  HIP_TRY(launch_precompute(a, c->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(c->T_rw, T_rw, sizeof c->T_rw);
  c->n_points = n;
  c->have_ref = true;
  return DPT_OK;
}

int dpt_track_frame(dpt_ctx* c, const double T_cw_init[16], dpt_result* out) {
  g_err.clear();
  if (!c || !T_cw_init || !out) return fail(DPT_E_ARG, "NULL argument");
  if (!finite16(T_cw_init)) return fail(DPT_E_ARG, "T_cw_init not finite");
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  if (!c->have_pyr[DPT_SLOT_CUR]) return fail(DPT_E_STATE, "no current pyramid");
  TrackArgs a;
  fill_track_args(c, a);
  rel_pose_f32(c, T_cw_init, a.T_init);
  HIP_TRY(launch_track(a, c->stream));
  HIP_TRY(hipMemcpyAsync(c->h_out, c->d_out, sizeof(TrackOut), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const TrackOut& o = *c->h_out;
  double Trel[16];
  for (int j = 0; j < 12; ++j) Trel[j] = (double)o.T[j];
  Trel[12] = Trel[13] = Trel[14] = 0.0;
  Trel[15] = 1.0;
  std::memset(out, 0, sizeof *out);
  compose(Trel, c->T_rw, out->T_cw);
  out->final_cost = o.n > 0 ? (double)o.E / (double)o.n : 0.0;
  out->iterations = o.iterations;
  for (int l = 0; l < kMaxLevels; ++l) out->iters_per_level[l] = o.iters_per_level[l];
  out->n_valid_points = o.n_valid_points;
  out->status = o.status;
  out->samples = o.samples;
  return DPT_OK;
}

int dpt_get_reference_cache(dpt_ctx* c, int32_t level, uint8_t* valid, float* I0, float* gx, float* gy, float* x0) {
  g_err.clear();
  if (!c) return fail(DPT_E_ARG, "NULL context");
  if (level < 0 || level >= c->prm.levels) return fail(DPT_E_ARG, "level %d", level);
  if (!c->have_ref) return fail(DPT_E_STATE, "no reference points");
  const size_t n = (size_t)c->n_points, K = (size_t)c->prm.n_pattern, cap = (size_t)c->cap;
  const size_t lo = (size_t)level * cap;
  if (n) {
    if (valid) HIP_TRY(hipMemcpyAsync(valid, c->valid + lo, n, hipMemcpyDeviceToHost, c->stream));
    if (I0) HIP_TRY(hipMemcpyAsync(I0, c->I0 + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (gx) HIP_TRY(hipMemcpyAsync(gx, c->gx + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (gy) HIP_TRY(hipMemcpyAsync(gy, c->gy + lo * K, n * K * 4, hipMemcpyDeviceToHost, c->stream));
    if (x0) HIP_TRY(hipMemcpyAsync(x0, c->x0, n * 3 * 4, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DPT_OK;
}

int dpt_normal_equations(dpt_ctx* c, int32_t level, const double T_rel[16], float* H21, float* b6, double* E,
                         int64_t* n, int32_t* npts) {
  g_err.clear();
  if (!c || !T_rel || !H21 || !b6 || !E || !n || !npts) return fail(DPT_E_ARG, "NULL argument");
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
  for (int j = 0; j < 21; ++j) H21[j] = c->h_tot[j];
  for (int j = 0; j < 6; ++j) b6[j] = c->h_tot[kSlotB + j];
  *E = c->h_tot[kSlotE];
  *n = (int64_t)c->h_tot[kSlotN];
  *npts = (int32_t)c->h_tot[kSlotPts];
  return DPT_OK;
}

}  // extern "C"
