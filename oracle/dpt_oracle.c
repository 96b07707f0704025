/*
 * FP64 CPU oracle of pose-only direct photometric tracking against a sparse map.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg load this code.  It shares no source, header,
 * table or helper with the HIP library, and neither side includes the other.
 *
 * What it follows (paper, Sec. IV "Direct Photometric Tracking"):
 *   Eq.(1)  u0_i = pi(T0 P_i), u_i(T) = pi(T P_i)
 *   Eq.(2)  r_ik = I0(u0_i + d_k) - I(u_i(T) + d_k), bilinear sampling
 *   Eq.(3)  least-squares cost over points and patch pixels
 *   Eq.(4)-(5) Gauss-Newton linearisation, H delta = b, H = J^T J, b = -J^T r
 *   Eq.(6)  inverse-compositional Jacobian J_ik = grad I0(u0_i + d_k) dpi/dx dx/ddelta at x = T0 P_i
 *   Sec. IV-C: pyramid, IC precompute per reference and level, per-level per-iteration
 *   track with reduction and a Cholesky solve, coarse to fine.
 *
 * Readings where the paper is silent (each restated where it is used):
 *   pyramid    uint8 2x2 box mean, round half up, floor sizes; or (flag) the paper's
 *              floating-point Gaussian pyramid: separable binomial [1 3 3 1]/8, vertical
 *              pass then horizontal pass, clamped borders, every second sample

 *   camera     f_l = f / 2^l, c_l = (c + 0.5) / 2^l - 0.5 (pixel centres at integers)
 *   gradient   central differences / 2 at integer pixels, bilinearly interpolated
 *   validity   a point counts only if Z > z_min and every pattern position p satisfies
 *              1 <= p.x < W_l - 2 and 1 <= p.y < H_l - 2
 *   twist      delta = (omega, v); left perturbation exp(delta) x0 in the reference frame
 *   update     T_rel <- T_rel exp(delta)^-1 with T_rel = T T0^-1 (inverse composition)
 *   robust     Huber, w = min(1, k/|r|), rho = r^2/2 or k(|r| - k/2); k <= 0: plain LS
 *   H          re-reduced with the weights at every iteration (iteratively reweighted);
 *              the paper's fixed H (reduced once per reference, no weights) is a flag
 *   stop       max_j |delta_j| < eps leaves a level; pivots <= 1e-12 max diag: not PD
 *   cost       mean rho over the valid level-0 samples of an extra pass at the result
 *
 * Everything is double precision, scalar loops in point order then pattern order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_MAX_ITERS = 1, ORC_TOO_FEW_POINTS = 2, ORC_NOT_PD = 3 };

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
} orc_camera;

typedef struct {
  int32_t levels;       /* 1..8 */
  int32_t max_iters;    /* per level */
  double huber_k;       /* <= 0: unweighted least squares */
  double step_eps;      /* convergence on max |delta_j| */
  int32_t min_points;   /* fewer valid points: TOO_FEW_POINTS */
  int32_t n_pattern;    /* K <= 128 */
  int32_t pattern[256]; /* (dx, dy) pairs, level pixels */
  double z_min;         /* metres */
  int32_t fixed_h;      /* 1: paper mode, H reduced once per reference, no weights */
  int32_t pyramid;      /* 0: uint8 box pyramid; 1: floating-point Gaussian pyramid */
} orc_params;

typedef struct {
  double T_cw[16];
  double final_cost;
  int32_t iterations;
  int32_t iters_per_level[8];
  int32_t n_valid_points;
  int32_t status;
  int64_t samples; /* residual samples evaluated over all passes */
} orc_result;

/* ------------------------------------------------------------------ pyramid */

int64_t orc_pyramid_bytes(int32_t W, int32_t H, int32_t L) {
  int64_t s = 0;
  for (int l = 0; l < L; ++l) s += (int64_t)(W >> l) * (H >> l);
  return s;
}

/* Level l+1 pixel = round-half-up mean of the 2x2 block of level l below it. */
void orc_pyramid(const uint8_t* img, int64_t pitch, int32_t W, int32_t H, int32_t L, uint8_t* out) {
  for (int y = 0; y < H; ++y) memcpy(out + (int64_t)y * W, img + y * pitch, (size_t)W);
  const uint8_t* src = out;
  int w = W, h = H;
  uint8_t* dst = out + (int64_t)W * H;
  for (int l = 1; l < L; ++l) {
    int w2 = w / 2, h2 = h / 2;
    for (int y = 0; y < h2; ++y)
      for (int x = 0; x < w2; ++x) {
        int s = src[(2 * y) * w + 2 * x] + src[(2 * y) * w + 2 * x + 1] + src[(2 * y + 1) * w + 2 * x] +
                src[(2 * y + 1) * w + 2 * x + 1];
        dst[y * w2 + x] = (uint8_t)((s + 2) >> 2);
      }
    src = dst;
    dst += (int64_t)w2 * h2;
    w = w2;
    h = h2;
  }
}

/* Floating-point Gaussian pyramid (Sec. IV-C, image pyramids): level 0 is the
 * image as numbers; level l+1 blurs level l vertically, then horizontally, with
 * the binomial kernel w = [1 3 3 1]/8 over samples 2y-1 .. 2y+2 (indices clamped
 * to the level) and keeps every second sample, so that level-(l+1) pixel x sits
 * at level-l position 2x + 1/2, the same pixel-centre convention as the box
 * pyramid.  Sizes floor(W/2) x floor(H/2).  out: sum over levels of w_l h_l doubles. */
void orc_pyramid_gauss(const uint8_t* img, int64_t pitch, int32_t W, int32_t H, int32_t L, double* out) {
  static const double w[4] = {1.0 / 8.0, 3.0 / 8.0, 3.0 / 8.0, 1.0 / 8.0};
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) out[(int64_t)y * W + x] = (double)img[y * pitch + x];
  const double* src = out;
  double* dst = out + (int64_t)W * H;
  int ww = W, hh = H;
  for (int l = 1; l < L; ++l) {
    int w2 = ww / 2, h2 = hh / 2;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)h2 * ww); /* vertical pass, kept rows only */
    for (int y = 0; y < h2; ++y)
      for (int x = 0; x < ww; ++x) {
        double acc = 0.0;
        for (int i = 0; i < 4; ++i) {
          int yy = 2 * y - 1 + i;
          yy = yy < 0 ? 0 : (yy > hh - 1 ? hh - 1 : yy);
          acc += w[i] * src[(int64_t)yy * ww + x];
        }
        tmp[(int64_t)y * ww + x] = acc;
      }
    for (int y = 0; y < h2; ++y)
      for (int x = 0; x < w2; ++x) {
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) {
          int xx = 2 * x - 1 + j;
          xx = xx < 0 ? 0 : (xx > ww - 1 ? ww - 1 : xx);
          acc += w[j] * tmp[(int64_t)y * ww + xx];
        }
        dst[(int64_t)y * w2 + x] = acc;
      }
    free(tmp);
    src = dst;
    dst += (int64_t)w2 * h2;
    ww = w2;
    hh = h2;
  }
}

/* The pyramid the tracker samples, as doubles: the box pyramid's uint8 values, or
 * the Gaussian pyramid (prm->pyramid). */
static double* orc_levels(const orc_params* prm, const uint8_t* img, int64_t pitch, int32_t W, int32_t H) {
  int64_t n = orc_pyramid_bytes(W, H, prm->levels);
  double* out = (double*)malloc(sizeof(double) * (size_t)n);
  if (prm->pyramid == 1) {
    orc_pyramid_gauss(img, pitch, W, H, prm->levels, out);
  } else {
    uint8_t* u = (uint8_t*)malloc((size_t)n);
    orc_pyramid(img, pitch, W, H, prm->levels, u);
    for (int64_t i = 0; i < n; ++i) out[i] = (double)u[i];
    free(u);
  }
  return out;
}

/* ------------------------------------------------------------------ point selection */

typedef struct {
  int32_t score, idx;
} orc_cand;

static int orc_cand_cmp(const void* a, const void* b) {
  const orc_cand* p = (const orc_cand*)a;
  const orc_cand* q = (const orc_cand*)b;
  if (p->score != q->score) return p->score > q->score ? -1 : 1;
  return (p->idx > q->idx) - (p->idx < q->idx);
}

static int orc_int_cmp(const void* a, const void* b) {
  int32_t p = *(const int32_t*)a, q = *(const int32_t*)b;
  return (p > q) - (p < q);
}

/* Stand-in for the map points the indirect pipeline provides: the n pixels of the
 * reference image with the largest squared central-difference gradient
 * s = (I[y][x+1]-I[y][x-1])^2 + (I[y+1][x]-I[y-1][x])^2 inside a margin, ties by
 * smaller linear index.  Returns the chosen indices in ascending order. */
int32_t orc_select_points(const uint8_t* img, int64_t pitch, int32_t W, int32_t H, int32_t n, int32_t margin,
                          int32_t* idx_out) {
  if (margin < 1) margin = 1;
  int64_t cap = (int64_t)(W > 2 * margin ? W - 2 * margin : 0) * (H > 2 * margin ? H - 2 * margin : 0);
  if (cap <= 0 || n <= 0) return 0;
  orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)cap);
  int64_t m = 0;
  for (int y = margin; y <= H - 1 - margin; ++y)
    for (int x = margin; x <= W - 1 - margin; ++x) {
      int dx = (int)img[y * pitch + x + 1] - (int)img[y * pitch + x - 1];
      int dy = (int)img[(y + 1) * pitch + x] - (int)img[(y - 1) * pitch + x];
      c[m].score = dx * dx + dy * dy;
      c[m].idx = y * W + x;
      ++m;
    }
  qsort(c, (size_t)m, sizeof(orc_cand), orc_cand_cmp);
  int32_t k = (int32_t)(m < n ? m : n);
  for (int32_t i = 0; i < k; ++i) idx_out[i] = c[i].idx;
  qsort(idx_out, (size_t)k, sizeof(int32_t), orc_int_cmp);
  free(c);
  return k;
}

/* ------------------------------------------------------------------ sampling */

static void orc_level_camera(const orc_camera* c, int l, double* fx, double* fy, double* cx, double* cy) {
  double s = ldexp(1.0, l);
  *fx = c->fx / s;
  *fy = c->fy / s;
  *cx = (c->cx + 0.5) / s - 0.5;
  *cy = (c->cy + 0.5) / s - 0.5;
}

/* Bilinear intensity, pixel centres at integer coordinates. */
double orc_sample(const uint8_t* img, int32_t W, double x, double y) {
  double fx = floor(x), fy = floor(y);
  int x0 = (int)fx, y0 = (int)fy;
  double a = x - fx, c = y - fy;
  const uint8_t* r0 = img + (int64_t)y0 * W + x0;
  const uint8_t* r1 = r0 + W;
  return (1 - a) * (1 - c) * r0[0] + a * (1 - c) * r0[1] + (1 - a) * c * r1[0] + a * c * r1[1];
}

/* Reference-side image gradient: central differences at the four taps, blended
 * with the bilinear weights of the sample position. */
void orc_gradient(const uint8_t* img, int32_t W, double x, double y, double* gx, double* gy) {
  double fx = floor(x), fy = floor(y);
  int x0 = (int)fx, y0 = (int)fy;
  double a = x - fx, c = y - fy;
  double wt[4] = {(1 - a) * (1 - c), a * (1 - c), (1 - a) * c, a * c};
  int px[4] = {x0, x0 + 1, x0, x0 + 1}, py[4] = {y0, y0, y0 + 1, y0 + 1};
  double sx = 0, sy = 0;
  for (int t = 0; t < 4; ++t) {
    const uint8_t* p = img + (int64_t)py[t] * W + px[t];
    sx += wt[t] * 0.5 * ((double)p[1] - (double)p[-1]);
    sy += wt[t] * 0.5 * ((double)p[W] - (double)p[-W]);
  }
  *gx = sx;
  *gy = sy;
}

/* orc_sample and orc_gradient on a level stored as doubles (what the tracker uses). */
double orc_sample_f(const double* img, int32_t W, double x, double y) {
  double fx = floor(x), fy = floor(y);
  int x0 = (int)fx, y0 = (int)fy;
  double a = x - fx, c = y - fy;
  const double* r0 = img + (int64_t)y0 * W + x0;
  const double* r1 = r0 + W;
  return (1 - a) * (1 - c) * r0[0] + a * (1 - c) * r0[1] + (1 - a) * c * r1[0] + a * c * r1[1];
}

void orc_gradient_f(const double* img, int32_t W, double x, double y, double* gx, double* gy) {
  double fx = floor(x), fy = floor(y);
  int x0 = (int)fx, y0 = (int)fy;
  double a = x - fx, c = y - fy;
  double wt[4] = {(1 - a) * (1 - c), a * (1 - c), (1 - a) * c, a * c};
  int px[4] = {x0, x0 + 1, x0, x0 + 1}, py[4] = {y0, y0, y0 + 1, y0 + 1};
  double sx = 0, sy = 0;
  for (int t = 0; t < 4; ++t) {
    const double* p = img + (int64_t)py[t] * W + px[t];
    sx += wt[t] * 0.5 * (p[1] - p[-1]);
    sy += wt[t] * 0.5 * (p[W] - p[-W]);
  }
  *gx = sx;
  *gy = sy;
}

static int orc_inside(double x, double y, int W, int H) { return x >= 1.0 && x < W - 2.0 && y >= 1.0 && y < H - 2.0; }

/* ------------------------------------------------------------------ SE(3) */

/* 3x4 row-major [R | t] */
static void orc_compose(const double* A, const double* B, double* C) {
  double T[12];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[4 * r + c] = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c];
    T[4 * r + 3] = A[4 * r] * B[3] + A[4 * r + 1] * B[7] + A[4 * r + 2] * B[11] + A[4 * r + 3];
  }
  memcpy(C, T, sizeof T);
}

static void orc_invert(const double* A, double* B) {
  double T[12];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[4 * r + c] = A[4 * c + r];
    T[4 * r + 3] = -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
  }
  memcpy(B, T, sizeof T);
}

/* exp of xi = (omega, v): R = I + A[w] + B[w]^2, t = (I + B[w] + C[w]^2) v, with
 * A = sin(th)/th, B = (1-cos th)/th^2, C = (th - sin th)/th^3 (Taylor below 1e-4). */
void orc_se3_exp(const double* xi, double* T16) {
  const double* w = xi;
  const double* v = xi + 3;
  double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double W2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
  memset(T16, 0, 16 * sizeof(double));
  for (int r = 0; r < 3; ++r) {
    double tv = 0;
    for (int c = 0; c < 3; ++c) {
      double id = (r == c) ? 1.0 : 0.0;
      T16[4 * r + c] = id + A * W[3 * r + c] + B * W2[3 * r + c];
      tv += (id + B * W[3 * r + c] + C * W2[3 * r + c]) * v[c];
    }
    T16[4 * r + 3] = tv;
  }
  T16[15] = 1.0;
}

/* log of a rigid transform: theta = atan2(|vee(R - R^T)| / 2, (tr R - 1) / 2),
 * omega = theta * axis, v = V^-1 t. */
void orc_se3_log(const double* T16, double* xi) {
  const double* T = T16;
  double s[3] = {T[9] - T[6], T[2] - T[8], T[4] - T[1]};
  double sn = 0.5 * sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  double cs = 0.5 * (T[0] + T[5] + T[10] - 1.0);
  double th = atan2(sn, cs);
  double f = (th < 1e-8) ? 0.5 : th / (2.0 * sin(th));
  double w[3] = {f * s[0], f * s[1], f * s[2]};
  double th2 = th * th;
  double D; /* V^-1 = I - 0.5 [w] + D [w]^2 */
  if (th < 1e-4) D = 1.0 / 12.0 + th2 / 720.0;
  else D = (1.0 - (th * sin(th)) / (2.0 * (1.0 - cos(th)))) / th2;
  double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double W2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
  double t[3] = {T[3], T[7], T[11]};
  for (int r = 0; r < 3; ++r) {
    double acc = 0;
    for (int c = 0; c < 3; ++c) acc += (((r == c) ? 1.0 : 0.0) - 0.5 * W[3 * r + c] + D * W2[3 * r + c]) * t[c];
    xi[3 + r] = acc;
    xi[r] = w[r];
  }
}

/* ------------------------------------------------------------------ linear algebra */

/* Solve H x = b for symmetric positive definite H (6x6, full) by H = L L^T.
 * Returns 0 on success, 1 if a pivot is <= rel_tol * max_j H_jj. */
int orc_cholesky_solve(const double* H, const double* b, double* x, double rel_tol) {
  double L[36] = {0};
  double dmax = 0;
  for (int j = 0; j < 6; ++j) dmax = H[7 * j] > dmax ? H[7 * j] : dmax;
  for (int j = 0; j < 6; ++j) {
    double d = H[7 * j];
    for (int k = 0; k < j; ++k) d -= L[6 * j + k] * L[6 * j + k];
    if (!(d > rel_tol * dmax)) return 1;
    L[7 * j] = sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double s = H[6 * i + j];
      for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = s / L[7 * j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
    y[i] = s / L[7 * i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
    x[i] = s / L[7 * i];
  }
  return 0;
}

/* ------------------------------------------------------------------ Jacobians */

/* 2x6 warp Jacobian d pi_l(exp(delta) x0) / d delta at delta = 0, columns
 * (w1 w2 w3 v1 v2 v3): dpi/dx times [-[x0]_x | I]. */
void orc_warp_jacobian(double fx, double fy, const double* x0, double* Jw) {
  double iz = 1.0 / x0[2], xp = x0[0] * iz, yp = x0[1] * iz;
  Jw[0] = -fx * xp * yp;
  Jw[1] = fx * (1.0 + xp * xp);
  Jw[2] = -fx * yp;
  Jw[3] = fx * iz;
  Jw[4] = 0.0;
  Jw[5] = -fx * xp * iz;
  Jw[6] = -fy * (1.0 + yp * yp);
  Jw[7] = fy * xp * yp;
  Jw[8] = fy * xp;
  Jw[9] = 0.0;
  Jw[10] = fy * iz;
  Jw[11] = -fy * yp * iz;
}

/* ------------------------------------------------------------------ reference cache */

typedef struct {
  orc_camera cam;
  orc_params prm;
  int32_t n;
  double T_rw[12];
  double* pyr;           /* reference pyramid (values as doubles) */
  int64_t off[8];        /* level offsets */
  double* x0;            /* [n][3] reference-camera points */
  uint8_t* refvalid;     /* [L][n] */
  double* I0;            /* [L][n][K] */
  double* g;             /* [L][n][K][2] */
  double* J;             /* [L][n][K][6] */
  double Hfix[8][36];    /* per-level unweighted H over reference-valid points */
} orc_ref;

static void orc_offsets(int W, int H, int L, int64_t* off) {
  int64_t s = 0;
  for (int l = 0; l < L; ++l) {
    off[l] = s;
    s += (int64_t)(W >> l) * (H >> l);
  }
}

/* IC precompute (Sec. IV-C, "Precompute Inverse Compositional"): per level and point,
 * project with T0, sample the reference patch and its gradients, and store I0 and
 * J_ik = grad I0 * Jw (Eq.6).  Also the per-level H of the paper's fixed-H mode. */
orc_ref* orc_ref_create(const orc_camera* cam, const orc_params* prm, const uint8_t* ref_img, int64_t pitch,
                        const float* P, int32_t n, const double* T_rw16) {
  orc_ref* R = (orc_ref*)calloc(1, sizeof(orc_ref));
  R->cam = *cam;
  R->prm = *prm;
  R->n = n;
  memcpy(R->T_rw, T_rw16, 12 * sizeof(double));
  int L = prm->levels, K = prm->n_pattern, W = cam->width, H = cam->height;
  R->pyr = orc_levels(prm, ref_img, pitch, W, H);
  orc_offsets(W, H, L, R->off);
  size_t nk = (size_t)n * K;
  R->x0 = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  R->refvalid = (uint8_t*)calloc((size_t)L * (n > 0 ? n : 1), 1);
  R->I0 = (double*)calloc((size_t)L * nk + 1, sizeof(double));
  R->g = (double*)calloc((size_t)L * nk * 2 + 1, sizeof(double));
  R->J = (double*)calloc((size_t)L * nk * 6 + 1, sizeof(double));
  for (int i = 0; i < n; ++i) {
    double p[3] = {P[3 * i], P[3 * i + 1], P[3 * i + 2]};
    for (int r = 0; r < 3; ++r)
      R->x0[3 * i + r] = R->T_rw[4 * r] * p[0] + R->T_rw[4 * r + 1] * p[1] + R->T_rw[4 * r + 2] * p[2] + R->T_rw[4 * r + 3];
  }
  for (int l = 0; l < L; ++l) {
    double fx, fy, cx, cy;
    orc_level_camera(cam, l, &fx, &fy, &cx, &cy);
    int Wl = W >> l, Hl = H >> l;
    const double* img = R->pyr + R->off[l];
    memset(R->Hfix[l], 0, sizeof R->Hfix[l]);
    for (int i = 0; i < n; ++i) {
      const double* x0 = R->x0 + 3 * i;
      if (!(x0[2] > prm->z_min)) continue;
      double u = fx * x0[0] / x0[2] + cx, v = fy * x0[1] / x0[2] + cy;
      int ok = 1;
      for (int k = 0; k < K && ok; ++k) ok = orc_inside(u + prm->pattern[2 * k], v + prm->pattern[2 * k + 1], Wl, Hl);
      if (!ok) continue;
      R->refvalid[(size_t)l * n + i] = 1;
      double Jw[12];
      orc_warp_jacobian(fx, fy, x0, Jw);
      for (int k = 0; k < K; ++k) {
        double px = u + prm->pattern[2 * k], py = v + prm->pattern[2 * k + 1];
        size_t s = (size_t)l * nk + (size_t)i * K + k;
        R->I0[s] = orc_sample_f(img, Wl, px, py);
        double gx, gy;
        orc_gradient_f(img, Wl, px, py, &gx, &gy);
        R->g[2 * s] = gx;
        R->g[2 * s + 1] = gy;
        double* J = R->J + 6 * s;
        for (int j = 0; j < 6; ++j) J[j] = gx * Jw[j] + gy * Jw[6 + j];
        for (int a = 0; a < 6; ++a)
          for (int c = 0; c < 6; ++c) R->Hfix[l][6 * a + c] += J[a] * J[c];
      }
    }
  }
  return R;
}

void orc_ref_free(orc_ref* R) {
  if (!R) return;
  free(R->pyr);
  free(R->x0);
  free(R->refvalid);
  free(R->I0);
  free(R->g);
  free(R->J);
  free(R);
}

/* Copies of the precompute cache of one level (test hook). */
void orc_ref_cache(const orc_ref* R, int32_t l, uint8_t* refvalid, double* I0, double* g, double* J, double* x0) {
  size_t n = (size_t)R->n, K = (size_t)R->prm.n_pattern, nk = n * K;
  if (refvalid) memcpy(refvalid, R->refvalid + (size_t)l * n, n);
  if (I0) memcpy(I0, R->I0 + (size_t)l * nk, nk * sizeof(double));
  if (g) memcpy(g, R->g + (size_t)l * nk * 2, nk * 2 * sizeof(double));
  if (J) memcpy(J, R->J + (size_t)l * nk * 6, nk * 6 * sizeof(double));
  if (x0) memcpy(x0, R->x0, n * 3 * sizeof(double));
}

void orc_ref_fixed_h(const orc_ref* R, int32_t l, double* H36) { memcpy(H36, R->Hfix[l], sizeof R->Hfix[l]); }

/* ------------------------------------------------------------------ normal equations */

typedef struct {
  double H[36], b[6], E;
  int64_t n;    /* valid samples */
  int32_t npts; /* valid points */
} orc_ne;

/* One Gauss-Newton linearisation at level l and relative pose T_rel (3x4):
 * residuals of Eq.(2) with the cached I0 and J, Huber weights, and the weighted
 * normal equations H = sum w J^T J, b = -sum w J^T r of Eq.(5). */
static void orc_accumulate(const orc_ref* R, const double* cur_pyr, int l, const double* Trel, int cost_only,
                           orc_ne* ne) {
  const orc_params* prm = &R->prm;
  int K = prm->n_pattern, n = R->n;
  int Wl = R->cam.width >> l, Hl = R->cam.height >> l;
  const double* img = cur_pyr + R->off[l];
  double fx, fy, cx, cy;
  orc_level_camera(&R->cam, l, &fx, &fy, &cx, &cy);
  double k = prm->huber_k;
  int robust = (k > 0) && !prm->fixed_h;
  memset(ne, 0, sizeof *ne);
  size_t nk = (size_t)n * K;
  for (int i = 0; i < n; ++i) {
    if (!R->refvalid[(size_t)l * n + i]) continue;
    const double* x0 = R->x0 + 3 * i;
    double x[3];
    for (int r = 0; r < 3; ++r) x[r] = Trel[4 * r] * x0[0] + Trel[4 * r + 1] * x0[1] + Trel[4 * r + 2] * x0[2] + Trel[4 * r + 3];
    if (!(x[2] > prm->z_min)) continue;
    double u = fx * x[0] / x[2] + cx, v = fy * x[1] / x[2] + cy;
    int ok = 1;
    for (int q = 0; q < K && ok; ++q) ok = orc_inside(u + prm->pattern[2 * q], v + prm->pattern[2 * q + 1], Wl, Hl);
    if (!ok) continue;
    ne->npts++;
    for (int q = 0; q < K; ++q) {
      size_t s = (size_t)l * nk + (size_t)i * K + q;
      double r = R->I0[s] - orc_sample_f(img, Wl, u + prm->pattern[2 * q], v + prm->pattern[2 * q + 1]);
      double ar = fabs(r), w, rho;
      if (robust && ar > k) {
        w = k / ar;
        rho = k * (ar - 0.5 * k);
      } else {
        w = 1.0;
        rho = 0.5 * r * r;
      }
      ne->E += rho;
      ne->n++;
      if (cost_only) continue;
      const double* J = R->J + 6 * s;
      for (int a = 0; a < 6; ++a) {
        ne->b[a] -= w * J[a] * r;
        if (!prm->fixed_h)
          for (int c = 0; c < 6; ++c) ne->H[6 * a + c] += w * J[a] * J[c];
      }
    }
  }
  if (prm->fixed_h && !cost_only) memcpy(ne->H, R->Hfix[l], sizeof ne->H);
}

/* Test hook: normal equations at level l for T_rel (4x4 row-major). */
void orc_ref_normal_equations(const orc_ref* R, const uint8_t* cur_img, int64_t pitch, int32_t l, const double* Trel16,
                              double* H36, double* b6, double* E, int64_t* n, int32_t* npts) {
  double* cur = orc_levels(&R->prm, cur_img, pitch, R->cam.width, R->cam.height);
  orc_ne ne;
  orc_accumulate(R, cur, l, Trel16, 0, &ne);
  memcpy(H36, ne.H, sizeof ne.H);
  memcpy(b6, ne.b, sizeof ne.b);
  *E = ne.E;
  *n = ne.n;
  *npts = ne.npts;
  free(cur);
}

/* ------------------------------------------------------------------ tracker */

/* Coarse-to-fine Gauss-Newton (Sec. IV-A, Sec. IV-C "Track"): at each level from the
 * coarsest, up to max_iters linearisations, each solved by Cholesky and applied by
 * inverse composition; the pose of one level starts the next.  A final cost-only
 * pass at level 0 gives the mean robust cost that the switch criterion reads. */
int32_t orc_ref_track(const orc_ref* R, const uint8_t* cur_img, int64_t pitch, const double* T_cw_init16,
                      orc_result* out) {
  const orc_params* prm = &R->prm;
  int L = prm->levels;
  double* cur = orc_levels(prm, cur_img, pitch, R->cam.width, R->cam.height);
  memset(out, 0, sizeof *out);
  double Tinv[12], Trel[12];
  orc_invert(R->T_rw, Tinv);
  orc_compose(T_cw_init16, Tinv, Trel);
  int status = ORC_OK;
  for (int l = L - 1; l >= 0 && status == ORC_OK; --l) {
    int converged = 0;
    for (int it = 0; it < prm->max_iters; ++it) {
      orc_ne ne;
      orc_accumulate(R, cur, l, Trel, 0, &ne);
      out->samples += ne.n;
      if (ne.npts < prm->min_points) {
        status = ORC_TOO_FEW_POINTS;
        break;
      }
      double delta[6];
      if (orc_cholesky_solve(ne.H, ne.b, delta, 1e-12)) {
        status = ORC_NOT_PD;
        break;
      }
      double xi[6], E16[16];
      for (int j = 0; j < 6; ++j) xi[j] = -delta[j];
      orc_se3_exp(xi, E16);
      orc_compose(Trel, E16, Trel);
      out->iterations++;
      out->iters_per_level[l]++;
      double m = 0;
      for (int j = 0; j < 6; ++j) m = fabs(delta[j]) > m ? fabs(delta[j]) : m;
      if (m < prm->step_eps) {
        converged = 1;
        break;
      }
    }
    if (status == ORC_OK && l == 0 && !converged) status = ORC_MAX_ITERS;
  }
  orc_ne ne;
  orc_accumulate(R, cur, 0, Trel, 1, &ne);
  out->samples += ne.n;
  out->final_cost = ne.n > 0 ? ne.E / (double)ne.n : 0.0;
  out->n_valid_points = ne.npts;
  out->status = status;
  double Tcw[12];
  orc_compose(Trel, R->T_rw, Tcw);
  memcpy(out->T_cw, Tcw, sizeof Tcw);
  out->T_cw[12] = out->T_cw[13] = out->T_cw[14] = 0.0;
  out->T_cw[15] = 1.0;
  free(cur);
  return status;
}
