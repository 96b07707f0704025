/*
 * Seeded synthetic scene renderer: three textured planes ray-cast into a
 * pinhole camera, giving uint8 grayscale frames and exact per-pixel depth.
 *
 * This is input generation only.  It is shared by the FP64 oracle side and the
 * GPU side as a source of identical test inputs and holds none of the tracking
 * method's arithmetic (no pyramid, sampling, Jacobian, weighting or solve).
 *
 * Scene (world frame = camera frame of the first reference view; x right,
 * y down, z forward):
 *   plane 0  y = -1  texture coordinates (x, z)
 *   plane 1  z =  3  texture coordinates (x, y)
 *   plane 2  x =  2  texture coordinates (z, y)
 * Each pixel centre ray takes the nearest positive hit.  The texture is one
 * continuous field over 3-D space, restricted to the planes, so that the seams
 * where two planes meet carry no intensity jump:
 *   f(h) = 128 + sum_j a_j exp(-|h - c_j|^2 / (2 s_j^2)) + A * vnoise(h / cell)
 * Blob centres c_j lie on the planes (drawn per plane in plane coordinates),
 * blobs are truncated at 4 s_j, and the value noise is trilinear with a
 * smoothstep between lattice values drawn from a counter-based hash of
 * (seed, ix, iy, iz).  Pixel value: clip(rint(f + noise), 0, 255).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_PLANES 3
#define SYN_CELL 0.25
#define SYN_MAXREACH 1.6 /* 4 * max sigma (0.4 m) */

typedef struct {
  double lo0, hi0, lo1, hi1; /* grid window in plane coordinates */
  int n0, n1;                /* cells */
  int* start;                /* n0*n1+1 */
  int* items;                /* blob indices */
} syn_grid;

/* splitmix64 finaliser (Steele, Lea, Flood 2014) as a counter-based hash */
static uint64_t syn_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double syn_lattice(uint64_t seed, int64_t ix, int64_t iy, int64_t iz) {
  uint64_t h = syn_mix(seed ^ syn_mix((uint64_t)ix ^ syn_mix((uint64_t)iy ^ syn_mix((uint64_t)iz))));
  double u = (double)(h >> 11) * (1.0 / 9007199254740992.0); /* [0,1) */
  return 2.0 * u - 1.0;
}

static double syn_smooth(double t) { return t * t * (3.0 - 2.0 * t); }

static double syn_vnoise(uint64_t seed, const double* p) {
  double f[3], t[3];
  int64_t i[3];
  for (int a = 0; a < 3; ++a) {
    f[a] = floor(p[a]);
    i[a] = (int64_t)f[a];
    t[a] = syn_smooth(p[a] - f[a]);
  }
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
    double w = (dx ? t[0] : 1 - t[0]) * (dy ? t[1] : 1 - t[1]) * (dz ? t[2] : 1 - t[2]);
    acc += w * syn_lattice(seed, i[0] + dx, i[1] + dy, i[2] + dz);
  }
  return acc;
}

/* blobs: [n][4] = amplitude, sigma, c0, c1 */
static void syn_grid_build(syn_grid* g, const double* blobs, int n, const double win[4]) {
  g->lo0 = win[0] - SYN_MAXREACH;
  g->hi0 = win[1] + SYN_MAXREACH;
  g->lo1 = win[2] - SYN_MAXREACH;
  g->hi1 = win[3] + SYN_MAXREACH;
  g->n0 = (int)ceil((g->hi0 - g->lo0) / SYN_CELL);
  g->n1 = (int)ceil((g->hi1 - g->lo1) / SYN_CELL);
  int nc = g->n0 * g->n1;
  g->start = (int*)calloc((size_t)nc + 1, sizeof(int));
  int* count = (int*)calloc((size_t)nc, sizeof(int));
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int c = 0; c < nc; ++c) g->start[c + 1] = g->start[c] + count[c];
      g->items = (int*)malloc(sizeof(int) * (size_t)(g->start[nc] > 0 ? g->start[nc] : 1));
      memset(count, 0, sizeof(int) * (size_t)nc);
    }
    for (int j = 0; j < n; ++j) {
      double s = blobs[4 * j + 1], c0 = blobs[4 * j + 2], c1 = blobs[4 * j + 3];
      int a0 = (int)floor((c0 - 4 * s - g->lo0) / SYN_CELL), b0 = (int)floor((c0 + 4 * s - g->lo0) / SYN_CELL);
      int a1 = (int)floor((c1 - 4 * s - g->lo1) / SYN_CELL), b1 = (int)floor((c1 + 4 * s - g->lo1) / SYN_CELL);
      if (a0 < 0) a0 = 0;
      if (a1 < 0) a1 = 0;
      if (b0 >= g->n0) b0 = g->n0 - 1;
      if (b1 >= g->n1) b1 = g->n1 - 1;
      for (int q1 = a1; q1 <= b1; ++q1)
        for (int q0 = a0; q0 <= b0; ++q0) {
          int c = q1 * g->n0 + q0;
          if (pass == 1) g->items[g->start[c] + count[c]] = j;
          count[c]++;
        }
    }
  }
  free(count);
}

static void syn_grid_free(syn_grid* g) {
  free(g->start);
  free(g->items);
}

/* plane q coordinates of a 3-D point, and its distance to plane q */
static void syn_plane_coords(int q, const double* h, double* c0, double* c1, double* dperp) {
  if (q == 0) *c0 = h[0], *c1 = h[2], *dperp = fabs(h[1] + 1.0);
  else if (q == 1) *c0 = h[0], *c1 = h[1], *dperp = fabs(h[2] - 3.0);
  else *c0 = h[2], *c1 = h[1], *dperp = fabs(h[0] - 2.0);
}

static double syn_texture(const syn_grid* grids, const double* blobs, int n_blobs, uint64_t seed,
                          double noise_amp, double noise_cell, const double* h) {
  double f = 128.0;
  for (int q = 0; q < SYN_PLANES; ++q) {
    const syn_grid* g = &grids[q];
    const double* bq = blobs + (size_t)q * n_blobs * 4;
    double p0, p1, dp;
    syn_plane_coords(q, h, &p0, &p1, &dp);
    if (dp > SYN_MAXREACH || !(p0 >= g->lo0 && p0 < g->hi0 && p1 >= g->lo1 && p1 < g->hi1)) continue;
    int q0 = (int)((p0 - g->lo0) / SYN_CELL), q1 = (int)((p1 - g->lo1) / SYN_CELL);
    if (q0 >= g->n0) q0 = g->n0 - 1;
    if (q1 >= g->n1) q1 = g->n1 - 1;
    int c = q1 * g->n0 + q0;
    for (int e = g->start[c]; e < g->start[c + 1]; ++e) {
      const double* bl = bq + 4 * g->items[e];
      double d0 = p0 - bl[2], d1 = p1 - bl[3], s = bl[1];
      double d2 = d0 * d0 + d1 * d1 + dp * dp;
      if (d2 <= 16.0 * s * s) f += bl[0] * exp(-d2 / (2.0 * s * s));
    }
  }
  double pn[3] = {h[0] / noise_cell, h[1] / noise_cell, h[2] / noise_cell};
  f += noise_amp * syn_vnoise(seed, pn);
  return f;
}

/*
 * Render one view.
 *   blobs      [3][n_blobs][4] (amplitude, sigma, c0, c1) per plane
 *   windows    [3][4] blob-centre window per plane (lo0, hi0, lo1, hi1)
 *   T_cw       row-major 4x4 world -> camera
 *   noise      optional [H][W] additive noise (NULL = none)
 *   img        out [H][W] uint8
 *   depth      out [H][W] camera-frame z of the hit (NULL = skip); 0 if no hit
 * Returns the number of pixels without a hit.
 */
int syn_render(int32_t width, int32_t height, double fx, double fy, double cx, double cy,
               const double* T_cw, int32_t n_blobs, const double* blobs, const double* windows,
               uint64_t seed, double noise_amp, double noise_cell, const float* noise,
               uint8_t* img, double* depth) {
  syn_grid grids[SYN_PLANES];
  for (int p = 0; p < SYN_PLANES; ++p)
    syn_grid_build(&grids[p], blobs + (size_t)p * n_blobs * 4, n_blobs, windows + 4 * p);
  /* camera centre and rotation transpose */
  const double* T = T_cw;
  double Rt[9] = {T[0], T[4], T[8], T[1], T[5], T[9], T[2], T[6], T[10]};
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = -(Rt[3 * a + 0] * T[3] + Rt[3 * a + 1] * T[7] + Rt[3 * a + 2] * T[11]);
  int misses = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : misses)
  for (int v = 0; v < height; ++v) {
    for (int u = 0; u < width; ++u) {
      double rc[3] = {(u - cx) / fx, (v - cy) / fy, 1.0};
      double d[3];
      for (int a = 0; a < 3; ++a) d[a] = Rt[3 * a + 0] * rc[0] + Rt[3 * a + 1] * rc[1] + Rt[3 * a + 2] * rc[2];
      double best = INFINITY;
      int plane = -1;
      if (d[1] != 0.0) {
        double t = (-1.0 - o[1]) / d[1];
        if (t > 1e-9 && t < best) best = t, plane = 0;
      }
      if (d[2] != 0.0) {
        double t = (3.0 - o[2]) / d[2];
        if (t > 1e-9 && t < best) best = t, plane = 1;
      }
      if (d[0] != 0.0) {
        double t = (2.0 - o[0]) / d[0];
        if (t > 1e-9 && t < best) best = t, plane = 2;
      }
      size_t pix = (size_t)v * width + u;
      if (plane < 0) {
        misses++;
        img[pix] = 0;
        if (depth) depth[pix] = 0.0;
        continue;
      }
      double h[3] = {o[0] + best * d[0], o[1] + best * d[1], o[2] + best * d[2]};
      double f = syn_texture(grids, blobs, n_blobs, seed, noise_amp, noise_cell, h);
      if (noise) f += noise[pix];
      double q = rint(f);
      if (q < 0) q = 0;
      if (q > 255) q = 255;
      img[pix] = (uint8_t)q;
      if (depth) depth[pix] = best; /* ray camera-frame z component is 1 */
    }
  }
  for (int p = 0; p < SYN_PLANES; ++p) syn_grid_free(&grids[p]);
  return misses;
}
