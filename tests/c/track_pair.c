/* Plain C client of the C ABI (include/dptrack.h): tracks one frame against a
 * reference and its map points, with no Python in the process.  Test
 * infrastructure: tests/test_c_abi.py writes the job file and checks the
 * result against the oracle.
 *
 * Job file (native byte order): int32 W, H, levels, n; double fx, fy, cx, cy;
 * double T_rw[16], T_init[16]; uint8 ref[W*H], cur[W*H]; float xyz[n*3].
 * Output file: the dpt_result of dpt_track_frame, then that of a one-frame
 * window track of the same host frame from the same start.
 *
 * usage: track_pair JOB OUT */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dptrack.h"

static int check(int rc, const char* what) {
  if (rc != DPT_OK) fprintf(stderr, "%s failed (%d): %s\n", what, rc, dpt_last_error());
  return rc != DPT_OK;
}

static int read_all(FILE* f, void* dst, size_t bytes) { return fread(dst, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s JOB OUT\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) {
    perror(argv[1]);
    return 2;
  }
  int32_t hdr[4];
  double intr[4], T_rw[16], T_init[16];
  int ok = read_all(f, hdr, sizeof hdr) && read_all(f, intr, sizeof intr) && read_all(f, T_rw, sizeof T_rw) &&
           read_all(f, T_init, sizeof T_init);
  const int32_t W = hdr[0], H = hdr[1], levels = hdr[2], n = hdr[3];
  if (!ok || W <= 0 || H <= 0 || n < 0) {
    fprintf(stderr, "bad job header\n");
    fclose(f);
    return 2;
  }
  uint8_t* ref = (uint8_t*)malloc((size_t)W * H);
  uint8_t* cur = (uint8_t*)malloc((size_t)W * H);
  float* xyz = (float*)malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
  ok = ref && cur && xyz && read_all(f, ref, (size_t)W * H) && read_all(f, cur, (size_t)W * H) &&
       read_all(f, xyz, sizeof(float) * 3 * (size_t)n);
  fclose(f);
  if (!ok) {
    fprintf(stderr, "short job file\n");
    return 2;
  }

  dpt_camera cam = {W, H, intr[0], intr[1], intr[2], intr[3]};
  dpt_params prm;
  memset(&prm, 0, sizeof prm);
  prm.levels = levels;
  prm.max_iters = 10;
  prm.huber_k = 9.0f;
  prm.step_eps = 1e-5f;
  prm.z_min = 1e-3f;
  prm.min_points = 10;
  static const int32_t diamond[16] = {-2, 0, 2, 0, 0, -2, 0, 2, -1, -1, 1, -1, -1, 1, 1, 1};
  prm.n_pattern = 8;
  for (int k = 0; k < 16; ++k) prm.pattern[k] = diamond[k];
  prm.precision = DPT_PREC_FP32;
  prm.flags = 0;

  dpt_ctx* ctx = NULL;
  dpt_result res, win;
  int rc = 1;
  if (check(dpt_create(&cam, &prm, n > 0 ? n : 1, NULL, &ctx), "dpt_create")) goto done;
  if (check(dpt_build_pyramid(ctx, DPT_SLOT_REF, ref, W, 0), "dpt_build_pyramid(REF)")) goto done;
  if (check(dpt_set_reference_points(ctx, xyz, n, T_rw, 0), "dpt_set_reference_points")) goto done;
  if (check(dpt_build_pyramid(ctx, DPT_SLOT_CUR, cur, W, 0), "dpt_build_pyramid(CUR)")) goto done;
  if (check(dpt_track_frame(ctx, T_init, &res), "dpt_track_frame")) goto done;
  if (check(dpt_track_window_enqueue(ctx, cur, W, (int64_t)W * H, 1, 0, DPT_INIT_GIVEN, T_init, &win),
            "dpt_track_window_enqueue") ||
      check(dpt_synchronize(ctx), "dpt_synchronize"))
    goto done;
  f = fopen(argv[2], "wb");
  if (!f || fwrite(&res, sizeof res, 1, f) != 1 || fwrite(&win, sizeof win, 1, f) != 1) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    if (f) fclose(f);
    goto done;
  }
  fclose(f);
  printf("status %d iterations %d final_cost %.6f t = (%.6f, %.6f, %.6f)\n", res.status, res.iterations,
         res.final_cost, res.T_cw[3], res.T_cw[7], res.T_cw[11]);
  rc = 0;
done:
  if (ctx) dpt_destroy(ctx);
  free(ref);
  free(cur);
  free(xyz);
  return rc;
}
