/* Drives the gapsim C ABI from plain C (no Python, no PyTorch): reads one gap's
 * parameters (a gs_gap_params as bytes) and its initial particles from files,
 * runs strict or weak steps on the default stream with the library's own
 * allocator, and prints the diagnostics of every level.  Used by the tests. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gapsim.h"

static int read_all(const char *path, void **buf, long *len) {
  FILE *f = fopen(path, "rb");
  if (!f) return -1;
  fseek(f, 0, SEEK_END);
  *len = ftell(f);
  fseek(f, 0, SEEK_SET);
  *buf = malloc((size_t)*len + 1);
  if (!*buf || fread(*buf, 1, (size_t)*len, f) != (size_t)*len) {
    fclose(f);
    return -1;
  }
  fclose(f);
  return 0;
}

int main(int argc, char **argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: abi_run PARAMS PARTICLES MODE(0 strict, 1 weak) STEPS\n");
    return 2;
  }
  void *pb = NULL, *qb = NULL;
  long pl = 0, ql = 0;
  if (read_all(argv[1], &pb, &pl) || pl != (long)sizeof(gs_gap_params)) {
    fprintf(stderr, "bad parameter file (%ld bytes, want %zu)\n", pl, sizeof(gs_gap_params));
    return 2;
  }
  gs_gap_params p;
  memcpy(&p, pb, sizeof p);
  p.beam_schedule = NULL;
  p.beam_schedule_len = 0;
  char msg[256];
  if (gs_validate_params(&p, msg, sizeof msg) != GS_OK) {
    fprintf(stderr, "invalid parameters: %s\n", msg);
    return 2;
  }
  gs_ctx *ctx = NULL;
  gs_status st = gs_init_gap(&ctx, 1, &p, NULL, NULL);
  if (st != GS_OK) {
    fprintf(stderr, "gs_init_gap: %d %s\n", (int)st, gs_last_error(NULL));
    return 1;
  }
  /* particle file: for species 0 then 1, an int64 count n and n x then n v (binary64) */
  if (read_all(argv[2], &qb, &ql)) return 2;
  const char *cur = (const char *)qb;
  for (int sp = 0; sp < 2; ++sp) {
    int64_t n;
    memcpy(&n, cur, 8);
    cur += 8;
    const double *x = (const double *)cur, *v = x + n;
    if ((st = gs_inject(ctx, 0, sp, n, x, v, 0)) != GS_OK) {
      fprintf(stderr, "gs_inject: %d %s\n", (int)st, gs_last_error(ctx));
      return 1;
    }
    cur += 16 * n;
  }
  const int mode = atoi(argv[3]), steps = atoi(argv[4]);
  for (int k = 0; k < steps; ++k) {
    st = mode == 0 ? gs_step_strict(ctx, 1, GS_GUESS_DIRECT) : gs_step_weak(ctx, 1);
    gs_diag d;
    if (st == GS_OK) st = gs_read_diagnostics(ctx, 0, &d, NULL, NULL, NULL);
    if (st != GS_OK) {
      fprintf(stderr, "step %d: %d %s\n", k, (int)st, gs_last_error(ctx));
      return 1;
    }
    printf("%lld %.17g %.17g %.17g %lld %lld %lld %lld %lld %lld %lld\n", (long long)d.step, d.phi0, d.sigma,
           d.qcirc, (long long)d.abs_cum[0][0], (long long)d.abs_cum[0][1], (long long)d.abs_cum[1][0],
           (long long)d.abs_cum[1][1], (long long)d.emit_cum[0], (long long)d.emit_cum[1],
           (long long)(d.n_live[0] + d.n_live[1]));
  }
  gs_destroy(ctx);
  free(pb);
  free(qb);
  return 0;
}
