/* A plain C99 client of libmabd: reads an assembly from a binary file, steps
   it through the C ABI only and writes the state and multipliers.  Built and
   run by tests/test_gpu_c_client.py, which compares its output with the
   Python binding's on the same input.

   Input file: int32 n, m, nsteps; double h; then dims (n*3), density (n),
   k_orth (n), pinned (n bytes), q0 (n*12), qd0 (n*12), type (m bytes), a (m
   int32), b (m int32), pa (m*3), pb (m*3), axis (m*3), cp_len (m), axis2
   (m*3).  Output file: int32 status, rows (int32); q (n*12), qd (n*12), lam (rows),
   then five doubles of mabd_residual. */
#include <stdio.h>
#include <stdlib.h>

#include "mabd.h"

static void *readn(FILE *f, size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[3];
  double h;
  if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&h, sizeof h, 1, f) != 1) return 2;
  const int32_t n = hdr[0], m = hdr[1], nsteps = hdr[2];
  mabd_bodies B;
  mabd_joints J;
  B.n = n;
  B.dims = readn(f, sizeof(double) * 3 * n);
  B.density = readn(f, sizeof(double) * n);
  B.k_orth = readn(f, sizeof(double) * n);
  B.poisson = NULL;
  B.pinned = readn(f, n);
  B.q0 = readn(f, sizeof(double) * 12 * n);
  B.qd0 = readn(f, sizeof(double) * 12 * n);
  J.m = m;
  J.type = readn(f, m);
  J.a = readn(f, sizeof(int32_t) * m);
  J.b = readn(f, sizeof(int32_t) * m);
  J.pa = readn(f, sizeof(double) * 3 * m);
  J.pb = readn(f, sizeof(double) * 3 * m);
  J.axis = readn(f, sizeof(double) * 3 * m);
  J.cp_len = readn(f, sizeof(double) * m);
  J.axis2 = readn(f, sizeof(double) * 3 * m);
  fclose(f);

  mabd_options opt;
  mabd_options_default(&opt);
  mabd_ctx *ctx = NULL;
  mabd_status st = mabd_create(&B, &J, &opt, &ctx);
  if (st != MABD_OK) {
    fprintf(stderr, "create: %s\n", mabd_last_error(NULL));
    return 3;
  }
  st = mabd_step(ctx, h, nsteps);
  double *q = malloc(sizeof(double) * 12 * n), *qd = malloc(sizeof(double) * 12 * n);
  const int64_t rows = mabd_rows(ctx);
  double *lam = malloc(sizeof(double) * (rows > 0 ? rows : 1));
  double res[5] = {0, 0, 0, 0, 0};
  if (st == MABD_OK) st = mabd_state(ctx, q, qd);
  if (st == MABD_OK) st = mabd_multipliers(ctx, lam);
  if (st == MABD_OK) st = mabd_residual(ctx, res);
  if (st != MABD_OK) fprintf(stderr, "step: %s\n", mabd_last_error(ctx));
  mabd_destroy(ctx);

  FILE *o = fopen(argv[2], "wb");
  if (!o) return 2;
  const int32_t out_hdr[2] = {(int32_t)st, (int32_t)rows};
  fwrite(out_hdr, sizeof out_hdr, 1, o);
  fwrite(q, sizeof(double), 12 * (size_t)n, o);
  fwrite(qd, sizeof(double), 12 * (size_t)n, o);
  fwrite(lam, sizeof(double), (size_t)rows, o);
  fwrite(res, sizeof(double), 5, o);
  fclose(o);
  return st == MABD_OK ? 0 : 1;
}
