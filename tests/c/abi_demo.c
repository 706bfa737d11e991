/* A plain C caller of the library: reads a problem written by the test
 * (raw little-endian arrays in a directory), builds the hierarchy from host
 * arrays, solves, checks the commuting relation on every level and writes u.
 * Usage: abi_demo DIR.  Prints "levels iters relres commute_rel". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hcurl_amg.h"

static void* load(const char* dir, const char* name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
  void* p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
  fclose(f);
  return p;
}

int main(int argc, char** argv) {
  if (argc != 2) { fprintf(stderr, "usage: %s DIR\n", argv[0]); return 2; }
  const char* dir = argv[1];
  int64_t* meta = (int64_t*)load(dir, "meta.bin", 4 * sizeof(int64_t));
  const int64_t n = meta[0], m = meta[1], nnz = meta[2], mH = meta[3];
  hcurl_csr A = {n, n, nnz, (const int64_t*)load(dir, "A_rowptr.bin", (n + 1) * 8),
                 (const int32_t*)load(dir, "A_col.bin", nnz * 4), (const double*)load(dir, "A_val.bin", nnz * 8)};
  hcurl_csr D = {n, m, 2 * n, (const int64_t*)load(dir, "D_rowptr.bin", (n + 1) * 8),
                 (const int32_t*)load(dir, "D_col.bin", 2 * n * 4), (const double*)load(dir, "D_val.bin", 2 * n * 8)};
  const int32_t* agg = (const int32_t*)load(dir, "agg.bin", m * 4);
  const double* f = (const double*)load(dir, "f.bin", n * 8);
  (void)mH;
  hcurl_amg_opts o;
  hcurl_amg_default_opts(&o);
  hcurl_amg h = NULL;
  const int32_t* maps[1] = {agg};
  int rc = hcurl_amg_setup(&A, &D, NULL, maps, 1, &o, &h);
  if (rc != HCURL_OK) { fprintf(stderr, "setup: %s (%s)\n", hcurl_error_string(rc), hcurl_last_error()); return 1; }
  double* u = (double*)malloc(n * 8);
  int iters = 0;
  double relres = 0.0;
  rc = hcurl_amg_solve(h, f, u, 1e-8, 500, &iters, &relres);
  if (rc != HCURL_OK) { fprintf(stderr, "solve: %s (%s)\n", hcurl_error_string(rc), hcurl_last_error()); return 1; }
  const int levels = hcurl_amg_num_levels(h);
  double worst = 0.0;
  for (int l = 0; l + 1 < levels; ++l) {
    double a = 0.0, r = 0.0;
    rc = hcurl_amg_commute_residual(h, l, &a, &r);
    if (rc != HCURL_OK) { fprintf(stderr, "commute: %s\n", hcurl_last_error()); return 1; }
    if (a / r > worst) worst = a / r;
  }
  /* a level past the last is refused */
  hcurl_level_info info;
  if (hcurl_amg_level_info(h, levels, &info) != HCURL_EINVAL) { fprintf(stderr, "level check\n"); return 1; }
  hcurl_amg_destroy(h);
  char path[4096];
  snprintf(path, sizeof path, "%s/u.bin", dir);
  FILE* out = fopen(path, "wb");
  if (!out || fwrite(u, 8, n, out) != (size_t)n) { fprintf(stderr, "cannot write u\n"); return 2; }
  fclose(out);
  printf("%d %d %.17g %.17g\n", levels, iters, relres, worst);
  return 0;
}
