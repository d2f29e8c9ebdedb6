/* A plain C caller of libpf (no Python, no HIP calls of its own): host arrays
 * in, host arrays out.  Reads c and eta (float64, [4][n^3]) from argv[2],
 * advances by IMEX Euler (dt 0.05) to t = 0.15 on an n^3 grid (n = argv[1]),
 * writes the final state to argv[3] and prints the step count.  Exit status 0
 * on success, otherwise the failing call's pf_status. */
#include <stdio.h>
#include <stdlib.h>

#include "pf.h"

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const int n = atoi(argv[1]);
  const size_t np = (size_t)n * n * n;
  double* u = (double*)malloc(4 * np * sizeof(double));
  if (!u) return 3;
  FILE* f = fopen(argv[2], "rb");
  if (!f || fread(u, sizeof(double), 4 * np, f) != 4 * np) return 4;
  fclose(f);
  pf_params p;
  pf_status s = pf_default_params(&p);
  if (s != PF_OK) return (int)-s;
  p.nx = p.ny = p.nz = n;
  p.method = PF_IMEX_EULER;
  p.adaptive = 0;
  p.dt0 = 0.05;
  pf_ctx* ctx = NULL;
  if ((s = pf_init(&p, NULL, &ctx)) != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", pf_status_string(s));
    return 10;
  }
  if ((s = pf_set_state(ctx, u, u + np, 0, 0.0)) != PF_OK) return 11;
  pf_stats st;
  if ((s = pf_advance(ctx, 0.15, &st)) != PF_OK) return 12;
  if ((s = pf_get_state(ctx, u, u + np, 0)) != PF_OK) return 13;
  pf_finalize(ctx);
  f = fopen(argv[3], "wb");
  if (!f || fwrite(u, sizeof(double), 4 * np, f) != 4 * np) return 5;
  fclose(f);
  printf("%lld\n", (long long)st.steps);
  free(u);
  return 0;
}
