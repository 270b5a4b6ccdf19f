/* A caller of the C ABI of include/crkdg.h with no Python and no torch: device
 * memory from hipMalloc, the default stream.  2D Euler, Q^2, 3-stage cRKDG on
 * a periodic 48 x 40 mesh in FP64: the cell averages are read from argv[1]
 * (V x Nc doubles, variable-major), limited, stepped `steps` times with
 * crkdg_step, and the final averages and the reached time are written to
 * argv[2].  Exit status 0 on success; any error is printed with
 * crkdg_last_error(). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "crkdg.h"

#define HIP(x)                                                              \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) {                                                 \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
      return 2;                                                             \
    }                                                                       \
  } while (0)
#define LIB(x)                                                              \
  do {                                                                      \
    int r_ = (x);                                                           \
    if (r_ < 0) {                                                           \
      fprintf(stderr, "%s returned %d: %s\n", #x, r_, crkdg_last_error()); \
      return 3;                                                             \
    }                                                                       \
  } while (0)

int main(int argc, char **argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: %s averages_in averages_out steps\n", argv[0]);
    return 1;
  }
  const int steps = atoi(argv[3]);
  crkdg_problem p;
  memset(&p, 0, sizeof p);
  p.dim = 2;
  p.n[0] = 48;
  p.n[1] = 40;
  p.n[2] = 1;
  for (int d = 0; d < 3; ++d) {
    p.lo[d] = 0.0;
    p.hi[d] = 1.0;
    p.bc[d] = CRKDG_BC_PERIODIC;
    p.vel[d] = 0.0;
  }
  p.system = CRKDG_SYS_EULER;
  p.gamma = 1.4;
  p.bound_lo = -INFINITY;
  p.bound_hi = INFINITY;
  p.eps = 1e-8;
  p.k = 2;
  p.space = CRKDG_SPACE_Q;
  p.stages = 3;
  p.precision = CRKDG_FP64;
  p.limiter = 1;
  p.cfl = 0.15;
  p.max_halvings = 40;
  p.scheme = CRKDG_SCHEME_CRKDG;

  crkdg_mesh *mesh = NULL;
  crkdg_layout lay;
  LIB(crkdg_init_mesh(&p, 1, &mesh, &lay));
  const int64_t nc = (int64_t)p.n[0] * p.n[1];
  const int V = 4;

  double *host = (double *)malloc(sizeof(double) * V * nc);
  FILE *f = fopen(argv[1], "rb");
  if (!f || fread(host, sizeof(double), V * nc, f) != (size_t)(V * nc)) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 1;
  }
  fclose(f);

  crkdg_state slots[8];
  for (int i = 0; i < lay.n_slots; ++i) {
    HIP(hipMalloc((void **)&slots[i].avg, sizeof(double) * lay.avg_elems));
    HIP(hipMalloc(&slots[i].hi, (size_t)lay.hi_bytes * lay.hi_elems));
    HIP(hipMemset(slots[i].hi, 0, (size_t)lay.hi_bytes * lay.hi_elems));
  }
  HIP(hipMemcpy(slots[0].avg, host, sizeof(double) * V * nc, hipMemcpyHostToDevice));
  crkdg_ctl *ctl = NULL;
  HIP(hipMalloc((void **)&ctl, lay.ctl_bytes));
  HIP(hipMemset(ctl, 0, lay.ctl_bytes));

  LIB(crkdg_limit(mesh, slots[0], ctl, NULL));
  const double t0 = 0.0;
  LIB(crkdg_start(mesh, slots, 0, ctl, &t0, NULL, NULL, NULL));
  crkdg_step_info info;
  memset(&info, 0, sizeof info);
  for (int n = 0; n < steps; ++n) {
    LIB(crkdg_step(mesh, slots, lay.n_slots, ctl, &info, NULL));
    if (info.status != 0) {
      fprintf(stderr, "step %d: status %d\n", n, info.status);
      return 4;
    }
  }
  HIP(hipMemcpy(host, slots[info.cur].avg, sizeof(double) * V * nc, hipMemcpyDeviceToHost));
  f = fopen(argv[2], "wb");
  if (!f) return 1;
  fwrite(host, sizeof(double), V * nc, f);
  fwrite(&info.t, sizeof(double), 1, f);
  fclose(f);
  printf("%d steps, t = %.17g, dt = %.17g\n", steps, info.t, info.dt);

  HIP(hipFree(ctl));
  for (int i = 0; i < lay.n_slots; ++i) {
    HIP(hipFree(slots[i].avg));
    HIP(hipFree(slots[i].hi));
  }
  LIB(crkdg_free_mesh(mesh));
  free(host);
  return 0;
}
