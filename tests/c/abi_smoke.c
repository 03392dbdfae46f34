/* Plain-C use of libplbm (no Python, no PyTorch): a D3Q19 droplet on a
 * caller-owned hipMalloc buffer and the legacy null stream, 40 steps, checked
 * for the health flags and exact mass conservation (float64 storage), the
 * allocation-free reduction (plbm_reduce_static, equal to plbm_reduce), and the
 * error path of an undersized buffer.  Prints one line; exit status 0 on
 * success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "plbm.h"

int main(void) {
  if (plbm_abi_version() != PLBM_ABI_VERSION) {
    fprintf(stderr, "ABI version mismatch\n");
    return 1;
  }
  plbm_lattice_params prm;
  if (plbm_params_pr_lattice(0.8, 0.326, 2.0, 1.0, 1.0, 1.0, NULL, &prm) != PLBM_OK) {
    fprintf(stderr, "params: %s\n", plbm_last_error());
    return 1;
  }
  plbm_lattice_desc d;
  memset(&d, 0, sizeof(d));
  d.lattice = PLBM_D3Q19;
  d.collision = PLBM_MRT;
  d.storage = PLBM_F64;
  d.nx = 40;
  d.ny = 33;
  d.nz = 27;
  d.bc[0] = d.bc[1] = d.bc[2] = PLBM_PERIODIC;
  d.pattern = PLBM_PATTERN_AB;
  uint64_t bytes = 0;
  if (plbm_lattice_bytes(&d, &bytes) != PLBM_OK) {
    fprintf(stderr, "bytes: %s\n", plbm_last_error());
    return 1;
  }
  void* mem = NULL;
  if (hipMalloc(&mem, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  plbm_lattice* lat = NULL;
  /* an undersized buffer is refused with PLBM_E_NOMEM before anything is touched */
  if (plbm_create(&d, &prm, mem, bytes - 1, NULL, &lat) != PLBM_E_NOMEM || lat != NULL) {
    fprintf(stderr, "undersized buffer accepted\n");
    return 1;
  }
  if (plbm_create(&d, &prm, mem, bytes, NULL, &lat) != PLBM_OK) {
    fprintf(stderr, "create: %s\n", plbm_last_error());
    return 1;
  }
  plbm_shape s;
  memset(&s, 0, sizeof(s));
  s.kind = PLBM_SHAPE_DROPLET;
  s.rho_in = prm.rho_l;
  s.rho_out = prm.rho_v;
  s.W = 5.0;
  s.R = 8.0;
  s.centre[0] = 20.0;
  s.centre[1] = 16.5;
  s.centre[2] = 13.5;
  plbm_diag d0, d1, d2;
  if (plbm_init_shape(lat, &s) != PLBM_OK || plbm_reduce(lat, &d0) != PLBM_OK) {
    fprintf(stderr, "init: %s\n", plbm_last_error());
    return 1;
  }
  if (plbm_step(lat, 40) != PLBM_OK || plbm_reduce(lat, &d1) != PLBM_OK) {
    fprintf(stderr, "step: %s\n", plbm_last_error());
    return 1;
  }
  /* the same reduction from the library's static workspace: identical result */
  if (plbm_reduce_static(lat, &d2) != PLBM_OK) {
    fprintf(stderr, "reduce_static: %s\n", plbm_last_error());
    return 1;
  }
  const int same = d2.mass == d1.mass && d2.max_u == d1.max_u && d2.momentum[0] == d1.momentum[0] &&
                   d2.flags == d1.flags && d2.time == d1.time;
  int64_t t = 0;
  plbm_get_time(lat, &t);
  const double drift = fabs(d1.mass - d0.mass) / d0.mass;
  printf("c_abi t=%lld mass0=%.15e mass=%.15e drift=%.2e max_u=%.3e flags=%d static_equal=%d\n", (long long)t,
         d0.mass, d1.mass, drift, d1.max_u, d1.flags, same);
  plbm_destroy(lat);
  hipFree(mem);
  return (t == 40 && d1.flags == 0 && drift <= 1e-13 && d1.max_u > 0.0 && same) ? 0 : 1;
}
