/*
 * The C ABI without Python or PyTorch: a periodic cuboid Taylor-Green run.
 *
 *   c_taylor_green NX NY NZ STEPS U_FILE [U_OUT]
 *
 * U_FILE holds the initial velocity as raw float64 [3][NZ][NY][NX] (SoA, x
 * fastest).  The program allocates two FP32 states and the fields with the
 * HIP runtime, runs lbm_init, STEPS steps of lbm_step and lbm_moments, and
 * prints the five FP64 totals (mass, momentum x/y/z, kinetic energy) on one
 * line; with U_OUT it also writes the final velocity field there as raw
 * float32 [3][NZ][NY][NX].  Grid spacing r = 1, s = 1/2, cs2 = 1/12,
 * nu = xi = 0.016 (eq. 53), local corrections (Sec. 2.4).
 *
 * Build (host compiler only):
 *   gcc -std=c11 -O2 -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include -Iinclude \
 *       examples/c_taylor_green.c -Lpaper_2107_14774_amd -llbm -L/opt/rocm/lib -lamdhip64 \
 *       -Wl,-rpath,$PWD/paper_2107_14774_amd -Wl,-rpath,/opt/rocm/lib -o c_taylor_green
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define HIP_OK(call)                                                           \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));               \
      return 2;                                                                \
    }                                                                          \
  } while (0)

#define LBM_OK(call)                                                           \
  do {                                                                         \
    int s_ = (call);                                                           \
    if (s_ != LBM_OK) {                                                        \
      fprintf(stderr, "%s: status %d: %s\n", #call, s_, lbm_last_error());     \
      return 3;                                                                \
    }                                                                          \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 6 && argc != 7) {
    fprintf(stderr, "usage: %s NX NY NZ STEPS U_FILE [U_OUT]\n", argv[0]);
    return 1;
  }
  const int nx = atoi(argv[1]), ny = atoi(argv[2]), nz = atoi(argv[3]), steps = atoi(argv[4]);
  const size_t n = (size_t)nx * ny * nz;

  lbm_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx; p.ny = ny; p.nz = nz;
  p.r = 1.0; p.s = 0.5; p.cs2 = 1.0 / 12.0;
  const double nu = 0.016;
  p.omega_nu = 1.0 / (nu / p.cs2 + 0.5);              /* eq. 53 */
  p.omega_xi = 1.0 / (1.5 * nu / p.cs2 + 0.5);        /* xi = nu */
  p.omega_hi = 1.0;
  p.bc_x = p.bc_y = p.bc_z = LBM_PERIODIC;
  p.storage = LBM_F32;
  p.corr = LBM_CORR_LOCAL;
  p.moments = LBM_CENTRAL;
  p.layout = LBM_LAYOUT_AB;
  p.rho0 = 1.0;

  double* u_host = (double*)malloc(3 * n * sizeof(double));
  FILE* f = fopen(argv[5], "rb");
  if (!f || fread(u_host, sizeof(double), 3 * n, f) != 3 * n) {
    fprintf(stderr, "cannot read %zu doubles from %s\n", 3 * n, argv[5]);
    return 1;
  }
  fclose(f);

  lbm_handle* h = NULL;
  LBM_OK(lbm_create(&p, &h));
  const size_t bytes = lbm_state_bytes(h);
  void *a = NULL, *b = NULL;
  double *u = NULL, *sums = NULL;
  float* u_out = NULL;
  HIP_OK(hipMalloc(&a, bytes));
  HIP_OK(hipMalloc(&b, bytes));
  HIP_OK(hipMalloc((void**)&u, 3 * n * sizeof(double)));
  HIP_OK(hipMalloc((void**)&sums, 5 * sizeof(double)));
  HIP_OK(hipMalloc((void**)&u_out, 3 * n * sizeof(float)));
  HIP_OK(hipMemcpy(u, u_host, 3 * n * sizeof(double), hipMemcpyHostToDevice));

  hipStream_t stream;
  HIP_OK(hipStreamCreate(&stream));
  LBM_OK(lbm_init(h, a, NULL, u, NULL, stream));
  LBM_OK(lbm_step(h, steps, a, b, NULL, stream));
  void* cur = (steps % 2 == 0) ? a : b;
  LBM_OK(lbm_moments(h, cur, NULL, NULL, u_out, sums, stream));
  double out[5];
  LBM_OK(lbm_check_sums(sums, out, stream));           /* synchronises the stream */
  printf("%.17g %.17g %.17g %.17g %.17g\n", out[0], out[1], out[2], out[3], out[4]);
  if (argc == 7) {
    float* host = (float*)malloc(3 * n * sizeof(float));
    HIP_OK(hipMemcpy(host, u_out, 3 * n * sizeof(float), hipMemcpyDeviceToHost));
    FILE* g = fopen(argv[6], "wb");
    if (!g || fwrite(host, sizeof(float), 3 * n, g) != 3 * n) {
      fprintf(stderr, "cannot write %s\n", argv[6]);
      return 1;
    }
    fclose(g);
    free(host);
  }

  HIP_OK(hipStreamDestroy(stream));
  HIP_OK(hipFree(a));
  HIP_OK(hipFree(b));
  HIP_OK(hipFree(u));
  HIP_OK(hipFree(sums));
  HIP_OK(hipFree(u_out));
  lbm_destroy(h);
  free(u_host);
  return 0;
}
