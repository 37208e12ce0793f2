/* A C99 consumer of the PWF library, for the tests: reads one problem's
 * description, its measured intensity and its diffuser from files, runs
 * pwf_solve on the GPU and writes the retrieved field and the loss history.
 * The HIP runtime supplies only device memory and a stream; there is no C++
 * and no PyTorch on this path.
 *
 *   pwf_c_solve PARAMS Y T PSI_OUT LOSS_OUT
 *
 * PARAMS: text "nx ny pixel_m wavelength_m z1_m z2_m sigma_x_px sigma_y_px
 *          eta alpha_re alpha_im gamma precond_scale iters"
 * Y: float32 [ny][nx]; T: complex64 [ny][nx] (interleaved re, im)
 * PSI_OUT: complex64 [ny][nx]; LOSS_OUT: float64 [iters]
 * Exit status 0 on success, 1 on a usage or file error, 2 on a library or
 * HIP error (the message names it). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "pwf.h"

static int read_file(const char* path, void* dst, size_t bytes) {
  FILE* f = fopen(path, "rb");
  if (!f) return 1;
  const size_t got = fread(dst, 1, bytes, f);
  fclose(f);
  return got == bytes ? 0 : 1;
}

static int write_file(const char* path, const void* src, size_t bytes) {
  FILE* f = fopen(path, "wb");
  if (!f) return 1;
  const size_t put = fwrite(src, 1, bytes, f);
  fclose(f);
  return put == bytes ? 0 : 1;
}

#define HIP_OK(call)                                                    \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) {                                             \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
      return 2;                                                         \
    }                                                                   \
  } while (0)

#define PWF_OK_(call)                                                   \
  do {                                                                  \
    pwf_status s_ = (call);                                             \
    if (s_ != PWF_OK) {                                                 \
      fprintf(stderr, "%s: %s\n", #call, pwf_status_string(s_));        \
      return 2;                                                         \
    }                                                                   \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s PARAMS Y T PSI_OUT LOSS_OUT\n", argv[0]);
    return 1;
  }
  pwf_problem p;
  memset(&p, 0, sizeof(p));
  int iters = 0;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 1;
  const int n = fscanf(f, "%d %d %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %d", &p.geom.nx, &p.geom.ny,
                       &p.geom.pixel_m, &p.geom.wavelength_m, &p.geom.z1_m, &p.geom.z2_m, &p.source.sigma_x_px,
                       &p.source.sigma_y_px, &p.params.eta, &p.params.alpha_re, &p.params.alpha_im,
                       &p.params.gamma, &p.params.precond_scale, &iters);
  fclose(f);
  if (n != 14 || p.geom.nx <= 0 || p.geom.ny <= 0 || iters < 1) return 1;
  p.source.kind = PWF_SRC_GAUSS;
  p.params.precondition = 1;
  const size_t m = (size_t)p.geom.nx * (size_t)p.geom.ny;

  float* y_h = malloc(sizeof(float) * m);
  float* t_h = malloc(2 * sizeof(float) * m);
  float* psi_h = malloc(2 * sizeof(float) * m);
  double* loss_h = malloc(sizeof(double) * (size_t)iters);
  if (!y_h || !t_h || !psi_h || !loss_h) return 1;
  if (read_file(argv[2], y_h, sizeof(float) * m) || read_file(argv[3], t_h, 2 * sizeof(float) * m)) return 1;

  void *y_d, *t_d, *psi_d, *loss_d, *ws;
  hipStream_t st;
  HIP_OK(hipStreamCreate(&st));
  HIP_OK(hipMalloc(&y_d, sizeof(float) * m));
  HIP_OK(hipMalloc(&t_d, 2 * sizeof(float) * m));
  HIP_OK(hipMalloc(&psi_d, 2 * sizeof(float) * m));
  HIP_OK(hipMalloc(&loss_d, sizeof(double) * (size_t)iters));
  HIP_OK(hipMemcpy(y_d, y_h, sizeof(float) * m, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(t_d, t_h, 2 * sizeof(float) * m, hipMemcpyHostToDevice));
  p.diffuser = t_d;

  const size_t ws_bytes = pwf_workspace_size(&p, 1);
  if (ws_bytes == 0) {
    fprintf(stderr, "pwf_workspace_size: problem rejected\n");
    return 2;
  }
  HIP_OK(hipMalloc(&ws, ws_bytes));
  const float* ys[1] = {(const float*)y_d};
  void* outs[1] = {psi_d};
  int32_t done = 0;
  PWF_OK_(pwf_solve(&p, 1, ys, outs, iters, 0.0, (double*)loss_d, &done, ws, ws_bytes, st));
  HIP_OK(hipStreamSynchronize(st));
  PWF_OK_(pwf_sync_status(ws, st));
  HIP_OK(hipMemcpy(psi_h, psi_d, 2 * sizeof(float) * m, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(loss_h, loss_d, sizeof(double) * (size_t)iters, hipMemcpyDeviceToHost));
  if (write_file(argv[4], psi_h, 2 * sizeof(float) * m) || write_file(argv[5], loss_h, sizeof(double) * (size_t)iters))
    return 1;
  printf("pwf_c_solve: %d x %d, %d iterations, final loss %.6e\n", p.geom.nx, p.geom.ny, (int)done, loss_h[iters - 1]);
  HIP_OK(hipFree(ws));
  HIP_OK(hipFree(loss_d));
  HIP_OK(hipFree(psi_d));
  HIP_OK(hipFree(t_d));
  HIP_OK(hipFree(y_d));
  HIP_OK(hipStreamDestroy(st));
  free(y_h);
  free(t_h);
  free(psi_h);
  free(loss_h);
  return 0;
}
