/* One gradient evaluation through the C ABI alone, without Python or torch: reads a problem
 * (n, p, K, then X float32 n x p, labels int32 n, B float32 p x K) from a binary file, puts
 * it in device memory with the HIP runtime, calls hmc_logpost_grad (equations (logkernel)
 * and (fullgrad)) and writes log K (float64) and G (float32 p x K). It also checks that a
 * workspace one byte short is refused on the host with HMC_ERR_WORKSPACE. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hmc.h"

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                 \
      return 2;                                                                \
    }                                                                          \
  } while (0)

static int read_all(FILE* f, void* dst, size_t bytes) { return fread(dst, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s problem.bin result.bin\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  int64_t hdr[3];
  if (!f || !read_all(f, hdr, sizeof hdr)) return 2;
  const int64_t n = hdr[0], p = hdr[1], K = hdr[2];
  const size_t xb = (size_t)(n * p) * sizeof(float), yb = (size_t)n * sizeof(int32_t),
               bb = (size_t)(p * K) * sizeof(float);
  float* X = malloc(xb);
  int32_t* y = malloc(yb);
  float* B = malloc(bb);
  float* G = malloc(bb);
  if (!X || !y || !B || !G || !read_all(f, X, xb) || !read_all(f, y, yb) || !read_all(f, B, bb))
    return 2;
  fclose(f);

  void *dX, *dy, *dB, *dG, *ws;
  double* dlogk;
  double logk = 0.0;
  HIP_OK(hipMalloc(&dX, xb));
  HIP_OK(hipMalloc(&dy, yb));
  HIP_OK(hipMalloc(&dB, bb));
  HIP_OK(hipMalloc(&dG, bb));
  HIP_OK(hipMalloc((void**)&dlogk, sizeof(double)));
  HIP_OK(hipMemcpy(dX, X, xb, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dy, y, yb, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dB, B, bb, hipMemcpyHostToDevice));

  hmc_problem prob;
  memset(&prob, 0, sizeof prob);
  prob.n = n;
  prob.p = p;
  prob.K = (int32_t)K;
  prob.xfmt = HMC_X_F32;
  prob.X = dX;
  prob.X_lo = NULL;
  prob.ldx = p;
  prob.y = dy;
  prob.prior = HMC_PRIOR_GAUSS;
  prob.prior_scale = 1.0;
  prob.pin_last_class = 1;
  size_t ws_bytes = 0;
  hmc_status st = hmc_workspace_bytes(&prob, &ws_bytes);
  if (st != HMC_OK) {
    fprintf(stderr, "hmc_workspace_bytes: %s (%s)\n", hmc_status_string(st), hmc_last_error());
    return 1;
  }
  HIP_OK(hipMalloc(&ws, ws_bytes));
  st = hmc_logpost_grad(&prob, dB, dlogk, dG, ws, ws_bytes - 1, NULL);
  if (st != HMC_ERR_WORKSPACE) {
    fprintf(stderr, "a short workspace gave %s\n", hmc_status_string(st));
    return 1;
  }
  st = hmc_logpost_grad(&prob, dB, dlogk, dG, ws, ws_bytes, NULL);
  if (st != HMC_OK) {
    fprintf(stderr, "hmc_logpost_grad: %s (%s)\n", hmc_status_string(st), hmc_last_error());
    return 1;
  }
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(&logk, dlogk, sizeof(double), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(G, dG, bb, hipMemcpyDeviceToHost));
  f = fopen(argv[2], "wb");
  if (!f || fwrite(&logk, sizeof logk, 1, f) != 1 || fwrite(G, 1, bb, f) != bb) return 2;
  fclose(f);
  printf("workspace %zu bytes, log K %.17g\n", ws_bytes, logk);
  HIP_OK(hipFree(ws));
  HIP_OK(hipFree(dlogk));
  HIP_OK(hipFree(dG));
  HIP_OK(hipFree(dB));
  HIP_OK(hipFree(dy));
  HIP_OK(hipFree(dX));
  free(X);
  free(y);
  free(B);
  free(G);
  return 0;
}
