/* A plain C99 client of the library, through include/adct16.h alone (no
 * Python, no PyTorch): the test suite compiles it with gcc and runs it.
 *
 *   abi_client host     status strings and argument validation; plan
 *                       creation reaches the device check (no GPU needed)
 *   abi_client device   on a gfx950 device: a lossless round trip (no
 *                       retention reconstructs every pixel, Section 4) through
 *                       the fused call and through forward + inverse
 *
 * Prints one line and exits 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "adct16.h"

static int failures = 0;

static void check(int ok, const char *what) {
  if (!ok) {
    printf("FAIL: %s (%s)\n", what, adct16_last_error_string());
    ++failures;
  }
}

static adct16_desc desc_of(const int32_t *h, const int32_t *w, const int32_t *p, const int64_t *o, int n) {
  adct16_desc d;
  memset(&d, 0, sizeof d);
  d.n_images = n;
  d.height = h;
  d.width = w;
  d.pitch = p;
  d.offset = o;
  d.in_dtype = ADCT16_U8;
  d.coef_dtype = ADCT16_I32;
  d.qcoef_dtype = ADCT16_I32;
  d.out_dtype = ADCT16_U8;
  d.qmode = ADCT16_Q_NONE;
  d.r = 16;
  d.q = 1;
  d.backend = ADCT16_BACKEND_AUTO;
  d.flags = 0;
  d.matrix = ADCT16_MATRIX_APPROX;
  return d;
}

static int host_checks(void) {
  int s;
  for (s = ADCT16_OK; s <= ADCT16_E_STATE; ++s) {
    const char *t = adct16_status_string((adct16_status)s);
    check(t != NULL && t[0] != '\0', "status string");
  }
  const int32_t h[1] = {64}, w[1] = {64}, p[1] = {64};
  const int64_t o[1] = {0};
  adct16_plan plan = NULL;
  check(adct16_plan_create(NULL, &plan) == ADCT16_E_NULL && plan == NULL, "NULL desc");
  adct16_desc d = desc_of(h, w, p, o, 1);
  check(adct16_plan_create(&d, NULL) == ADCT16_E_NULL, "NULL out");
  const int32_t h0[1] = {0};
  adct16_desc bad = desc_of(h0, w, p, o, 1);
  check(adct16_plan_create(&bad, &plan) == ADCT16_E_SHAPE, "zero height");
  bad = desc_of(h, w, p, o, 1);
  bad.qmode = ADCT16_Q_ZONAL;
  bad.r = 17;
  check(adct16_plan_create(&bad, &plan) == ADCT16_E_MODE, "zonal r = 17");
  const adct16_status st = adct16_plan_create(&d, &plan);
  check(st == ADCT16_OK || st == ADCT16_E_DEVICE, "valid desc");
  if (plan) adct16_plan_destroy(plan);
  double m[256];
  check(adct16_transform_matrix(ADCT16_MATRIX_T, m) == ADCT16_OK && m[0] == 1.0, "transform matrix");
  printf("abi_client host %s (valid desc: %s)\n", failures ? "FAILED" : "ok", adct16_status_string(st));
  return failures ? 1 : 0;
}

#define HIP_OK(call) check((call) == hipSuccess, #call)

static int device_checks(void) {
  /* two images: 40 x 50 (ragged in both directions) and 16 x 16 */
  const int32_t h[2] = {40, 16}, w[2] = {50, 16}, p[2] = {64, 16};
  const int64_t o[2] = {0, 40 * 64};
  const size_t bytes = (size_t)(40 * 64 + 16 * 16);
  unsigned char *host_in = (unsigned char *)malloc(bytes), *host_out = (unsigned char *)malloc(bytes);
  unsigned state = 12345u;
  size_t i;
  for (i = 0; i < bytes; ++i) {
    state = state * 1664525u + 1013904223u;
    host_in[i] = (unsigned char)(state >> 24);
  }
  adct16_desc d = desc_of(h, w, p, o, 2);
  adct16_plan plan = NULL;
  check(adct16_plan_create(&d, &plan) == ADCT16_OK, "plan_create");
  if (!plan) return 1;
  int64_t nb = 0;
  check(adct16_plan_num_blocks(plan, &nb) == ADCT16_OK && nb == 4 * 3 + 1, "num_blocks");
  void *d_in = NULL, *d_out = NULL, *d_coef = NULL;
  int64_t *d_sse = NULL;
  double *d_psnr = NULL;
  HIP_OK(hipMalloc(&d_in, bytes));
  HIP_OK(hipMalloc(&d_out, bytes));
  HIP_OK(hipMalloc(&d_coef, (size_t)nb * 256 * sizeof(int32_t)));
  HIP_OK(hipMalloc((void **)&d_sse, 2 * sizeof(int64_t)));
  HIP_OK(hipMalloc((void **)&d_psnr, 2 * sizeof(double)));
  HIP_OK(hipMemcpy(d_in, host_in, bytes, hipMemcpyHostToDevice));

  /* fused: reconstruction, SSE, PSNR */
  HIP_OK(hipMemset(d_out, 0, bytes));
  check(adct16_compress_and_measure(plan, d_in, d_out, NULL, d_sse, d_psnr, NULL) == ADCT16_OK, "fused call");
  HIP_OK(hipDeviceSynchronize());
  int64_t sse[2];
  double psnr[2];
  HIP_OK(hipMemcpy(host_out, d_out, bytes, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(sse, d_sse, sizeof sse, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(psnr, d_psnr, sizeof psnr, hipMemcpyDeviceToHost));
  int k, y, x, same = 1;
  for (k = 0; k < 2; ++k)
    for (y = 0; y < h[k]; ++y)
      for (x = 0; x < w[k]; ++x) same &= host_out[o[k] + (int64_t)y * p[k] + x] == host_in[o[k] + (int64_t)y * p[k] + x];
  check(same, "fused lossless reconstruction");
  check(sse[0] == 0 && sse[1] == 0, "fused SSE = 0");
  check(isinf(psnr[0]) && isinf(psnr[1]), "fused PSNR = +inf");

  /* unfused: forward, then inverse of every coefficient */
  HIP_OK(hipMemset(d_out, 0, bytes));
  check(adct16_forward(plan, d_in, d_coef, NULL) == ADCT16_OK, "forward");
  check(adct16_inverse(plan, d_coef, d_out, NULL) == ADCT16_OK, "inverse");
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(host_out, d_out, bytes, hipMemcpyDeviceToHost));
  same = 1;
  for (k = 0; k < 2; ++k)
    for (y = 0; y < h[k]; ++y)
      for (x = 0; x < w[k]; ++x) same &= host_out[o[k] + (int64_t)y * p[k] + x] == host_in[o[k] + (int64_t)y * p[k] + x];
  check(same, "forward + inverse lossless");
  /* DC of the 16 x 16 image (block 12): 256 times its mean pixel, exactly */
  int32_t z[256];
  HIP_OK(hipMemcpy(z, (const int32_t *)d_coef + 12 * 256, sizeof z, hipMemcpyDeviceToHost));
  int64_t sum = 0;
  for (y = 0; y < 16; ++y)
    for (x = 0; x < 16; ++x) sum += host_in[o[1] + y * 16 + x];
  check(z[0] == sum, "DC = sum of the block");

  adct16_plan_destroy(plan);
  (void)hipFree(d_in);
  (void)hipFree(d_out);
  (void)hipFree(d_coef);
  (void)hipFree(d_sse);
  (void)hipFree(d_psnr);
  free(host_in);
  free(host_out);
  printf("abi_client device %s\n", failures ? "FAILED" : "ok");
  return failures ? 1 : 0;
}

int main(int argc, char **argv) {
  if (argc > 1 && strcmp(argv[1], "device") == 0) return device_checks();
  return host_checks();
}
