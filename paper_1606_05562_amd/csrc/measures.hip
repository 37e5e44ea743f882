// Host-side library functions: the 16-point transform matrices and the
// similarity and coding measures of Section 3 (the quantities of Table 2).
// No device is involved; these are plain float64 computations on 16x16
// matrices.
#include <math.h>
#include <string.h>

#include "adct16.h"

namespace {

constexpr int N = 16;

// Section 2: the {0, +1, -1} matrix of the proposed transform.
constexpr signed char kTHost[N][N] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, 1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1, -1, -1},
    {1, 1, 1, 0, 0, -1, -1, -1, -1, -1, -1, 0, 0, 1, 1, 1},
    {1, 1, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, -1, -1},
    {1, 0, 0, -1, -1, 0, 0, 1, 1, 0, 0, -1, -1, 0, 0, 1},
    {1, 1, -1, -1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1},
    {1, 0, -1, -1, 1, 1, 0, -1, -1, 0, 1, 1, -1, -1, 0, 1},
    {0, 0, -1, 1, 1, -1, -1, 1, -1, 1, 1, -1, -1, 1, 0, 0},
    {1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1},
    {1, -1, -1, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, 1, -1},
    {1, -1, 0, 1, -1, 0, 1, -1, -1, 1, 0, -1, 1, 0, -1, 1},
    {0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0},
    {0, -1, 1, 0, 0, 1, -1, 0, 0, -1, 1, 0, 0, 1, -1, 0},
    {1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1},
    {0, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1, 1, -1, 1, -1, 0},
    {1, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1},
};

// Orthonormal DCT-II: C[k][m] = a_k cos(pi (2m + 1) k / 32), a_0 = 1/4,
// a_k = 1/sqrt(8).
void dct2(double (&c)[N][N]) {
  for (int k = 0; k < N; ++k)
    for (int m = 0; m < N; ++m)
      c[k][m] = (k == 0 ? 0.25 : 1.0 / sqrt(8.0)) * cos(M_PI * (2 * m + 1) * k / (2.0 * N));
}


}  // namespace

// The error text is kept by the main API translation unit.
namespace adct16 {
void set_last_error(const char* msg);
}

extern "C" {

adct16_status adct16_transform_matrix(int32_t which, double* m) {
  if (!m) {
    adct16::set_last_error("m is NULL");
    return ADCT16_E_NULL;
  }
  double c[N][N];
  switch (which) {
    case ADCT16_MATRIX_APPROX:
      // C_hat = S T with S = diag(1 / sqrt(n_i)), n_i the squared row norms.
      for (int i = 0; i < N; ++i) {
        int n = 0;
        for (int j = 0; j < N; ++j) n += kTHost[i][j] * kTHost[i][j];
        for (int j = 0; j < N; ++j) c[i][j] = kTHost[i][j] / sqrt((double)n);
      }
      break;
    case ADCT16_MATRIX_T:
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) c[i][j] = kTHost[i][j];
      break;
    case ADCT16_MATRIX_WHT:
      // Walsh-Hadamard in natural (Sylvester) order: H[i][j] = (-1)^popcount(i & j), / 4.
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) c[i][j] = (__builtin_popcount(i & j) & 1 ? -1.0 : 1.0) / 4.0;
      break;
    case ADCT16_MATRIX_DCT:
      dct2(c);
      break;
    default:
      adct16::set_last_error("unknown matrix");
      return ADCT16_E_MODE;
  }
  memcpy(m, c, sizeof c);
  return ADCT16_OK;
}

adct16_status adct16_transform_measures(const double* ct, double rho, double* out) {
  if (!ct || !out) {
    adct16::set_last_error("ct / out is NULL");
    return ADCT16_E_NULL;
  }
  if (!(rho > 0.0 && rho < 1.0)) {
    adct16::set_last_error("rho must lie in (0, 1)");
    return ADCT16_E_MODE;
  }
  double a[N][N], c[N][N], r[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      a[i][j] = ct[i * N + j];
      if (!isfinite(a[i][j])) {
        adct16::set_last_error("ct holds a non-finite entry");
        return ADCT16_E_MODE;
      }
    }
  dct2(c);
  // Section 3.2: first-order Markov covariance R_ij = rho^|i - j|.
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r[i][j] = pow(rho, fabs((double)(i - j)));

  // DCT distortion d2 = 1 - (1/N) sum_i (C ct^T)_ii^2.
  double dsum = 0.0;
  for (int i = 0; i < N; ++i) {
    double d = 0.0;
    for (int k = 0; k < N; ++k) d += c[i][k] * a[i][k];
    dsum += d * d;
  }
  const double d2 = 1.0 - dsum / N;

  // Total error energy pi ||C - ct||_F^2 and MSE (1/N) tr((C - ct) R (C - ct)^T).
  double e[N][N], fro = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      e[i][j] = c[i][j] - a[i][j];
      fro += e[i][j] * e[i][j];
    }
  double tr = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) tr += e[i][j] * r[j][k] * e[i][k];

  // Section 3.3: s = ct R ct^T; coding gain and transform efficiency.
  double s[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double v = 0.0;
      for (int k = 0; k < N; ++k)
        for (int l = 0; l < N; ++l) v += a[i][k] * r[k][l] * a[j][l];
      s[i][j] = v;
    }
  double trace = 0.0, logprod = 0.0, diag_abs = 0.0, all_abs = 0.0;
  for (int i = 0; i < N; ++i) {
    double norm2 = 0.0;
    for (int j = 0; j < N; ++j) norm2 += a[i][j] * a[i][j];
    if (!(s[i][i] > 0.0) || !(norm2 > 0.0)) {
      adct16::set_last_error("ct has a zero row");
      return ADCT16_E_MODE;
    }
    trace += s[i][i];
    logprod += log(s[i][i] * sqrt(norm2));
    diag_abs += fabs(s[i][i]);
    for (int j = 0; j < N; ++j) all_abs += fabs(s[i][j]);
  }
  out[0] = d2;
  out[1] = M_PI * fro;
  out[2] = tr / N;
  out[3] = 10.0 * log10((trace / N) / exp(logprod / N));
  out[4] = diag_abs / all_abs * 100.0;
  return ADCT16_OK;
}

}  // extern "C"
