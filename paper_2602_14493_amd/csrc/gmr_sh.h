// View-dependent colour: the extension named with the colour assignment of Sec. 2.2.
//
// Every vertex carries K = (D + 1)^2 coefficients per channel (layout [V][K][3]); a face takes
// their mean, as Eq. 16 does for a single colour.  In a view, the face's colour is
//   max(0, c_0 + sum_{k=1}^{K-1} c_k Y_k(d)),   d = (mu - camera centre) / |mu - camera centre|,
// with Y_k the real spherical harmonics of degrees 1..D (orthonormal on the sphere, 3DGS sign
// convention).  c_0 is the colour itself, so D = 0 is Eq. 16.
#pragma once

#include <hip/hip_runtime.h>

namespace gmr {

// Normalisations of the real harmonics: sqrt((2l + 1) / (4 pi) * (l - |m|)! / (l + |m|)!) times
// the factors that make the Cartesian polynomials below orthonormal.
constexpr double kShC1 = 0.48860251190291992;    // sqrt(3 / (4 pi))
constexpr double kShC2a = 1.0925484305920792;    // sqrt(15 / (4 pi))
constexpr double kShC2b = 0.31539156525252005;   // sqrt(5 / (16 pi))
constexpr double kShC2c = 0.54627421529603959;   // sqrt(15 / (16 pi))
constexpr double kShC3a = 0.59004358992664352;   // sqrt(35 / (32 pi))
constexpr double kShC3b = 2.8906114426405538;    // sqrt(105 / (4 pi))
constexpr double kShC3c = 0.4570457994644658;    // sqrt(21 / (32 pi))
constexpr double kShC3d = 0.37317633259011540;   // sqrt(7 / (16 pi))
constexpr double kShC3e = 1.4453057213202769;    // sqrt(105 / (16 pi))

template <int D>
constexpr int sh_count() { return (D + 1) * (D + 1); }

// Y[0..K) at the unit direction (x, y, z); Y[0] = 1.
template <int D>
__device__ inline void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = 1.0;
  if constexpr (D >= 1) {
    Y[1] = -kShC1 * y;
    Y[2] = kShC1 * z;
    Y[3] = -kShC1 * x;
  }
  if constexpr (D >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kShC2a * (x * y);
    Y[5] = -kShC2a * (y * z);
    Y[6] = kShC2b * (2.0 * zz - xx - yy);
    Y[7] = -kShC2a * (x * z);
    Y[8] = kShC2c * (xx - yy);
    if constexpr (D >= 3) {
      Y[9] = -kShC3a * (y * (3.0 * xx - yy));
      Y[10] = kShC3b * (x * y * z);
      Y[11] = -kShC3c * (y * (4.0 * zz - xx - yy));
      Y[12] = kShC3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
      Y[13] = -kShC3c * (x * (4.0 * zz - xx - yy));
      Y[14] = kShC3e * (z * (xx - yy));
      Y[15] = -kShC3a * (x * (xx - 3.0 * yy));
    }
  }
}

// Gradient of sum_{k >= 1} w[k] Y_k with the Y_k taken as polynomials in (x, y, z) (the caller
// projects out the radial part).
template <int D>
__device__ inline void sh_poly_grad(double x, double y, double z, const double* w, double& gx, double& gy,
                                    double& gz) {
  gx = gy = gz = 0.0;
  if constexpr (D >= 1) {
    gy -= kShC1 * w[1];
    gz += kShC1 * w[2];
    gx -= kShC1 * w[3];
  }
  if constexpr (D >= 2) {
    gx += kShC2a * w[4] * y;  gy += kShC2a * w[4] * x;
    gy -= kShC2a * w[5] * z;  gz -= kShC2a * w[5] * y;
    gx -= 2.0 * kShC2b * w[6] * x;  gy -= 2.0 * kShC2b * w[6] * y;  gz += 4.0 * kShC2b * w[6] * z;
    gx -= kShC2a * w[7] * z;  gz -= kShC2a * w[7] * x;
    gx += 2.0 * kShC2c * w[8] * x;  gy -= 2.0 * kShC2c * w[8] * y;
    if constexpr (D >= 3) {
      const double xx = x * x, yy = y * y, zz = z * z;
      gx -= 6.0 * kShC3a * w[9] * x * y;  gy -= 3.0 * kShC3a * w[9] * (xx - yy);
      gx += kShC3b * w[10] * y * z;  gy += kShC3b * w[10] * x * z;  gz += kShC3b * w[10] * x * y;
      gx += 2.0 * kShC3c * w[11] * x * y;  gy -= kShC3c * w[11] * (4.0 * zz - xx - 3.0 * yy);
      gz -= 8.0 * kShC3c * w[11] * y * z;
      gx -= 6.0 * kShC3d * w[12] * x * z;  gy -= 6.0 * kShC3d * w[12] * y * z;
      gz += kShC3d * w[12] * (6.0 * zz - 3.0 * xx - 3.0 * yy);
      gx -= kShC3c * w[13] * (4.0 * zz - 3.0 * xx - yy);  gy += 2.0 * kShC3c * w[13] * x * y;
      gz -= 8.0 * kShC3c * w[13] * x * z;
      gx += 2.0 * kShC3e * w[14] * x * z;  gy -= 2.0 * kShC3e * w[14] * y * z;  gz += kShC3e * w[14] * (xx - yy);
      gx -= 3.0 * kShC3a * w[15] * (xx - yy);  gy += 6.0 * kShC3a * w[15] * x * y;
    }
  }
}

// Camera centre -R^T t of a view (R row-major).
__device__ inline void view_centre(const float* R, const float* t, double* c) {
  for (int i = 0; i < 3; ++i)
    c[i] = -((double)R[i] * t[0] + (double)R[3 + i] * t[1] + (double)R[6 + i] * t[2]);
}

// Mean over a face's three vertices of each colour coefficient: coef[k][c].
template <int D>
__device__ inline void face_coefs(const float* __restrict__ colors, int32_t i0, int32_t i1, int32_t i2,
                                  float (*coef)[3]) {
  constexpr int K = sh_count<D>();
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      coef[k][c] = (float)(((double)colors[((int64_t)i0 * K + k) * 3 + c] + (double)colors[((int64_t)i1 * K + k) * 3 + c] +
                            (double)colors[((int64_t)i2 * K + k) * 3 + c]) * (1.0 / 3.0));
}

}  // namespace gmr
