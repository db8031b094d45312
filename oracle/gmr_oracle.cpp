// FP64 CPU oracle of the Gaussian Mesh Renderer hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or load this file's
// library; only the tests, the smoke check and the bench's CPU-baseline leg use it.  It shares no
// code, header, table or constant generator with the HIP kernels.
//
// What it computes (Liu & Okura, "Gaussian Mesh Renderer for Lightweight Differentiable
// Rendering"):
//   * mesh -> Gaussian conversion, following Sec. 2.2 step by step: local facet frame (Eq. 3),
//     2D vertex coordinates, centroid (Eq. 4), second moments of the uniform triangle through the
//     barycentric map (Eq. 5-8) integrated exactly, 2D covariance (Eq. 9), 2x2 eigen
//     decomposition (Eq. 10), lifted eigenvectors (Eq. 11), area matching (Eq. 12), the 3D
//     covariance (Eq. 13 with R_local of Eq. 14, or the embedded form Eq. 15), opacity 1 and the
//     vertex-average colour (Eq. 16);
//   * the "3DGS-based" baseline conversion the paper compares against (Sec. 3.1, Baselines): the
//     mean at the centroid, the frame from the facet normal (z) and the first edge (x); its scales
//     are not given, so they are read as the area-matched covariance's variances along those two
//     axes (kappa Sigma2D_xx, kappa Sigma2D_yy) and s_z along the normal -- the two conversions
//     then differ only in the frame, which is what the comparison is about;
//   * the standard 3DGS splatting the paper adopts (Sec. 2.1): first-order EWA projection of
//     each Gaussian to a screen-space conic with a 0.3 px^2 low-pass dilation, a 3-sigma
//     axis-aligned extent tested per pixel centre, and front-to-back alpha compositing with the
//     alpha cutoff 1/255, alpha clamp 0.99 and transmittance stop 1e-4 (all three as the
//     float32-rounded constants the caller passes in), per pixel over that pixel's Gaussians
//     ordered by (float32(depth), global id) -- no tiles;
//   * view-dependent colour, the extension named with the colour assignment of Sec. 2.2: each
//     vertex carries K = (degree + 1)^2 coefficients per channel; a face takes their mean (as in
//     Eq. 16); per view its colour is max(0, c_0 + sum_{k >= 1} c_k Y_k(d)), d the unit direction
//     from the camera centre to the Gaussian's mean and Y_k the real spherical harmonics of degree
//     1-3 in the sign convention of 3DGS.  c_0 is the colour itself (the DC encode/decode cancel),
//     so degree 0, or zero higher coefficients, is exactly Eq. 16;
//   * the exact adjoint of that composite, chained to vertices and colours.  The chain through
//     projection and conversion uses forward-mode dual numbers over the closed form
//     Sigma = kappa/12 * sum_q q q^T + s_z^2 n n^T, which equals Eq. 13 exactly (pinned against
//     the literal route by the tests).
//
// Precision: every floating-point quantity is double.  Inputs are the float32 arrays the GPU
// receives, promoted exactly.
//
// Build: g++ -O2 -std=c++17 -fopenmp -fPIC -shared gmr_oracle.cpp -o libgmr_oracle.so

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------------------------------------
// scalar helpers: the same code runs on double and on dual numbers (value + 9 partials)
// ------------------------------------------------------------------------------------------------

constexpr int ND = 9;  // partials w.r.t. the 9 coordinates of (v_i, v_j, v_k)

struct Dual {
  double v;
  double d[ND];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof d); }  // NOLINT: implicit by design
};

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int i = 0; i < ND; ++i) r.d[i] = -a.d[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  Dual r(s);
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] / (2.0 * s);
  return r;
}
using std::sqrt;

template <class T>
inline T dot3(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T>
inline void cross3(const T* a, const T* b, T* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

const double kPi = 3.14159265358979323846;
const double kEps = 1e-14;   // Eq. 12 (epsilon on lambda1*lambda2)
const double kSz = 1e-6;     // s_z, Sec. 2.2 after Eq. 12

// ------------------------------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 on a unit direction d = (x, y, z): Y[0] = 1 (the colour
// itself), then the orthonormal real harmonics with the normalisations sqrt((2l+1)/(4 pi) ...)
// written out and the sign convention of 3DGS.
// ------------------------------------------------------------------------------------------------
template <class T>
void sh_basis(int degree, const T* d, T* Y) {
  const double c1 = std::sqrt(3.0 / (4.0 * kPi));
  const double c2a = std::sqrt(15.0 / (4.0 * kPi)), c2b = std::sqrt(5.0 / (16.0 * kPi)),
               c2c = std::sqrt(15.0 / (16.0 * kPi));
  const double c3a = std::sqrt(35.0 / (32.0 * kPi)), c3b = std::sqrt(105.0 / (4.0 * kPi)),
               c3c = std::sqrt(21.0 / (32.0 * kPi)), c3d = std::sqrt(7.0 / (16.0 * kPi)),
               c3e = std::sqrt(105.0 / (16.0 * kPi));
  const T x = d[0], y = d[1], z = d[2];
  Y[0] = T(1.0);
  if (degree < 1) return;
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (degree < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[4] = c2a * (x * y);
  Y[5] = -c2a * (y * z);
  Y[6] = c2b * (2.0 * zz - xx - yy);
  Y[7] = -c2a * (x * z);
  Y[8] = c2c * (xx - yy);
  if (degree < 3) return;
  Y[9] = -c3a * (y * (3.0 * xx - yy));
  Y[10] = c3b * (x * y * z);
  Y[11] = -c3c * (y * (4.0 * zz - xx - yy));
  Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
  Y[13] = -c3c * (x * (4.0 * zz - xx - yy));
  Y[14] = c3e * (z * (xx - yy));
  Y[15] = -c3a * (x * (xx - 3.0 * yy));
}

// ------------------------------------------------------------------------------------------------
// Conversion, literal route of Sec. 2.2 (double only)
// ------------------------------------------------------------------------------------------------

// Integral over the unit simplex {a, b >= 0, a + b <= 1} of a^p b^q: p! q! / (p + q + 2)!.
double simplex_monomial(int p, int q) {
  double num = 1.0, den = 1.0;
  for (int i = 2; i <= p; ++i) num *= i;
  for (int i = 2; i <= q; ++i) num *= i;
  for (int i = 2; i <= p + q + 2; ++i) den *= i;
  return num / den;
}

// E[f g] over the triangle for f, g affine in the barycentric parameters (Eq. 5):
// f = f0 + f1*alpha + f2*beta, g likewise.  With dA = 2|A| dalpha dbeta, Eq. 6-8 become
// E[f g] = 2 * integral over the simplex of f*g.
double tri_moment(const double f[3], const double g[3]) {
  // f*g = f0g0 + (f0g1+f1g0) a + (f0g2+f2g0) b + f1g1 a^2 + (f1g2+f2g1) a b + f2g2 b^2
  double s = f[0] * g[0] * simplex_monomial(0, 0) + (f[0] * g[1] + f[1] * g[0]) * simplex_monomial(1, 0) +
             (f[0] * g[2] + f[2] * g[0]) * simplex_monomial(0, 1) + f[1] * g[1] * simplex_monomial(2, 0) +
             (f[1] * g[2] + f[2] * g[1]) * simplex_monomial(1, 1) + f[2] * g[2] * simplex_monomial(0, 2);
  return 2.0 * s;
}

// Symmetric 2x2 eigen decomposition (Eq. 10): lambda1 >= lambda2, u1 unit, u2 = u1 rotated +90.
void eig2(double a, double b, double c, double* l1, double* l2, double u1[2], double u2[2]) {
  double m = 0.5 * (a + c), d = 0.5 * (a - c);
  double r = std::sqrt(d * d + b * b);
  *l1 = m + r;
  *l2 = m - r;
  if (r == 0.0) {  // repeated eigenvalue: any orthonormal basis
    u1[0] = 1.0; u1[1] = 0.0;
  } else if (d >= 0.0) {
    double x = d + r, y = b, n = std::sqrt(x * x + y * y);
    u1[0] = x / n; u1[1] = y / n;
  } else {
    double x = b, y = r - d, n = std::sqrt(x * x + y * y);
    u1[0] = x / n; u1[1] = y / n;
  }
  u2[0] = -u1[1];
  u2[1] = u1[0];
}

// Per-face intermediates of the literal route, exported for the pin tests.
struct FaceSteps {
  double x_axis[3], y_axis[3], n_f[3];    // local orthonormal frame (Sec. 2.2, Eq. 3)
  double xj, xk, yk;                      // 2D vertices (0,0), (xj,0), (xk,yk)
  double mux, muy;                        // centroid, Eq. 4
  double Exx, Exy, Eyy;                   // Eq. 6-8
  double S2[3];                           // Eq. 9: (xx, xy, yy)
  double l1, l2, u1[2], u2[2];            // Eq. 10
  double xp[3], yp[3];                    // Eq. 11 lifted eigenvectors
  double area, kappa;                     // |A|, Eq. 12
  double mu[3];                           // 3D mean: Eq. 3 applied to Eq. 4
  double S[9];                            // Eq. 13 (cov_mode 0), Eq. 15 (1), edge-frame baseline (2)
};

bool face_literal(const double* vi, const double* vj, const double* vk, int cov_mode, FaceSteps* o) {
  double e1[3], e2[3], m[3];
  for (int i = 0; i < 3; ++i) { e1[i] = vj[i] - vi[i]; e2[i] = vk[i] - vi[i]; }
  cross3(e1, e2, m);
  double mm = std::sqrt(dot3(m, m));
  if (!(mm > 0.0) || !std::isfinite(mm)) return false;  // collinear / non-finite: culled
  o->area = 0.5 * mm;  // |A|, the triangle's size on its plane
  // Local frame: origin v_i, x along v_j - v_i, y by Gram-Schmidt of v_k - v_i, normal implicit z.
  double L1 = std::sqrt(dot3(e1, e1));
  for (int i = 0; i < 3; ++i) o->x_axis[i] = e1[i] / L1;
  double p = dot3(e2, o->x_axis), w[3];
  for (int i = 0; i < 3; ++i) w[i] = e2[i] - p * o->x_axis[i];
  double Lw = std::sqrt(dot3(w, w));
  for (int i = 0; i < 3; ++i) o->y_axis[i] = w[i] / Lw;
  cross3(o->x_axis, o->y_axis, o->n_f);
  // 2D vertex positions in the local frame.
  o->xj = L1;
  o->xk = dot3(e2, o->x_axis);
  o->yk = dot3(e2, o->y_axis);
  // Eq. 4: centroid.
  o->mux = (o->xj + o->xk) / 3.0;
  o->muy = o->yk / 3.0;
  // Eq. 5: x(a,b) = x_i + a (x_j - x_i) + b (x_k - x_i) with x_i = y_i = 0.
  const double xi = 0.0, yi = 0.0, yj = 0.0;
  double fx[3] = {xi, o->xj - xi, o->xk - xi};
  double fy[3] = {yi, yj - yi, o->yk - yi};
  // Eq. 6-8.
  o->Exx = tri_moment(fx, fx);
  o->Exy = tri_moment(fx, fy);
  o->Eyy = tri_moment(fy, fy);
  // Eq. 9.
  o->S2[0] = o->Exx - o->mux * o->mux;
  o->S2[1] = o->Exy - o->mux * o->muy;
  o->S2[2] = o->Eyy - o->muy * o->muy;
  // Eq. 10.
  eig2(o->S2[0], o->S2[1], o->S2[2], &o->l1, &o->l2, o->u1, o->u2);
  // Eq. 11.
  for (int i = 0; i < 3; ++i) {
    o->xp[i] = o->u1[0] * o->x_axis[i] + o->u1[1] * o->y_axis[i];
    o->yp[i] = o->u2[0] * o->x_axis[i] + o->u2[1] * o->y_axis[i];
  }
  // Eq. 12.
  o->kappa = o->area / (kPi * std::sqrt(std::max(o->l1 * o->l2, kEps)));
  // 3D mean.
  for (int i = 0; i < 3; ++i) o->mu[i] = vi[i] + o->mux * o->x_axis[i] + o->muy * o->y_axis[i];
  if (cov_mode == 0) {
    // Eq. 13 with R_local = [x', y', n_f] (Eq. 14).
    double sx2 = o->kappa * o->l1, sy2 = o->kappa * o->l2, sz2 = kSz * kSz;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        o->S[3 * r + c] = sx2 * o->xp[r] * o->xp[c] + sy2 * o->yp[r] * o->yp[c] + sz2 * o->n_f[r] * o->n_f[c];
  } else if (cov_mode == 2) {
    // Baseline: rotation [x_axis (first edge), y_axis, n_f], diagonal scales in that frame.
    const double sx2 = o->kappa * o->S2[0], sy2 = o->kappa * o->S2[2], sz2 = kSz * kSz;
    const double* X = o->x_axis;
    const double* Y = o->y_axis;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        o->S[3 * r + c] = sx2 * X[r] * X[c] + sy2 * Y[r] * Y[c] + sz2 * o->n_f[r] * o->n_f[c];
  } else {
    // Eq. 15: R_f blockdiag(Sigma2D, 0) R_f^T, R_f = [x_axis, y_axis, n_f].
    const double* X = o->x_axis;
    const double* Y = o->y_axis;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        o->S[3 * r + c] = o->S2[0] * X[r] * X[c] + o->S2[1] * (X[r] * Y[c] + Y[r] * X[c]) + o->S2[2] * Y[r] * Y[c];
  }
  return true;
}

// ------------------------------------------------------------------------------------------------
// Conversion, closed form (templated; used by the adjoint).  The uniform triangle's covariance is
// (1/12) sum_{q in {v_i,v_j,v_k}} (q - mu)(q - mu)^T; it equals R_f blockdiag(Sigma2D,0) R_f^T
// (Eq. 15).  Its determinant on the plane is |A|^2/108 = lambda1*lambda2, so Eq. 13 equals
// kappa * that + s_z^2 n n^T.
// ------------------------------------------------------------------------------------------------

template <class T>
bool convert_closed(const T* vi, const T* vj, const T* vk, int cov_mode, T* mu, T* S) {
  T e1[3], e2[3], m[3];
  for (int i = 0; i < 3; ++i) { e1[i] = vj[i] - vi[i]; e2[i] = vk[i] - vi[i]; }
  cross3(e1, e2, m);
  T mm2 = dot3(m, m);
  if (!(val(mm2) > 0.0) || !std::isfinite(val(mm2))) return false;
  T mm = sqrt(mm2);
  T area = 0.5 * mm;
  for (int i = 0; i < 3; ++i) mu[i] = (vi[i] + vj[i] + vk[i]) / 3.0;
  T q[3][3];
  for (int i = 0; i < 3; ++i) { q[0][i] = vi[i] - mu[i]; q[1][i] = vj[i] - mu[i]; q[2][i] = vk[i] - mu[i]; }
  T C[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[3 * r + c] = (q[0][r] * q[0][c] + q[1][r] * q[1][c] + q[2][r] * q[2][c]) / 12.0;
  if (cov_mode == 1) {
    for (int i = 0; i < 9; ++i) S[i] = C[i];
    return true;
  }
  T det2 = area * area / 108.0;
  T kappa = (val(det2) >= kEps) ? area / (kPi * sqrt(det2)) : area / (kPi * std::sqrt(kEps));
  T n[3] = {m[0] / mm, m[1] / mm, m[2] / mm};
  if (cov_mode == 2) {
    // edge-frame baseline: x = e1 / |e1|, y = n x x; variances of kappa C along x and y
    T l1 = sqrt(dot3(e1, e1));
    T x[3] = {e1[0] / l1, e1[1] / l1, e1[2] / l1};
    T y[3];
    cross3(n, x, y);
    T Cx[3], Cy[3];
    for (int r = 0; r < 3; ++r) {
      Cx[r] = C[3 * r] * x[0] + C[3 * r + 1] * x[1] + C[3 * r + 2] * x[2];
      Cy[r] = C[3 * r] * y[0] + C[3 * r + 1] * y[1] + C[3 * r + 2] * y[2];
    }
    T sx2 = kappa * dot3(x, Cx), sy2 = kappa * dot3(y, Cy);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) S[3 * r + c] = sx2 * x[r] * x[c] + sy2 * y[r] * y[c] + (kSz * kSz) * n[r] * n[c];
    return true;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) S[3 * r + c] = kappa * C[3 * r + c] + (kSz * kSz) * n[r] * n[c];
  return true;
}

// ------------------------------------------------------------------------------------------------
// Camera and EWA projection (3DGS lineage, Sec. 2.1)
// ------------------------------------------------------------------------------------------------

struct Cam {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H;
  double znear, zfar;
};

Cam make_cam(const double* a) {
  Cam c;
  for (int i = 0; i < 9; ++i) c.R[i] = a[i];
  for (int i = 0; i < 3; ++i) c.t[i] = a[9 + i];
  c.fx = a[12]; c.fy = a[13]; c.cx = a[14]; c.cy = a[15];
  c.W = (int)a[16]; c.H = (int)a[17];
  c.znear = a[18]; c.zfar = a[19];
  return c;
}

template <class T>
struct Proj {
  T u, v, conic[3];  // conic (a, b, c) = inverse of the 2x2 screen covariance
  T depth;
  double rx, ry;     // 3-sigma half extents (no gradient flows through the extent)
};

// p = R mu + t; J = d(u,v)/dp at p; Sigma' = J R Sigma R^T J^T + dilation * I.
template <class T>
bool project(const T* mu, const T* S, const Cam& cam, double dilation, double nsig, Proj<T>* o) {
  T p[3];
  for (int r = 0; r < 3; ++r) p[r] = cam.R[3 * r] * mu[0] + cam.R[3 * r + 1] * mu[1] + cam.R[3 * r + 2] * mu[2] + cam.t[r];
  if (!(val(p[2]) > cam.znear) || !(val(p[2]) < cam.zfar)) return false;
  T iz = 1.0 / p[2];
  T J[6] = {cam.fx * iz, T(0.0), -cam.fx * p[0] * iz * iz, T(0.0), cam.fy * iz, -cam.fy * p[1] * iz * iz};
  // W = R S R^T
  T RS[9], Wm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      RS[3 * r + c] = cam.R[3 * r] * S[c] + cam.R[3 * r + 1] * S[3 + c] + cam.R[3 * r + 2] * S[6 + c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      Wm[3 * r + c] = RS[3 * r] * cam.R[3 * c] + RS[3 * r + 1] * cam.R[3 * c + 1] + RS[3 * r + 2] * cam.R[3 * c + 2];
  T JW[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      JW[3 * r + c] = J[3 * r] * Wm[c] + J[3 * r + 1] * Wm[3 + c] + J[3 * r + 2] * Wm[6 + c];
  T sxx = JW[0] * J[0] + JW[1] * J[1] + JW[2] * J[2] + dilation;
  T sxy = JW[0] * J[3] + JW[1] * J[4] + JW[2] * J[5];
  T syy = JW[3] * J[3] + JW[4] * J[4] + JW[5] * J[5] + dilation;
  T det = sxx * syy - sxy * sxy;
  if (!(val(det) > 0.0)) return false;
  o->conic[0] = syy / det;
  o->conic[1] = -sxy / det;
  o->conic[2] = sxx / det;
  o->u = cam.fx * p[0] * iz + cam.cx;
  o->v = cam.fy * p[1] * iz + cam.cy;
  o->depth = p[2];
  o->rx = nsig * std::sqrt(val(sxx));
  o->ry = nsig * std::sqrt(val(syy));
  return true;
}

// ------------------------------------------------------------------------------------------------
// Scene set-up for one (mesh, view)
// ------------------------------------------------------------------------------------------------

struct Params {
  int cov_mode;
  int sh_degree;     // 0: one colour per vertex (Eq. 16); 1-3: view-dependent colour
  double dilation, amin, amax, teps, bg[3];
  double d_ext;      // extent margin (px) within which the inside/outside decision counts as near
  double d_alpha;    // relative margin around the alpha cutoff and the alpha clamp
  double alpha_err;  // relative error bound of a float32 alpha; drives the transmittance bound
  double nsig;
};

Params make_params(const double* a) {
  Params p;
  p.cov_mode = (int)a[0];
  p.dilation = a[1]; p.amin = a[2]; p.amax = a[3]; p.teps = a[4];
  p.bg[0] = a[5]; p.bg[1] = a[6]; p.bg[2] = a[7];
  p.d_ext = a[8]; p.d_alpha = a[9]; p.alpha_err = a[10];
  p.nsig = a[11];
  p.sh_degree = (int)a[12];
  return p;
}

struct Gauss {
  bool ok;
  double u, v, a, b, c, rx, ry, depth, col[3];
  uint64_t key;  // (bits of float32(depth)) << 32 | global id
};

uint32_t f32bits(double x) {
  float f = (float)x;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

// Camera centre in world coordinates: -R^T t.
void cam_centre(const Cam& cam, double* c) {
  for (int i = 0; i < 3; ++i) c[i] = -(cam.R[i] * cam.t[0] + cam.R[3 + i] * cam.t[1] + cam.R[6 + i] * cam.t[2]);
}

// Mean colour coefficients of a face (Eq. 16 applied to every coefficient): coef[k][c].
void face_coefs(const float* Cc, int K, const int32_t* id, double (*coef)[3]) {
  for (int k = 0; k < K; ++k)
    for (int c = 0; c < 3; ++c)
      coef[k][c] = ((double)Cc[((size_t)id[0] * K + k) * 3 + c] + (double)Cc[((size_t)id[1] * K + k) * 3 + c] +
                    (double)Cc[((size_t)id[2] * K + k) * 3 + c]) / 3.0;
}

// The face's colour in this view (before the clamp at 0), from its mean and coefficients.
template <class T>
void view_colour(int degree, const double (*coef)[3], const T* mu, const double* centre, T* raw, T* Y) {
  const int K = (degree + 1) * (degree + 1);
  T d[3] = {mu[0] - centre[0], mu[1] - centre[1], mu[2] - centre[2]};
  T r = sqrt(dot3(d, d));
  for (int i = 0; i < 3; ++i) d[i] = d[i] / r;
  sh_basis(degree, d, Y);
  for (int c = 0; c < 3; ++c) {
    raw[c] = T(0.0);
    for (int k = 0; k < K; ++k) raw[c] = raw[c] + coef[k][c] * Y[k];
  }
}

void setup(long nv, const float* V, long nf, const int32_t* F, const float* Cc, long gid_base,
           const Cam& cam, const Params& P, std::vector<Gauss>& G) {
  const int K = (P.sh_degree + 1) * (P.sh_degree + 1);
  double centre[3];
  cam_centre(cam, centre);
  G.assign(nf, Gauss{});
#pragma omp parallel for schedule(static)
  for (long f = 0; f < nf; ++f) {
    Gauss& g = G[f];
    g.ok = false;
    int32_t id[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
    if (id[0] < 0 || id[1] < 0 || id[2] < 0 || id[0] >= nv || id[1] >= nv || id[2] >= nv) continue;
    double v[3][3];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) v[k][i] = (double)V[3 * id[k] + i];
    FaceSteps st;
    if (!face_literal(v[0], v[1], v[2], P.cov_mode, &st)) continue;
    Proj<double> pr;
    if (!project(st.mu, st.S, cam, P.dilation, P.nsig, &pr)) continue;
    g.ok = true;
    g.u = pr.u; g.v = pr.v;
    g.a = pr.conic[0]; g.b = pr.conic[1]; g.c = pr.conic[2];
    g.rx = pr.rx; g.ry = pr.ry; g.depth = pr.depth;
    double coef[16][3];
    face_coefs(Cc, K, id, coef);  // Eq. 16
    if (P.sh_degree == 0) {
      for (int i = 0; i < 3; ++i) g.col[i] = coef[0][i];
    } else {
      double raw[3], Y[16];
      view_colour(P.sh_degree, coef, st.mu, centre, raw, Y);
      for (int i = 0; i < 3; ++i) g.col[i] = std::max(0.0, raw[i]);
    }
    g.key = ((uint64_t)f32bits(pr.depth) << 32) | (uint64_t)(uint32_t)(gid_base + f);
  }
}

// Pixel range [lo, hi] whose centres i + 0.5 satisfy |i + 0.5 - u| <= r + margin.
inline void pix_range(double u, double r, double margin, long* lo, long* hi) {
  *lo = (long)std::ceil(u - r - margin - 0.5);
  *hi = (long)std::floor(u + r + margin - 0.5);
}

// Candidate lists per pixel of the window, gathered Gaussian by Gaussian (CSR).  A Gaussian is
// listed at every pixel of its extent enlarged by the near-threshold margin.
struct PixLists {
  int x0, y0, w, h;
  std::vector<int64_t> off;
  std::vector<int32_t> idx;
};

void build_lists(const std::vector<Gauss>& G, const Cam& cam, const Params& P, const int32_t* win, PixLists& L) {
  int x0 = std::max(0, win[0]), y0 = std::max(0, win[1]);
  int x1 = std::min(cam.W, win[2]), y1 = std::min(cam.H, win[3]);
  L.x0 = x0; L.y0 = y0; L.w = std::max(0, x1 - x0); L.h = std::max(0, y1 - y0);
  long np = (long)L.w * L.h;
  std::vector<int64_t> cnt(np + 1, 0);
  long nf = (long)G.size();
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      L.off.assign(np + 1, 0);
      for (long i = 0; i < np; ++i) L.off[i + 1] = L.off[i] + cnt[i];
      L.idx.assign(L.off[np], 0);
      std::fill(cnt.begin(), cnt.end(), 0);
    }
    for (long f = 0; f < nf; ++f) {
      const Gauss& g = G[f];
      if (!g.ok) continue;
      long ilo, ihi, jlo, jhi;
      pix_range(g.u, g.rx, P.d_ext, &ilo, &ihi);
      pix_range(g.v, g.ry, P.d_ext, &jlo, &jhi);
      ilo = std::max<long>(ilo, x0); ihi = std::min<long>(ihi, x1 - 1);
      jlo = std::max<long>(jlo, y0); jhi = std::min<long>(jhi, y1 - 1);
      for (long j = jlo; j <= jhi; ++j)
        for (long i = ilo; i <= ihi; ++i) {
          long p = (j - y0) * (long)L.w + (i - x0);
          if (pass == 0) cnt[p]++;
          else L.idx[L.off[p] + cnt[p]++] = (int32_t)f;
        }
    }
  }
}

// One composited entry of a pixel.
struct Hit {
  int32_t f;
  double alpha, e, T, dx, dy;
};

// Composite one pixel (front to back).  Returns the number composited; fills hits, the final
// transmittance, rgb, and whether the pixel lies near a decision threshold.
int composite_pixel(const std::vector<Gauss>& G, const Params& P, const int32_t* cand, long nc,
                    double px, double py, std::vector<int32_t>& order, std::vector<Hit>& hits,
                    double* rgb, double* Tf, bool* near) {
  order.assign(cand, cand + nc);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return G[a].key < G[b].key; });
  hits.clear();
  double T = 1.0, C[3] = {0, 0, 0};
  double errT = 0.0;  // relative error bound of a float32 evaluation of T (rounding + alpha error)
  bool nr = false;
  for (long k = 0; k < nc; ++k) {
    const Gauss& g = G[order[k]];
    double dx = g.u - px, dy = g.v - py;
    double mx = g.rx - std::fabs(dx), my = g.ry - std::fabs(dy);
    bool inside = (mx >= 0.0) && (my >= 0.0);
    bool edge = std::fabs(std::min(mx, my)) < P.d_ext;
    double power = -0.5 * (g.a * dx * dx + g.c * dy * dy) - g.b * dx * dy;
    double e = std::exp(power);
    double alpha = std::min(P.amax, e);
    if (edge && alpha >= P.amin * (1.0 - P.d_alpha)) nr = true;  // extent decision could flip
    if (!inside) continue;
    if (power > 0.0) continue;
    if (std::fabs(alpha - P.amin) < P.d_alpha * P.amin) nr = true;  // cutoff decision could flip
    if (alpha < P.amin) continue;
    if (std::fabs(e - P.amax) < P.d_alpha * P.amax) nr = true;      // clamp kink (gradient only)
    double Tn = T * (1.0 - alpha);
    double errn = errT + 1.2e-7 + (e < P.amax ? P.alpha_err * alpha / (1.0 - alpha) : 0.0);
    if (std::fabs(Tn - P.teps) <= 4.0 * errn * P.teps) nr = true;   // stop decision could flip
    if (Tn < P.teps) break;                                         // stop, not composited
    hits.push_back(Hit{order[k], alpha, e, T, dx, dy});
    for (int i = 0; i < 3; ++i) C[i] += g.col[i] * alpha * T;
    T = Tn;
    errT = errn;
  }
  for (int i = 0; i < 3; ++i) rgb[i] = C[i] + T * P.bg[i];
  *Tf = T;
  *near = nr;
  return (int)hits.size();
}

}  // namespace

// ================================================================================================
// C ABI (ctypes)
// ================================================================================================
extern "C" {

int gmro_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Literal conversion of every face (Sec. 2.2).  Outputs: mu[nf][3], S[nf][9], col[nf][3],
// valid[nf].  Returns the number of valid faces.
long gmro_convert(long nv, const float* V, long nf, const int32_t* F, const float* C, int cov_mode,
                  double* mu, double* S, double* col, uint8_t* valid) {
  long nvalid = 0;
#pragma omp parallel for reduction(+ : nvalid)
  for (long f = 0; f < nf; ++f) {
    valid[f] = 0;
    int32_t id[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
    if (id[0] < 0 || id[1] < 0 || id[2] < 0 || id[0] >= nv || id[1] >= nv || id[2] >= nv) continue;
    double v[3][3];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) v[k][i] = (double)V[3 * id[k] + i];
    FaceSteps st;
    if (!face_literal(v[0], v[1], v[2], cov_mode, &st)) continue;
    for (int i = 0; i < 3; ++i) mu[3 * f + i] = st.mu[i];
    for (int i = 0; i < 9; ++i) S[9 * f + i] = st.S[i];
    for (int i = 0; i < 3; ++i) col[3 * f + i] = ((double)C[3 * id[0] + i] + (double)C[3 * id[1] + i] + (double)C[3 * id[2] + i]) / 3.0;
    valid[f] = 1;
    ++nvalid;
  }
  return nvalid;
}

// Closed-form conversion (the form the adjoint differentiates), same outputs as gmro_convert.
long gmro_convert_closed(long nv, const float* V, long nf, const int32_t* F, int cov_mode,
                         double* mu, double* S, uint8_t* valid) {
  long nvalid = 0;
  for (long f = 0; f < nf; ++f) {
    valid[f] = 0;
    double v[3][3];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) v[k][i] = (double)V[3 * F[3 * f + k] + i];
    if (!convert_closed(v[0], v[1], v[2], cov_mode, mu + 3 * f, S + 9 * f)) continue;
    valid[f] = 1;
    ++nvalid;
  }
  (void)nv;
  return nvalid;
}

// All intermediates of the literal route for one triangle given in double (pin tests).
// out[0..]: x_axis3 y_axis3 n3 xj xk yk mux muy Exx Exy Eyy S2xx S2xy S2yy l1 l2 u1(2) u2(2)
//           xp3 yp3 area kappa mu3 S9   (56 values)
int gmro_face_steps(const double* vi, const double* vj, const double* vk, int cov_mode, double* out) {
  FaceSteps s;
  if (!face_literal(vi, vj, vk, cov_mode, &s)) return 0;
  double* o = out;
  for (int i = 0; i < 3; ++i) *o++ = s.x_axis[i];
  for (int i = 0; i < 3; ++i) *o++ = s.y_axis[i];
  for (int i = 0; i < 3; ++i) *o++ = s.n_f[i];
  *o++ = s.xj; *o++ = s.xk; *o++ = s.yk; *o++ = s.mux; *o++ = s.muy;
  *o++ = s.Exx; *o++ = s.Exy; *o++ = s.Eyy;
  for (int i = 0; i < 3; ++i) *o++ = s.S2[i];
  *o++ = s.l1; *o++ = s.l2;
  *o++ = s.u1[0]; *o++ = s.u1[1]; *o++ = s.u2[0]; *o++ = s.u2[1];
  for (int i = 0; i < 3; ++i) *o++ = s.xp[i];
  for (int i = 0; i < 3; ++i) *o++ = s.yp[i];
  *o++ = s.area; *o++ = s.kappa;
  for (int i = 0; i < 3; ++i) *o++ = s.mu[i];
  for (int i = 0; i < 9; ++i) *o++ = s.S[i];
  return 1;
}

// Projection of one face's Gaussian (mu, S full 3x3) for one camera.  out: u v a b c rx ry depth.
int gmro_project_one(const double* mu, const double* S, const double* cam, double dilation, double nsig, double* out) {
  Cam c = make_cam(cam);
  Proj<double> p;
  if (!project(mu, S, c, dilation, nsig, &p)) return 0;
  out[0] = p.u; out[1] = p.v; out[2] = p.conic[0]; out[3] = p.conic[1]; out[4] = p.conic[2];
  out[5] = p.rx; out[6] = p.ry; out[7] = p.depth;
  return 1;
}

// The colour basis on n unit directions: out[n][16] (entries past (degree + 1)^2 left untouched).
long gmro_sh_basis(int degree, long n, const double* dirs, double* out) {
  for (long i = 0; i < n; ++i) sh_basis(degree, dirs + 3 * i, out + 16 * i);
  return n;
}

// Per-Gaussian screen-space record for one view: out[nf][12] = ok u v a b c rx ry depth r g b.
long gmro_gaussians(long nv, const float* V, long nf, const int32_t* F, const float* C, const double* cam,
                    const double* prm, double* out) {
  Cam cm = make_cam(cam);
  Params P = make_params(prm);
  std::vector<Gauss> G;
  setup(nv, V, nf, F, C, 0, cm, P, G);
  long n = 0;
  for (long f = 0; f < nf; ++f) {
    const Gauss& g = G[f];
    double* o = out + 12 * f;
    o[0] = g.ok ? 1.0 : 0.0;
    o[1] = g.u; o[2] = g.v; o[3] = g.a; o[4] = g.b; o[5] = g.c; o[6] = g.rx; o[7] = g.ry; o[8] = g.depth;
    o[9] = g.col[0]; o[10] = g.col[1]; o[11] = g.col[2];
    n += g.ok;
  }
  return n;
}

// Render the pixels of window win = [x0, y0, x1, y1) of one view of one mesh.  Outputs are laid
// out over the window, row-major: rgb[h][w][3], Tf[h][w], ncomp[h][w], mask[h][w] (near a
// decision threshold), lhash[h][w] (may be NULL: a hash of the composited face sequence).
// gid_base is the global id of face 0 (ties in depth are broken by it).
// Returns the total number of candidate entries.
long gmro_render(long nv, const float* V, long nf, const int32_t* F, const float* C, long gid_base,
                 const double* cam, const double* prm, const int32_t* win,
                 double* rgb, double* Tf, int32_t* ncomp, uint8_t* mask, uint64_t* lhash) {
  Cam cm = make_cam(cam);
  Params P = make_params(prm);
  std::vector<Gauss> G;
  setup(nv, V, nf, F, C, gid_base, cm, P, G);
  PixLists L;
  build_lists(G, cm, P, win, L);
  long np = (long)L.w * L.h;
#pragma omp parallel
  {
    std::vector<int32_t> order;
    std::vector<Hit> hits;
#pragma omp for schedule(dynamic, 256)
    for (long p = 0; p < np; ++p) {
      long i = L.x0 + p % L.w, j = L.y0 + p / L.w;
      bool nr;
      ncomp[p] = composite_pixel(G, P, L.idx.data() + L.off[p], L.off[p + 1] - L.off[p], i + 0.5, j + 0.5,
                                 order, hits, rgb + 3 * p, Tf + p, &nr);
      mask[p] = nr ? 1 : 0;
      if (lhash) {  // FNV-1a over the composited face indices: a summary of the pixel's decisions
        uint64_t h = 1469598103934665603ull;
        for (const Hit& x : hits) { h ^= (uint64_t)(uint32_t)x.f; h *= 1099511628211ull; }
        lhash[p] = h;
      }
    }
  }
  return (long)L.idx.size();
}

// Exact adjoint of gmro_render over the same window.  g_rgb[h][w][3] and g_alpha[h][w] (may be
// NULL) are dL/d(rgb) and dL/d(alpha = 1 - Tf).  Accumulates dL/dV into dV[nv][3] and dL/dC into
// dC[nv][3] (caller zeroes them).  If gG is not NULL it receives the per-Gaussian screen-space
// gradients [nf][8] = du dv da db dc dr dg db (accumulated).
long gmro_render_adjoint(long nv, const float* V, long nf, const int32_t* F, const float* C, long gid_base,
                         const double* cam, const double* prm, const int32_t* win,
                         const double* g_rgb, const double* g_alpha, double* dV, double* dC, double* gG) {
  Cam cm = make_cam(cam);
  Params P = make_params(prm);
  std::vector<Gauss> G;
  setup(nv, V, nf, F, C, gid_base, cm, P, G);
  PixLists L;
  build_lists(G, cm, P, win, L);
  long np = (long)L.w * L.h;
  std::vector<double> GG(8 * (size_t)nf, 0.0);
#pragma omp parallel
  {
    std::vector<int32_t> order;
    std::vector<Hit> hits;
#pragma omp for schedule(dynamic, 256)
    for (long p = 0; p < np; ++p) {
      long i = L.x0 + p % L.w, j = L.y0 + p / L.w;
      double rgb[3], Tf;
      bool nr;
      int K = composite_pixel(G, P, L.idx.data() + L.off[p], L.off[p + 1] - L.off[p], i + 0.5, j + 0.5,
                              order, hits, rgb, &Tf, &nr);
      const double* gc = g_rgb + 3 * p;
      double ga = g_alpha ? g_alpha[p] : 0.0;
      if (gc[0] == 0.0 && gc[1] == 0.0 && gc[2] == 0.0 && ga == 0.0) continue;
      double bgg = P.bg[0] * gc[0] + P.bg[1] * gc[1] + P.bg[2] * gc[2];
      // C = sum_k c_k a_k T_k + T_f bg ; alpha_out = 1 - T_f ; T_{k+1} = T_k (1 - a_k).
      double S = 0.0;  // sum over later entries of a_j T_j (c_j . g_C)
      for (int k = K - 1; k >= 0; --k) {
        const Hit& h = hits[k];
        const Gauss& g = G[h.f];
        double cg = g.col[0] * gc[0] + g.col[1] * gc[1] + g.col[2] * gc[2];
        double d_alpha = h.T * cg - (S + Tf * bgg - Tf * ga) / (1.0 - h.alpha);
        S += h.alpha * h.T * cg;
        double d_pow = (h.e < P.amax) ? h.e * d_alpha : 0.0;  // alpha = min(amax, e^power)
        double out[8];
        out[0] = -d_pow * (g.a * h.dx + g.b * h.dy);
        out[1] = -d_pow * (g.b * h.dx + g.c * h.dy);
        out[2] = -0.5 * d_pow * h.dx * h.dx;
        out[3] = -d_pow * h.dx * h.dy;
        out[4] = -0.5 * d_pow * h.dy * h.dy;
        for (int c = 0; c < 3; ++c) out[5 + c] = h.alpha * h.T * gc[c];
        for (int c = 0; c < 8; ++c) {
#pragma omp atomic
          GG[8 * (size_t)h.f + c] += out[c];
        }
      }
    }
  }
  // Chain (u, v, a, b, c) -> vertices with dual numbers; colours by Eq. 16 (and, with view-dependent
  // colour, through the coefficients and through the viewing direction's dependence on the mean).
  const int K = (P.sh_degree + 1) * (P.sh_degree + 1);
  double centre[3];
  cam_centre(cm, centre);
  std::vector<double> dVl(3 * (size_t)nv, 0.0), dCl(3 * (size_t)nv * K, 0.0);
  for (long f = 0; f < nf; ++f) {
    const double* gg = GG.data() + 8 * f;
    if (gG)
      for (int c = 0; c < 8; ++c) gG[8 * f + c] += gg[c];
    bool any = false;
    for (int c = 0; c < 8; ++c) any |= (gg[c] != 0.0);
    if (!any || !G[f].ok) continue;
    int32_t id[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
    Dual v[3][3];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) {
        v[k][i] = Dual((double)V[3 * id[k] + i]);
        v[k][i].d[3 * k + i] = 1.0;
      }
    Dual mu[3], S[9];
    if (!convert_closed(v[0], v[1], v[2], P.cov_mode, mu, S)) continue;
    Proj<Dual> pr;
    if (!project(mu, S, cm, P.dilation, P.nsig, &pr)) continue;
    const Dual* outs[5] = {&pr.u, &pr.v, &pr.conic[0], &pr.conic[1], &pr.conic[2]};
    double coef[16][3];
    face_coefs(C, K, id, coef);
    Dual raw[3], Y[16];
    double gcol[3] = {gg[5], gg[6], gg[7]};  // dL/d(colour), zero where the clamp at 0 is active
    if (P.sh_degree > 0) {
      view_colour(P.sh_degree, coef, mu, centre, raw, Y);
      for (int c = 0; c < 3; ++c)
        if (!(val(raw[c]) > 0.0)) gcol[c] = 0.0;
    }
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int q = 0; q < 5; ++q) s += gg[q] * outs[q]->d[3 * k + i];
        if (P.sh_degree > 0)
          for (int c = 0; c < 3; ++c) s += gcol[c] * raw[c].d[3 * k + i];  // through the direction
        dVl[3 * (size_t)id[k] + i] += s;
      }
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < K; ++j)
        for (int c = 0; c < 3; ++c)
          dCl[((size_t)id[k] * K + j) * 3 + c] += gcol[c] * (P.sh_degree > 0 ? val(Y[j]) : 1.0) / 3.0;
  }
  for (long i = 0; i < 3 * nv; ++i) dV[i] += dVl[i];
  for (long i = 0; i < 3 * nv * K; ++i) dC[i] += dCl[i];
  return np;
}

// Per-tile Gaussian lists of one view for a tile grid of tw x th pixels.  A Gaussian belongs to
// a tile iff some pixel centre of the tile lies in its 3-sigma extent.  Lists are ordered by
// (float32(depth), global id).  amb[n] = 1 marks an entry whose membership could flip within the
// margin d_ext.  Writes tile_off[ntiles+1]; ids/amb up to cap entries.  Returns the total count.
long gmro_tile_lists(long nv, const float* V, long nf, const int32_t* F, const float* C, long gid_base,
                     const double* cam, const double* prm, int tw, int th,
                     int64_t* tile_off, int32_t* ids, uint8_t* amb, long cap) {
  Cam cm = make_cam(cam);
  Params P = make_params(prm);
  std::vector<Gauss> G;
  setup(nv, V, nf, F, C, gid_base, cm, P, G);
  int ntx = (cm.W + tw - 1) / tw, nty = (cm.H + th - 1) / th;
  long ntiles = (long)ntx * nty;
  std::vector<std::vector<std::pair<uint64_t, std::pair<int32_t, uint8_t>>>> lists(ntiles);
  for (long f = 0; f < nf; ++f) {
    const Gauss& g = G[f];
    if (!g.ok) continue;
    long oi0, oi1, oj0, oj1, ii0, ii1, ij0, ij1;
    pix_range(g.u, g.rx, P.d_ext, &oi0, &oi1);
    pix_range(g.v, g.ry, P.d_ext, &oj0, &oj1);
    pix_range(g.u, g.rx, -P.d_ext, &ii0, &ii1);
    pix_range(g.v, g.ry, -P.d_ext, &ij0, &ij1);
    long e_i0, e_i1, e_j0, e_j1;  // exact extent
    pix_range(g.u, g.rx, 0.0, &e_i0, &e_i1);
    pix_range(g.v, g.ry, 0.0, &e_j0, &e_j1);
    auto clampx = [&](long& a, long& b) { a = std::max<long>(a, 0); b = std::min<long>(b, cm.W - 1); };
    auto clampy = [&](long& a, long& b) { a = std::max<long>(a, 0); b = std::min<long>(b, cm.H - 1); };
    clampx(oi0, oi1); clampy(oj0, oj1); clampx(ii0, ii1); clampy(ij0, ij1); clampx(e_i0, e_i1); clampy(e_j0, e_j1);
    if (oi0 > oi1 || oj0 > oj1) continue;
    for (long ty = oj0 / th; ty <= oj1 / th; ++ty)
      for (long tx = oi0 / tw; tx <= oi1 / tw; ++tx) {
        bool in_exact = e_i0 <= e_i1 && e_j0 <= e_j1 && tx >= e_i0 / tw && tx <= e_i1 / tw && ty >= e_j0 / th && ty <= e_j1 / th;
        bool in_inner = ii0 <= ii1 && ij0 <= ij1 && tx >= ii0 / tw && tx <= ii1 / tw && ty >= ij0 / th && ty <= ij1 / th;
        bool ambiguous = !in_inner;  // in the enlarged set but not the shrunk one
        if (!in_exact && !ambiguous) continue;
        lists[ty * ntx + tx].push_back({g.key, {(int32_t)(gid_base + f), (uint8_t)(ambiguous ? (in_exact ? 1 : 2) : 0)}});
      }
  }
  long n = 0;
  for (long t = 0; t < ntiles; ++t) {
    std::sort(lists[t].begin(), lists[t].end());
    tile_off[t] = n;
    for (auto& e : lists[t]) {
      if (n < cap) { ids[n] = e.second.first; amb[n] = e.second.second; }
      ++n;
    }
  }
  tile_off[ntiles] = n;
  return n;
}

}  // extern "C"
