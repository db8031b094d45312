// Backward of the EWA projection and of the conversion, then the per-vertex gather.
//
// k_face_bwd: one thread per face (double precision).  For every view of the face's mesh it reads
// the face-view's gradient sums {A, B, C, D, E, dr, dg, db} (the rasteriser's sums in the scaled
// Cholesky frame of the conic, turned into {du, dv, da, db, dc} below), re-derives the projection
// and accumulates dL/dmu and dL/dSigma over views (gradients as full symmetric matrices:
// dL = tr(G dX)):
//   conic Q = Sigma'^-1:           G_Sigma' = -Q Gq Q, Gq = [[da, db/2], [db/2, dc]]
//   Sigma' = J W J^T + d I:        G_W = J^T G_Sigma' J,  G_J = 2 G_Sigma' J W
//   W = R Sigma R^T:               G_Sigma = R^T G_W R
//   J(p), (u, v)(p), p = R mu + t: G_mu = R^T G_p
// then differentiates the closed-form conversion (same expressions as the forward):
//   Sigma = kappa/36 M + s_z^2 n n^T, M = 2 e1 e1^T + 2 e2 e2^T - e1 e2^T - e2 e1^T
//   dM: G_e1 = G (4 e1 - 2 e2), G_e2 = G (4 e2 - 2 e1)
//   n = m/|m|, m = e1 x e2: G_n = 2 s_z^2 G n, G_m = (I - n n^T) G_n / |m|
//   clamped kappa = |A| / (pi sqrt(eps)), |A| = |m|/2: G_m += tr(G M)/36 / (pi sqrt(eps)) n / 2
//   m = e1 x e2: G_e1 += e2 x G_m, G_e2 += G_m x e1; mu = (v_i + v_j + v_k)/3
// and writes per-corner vertex gradients and the face's colour gradient (12 floats per face).
// With view-dependent colour (degree SHD > 0) the colour of face-view (f, v) is
// max(0, sum_k c_k Y_k(d_v)), d_v = (mu - centre_v) / r_v: the clamp passes dL/dcolour where the
// sum is positive, G_c_k += dL/dcolour Y_k(d_v) (the face's coefficient gradients, 3K floats in
// `fsh`), and G_mu += (I - d d^T) / r_v grad_d(sum_k w_k Y_k), w_k = sum_channels dL/dcolour c_k.
// k_vertex_gather: one thread per vertex sums its corners through the (vertex -> face, corner)
// CSR in a fixed order, so the vertex gradients do not depend on atomic ordering (a vertex with
// more than 32 corners is summed by its whole wavefront, lane-strided, in a fixed tree order).  With a fused
// loss its first blocks also sum the per-item loss slots (one launch fewer per backward).
#include "gmr_common.h"
#include "gmr_launch.h"
#include "gmr_sh.h"

namespace gmr {

__device__ inline void sym3_from6(const double* s, double (&M)[3][3]) {
  M[0][0] = s[0]; M[0][1] = s[1]; M[0][2] = s[2];
  M[1][0] = s[1]; M[1][1] = s[3]; M[1][2] = s[4];
  M[2][0] = s[2]; M[2][1] = s[4]; M[2][2] = s[5];
}

// LPF lanes per face (1 or 8, consecutive lanes of a wavefront): with LPF > 1 lane u of a face's
// group takes views u, u + LPF, ... of its mesh, the group sums its per-view partials in a fixed
// tree order, and the group's first lane differentiates the conversion -- small batches then run
// LPF times as many wavefronts, each with a shorter chain of dependent FP64 work.
template <int SHD, int LPF>
__global__ __launch_bounds__(256) void k_face_bwd(const void* __restrict__ table, const float* __restrict__ verts,
                                                  const int32_t* __restrict__ faces, const float* __restrict__ colors,
                                                  KOpts o, const float4* __restrict__ dfv, float4* __restrict__ fgrad,
                                                  float* __restrict__ fsh) {
  static_assert(LPF == 1 || (SHD == 0 && (LPF & (LPF - 1)) == 0 && LPF <= kWave), "LPF: 1, or a power of two without SH");
  constexpr int K = sh_count<SHD>();
  const TableHdr* th = static_cast<const TableHdr*>(table);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t f = t / LPF;
  const int u = (int)(t - f * LPF);
  if (f >= th->faces_total) return;  // the whole group (same face)
  const int32_t* mfo = table_i32(table, th->mesh_face_off);
  const int32_t* mvo = table_i32(table, th->mesh_view_off);
  const int32_t* mvs = table_i32(table, th->mesh_views_off);
  const ViewDev* views = table_views(table);
  const int m = find_mesh(mfo, th->num_meshes, (int32_t)f);
  const int32_t i0 = faces[3 * f], i1 = faces[3 * f + 1], i2 = faces[3 * f + 2];
  double vi[3], vj[3], vk[3];
  for (int a = 0; a < 3; ++a) {
    vi[a] = verts[3 * (int64_t)i0 + a];
    vj[a] = verts[3 * (int64_t)i1 + a];
    vk[a] = verts[3 * (int64_t)i2 + a];
  }
  float4* out = fgrad + 3 * f;
  // only the mean and covariance stay live through the view loop; the rest of the conversion is
  // recomputed after it (fewer registers held across the loop's FP64 work)
  double mu[3], Sg[6];
  {
    FaceGeo g0;
    const bool ok = face_convert(vi, vj, vk, o.cov_mode, g0);
    for (int a = 0; a < 3; ++a) mu[a] = g0.mu[a];
    for (int a = 0; a < 6; ++a) Sg[a] = g0.S[a];
    if (!ok) {  // uniform over the face's group
      if (u == 0) {
        out[0] = out[1] = out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (SHD > 0)
          for (int k = 0; k < 3 * K; ++k) fsh[3 * K * f + k] = 0.f;
      }
      return;
    }
  }
  float coef[K][3], gsh[K][3];
  if constexpr (SHD > 0) {
    face_coefs<SHD>(colors, i0, i1, i2, coef);
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
  }
  double Gmu[3] = {0.0, 0.0, 0.0};
  double GS6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // G_Sigma (symmetric): xx xy xz yy yz zz
  float gcol[3] = {0.f, 0.f, 0.f};
  for (int k = mvo[m] + u; k < mvo[m + 1]; k += LPF) {
    const ViewDev& V = views[mvs[k]];
    const int64_t fv = V.fv_offset + (f - V.face_begin);
    const float4 d0 = dfv[2 * fv], d1 = dfv[2 * fv + 1];
    if (d0.x == 0.f && d0.y == 0.f && d0.z == 0.f && d0.w == 0.f && d1.x == 0.f && d1.y == 0.f && d1.z == 0.f &&
        d1.w == 0.f)
      continue;
    if constexpr (SHD == 0) {
      gcol[0] += d1.y; gcol[1] += d1.z; gcol[2] += d1.w;
    } else {
      double cc[3];
      view_centre(V.R, V.t, cc);
      const double px = mu[0] - cc[0], py = mu[1] - cc[1], pz = mu[2] - cc[2];
      const double ir = 1.0 / sqrt(px * px + py * py + pz * pz);
      const double x = px * ir, y = py * ir, z = pz * ir;
      double Y[K];
      sh_basis<SHD>(x, y, z, Y);
      double gc[3] = {d1.y, d1.z, d1.w};
      for (int a = 0; a < 3; ++a) {
        double raw = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) raw += (double)coef[k][a] * Y[k];
        if (!(raw > 0.0)) gc[a] = 0.0;  // the clamp at 0
      }
      double w[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        gsh[k][0] += (float)(gc[0] * Y[k]);
        gsh[k][1] += (float)(gc[1] * Y[k]);
        gsh[k][2] += (float)(gc[2] * Y[k]);
        w[k] = gc[0] * coef[k][0] + gc[1] * coef[k][1] + gc[2] * coef[k][2];
      }
      double gx, gy, gz;
      sh_poly_grad<SHD>(x, y, z, w, gx, gy, gz);
      const double dd = x * gx + y * gy + z * gz;
      Gmu[0] += (gx - x * dd) * ir;
      Gmu[1] += (gy - y * dd) * ir;
      Gmu[2] += (gz - z * dd) * ir;
    }
    ProjGeo q;
    if (!view_project(V, mu, Sg, (double)o.dilation, q)) continue;
    // the rasteriser's sums over the face-view's pixels, {A, B, C, D, E} = sum of gq {w1, w2,
    // w1 dx, w1 dy, w2 dy} with gq = dL/d(ln alpha) and w = k L (dx, dy), L the conic's Cholesky
    // factor (k^2 = log2(e) / 2, the record's scale): exp2(-|w|^2) = exp(-d^T Q d / 2), so
    // dL/d(u, v) = -2 ln2 k (L^T (A, B)) and the sums of gq dx^2, gq dx dy, gq dy^2 follow from
    // the triangular system C = k (l11 Sxx + l12 Sxy), D = k (l11 Sxy + l12 Syy), E = k l22 Syy;
    // dL/d(a, b, c) = -(Sxx / 2, Sxy, Syy / 2)
    const double l11 = sqrt(q.a), l12 = q.b / l11, l22 = 1.0 / (l11 * sqrt(q.det));
    const double kl11 = kRasterScale * l11, kl12 = kRasterScale * l12, kl22 = kRasterScale * l22;
    const double sA = d0.x, sB = d0.y, sC = d0.z, sD = d0.w, sE = d1.x;
    const double Syy = sE / kl22;
    const double Sxy = (sD - kl12 * Syy) / kl11;
    const double Sxx = (sC - kl12 * Sxy) / kl11;
    const double du = -2.0 * kLn2 * kl11 * sA, dv = -2.0 * kLn2 * (kl12 * sA + kl22 * sB);
    const double da = -0.5 * Sxx, db = -Sxy, dc = -0.5 * Syy;
    // G_Sigma' = -Q Gq Q
    const double a = q.a, b = q.b, c = q.c;
    const double m00 = a * da + b * 0.5 * db, m01 = a * 0.5 * db + b * dc;
    const double m10 = b * da + c * 0.5 * db, m11 = b * 0.5 * db + c * dc;
    const double gxx = -(m00 * a + m01 * b), gxy = -(m00 * b + m01 * c), gyy = -(m10 * b + m11 * c);
    const double j0 = q.J[0], j2 = q.J[2], j4 = q.J[4], j5 = q.J[5];
    // G J (2x3)
    const double GJ[2][3] = {{gxx * j0, gxy * j4, gxx * j2 + gxy * j5}, {gxy * j0, gyy * j4, gxy * j2 + gyy * j5}};
    // G_W = J^T (G J); J^T rows: (j0, 0), (0, j4), (j2, j5)
    double GW[3][3];
    for (int cc = 0; cc < 3; ++cc) {
      GW[0][cc] = j0 * GJ[0][cc];
      GW[1][cc] = j4 * GJ[1][cc];
      GW[2][cc] = j2 * GJ[0][cc] + j5 * GJ[1][cc];
    }
    // G_J = 2 (G J) W
    double Wm[3][3];
    sym3_from6(q.W, Wm);
    double GJm[2][3];
    for (int r = 0; r < 2; ++r)
      for (int cc = 0; cc < 3; ++cc)
        GJm[r][cc] = 2.0 * (GJ[r][0] * Wm[0][cc] + GJ[r][1] * Wm[1][cc] + GJ[r][2] * Wm[2][cc]);
    // G_Sigma += R^T G_W R
    double R[3][3];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) R[r][cc] = (double)V.R[3 * r + cc];
    double GWR[3][3];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) GWR[r][cc] = GW[r][0] * R[0][cc] + GW[r][1] * R[1][cc] + GW[r][2] * R[2][cc];
    // R^T G_W R is symmetric (G_W is): its upper triangle
    for (int r = 0, i6 = 0; r < 3; ++r)
      for (int cc = r; cc < 3; ++cc, ++i6)
        GS6[i6] += R[0][r] * GWR[0][cc] + R[1][r] * GWR[1][cc] + R[2][r] * GWR[2][cc];
    // G_p from J(p) and (u, v)(p)
    const double x = q.p[0], y = q.p[1], iz = 1.0 / q.p[2];
    const double fx = V.fx, fy = V.fy;
    double Gp[3];
    Gp[0] = GJm[0][2] * (-fx * iz * iz) + du * fx * iz;
    Gp[1] = GJm[1][2] * (-fy * iz * iz) + dv * fy * iz;
    Gp[2] = GJm[0][0] * (-fx * iz * iz) + GJm[0][2] * (2.0 * fx * x * iz * iz * iz) + GJm[1][1] * (-fy * iz * iz) +
            GJm[1][2] * (2.0 * fy * y * iz * iz * iz) - du * fx * x * iz * iz - dv * fy * y * iz * iz;
    for (int r = 0; r < 3; ++r) Gmu[r] += R[0][r] * Gp[0] + R[1][r] * Gp[1] + R[2][r] * Gp[2];
  }
  if constexpr (LPF > 1) {
#pragma unroll
    for (int d = LPF / 2; d > 0; d >>= 1) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Gmu[r] += __shfl_xor(Gmu[r], d, kWave);
        gcol[r] += __shfl_xor(gcol[r], d, kWave);
      }
#pragma unroll
      for (int i6 = 0; i6 < 6; ++i6) GS6[i6] += __shfl_xor(GS6[i6], d, kWave);
    }
    if (u != 0) return;
  }
  double GS[3][3];
  sym3_from6(GS6, GS);
  // the conversion again, from the vertices (read back: they were not kept in registers)
  FaceGeo g;
  {
    for (int a = 0; a < 3; ++a) {
      vi[a] = verts[3 * (int64_t)i0 + a];
      vj[a] = verts[3 * (int64_t)i1 + a];
      vk[a] = verts[3 * (int64_t)i2 + a];
    }
    face_convert(vi, vj, vk, o.cov_mode, g);
  }
  const double* e1 = g.e1;
  const double* e2 = g.e2;
  double Ge1[3], Ge2[3];
  if (o.cov_mode == 2) {
    // S = kappa a x x' + kappa b y y' + s_z^2 n n', a = x'Cx, b = y'Cy, x = e1/|e1|, y = n x x
    const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    const double inv = 1.0 / g.mm;
    const double n[3] = {g.m[0] * inv, g.m[1] * inv, g.m[2] * inv};
    const double x[3] = {e1[0] / l1, e1[1] / l1, e1[2] / l1};
    const double y[3] = {n[1] * x[2] - n[2] * x[1], n[2] * x[0] - n[0] * x[2], n[0] * x[1] - n[1] * x[0]};
    double Cm[3][3];  // C = M / 36
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc)
        Cm[r][cc] = (2.0 * e1[r] * e1[cc] + 2.0 * e2[r] * e2[cc] - e1[r] * e2[cc] - e2[r] * e1[cc]) * (1.0 / 36.0);
    double Cx[3], Cy[3], Gx_[3], Gy_[3];
    for (int r = 0; r < 3; ++r) {
      Cx[r] = Cm[r][0] * x[0] + Cm[r][1] * x[1] + Cm[r][2] * x[2];
      Cy[r] = Cm[r][0] * y[0] + Cm[r][1] * y[1] + Cm[r][2] * y[2];
      Gx_[r] = GS[r][0] * x[0] + GS[r][1] * x[1] + GS[r][2] * x[2];
      Gy_[r] = GS[r][0] * y[0] + GS[r][1] * y[1] + GS[r][2] * y[2];
    }
    const double a = x[0] * Cx[0] + x[1] * Cx[1] + x[2] * Cx[2];
    const double b = y[0] * Cy[0] + y[1] * Cy[1] + y[2] * Cy[2];
    const double gxs = x[0] * Gx_[0] + x[1] * Gx_[1] + x[2] * Gx_[2];
    const double gys = y[0] * Gy_[0] + y[1] * Gy_[1] + y[2] * Gy_[2];
    const double kp = g.kappa;
    // through C: G_C = kappa (gxs x x' + gys y y'), and C's edge form as in the other modes
    for (int r = 0; r < 3; ++r) {
      const double xe1 = x[0] * e1[0] + x[1] * e1[1] + x[2] * e1[2], xe2 = x[0] * e2[0] + x[1] * e2[1] + x[2] * e2[2];
      const double ye1 = y[0] * e1[0] + y[1] * e1[1] + y[2] * e1[2], ye2 = y[0] * e2[0] + y[1] * e2[1] + y[2] * e2[2];
      const double G1 = kp * (gxs * x[r] * xe1 + gys * y[r] * ye1);
      const double G2 = kp * (gxs * x[r] * xe2 + gys * y[r] * ye2);
      Ge1[r] = (4.0 * G1 - 2.0 * G2) * (1.0 / 36.0);
      Ge2[r] = (4.0 * G2 - 2.0 * G1) * (1.0 / 36.0);
    }
    // through the frame
    double Gx[3], Gy[3], Gn[3];
    for (int r = 0; r < 3; ++r) {
      Gx[r] = 2.0 * kp * (gxs * Cx[r] + a * Gx_[r]);
      Gy[r] = 2.0 * kp * (gys * Cy[r] + b * Gy_[r]);
      Gn[r] = 2.0 * kSz2 * (GS[r][0] * n[0] + GS[r][1] * n[1] + GS[r][2] * n[2]);
    }
    // y = n x x: dL/dn += x x Gy, dL/dx += Gy x n
    Gn[0] += x[1] * Gy[2] - x[2] * Gy[1];
    Gn[1] += x[2] * Gy[0] - x[0] * Gy[2];
    Gn[2] += x[0] * Gy[1] - x[1] * Gy[0];
    Gx[0] += Gy[1] * n[2] - Gy[2] * n[1];
    Gx[1] += Gy[2] * n[0] - Gy[0] * n[2];
    Gx[2] += Gy[0] * n[1] - Gy[1] * n[0];
    const double xGx = x[0] * Gx[0] + x[1] * Gx[1] + x[2] * Gx[2];
    for (int r = 0; r < 3; ++r) Ge1[r] += (Gx[r] - x[r] * xGx) / l1;
    const double nGn = n[0] * Gn[0] + n[1] * Gn[1] + n[2] * Gn[2];
    double Gm[3];
    for (int r = 0; r < 3; ++r) Gm[r] = (Gn[r] - n[r] * nGn) * inv;
    if (g.clamped) {  // kappa = |m| / (2 pi sqrt(eps))
      const double gk = a * gxs + b * gys;
      for (int r = 0; r < 3; ++r) Gm[r] += gk * n[r] / (2.0 * kPi * sqrt(kEpsL));
    }
    Ge1[0] += e2[1] * Gm[2] - e2[2] * Gm[1];
    Ge1[1] += e2[2] * Gm[0] - e2[0] * Gm[2];
    Ge1[2] += e2[0] * Gm[1] - e2[1] * Gm[0];
    Ge2[0] += Gm[1] * e1[2] - Gm[2] * e1[1];
    Ge2[1] += Gm[2] * e1[0] - Gm[0] * e1[2];
    Ge2[2] += Gm[0] * e1[1] - Gm[1] * e1[0];
  } else {
  const double scale = (o.cov_mode == 1 ? 1.0 : g.kappa) / 36.0;
  for (int r = 0; r < 3; ++r) {
    const double G1 = GS[r][0] * e1[0] + GS[r][1] * e1[1] + GS[r][2] * e1[2];
    const double G2 = GS[r][0] * e2[0] + GS[r][1] * e2[1] + GS[r][2] * e2[2];
    Ge1[r] = scale * (4.0 * G1 - 2.0 * G2);
    Ge2[r] = scale * (4.0 * G2 - 2.0 * G1);
  }
  if (o.cov_mode == 0) {
    const double inv = 1.0 / g.mm;
    const double n[3] = {g.m[0] * inv, g.m[1] * inv, g.m[2] * inv};
    double Gn[3];
    for (int r = 0; r < 3; ++r) Gn[r] = 2.0 * kSz2 * (GS[r][0] * n[0] + GS[r][1] * n[1] + GS[r][2] * n[2]);
    const double nGn = n[0] * Gn[0] + n[1] * Gn[1] + n[2] * Gn[2];
    double Gm[3];
    for (int r = 0; r < 3; ++r) Gm[r] = (Gn[r] - n[r] * nGn) * inv;
    if (g.clamped) {
      double M[6];
      M[0] = 2.0 * e1[0] * e1[0] + 2.0 * e2[0] * e2[0] - 2.0 * e1[0] * e2[0];
      M[1] = 2.0 * e1[0] * e1[1] + 2.0 * e2[0] * e2[1] - e1[0] * e2[1] - e2[0] * e1[1];
      M[2] = 2.0 * e1[0] * e1[2] + 2.0 * e2[0] * e2[2] - e1[0] * e2[2] - e2[0] * e1[2];
      M[3] = 2.0 * e1[1] * e1[1] + 2.0 * e2[1] * e2[1] - 2.0 * e1[1] * e2[1];
      M[4] = 2.0 * e1[1] * e1[2] + 2.0 * e2[1] * e2[2] - e1[1] * e2[2] - e2[1] * e1[2];
      M[5] = 2.0 * e1[2] * e1[2] + 2.0 * e2[2] * e2[2] - 2.0 * e1[2] * e2[2];
      const double trGM = GS[0][0] * M[0] + GS[1][1] * M[3] + GS[2][2] * M[5] +
                          2.0 * (GS[0][1] * M[1] + GS[0][2] * M[2] + GS[1][2] * M[4]);
      const double gA = trGM / 36.0 / (kPi * sqrt(kEpsL));
      for (int r = 0; r < 3; ++r) Gm[r] += 0.5 * gA * n[r];
    }
    // m = e1 x e2
    Ge1[0] += e2[1] * Gm[2] - e2[2] * Gm[1];
    Ge1[1] += e2[2] * Gm[0] - e2[0] * Gm[2];
    Ge1[2] += e2[0] * Gm[1] - e2[1] * Gm[0];
    Ge2[0] += Gm[1] * e1[2] - Gm[2] * e1[1];
    Ge2[1] += Gm[2] * e1[0] - Gm[0] * e1[2];
    Ge2[2] += Gm[0] * e1[1] - Gm[1] * e1[0];
  }
  }
  float gv[9];
  for (int r = 0; r < 3; ++r) {
    const double gm3 = Gmu[r] * (1.0 / 3.0);
    gv[r] = (float)(-Ge1[r] - Ge2[r] + gm3);
    gv[3 + r] = (float)(Ge1[r] + gm3);
    gv[6 + r] = (float)(Ge2[r] + gm3);
  }
  out[0] = make_float4(gv[0], gv[1], gv[2], gv[3]);
  out[1] = make_float4(gv[4], gv[5], gv[6], gv[7]);
  out[2] = make_float4(gv[8], gcol[0], gcol[1], gcol[2]);
  if constexpr (SHD > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int a = 0; a < 3; ++a) fsh[3 * K * f + 3 * k + a] = gsh[k][a];
  }
}

namespace {
// Sum of (a, b) over the 256 threads of a block in a fixed order; valid in thread 0.
__device__ inline void block_sum2(double& a, double& b, double* s_a, double* s_b) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    a += __shfl_xor(a, d, kWave);
    b += __shfl_xor(b, d, kWave);
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { s_a[w] = a; s_b[w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = s_a[0]; b = s_b[0];
    for (int i = 1; i < 256 / kWave; ++i) { a += s_a[i]; b += s_b[i]; }
  }
  __syncthreads();
}
__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ inline double bitsd(unsigned long long x) { return __longlong_as_double((long long)x); }
}  // namespace

// Fused-loss backward: the colour and silhouette losses as a deterministic sum of the per-item
// slots.  Block b < r.nb sums a contiguous chunk; the block that takes the last ticket sums the
// block results in block order and writes the header (and `out`, n_out floats, when given).
// Every thread of the block calls it (it synchronises the block).
__device__ inline void loss_reduce_block(const LossRed& r, int b) {
  __shared__ double s_a[256 / kWave], s_b[256 / kWave];
  __shared__ bool s_last;
  const int nb = r.nb;
  const int chunk = (r.items + nb - 1) / nb;
  const int lo = b * chunk, hi = min(r.items, lo + chunk);
  double l = 0.0, ls = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
    const float4 v = r.stats[i];
    l += (double)v.x;
    ls += (double)v.y;
  }
  block_sum2(l, ls, s_a, s_b);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&r.part[2 * b], dbits(l), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&r.part[2 * b + 1], dbits(ls), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t t = __hip_atomic_fetch_add(&r.hdr->red_ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = t == (uint32_t)nb - 1u;
  }
  __syncthreads();
  if (!s_last) return;  // uniform across the block
  __threadfence();
  l = 0.0; ls = 0.0;
  if ((int)threadIdx.x < nb) {
    l = bitsd(__hip_atomic_load(&r.part[2 * threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    ls = bitsd(__hip_atomic_load(&r.part[2 * threadIdx.x + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  block_sum2(l, ls, s_a, s_b);
  if (threadIdx.x == 0) {
    r.hdr->loss = (float)l;
    r.hdr->loss_sil = (float)ls;
    if (r.out) {
      r.out[0] = (float)l;
      if (r.n_out > 1) r.out[1] = (float)ls;
    }
    r.hdr->red_ticket = 0u;
  }
}

__global__ __launch_bounds__(256) void k_loss_reduce(LossRed r) { loss_reduce_block(r, (int)blockIdx.x); }

// Corner sums of one vertex: x[0..3) position gradient, x[3 + 3k + channel] colour (coefficient k)
// gradient.
template <int SHD>
struct VertexAcc {
  static constexpr int n = 3 + 3 * sh_count<SHD>();
  float x[n];
};

// Adds the corners e0, e0 + step, ... < e1 of the (vertex -> face, corner) CSR to a.
template <int SHD>
__device__ inline void gather_corners(const int32_t* __restrict__ ent, const float* __restrict__ fgrad,
                                      const float* __restrict__ fsh, int32_t e0, int32_t e1, int32_t step,
                                      VertexAcc<SHD>& a) {
  constexpr int K = sh_count<SHD>();
  for (int32_t e = e0; e < e1; e += step) {
    const int32_t fc = ent[e];
    const int32_t f = fc / 3, corner = fc - 3 * f;
    const float* p = fgrad + 12 * (int64_t)f;
    a.x[0] += p[3 * corner];
    a.x[1] += p[3 * corner + 1];
    a.x[2] += p[3 * corner + 2];
    if constexpr (SHD == 0) {
      a.x[3] += p[9];
      a.x[4] += p[10];
      a.x[5] += p[11];
    } else {
      const float* q = fsh + (int64_t)3 * K * f;
#pragma unroll
      for (int k = 0; k < 3 * K; ++k) a.x[3 + k] += q[k];
    }
  }
}

template <int SHD>
__device__ inline void write_vertex(const VertexAcc<SHD>& a, int64_t v, float* __restrict__ dV, float* __restrict__ dC) {
  constexpr int K = sh_count<SHD>();
  const float third = 1.f / 3.f;
  dV[3 * v] = a.x[0]; dV[3 * v + 1] = a.x[1]; dV[3 * v + 2] = a.x[2];
#pragma unroll
  for (int k = 0; k < 3 * K; ++k) dC[(int64_t)v * 3 * K + k] = a.x[3 + k] * third;
}

// Vertices with more corners than this (the poles of a UV sphere have hundreds) are gathered by a
// whole wavefront, so no lane serialises a long run of dependent loads while the others wait.
constexpr int32_t kCoopCorners = 32;

template <int SHD>
__global__ __launch_bounds__(256) void k_vertex_gather(const int32_t* __restrict__ off, const int32_t* __restrict__ ent,
                                                       const float* __restrict__ fgrad, const float* __restrict__ fsh,
                                                       int64_t nv, float* __restrict__ dV, float* __restrict__ dC,
                                                       LossRed red) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int32_t e0 = 0, e1 = 0;
  if (v < nv) {
    e0 = off[v];
    e1 = off[v + 1];
  }
  const bool coop = e1 - e0 > kCoopCorners;
  if (v < nv && !coop) {
    VertexAcc<SHD> a{};
    gather_corners<SHD>(ent, fgrad, fsh, e0, e1, 1, a);
    write_vertex<SHD>(a, v, dV, dC);
  }
  // high-degree vertices, one at a time: lane l takes corners l, l + 64, ..., then a fixed-order
  // tree sum over the wavefront (deterministic)
  uint64_t m = __ballot(coop);
  while (m) {
    const int l = __builtin_ctzll(m);
    m &= m - 1;
    const int32_t b0 = __shfl(e0, l, kWave), b1 = __shfl(e1, l, kWave);
    VertexAcc<SHD> a{};
    gather_corners<SHD>(ent, fgrad, fsh, b0 + lane, b1, kWave, a);
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1)
#pragma unroll
      for (int i = 0; i < VertexAcc<SHD>::n; ++i) a.x[i] += __shfl_xor(a.x[i], d, kWave);
    if (lane == 0) write_vertex<SHD>(a, (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane) + l, dV, dC);
  }
  if (red.stats && (int)blockIdx.x < red.nb) loss_reduce_block(red, (int)blockIdx.x);  // block-uniform
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int64_t n, float val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = val;
}

// Start of a backward: the workspace's backward counters and, unless a rebuild of the lists has
// already cleared them, the face-view gradient accumulators.
__global__ __launch_bounds__(256) void k_bwd_prologue(WsHdr* __restrict__ hdr, float* __restrict__ dfv, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < n; i += (int64_t)gridDim.x * blockDim.x) dfv[i] = 0.f;
  if (t == 0) {
    hdr->bwd_stats = 1u;
    hdr->loss = 0.f;
    hdr->loss_sil = 0.f;
    hdr->red_ticket = 0u;
  }
}


// Adam with bias correction; t = step + 1 is read from the device (advanced by k_adam_tick).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                              const int32_t* __restrict__ step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float t = (float)(*step + 1);
  const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_adam_tick(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

void launch_face_bwd(const void* table, int64_t faces_total, const float* verts, const int32_t* faces,
                     const float* colors, const KOpts& o, const float4* dfv, float4* fgrad, float* fsh, int max_views,
                     hipStream_t s) {
  if (faces_total <= 0) return;
  // 8 lanes per face when the faces alone would leave most of the GPU idle (fewer than 256 per CU)
  const bool split = o.sh_degree == 0 && max_views > 1 && faces_total < 256 * 256;
  const int lpf = split ? 8 : 1;
  const dim3 grid((unsigned)((faces_total * lpf + 255) / 256));
  if (split) {
    hipLaunchKernelGGL((k_face_bwd<0, 8>), grid, dim3(256), 0, s, table, verts, faces, colors, o, dfv, fgrad, fsh);
    return;
  }
  switch (o.sh_degree) {
    case 1: hipLaunchKernelGGL((k_face_bwd<1, 1>), grid, dim3(256), 0, s, table, verts, faces, colors, o, dfv, fgrad, fsh); break;
    case 2: hipLaunchKernelGGL((k_face_bwd<2, 1>), grid, dim3(256), 0, s, table, verts, faces, colors, o, dfv, fgrad, fsh); break;
    case 3: hipLaunchKernelGGL((k_face_bwd<3, 1>), grid, dim3(256), 0, s, table, verts, faces, colors, o, dfv, fgrad, fsh); break;
    default: hipLaunchKernelGGL((k_face_bwd<0, 1>), grid, dim3(256), 0, s, table, verts, faces, colors, o, dfv, fgrad, fsh); break;
  }
}

void launch_loss_reduce(const LossRed& r, hipStream_t s) {
  LossRed q = r;
  q.nb = std::max(1, std::min(kLossReduceBlocks, (r.items + 2047) / 2048));
  hipLaunchKernelGGL(k_loss_reduce, dim3((unsigned)q.nb), dim3(256), 0, s, q);
}

void launch_vertex_gather(const int32_t* off, const int32_t* ent, const float* fgrad, const float* fsh, int sh_degree,
                          int64_t nv, float* dV, float* dC, const LossRed* red, hipStream_t s) {
  if (nv <= 0) {
    if (red) launch_loss_reduce(*red, s);
    return;
  }
  const int64_t blocks = (nv + 255) / 256;
  LossRed q{};
  if (red) {
    q = *red;
    // every gather block up to kLossReduceBlocks takes a share (shorter chunks, shorter tail)
    q.nb = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kLossReduceBlocks, red->items), blocks));
  }
  const dim3 grid((unsigned)blocks);
  switch (sh_degree) {
    case 1: hipLaunchKernelGGL(k_vertex_gather<1>, grid, dim3(256), 0, s, off, ent, fgrad, fsh, nv, dV, dC, q); break;
    case 2: hipLaunchKernelGGL(k_vertex_gather<2>, grid, dim3(256), 0, s, off, ent, fgrad, fsh, nv, dV, dC, q); break;
    case 3: hipLaunchKernelGGL(k_vertex_gather<3>, grid, dim3(256), 0, s, off, ent, fgrad, fsh, nv, dV, dC, q); break;
    default: hipLaunchKernelGGL(k_vertex_gather<0>, grid, dim3(256), 0, s, off, ent, fgrad, fsh, nv, dV, dC, q); break;
  }
}

void launch_fill_f32(float* p, int64_t n, float val, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)nb), dim3(256), 0, s, p, n, val);
}

void launch_bwd_prologue(WsHdr* hdr, float* dfv, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  nb = nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
  hipLaunchKernelGGL(k_bwd_prologue, dim3((unsigned)nb), dim3(256), 0, s, hdr, dfv, n);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t* step, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, step);
  launch_adam_tick(step, s);
}

void launch_adam_tick(int32_t* step, hipStream_t s) { hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, step); }

}  // namespace gmr
