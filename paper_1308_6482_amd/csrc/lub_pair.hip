// lub_pair.hip -- per-pair closest points, local geometry, resistance and
// transfer (gfx950).  One lane per pair.
//
// Closest points (Sec. III.A).  The paper's fixed point -- outward normals
// antiparallel and along the line joining the tangent points -- is, with
// the tangent points written as support points y_i = r_i + M_i n / h_i(n),
// y_j = r_j - M_j n / h_j(n) (h_k(n) = sqrt(n.M_k n)), the stationary point
// of g(n) = n.d - h_i(n) - h_j(n) on the unit sphere; g there is the signed
// gap (negative for a small overlap).  It is found by Newton's method in the
// tangent plane of n (two unknowns), started from the line of centres
// mapped by (M_i + M_j)^-1 (the normal of an ellipsoid standing in for the
// two bodies' Minkowski sum), in FP64.  The Riemannian Hessian is shifted to stay negative definite far
// from the solution.  This replaces the paper's Lin-Han tangent-sphere
// iteration (linear convergence, ~40 iterations for aspect ratio 1/3) by a
// quadratically convergent one that needs no pole-safe parametrisation.
//
// Local geometry (Sec. III.B).  For a spheroid the outward normal at
// parametric latitude p satisfies tan(angle to the equator) =
// (R_par/R_perp) tan p, so (cos p, sin p) follows from the normal's axial
// component alone, and the principal direction x1 = d y / d p is the
// projection of the symmetry axis onto the tangent plane.  Radii S1, S2
// and the cubic coefficients Gamma_0, Gamma_2 follow Eq. lub:curvature-radii
// and the Gamma formulas of Sec. III.B; phi, lambda, chi, beta, k and kappa
// follow the Appendix.
//
// Resistance (Appendix, Eqs. app:first-element .. app:last-element), with
// the cut-off correction of Eq. lub:resistance-correction at the clipped gap
// max(h, h_c) and the Hookean contact of Eqs. lub:frep / lub:model; transfer
// to the particle centres as at the end of Sec. III.B.
//
// Records.  The kernels gather a 64-B copy per particle (centre, axis, radii)
// and form the support matrix M in registers with the staging's expression.
// The previous call's normal (warm start) comes from the previous slot range
// of one of the pair's particles (a few consecutive slots, each with the
// xor of its pair's input indices),
// or, with reused neighbour lists, from a slot per superset entry tagged with
// the search that made the superset.
//
// Precision.  R = double: every step in FP64.  R = float: the Newton solve,
// the gap, the frame vectors, the latitudes, the curvature radii and cubic
// coefficients, the eigen-decomposition of the gap matrix, the relative
// surface velocities and their projections, and the ln(h/Delta),
// 1/h - 1/Delta factors are computed in FP64; the 16 coefficients of K (from
// those inputs rounded to FP32), the 6 x 6 product and the transfer run in
// FP32.  (Taking the geometry to
// FP32 as well measured 1.5 % less pair-kernel time and three times the
// largest per-pair error on the full-scale suspension, 6.3e-6 against
// 1.9e-6, next to the 1e-5 bar.)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lub_internal.h"
#include "lub_newton.h"

namespace lub {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Canonical pair frame of a spheroid with unit symmetry axis ax seen from
// its partner at offset d: rows x, y, z; z = +-ax towards the partner,
// x = the part of d normal to z (any normal if d lies on the axis).
__host__ __device__ __forceinline__ void canonical_frame(const double ax[3],
                                                        const double d[3],
                                                        double F[3][3]) {
  const double sg = dot3(ax, d) < 0.0 ? -1.0 : 1.0;
  double z[3] = {sg * ax[0], sg * ax[1], sg * ax[2]};
  const double dz = dot3(d, z);
  double x[3] = {d[0] - dz * z[0], d[1] - dz * z[1], d[2] - dz * z[2]};
  const double nx = sqrt(dot3(x, x));
  if (nx <= 1e-12 * fmax(sqrt(dot3(d, d)), 1e-300)) {
    perp(z, x);
  } else {
    for (int k = 0; k < 3; ++k) x[k] /= nx;
  }
  double y[3];
  cross3(z, x, y);
  for (int k = 0; k < 3; ++k) {
    F[0][k] = x[k];
    F[1][k] = y[k];
    F[2][k] = z[k];
  }
}

// the ten seed features: d in frame i / R_perp,i; the rotation from frame i
// to frame j as a unit quaternion (w >= 0); three shape ratios
__host__ __device__ __forceinline__ void seed_features(const double d[3],
                                                      const PRec& A,
                                                      const PRec& B, float X[10]) {
  double Fi[3][3], Fj[3][3], md[3] = {-d[0], -d[1], -d[2]};
  canonical_frame(A.ax, d, Fi);
  canonical_frame(B.ax, md, Fj);
  const double rp = A.Rperp;
  for (int a = 0; a < 3; ++a) X[a] = (float)(dot3(Fi[a], d) / rp);
  double R[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R[a][b] = dot3(Fi[a], Fj[b]);
  const double tr = R[0][0] + R[1][1] + R[2][2];
  double q[4];
  q[0] = sqrt(fmax(0.0, 1.0 + tr)) / 2.0;
  q[1] = copysign(sqrt(fmax(0.0, 1.0 + R[0][0] - R[1][1] - R[2][2])) / 2.0, R[2][1] - R[1][2]);
  q[2] = copysign(sqrt(fmax(0.0, 1.0 - R[0][0] + R[1][1] - R[2][2])) / 2.0, R[0][2] - R[2][0]);
  q[3] = copysign(sqrt(fmax(0.0, 1.0 - R[0][0] - R[1][1] + R[2][2])) / 2.0, R[1][0] - R[0][1]);
  const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int a = 0; a < 4; ++a) X[3 + a] = (float)(q[a] / qn);
  X[7] = (float)(A.Rpar / rp);
  X[8] = (float)(B.Rpar / rp);
  X[9] = (float)(B.Rperp / rp);
}

// seed normal from predicted surface parameters (p, q) of both particles:
// the outward normal of i at its point and minus that of j, averaged
__host__ __device__ __forceinline__ bool seed_normal(const double d[3], const PRec& A,
                                                    const PRec& B, const float Y[4],
                                                    double n0[3]) {
  double Fi[3][3], Fj[3][3], md[3] = {-d[0], -d[1], -d[2]};
  canonical_frame(A.ax, d, Fi);
  canonical_frame(B.ax, md, Fj);
  double ni[3] = {0, 0, 0}, nj[3] = {0, 0, 0};
  const double nbi[3] = {cos((double)Y[0]) * cos((double)Y[1]) / A.Rperp,
                         cos((double)Y[0]) * sin((double)Y[1]) / A.Rperp,
                         sin((double)Y[0]) / A.Rpar};
  const double nbj[3] = {cos((double)Y[2]) * cos((double)Y[3]) / B.Rperp,
                         cos((double)Y[2]) * sin((double)Y[3]) / B.Rperp,
                         sin((double)Y[2]) / B.Rpar};
  const double ili = inv_sqrt(dot3(nbi, nbi)), ilj = inv_sqrt(dot3(nbj, nbj));
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      ni[k] += Fi[a][k] * (nbi[a] * ili);
      nj[k] += Fj[a][k] * (nbj[a] * ilj);
    }
  double m[3] = {ni[0] - nj[0], ni[1] - nj[1], ni[2] - nj[2]};
  const double mn2 = dot3(m, m);
  if (!(mn2 > 1e-12) || !(dot3(m, d) > 0.0)) return false;
  const double imn = inv_sqrt(mn2);
  for (int k = 0; k < 3; ++k) n0[k] = m[k] * imn;
  return true;
}

// (cos p, sin p) of the spheroid surface point whose outward unit normal is
// n, from the cosine c = n.ax of the angle between normal and symmetry axis,
// plus x1 = d y / d p: the axis projected onto the tangent plane
__host__ __device__ __forceinline__ void latitude(const double n[3],
                                                  const double ax[3], double Rpa,
                                                  double Rpe, double* cp,
                                                  double* sp, double e1[3]) {
  const double c = dot3(n, ax);
  double x[3];
  cross3(n, ax, x);
  double rho = sqrt(dot3(x, x));
  double a = Rpe * rho, b = Rpa * c;
  const double inr = inv_sqrt(a * a + b * b);
  *cp = a * inr;
  *sp = b * inr;
  double t[3] = {ax[0] - c * n[0], ax[1] - c * n[1], ax[2] - c * n[2]};
  const double tl2 = dot3(t, t);
  if (tl2 > 1e-24) {
    const double itl = inv_sqrt(tl2);
    for (int k = 0; k < 3; ++k) e1[k] = t[k] * itl;
  } else {
    perp(n, e1);  // pole: S1 = S2 and Gamma = 0, any tangent will do
  }
}

// principal radii, their reciprocals and the two non-zero cubic
// coefficients of a spheroid (two divisions: 1 / (Rpa Rpe), 1 / (s1^3 Rpe))
template <typename R>
__host__ __device__ __forceinline__ void radii(R Rpa, R Rpe, R cp, R sp, R* S1, R* S2,
                                      R* iS1, R* iS2, R* G0, R* G2) {
  R s1sq = Rpe * Rpe * sp * sp + Rpa * Rpa * cp * cp;
  R s1 = sqrt(s1sq);
  const R s3 = s1sq * s1;
  const R iab = R(1) / (Rpa * Rpe);
  const R x = R(1) / (s3 * Rpe);
  *S1 = s3 * iab;                 // s1^3 / (Rpa Rpe)
  *S2 = Rpe * Rpe * s1 * iab;     // Rpe s1 / Rpa
  *iS1 = Rpa * Rpe * Rpe * x;     // Rpa Rpe / s1^3
  *iS2 = Rpa * s1sq * x;          // Rpa / (Rpe s1)
  R num = (Rpa * Rpa - Rpe * Rpe) * Rpa * sp * cp;
  const R x2 = x * x;             // 1 / (s1^6 Rpe^2)
  *G0 = R(0.5) * num * Rpe * Rpe * Rpe * x2;  // num Rpe / (2 s1^6)
  *G2 = R(0.5) * num * s1sq * Rpe * x2;       // num / (2 Rpe s1^4)
}

// cubic coefficients a (given in axes rotated by +alpha) in unrotated axes
// ---------------------------------------------------------------------------
// Last resort: the tangent-sphere iteration of Sec. III.A (Lin and Han), on
// the surfaces x^T A x = 1, A = (I - a a^T) / Rperp^2 + a a^T / Rpar^2.

// quadratic form of a spheroid with unit axis a at x, and its bilinear form
__host__ __device__ __forceinline__ double sph_q(const PRec& P, const double x[3]) {
  const double ax = dot3(P.ax, x);
  return (dot3(x, x) - ax * ax) / (P.Rperp * P.Rperp) + ax * ax / (P.Rpar * P.Rpar);
}

__host__ __device__ __forceinline__ double sph_b(const PRec& P, const double x[3],
                                                 const double u[3]) {
  const double ax = dot3(P.ax, x), au = dot3(P.ax, u);
  return (dot3(x, u) - ax * au) / (P.Rperp * P.Rperp) + ax * au / (P.Rpar * P.Rpar);
}

// Where the ray x0 + t u (t > 0, u unit, x0 relative to the centre) leaves
// the surface: the larger root of q(x0 + t u) = 1, also from a start
// outside the body when the ray still crosses it.
__host__ __device__ __forceinline__ bool ray_exit(const PRec& P, const double x0[3],
                                                  const double u[3], double y[3]) {
  const double qa = sph_q(P, u), qb = sph_b(P, x0, u), qc = sph_q(P, x0) - 1.0;
  const double disc = qb * qb - qa * qc;
  if (!(disc >= 0.0) || !(qa > 0.0)) return false;
  const double t = (-qb + sqrt(disc)) / qa;
  if (!(t > 0.0)) return false;
  for (int k = 0; k < 3; ++k) y[k] = x0[k] + t * u[k];
  return true;
}

// outward unit normal at the surface point y (relative to the centre)
__host__ __device__ __forceinline__ void sph_normal(const PRec& P, const double y[3],
                                                    double n[3]) {
  const double ay = dot3(P.ax, y);
  const double ip = 1.0 / (P.Rperp * P.Rperp), ia = 1.0 / (P.Rpar * P.Rpar);
  for (int k = 0; k < 3; ++k) n[k] = (y[k] - ay * P.ax[k]) * ip + ay * P.ax[k] * ia;
  const double ln = sqrt(dot3(n, n));
  for (int k = 0; k < 3; ++k) n[k] /= ln;
}

// smaller principal radius of curvature at the surface point y (Eq.
// lub:curvature-radii), or the conservative radius of Eq. lub:minimum-radius
__host__ __device__ __forceinline__ double sph_radius(const PRec& P, const double y[3],
                                                      bool local) {
  if (!local) {
    if (P.Rpar < P.Rperp) return P.Rpar * P.Rpar / P.Rperp;
    if (P.Rpar > P.Rperp) return P.Rperp * P.Rperp / P.Rpar;
    return P.Rpar;
  }
  const double ay = dot3(P.ax, y);
  double sp = ay / P.Rpar;
  double cp = sqrt(fmax(dot3(y, y) - ay * ay, 0.0)) / P.Rperp;
  const double l = sqrt(sp * sp + cp * cp);
  sp /= l;
  cp /= l;
  double S1, S2, iS1, iS2, G0, G2;
  radii<double>(P.Rpar, P.Rperp, cp, sp, &S1, &S2, &iS1, &iS2, &G0, &G2);
  return fmin(S1, S2);
}

// The two-fold strategy: up to n1 iterations with the local radii (accepted
// only if the normals face the other centre and, for an overlap, each point
// lies inside the other particle), else from the line of centres again with
// the conservative radii for up to n2.  Returns the direction between the
// final sphere centres (i -> j), the start of a Newton polish.
__host__ __device__ bool tangent_spheres(const double d[3], const PRec& A, const PRec& B,
                                         double nout[3]) {
  constexpr int kN1 = 10, kN2 = 1000;
  constexpr double kEps = 1e-6;
  const double dn = sqrt(dot3(d, d));
  if (!(dn > 0.0)) return false;
  const double zero[3] = {0.0, 0.0, 0.0};
  for (int phase = 0; phase < 2; ++phase) {
    const bool local = phase == 0;
    double u[3] = {d[0] / dn, d[1] / dn, d[2] / dn}, mu[3] = {-u[0], -u[1], -u[2]};
    double yi[3], yj[3], ni[3], nj[3];  // yj relative to j's centre
    if (!ray_exit(A, zero, u, yi) || !ray_exit(B, zero, mu, yj)) return false;
    sph_normal(A, yi, ni);
    sph_normal(B, yj, nj);
    const int nmax = local ? kN1 : kN2;
    for (int it = 0; it < nmax; ++it) {
      const double si = sph_radius(A, yi, local), sj = sph_radius(B, yj, local);
      double zi[3], zj[3], w[3];
      for (int k = 0; k < 3; ++k) {
        zi[k] = yi[k] - si * ni[k];           // relative to i's centre
        zj[k] = yj[k] - sj * nj[k];           // relative to j's centre
        w[k] = d[k] + zj[k] - zi[k];          // z_j - z_i
      }
      const double lw = sqrt(dot3(w, w));
      if (!(lw > 0.0)) break;
      for (int k = 0; k < 3; ++k) {
        u[k] = w[k] / lw;
        mu[k] = -u[k];
      }
      // converged: both normals along the line of the sphere centres
      if (dot3(ni, u) > 1.0 - kEps && dot3(nj, mu) > 1.0 - kEps) {
        bool ok = dot3(ni, d) > 0.0 && dot3(nj, d) < 0.0;
        if (ok && lw < si + sj) {  // overlap: each point inside the other body
          double yi_j[3], yj_i[3];
          for (int k = 0; k < 3; ++k) {
            yi_j[k] = yi[k] - d[k];
            yj_i[k] = yj[k] + d[k];
          }
          ok = sph_q(B, yi_j) <= 1.0 && sph_q(A, yj_i) <= 1.0;
        }
        // the conservative phase's result is taken as it is: the Newton
        // polish that follows judges it
        if (!local || ok) {
          for (int k = 0; k < 3; ++k) nout[k] = u[k];
          return true;
        }
        break;  // the local radii gave no meaningful result: conservative phase
      }
      if (!ray_exit(A, zi, u, yi) || !ray_exit(B, zj, mu, yj)) break;
      sph_normal(A, yi, ni);
      sph_normal(B, yj, nj);
    }
  }
  return false;
}

template <typename R>
__host__ __device__ __forceinline__ void rotate_cubic(R c, R s, const R a[4], R m[4]) {
  R c2 = c * c, s2 = s * s;
  m[0] = a[0] * c2 * c - a[1] * s * c2 + a[2] * s2 * c - a[3] * s2 * s;
  m[1] = R(3) * a[0] * s * c2 + a[1] * (c2 * c - R(2) * s2 * c) +
         a[2] * (s2 * s - R(2) * s * c2) + R(3) * a[3] * s2 * c;
  m[2] = R(3) * a[0] * c * s2 + a[1] * (R(2) * c2 * s - s2 * s) +
         a[2] * (c2 * c - R(2) * c * s2) - R(3) * a[3] * c2 * s;
  m[3] = a[0] * s2 * s + a[1] * c * s2 + a[2] * c2 * s + a[3] * c2 * c;
}

// The 16 singular coefficients: K = C ln h (C33 / h for the normal one).
// Index order 11 12 13 14 15 22 23 24 25 33 34 35 36 44 45 55.
template <typename R>
__host__ __device__ __forceinline__ void k_coeffs(R S1, R S2, double iS1d, double iS2d, R G0,
                                         R G2, R iS1p, R iS2p, R G0p, R G2p, R cph,
                                         R sph, R C[16]) {
  const R pi = R(kPi);
  // quadratic gap matrix and its eigen-decomposition: a few flops, in FP64
  // (errors in chi propagate into every coupling term)
  double m11 = 0.5 * iS1d + 0.5 * ((double)cph * cph * iS1p + (double)sph * sph * iS2p);
  double m22 = 0.5 * iS2d + 0.5 * ((double)sph * sph * iS1p + (double)cph * cph * iS2p);
  double m12 = 0.5 * (double)sph * cph * ((double)iS1p - iS2p);
  double half = 0.5 * (m11 - m22);
  double rad = sqrt(half * half + m12 * m12);
  double dl1 = 0.5 * (m11 + m22) + rad;
  double dl2 = (m11 * m22 - m12 * m12) / dl1;
  // chi: eigenvector of l1 is (cos chi, -sin chi)
  double dc = 1.0, ds = 0.0;
  if (rad > 0.0) {
    const double irad = 1.0 / rad;
    double c2x = half * irad, s2x = -m12 * irad;
    if (c2x >= 0.0) {
      dc = sqrt(0.5 * (1.0 + c2x));
      ds = s2x / (2.0 * dc);
    } else {
      ds = sqrt(0.5 * (1.0 - c2x));
      ds = s2x < 0.0 ? -ds : ds;
      dc = s2x / (2.0 * ds);
    }
  }
  const R l1 = R(dl1), l2 = R(dl2), c = R(dc), s = R(ds);
  // beta = m(phi, Gamma'), k = Gamma + beta, kappa = m(chi, k) rescaled
  R gp[4] = {G0p, R(0), G2p, R(0)}, beta[4];
  rotate_cubic(cph, sph, gp, beta);
  R kk[4] = {G0 + beta[0], beta[1], G2 + beta[2], beta[3]};
  R mk[4];
  rotate_cubic(c, s, kk, mk);
  // the divisions by sqrt(l), l, A and B as products with their reciprocals
  const R iq1 = inv_sqrt(l1), iq2 = inv_sqrt(l2);
  const R q1 = l1 * iq1, q2 = l2 * iq2;
  const R il1 = iq1 * iq1, il2 = iq2 * iq2;
  R k0 = mk[0] * (il1 * iq1), k1 = mk[1] * (il1 * iq2);
  R k2 = mk[2] * (iq1 * il2), k3 = mk[3] * (il2 * iq2);

  R lsum = l1 + l2;
  R A = R(3) * l1 + R(2) * l2, B = R(2) * l1 + R(3) * l2;
  const R iA = R(1) / A, iB = R(1) / B;
  R p1 = iA * il1, p2 = iB * il2;
  R cc = c * c, ss = s * s, sc = s * c;
  R isl = iq1 * iq2;
  R u1 = R(1) - l1 * S1, u2 = R(1) - l2 * S1;
  R w1 = R(1) - l1 * S2, w2 = R(1) - l2 * S2;
  const R iS1 = R(iS1d), iS2 = R(iS2d);
  // translation-translation and translation-rotation (curvature only)
  C[0] = -pi * isl * iS1 * iS1 * (R(3) * cc * u1 * u1 * p1 + R(3) * ss * u2 * u2 * p2 + S1 * S1);
  C[1] = R(3) * pi * isl * iS1 * iS2 * sc * (u1 * w1 * p1 - u2 * w2 * p2);
  C[3] = R(3) * pi * isl * iS1 * sc * (u1 * p1 - u2 * p2);
  C[4] = R(3) * pi * isl * iS1 * (cc * u1 * p1 + ss * u2 * p2);
  C[5] = -pi * isl * iS2 * iS2 * (R(3) * ss * w1 * w1 * p1 + R(3) * cc * w2 * w2 * p2 + S2 * S2);
  C[7] = -R(3) * pi * isl * iS2 * (ss * w1 * p1 + cc * w2 * p2);
  C[8] = R(3) * pi * isl * iS2 * sc * (w2 * p2 - w1 * p1);
  // normal
  R f3 = R(3) * pi * isl / lsum;
  C[9] = f3;
  // cubic couplings
  R Qa = (R(7) * l1 + R(2) * l2) * k0 + (l1 + R(2) * l2) * k2;
  R Qb = (R(2) * l1 + l2) * k1 + (R(2) * l1 + R(7) * l2) * k3;
  R Pa = R(3) * k0 * l1 + k2 * l2;
  R Pb = k1 * l1 + R(3) * k3 * l2;
  R ra = Qa * (iq1 * iA), rb = Qb * (iq2 * iB);
  C[10] = R(0.75) * f3 * (rb * c - ra * s);
  C[11] = -R(0.75) * f3 * (ra * c + rb * s);
  R g0 = cc * il1 + ss * il2, g2 = ss * il1 + cc * il2, gx = sc * (il2 - il1);
  R t13 = (R(2) * q1 * Pa - R(1.5) * iS1 * Qa * iq1) * c * iA +
          (R(2) * q2 * Pb - R(1.5) * iS1 * Qb * iq2) * s * iB + R(3) * G0 * g0 + G2 * g2;
  R t23 = (-R(2) * q1 * Pa + R(1.5) * iS2 * Qa * iq1) * s * iA +
          (R(2) * q2 * Pb - R(1.5) * iS2 * Qb * iq2) * c * iB + R(2) * G2 * gx;
  C[2] = -R(0.5) * f3 * t13;
  C[6] = -R(0.5) * f3 * t23;
  C[12] = -R(0.5) * f3 * sc * (iS1 - iS2) * (il1 - il2);
  // rotation-rotation
  C[13] = -R(3) * pi * isl * (ss * p1 + cc * p2);
  C[14] = R(3) * pi * isl * sc * (p2 - p1);
  C[15] = -R(3) * pi * isl * (cc * p1 + ss * p2);
}

// Ladd's normal law for spheres, Eq. methods:llub: the force on i along the
// line of centres n (from i to j) is mu 6 pi (a b / (a + b))^2 times the
// approach rate n.(v_j - v_i) times (1/h - 1/delta_n), with b -> infinity
// (coefficient 6 pi mu a^2) for a wall; the gap is clipped at h_c and the
// contact force added as in the contact-based model.  It passes through
// both centres: no torque.
template <typename R>
__host__ __device__ void ladd_pair(const CallDesc& cd, const PRec& A, const KRec& KA,
                                   const PRec& Bp, const KRec* KB, bool pair, int side,
                                   PairOut<R>& out, double& hout, int& status) {
  const double a = A.Rperp;
  double n[3], h, g, vj[3];  // vj: velocity of the partner (its image) or the wall
  if (pair) {
    double d[3];
    const int m = pair_image(cd, A.r, Bp.r, d);
    const double dn = sqrt(dot3(d, d));
    for (int k = 0; k < 3; ++k) n[k] = d[k] / dn;
    const double b = Bp.Rperp;
    h = dn - a - b;
    g = a * b / (a + b);
    // velocity of the image of j that d points to
    vj[0] = KB->v[0] - m * cd.le_vel;
    vj[1] = KB->v[1];
    vj[2] = KB->v[2];
  } else {
    n[0] = n[1] = 0.0;
    n[2] = side == 0 ? -1.0 : 1.0;
    h = (side == 0 ? A.r[2] : cd.L[2] - A.r[2]) - a;
    g = a;
    for (int k = 0; k < 3; ++k) vj[k] = cd.wall_vel[side][k];
  }
  hout = h;
  const double heff = h > cd.h_c ? h : cd.h_c;
  if (heff >= cd.delta_n && h > cd.h_c) {
    status = 1;
    return;
  }
  if (!(heff > 0.0)) {
    status = 2;
    return;
  }
  status = 0;
  const double un = n[0] * (vj[0] - KA.v[0]) + n[1] * (vj[1] - KA.v[1]) +
                    n[2] * (vj[2] - KA.v[2]);
  double fn = cd.mu * 6.0 * kPi * g * g * (1.0 / heff - cd.inv_delta_n) * un;
  if (h <= cd.h_c) fn -= h > 0.0 ? cd.eps_c * (cd.h_c - h) : cd.eps_c * cd.h_c;
  for (int k = 0; k < 3; ++k) out.F[k] = R(fn * n[k]);
}

// nseed (used when use_nseed): the previous call's normal; fell_back and
// warm_used are set to 1 when the solve fell back to another start or
// started from nseed; nout receives the converged normal.
template <typename R, bool kTangent>
__host__ __device__ void eval_pair(const CallDesc& cd, const PRec& A, const KRec& KA,
                          const PRec& Bp, const KRec* KB, bool pair, int side,
                          PairOut<R>& out, double& hout, int& status,
                          int& iters, const float* seedY, int& fell_back,
                          const double (&nseed)[3], bool use_nseed, int& warm_used,
                          double (&nout)[3], double* det) {
  for (int k = 0; k < 3; ++k) out.F[k] = out.Ti[k] = out.Tj[k] = R(0);
  if (det)
    for (int k = 0; k < kDetailWords; ++k) det[k] = 0.0;
  if (cd.model == LUB_MODEL_LADD) {
    ladd_pair<R>(cd, A, KA, Bp, KB, pair, side, out, hout, status);
    iters = 0;
    return;
  }
  Solve sv;
  int le_m = 0;  // Lees-Edwards image of j: its velocity differs by -le_m le_vel in x
  if (pair) {
    double d[3];
    le_m = pair_image(cd, A.r, Bp.r, d);
    // start: the previous call's normal (warm start), else the learned
    // prediction, else the plain start (the line of centres mapped by
    // (M_i + M_j)^-1).  The plain start judges a seeded one: if the seeded
    // iteration does not converge, start again from the plain start
    double n0[3] = {0.0, 0.0, 0.0};
    bool seeded = false;
    if (use_nseed && dot3(nseed, d) > 0.0) {
      for (int k = 0; k < 3; ++k) n0[k] = nseed[k];
      seeded = true;
      warm_used = 1;
    } else if (seedY) {
      seeded = seed_normal(d, A, Bp, seedY, n0);
      if (!seeded) fell_back = 1;
    }
    // one call site of the solver (a second inlined copy only costs
    // instruction cache): the seeded attempt, then the plain one if needed
    bool from_seed = seeded;
    int used = 0;
#pragma clang loop unroll(disable)
    for (;;) {
      sv = closest_points(d, A.M, Bp.M, cd.max_iter, n0, from_seed, cd.newton_tol);
      if (sv.ok || !from_seed) break;
      used = sv.iters;
      from_seed = false;
      fell_back = 1;
    }
    sv.iters += used;
    if (kTangent && !sv.ok) {
      // last resort: the paper's tangent-sphere iteration, then a Newton
      // polish from its normal (at least 8 iterations: its start is only
      // within the iteration's tolerance)
      double nl[3];
      if (tangent_spheres(d, A, Bp, nl)) {
        const int used = sv.iters;
        Solve sp = closest_points(d, A.M, Bp.M, cd.max_iter > 8 ? cd.max_iter : 8, nl, true,
                                  cd.newton_tol);
        sp.iters += used;
        if (sp.ok) {
          sv = sp;
          fell_back = 1;
        }
      }
    }
    if (sv.ok)
      for (int k = 0; k < 3; ++k) nout[k] = sv.n[k];
  } else {
    // wall: the particle's support point towards the plane
    double nz = side == 0 ? -1.0 : 1.0;
    double hs = sqrt(A.M[5]);
    sv.n[0] = 0.0;
    sv.n[1] = 0.0;
    sv.n[2] = nz;
    sv.ai[0] = A.M[2] * nz / hs;
    sv.ai[1] = A.M[4] * nz / hs;
    sv.ai[2] = A.M[5] * nz / hs;
    sv.bj[0] = sv.bj[1] = sv.bj[2] = 0.0;
    sv.h = (side == 0 ? A.r[2] : cd.L[2] - A.r[2]) - hs;
    sv.iters = 0;
    sv.ok = true;
  }
  iters = sv.iters;
  hout = sv.h;
  if (!sv.ok) {
    status = 3;
    return;
  }
  if (det)
    for (int k = 0; k < 3; ++k) {
      det[k] = sv.n[k];
      det[3 + k] = sv.ai[k];
      det[6 + k] = -sv.bj[k];
    }
  const double h = sv.h;
  const double heff = h > cd.h_c ? h : cd.h_c;
  if (heff >= cd.dmax && h > cd.h_c) {
    status = 1;
    return;
  }
  if (!(heff > 0.0)) {
    status = 2;
    return;
  }
  status = 0;
  const double* n = sv.n;

  // frame of surface i and latitude of both closest points (FP64)
  double cpi, spi, e1[3], e2[3];
  latitude(n, A.ax, A.Rpar, A.Rperp, &cpi, &spi, e1);
  cross3(n, e1, e2);
  double S1, S2, G0, G2, iS1p = 0.0, iS2p = 0.0, G0p = 0.0, G2p = 0.0;
  double cph = 1.0, sph = 0.0;
  double iS1, iS2;
  radii<double>(A.Rpar, A.Rperp, cpi, spi, &S1, &S2, &iS1, &iS2, &G0, &G2);
  if (pair) {
    // surface j: outward normal -n; its x1' lies in the same tangent plane
    double cpj, spj, e1p[3];
    const double nj[3] = {-n[0], -n[1], -n[2]};
    latitude(nj, Bp.ax, Bp.Rpar, Bp.Rperp, &cpj, &spj, e1p);
    double S1p, S2p;
    radii<double>(Bp.Rpar, Bp.Rperp, cpj, spj, &S1p, &S2p, &iS1p, &iS2p, &G0p, &G2p);
    cph = dot3(e1p, e1);
    sph = dot3(e1p, e2);
  }
  R C[16];
  k_coeffs<R>(R(S1), R(S2), iS1, iS2, R(G0), R(G2), R(iS1p), R(iS2p), R(G0p),
              R(G2p), R(cph), R(sph), C);

  // cut-off factors (FP64), Eq. lub:resistance-correction; the "normal
  // only" model drops every element but K33
  const bool full = cd.model == LUB_MODEL_FULL;
  const double lh = full && heff < fmax(cd.delta_t, cd.delta_r) ? log(heff) : 0.0;
  double Lt = full && heff < cd.delta_t ? lh - cd.ln_delta_t : 0.0;
  double Lr = full && heff < cd.delta_r ? lh - cd.ln_delta_r : 0.0;
  // the contact-only law has no resistance: the repulsion below acts alone
  const bool lub = cd.model != LUB_MODEL_CONTACT;
  double Ln = lub && heff < cd.delta_n ? 1.0 / heff - cd.inv_delta_n : 0.0;
  if (det) {
    // the frame's x1 axis and the corrective elements K~ = C (ln h_eff - ln
    // Delta) or C33 (1/h_eff - 1/Delta_n), as the transfer below uses them
    for (int k = 0; k < 3; ++k) det[9 + k] = e1[k];
    for (int k = 0; k < 16; ++k) {
      const double fac = k == 9 ? Ln : (k >= 13 ? Lr : Lt);
      det[12 + k] = (double)C[k] * fac;
    }
  }

  // relative surface velocities in the local frame (FP64)
  double Vi[3], Vj[3], wr[3], tmp[3];
  cross3(KA.w, sv.ai, tmp);
  for (int k = 0; k < 3; ++k) Vi[k] = KA.v[k] + tmp[k];
  if (pair) {
    double yj[3] = {-sv.bj[0], -sv.bj[1], -sv.bj[2]};
    cross3(KB->w, yj, tmp);
    for (int k = 0; k < 3; ++k) {
      Vj[k] = KB->v[k] + tmp[k];
      wr[k] = KB->w[k] - KA.w[k];
    }
    Vj[0] -= le_m * cd.le_vel;
  } else {
    for (int k = 0; k < 3; ++k) {
      Vj[k] = cd.wall_vel[side][k];
      wr[k] = -KA.w[k];
    }
  }
  double dv[3] = {Vj[0] - Vi[0], Vj[1] - Vi[1], Vj[2] - Vi[2]};
  R U[6] = {R(dot3(e1, dv)), R(dot3(e2, dv)), R(dot3(n, dv)),
            R(dot3(e1, wr)), R(dot3(e2, wr)), R(dot3(n, wr))};
  R lt = R(Lt), lr = R(Lr), ln_ = R(Ln), mu = R(cd.mu);
  R Fb[6];
  Fb[0] = mu * lt * (C[0] * U[0] + C[1] * U[1] + C[2] * U[2] + C[3] * U[3] + C[4] * U[4]);
  Fb[1] = mu * lt * (C[1] * U[0] + C[5] * U[1] + C[6] * U[2] + C[7] * U[3] + C[8] * U[4]);
  Fb[2] = mu * (lt * (C[2] * U[0] + C[6] * U[1] + C[10] * U[3] + C[11] * U[4] + C[12] * U[5]) +
                ln_ * C[9] * U[2]);
  Fb[3] = mu * (lt * (C[3] * U[0] + C[7] * U[1] + C[10] * U[2]) + lr * (C[13] * U[3] + C[14] * U[4]));
  Fb[4] = mu * (lt * (C[4] * U[0] + C[8] * U[1] + C[11] * U[2]) + lr * (C[14] * U[3] + C[15] * U[4]));
  Fb[5] = mu * lt * C[12] * U[2];
  if (h <= cd.h_c) {
    double Fr = h > 0.0 ? cd.eps_c * (cd.h_c - h) : cd.eps_c * cd.h_c;
    Fb[2] -= R(Fr);
  }
  // back to the world frame; torques about the centres
  R E1[3] = {R(e1[0]), R(e1[1]), R(e1[2])};
  R E2[3] = {R(e2[0]), R(e2[1]), R(e2[2])};
  R E3[3] = {R(n[0]), R(n[1]), R(n[2])};
  R F[3], T[3];
  for (int k = 0; k < 3; ++k) {
    F[k] = Fb[0] * E1[k] + Fb[1] * E2[k] + Fb[2] * E3[k];
    T[k] = Fb[3] * E1[k] + Fb[4] * E2[k] + Fb[5] * E3[k];
  }
  R ai[3] = {R(sv.ai[0]), R(sv.ai[1]), R(sv.ai[2])};
  R bj[3] = {R(sv.bj[0]), R(sv.bj[1]), R(sv.bj[2])};
  R xa[3], xb[3];
  cross3(ai, F, xa);
  cross3(bj, F, xb);
  for (int k = 0; k < 3; ++k) {
    out.F[k] = F[k];
    out.Ti[k] = T[k] + xa[k];
    out.Tj[k] = pair ? -T[k] + xb[k] : R(0);
  }
}

constexpr int kPairBlock = 64;

// kTangent = false: the main pass over all slots; a particle pair whose
// Newton solve fails from every start is put on fail_list and left to the
// second pass (kTangent = true, a small grid over that list), which adds the
// tangent-sphere fallback.  The fallback's registers would otherwise lower
// the occupancy of the main pass.
template <typename R, bool kTangent>
__global__ void __launch_bounds__(kPairBlock) k_pairs(CallDesc cd,
                                              const PRecP* __restrict__ recp,
                                              const KRec* __restrict__ kin,
                                              const int32_t* __restrict__ work_s,
                                              const int32_t* __restrict__ work_t,
                                              const float* __restrict__ seedY,
                                              PairOut<R>* __restrict__ out,
                                              double* __restrict__ out_h,
                                              int8_t* __restrict__ out_status,
                                              uint8_t* __restrict__ out_iters,
                                              WarmTables warm,
                                              int32_t* __restrict__ fail_list,
                                              int64_t* __restrict__ stat_pair,
                                              Counters* cnt, double* __restrict__ detail) {
  // one wavefront per block: statistics are reduced in the wave (ballots,
  // shuffles) and written as this block's row, without atomics
  static_assert(kPairBlock == 64, "one wavefront per block");
  const int lane = threadIdx.x;
  // the grid is sized for the capacity; blocks past the device-side work
  // count leave at once (their rows are not read)
  const int nwork = cnt->error != 0 ? 0
                    : kTangent  ? min(cnt->failed, cd.cap_work)
                                : min(cnt->work, cd.cap_work);
  if ((int)(blockIdx.x * blockDim.x) >= nwork) return;
  int64_t n_iters = 0, n_active = 0, n_overlap = 0, n_unres = 0, n_uncon = 0, n_fb = 0,
          n_warm = 0;
  // reused lists: normals stored per superset entry carry the number of the
  // search that made the superset
  const int tag = cd.warm_slots ? (int)warm.state->builds : 0;
  int max_it = 0;
  int64_t my_hist = 0;  // lane b < 32 holds histogram bucket b
  for (int w0 = blockIdx.x * blockDim.x; w0 < nwork; w0 += gridDim.x * blockDim.x) {
    const bool on = w0 + lane < nwork;
    const int w = kTangent ? (on ? fail_list[w0 + lane] : 0) : w0 + lane;
    int status = -1, iters = 0, fb = 0, wu = 0;
    double h = 0.0;
    if (on) {
      const int s = work_s[w], t = work_t[w];
      const bool pp = t >= 0;  // a particle pair, else a wall pair
      // warm start: the previous normal of the pair, kept per superset
      // entry (reused lists) or found in the owner's previous slot range.
      // One call site of the pair evaluation for every kind (inlined copies
      // only cost instruction cache)
      const bool warm_on = pp && (cd.warm_slots || cd.warm_ranges);
      double nprev[3] = {0.0, 0.0, 0.0};
      double nnew[3] = {0.0, 0.0, 0.0};
      bool found = false;
      int e_sup = 0;
      int key = -1;  // input index of s xor that of t (slot ranges)
      if (warm_on && cd.warm_slots) {
        // made under the current superset?
        e_sup = warm.slot_sup[w];
        const float4 v = warm.sup_val[e_sup];
        found = __float_as_int(v.w) == tag;
        nprev[0] = v.x;
        nprev[1] = v.y;
        nprev[2] = v.z;
      } else if (warm_on) {
        // the pair sat in the range of one of its two particles (the one
        // that evaluated it, or the one whose search found it: the one
        // earlier in cell order, which moves little between calls); that
        // one's range first
        const int is = warm.orig[s], it = warm.orig[t];
        key = is ^ it;
        const bool s_first = cd.partner_codes != kPartnerRanges || s < t;
        const int pa = s_first ? is : it;  // the particle whose range holds w
        const int2 ra = warm.prev_range[pa];
        // first the slot at the same place in that particle's previous range
        // as w in its current one (the lists change little between calls),
        // then the two previous ranges
        const int g = ra.x + (w - warm.cur_range[pa].x);
        if (g >= 0 && g >= ra.x && g < ra.y && g < cd.cap_work) {
          const float4 v = warm.prev_val[g];
          if (__float_as_int(v.w) == key) {
            nprev[0] = v.x;
            nprev[1] = v.y;
            nprev[2] = v.z;
            found = true;
          }
        }
        for (int side = 0; side < 2 && !found; ++side) {
          const int2 rg = side == 0 ? ra : warm.prev_range[s_first ? it : is];
          const int lo = max(rg.x, 0);
          const int hi = min(min(rg.y, cd.cap_work), lo + kWarmScan);
          for (int k = lo; k < hi; ++k) {
            const float4 v = warm.prev_val[k];
            if (__float_as_int(v.w) == key) {
              nprev[0] = v.x;
              nprev[1] = v.y;
              nprev[2] = v.z;
              found = true;
              break;
            }
          }
        }
      }
      PairOut<R> o;
      // the full records, formed from the 64-B copies
      const PRec A = expand_record(recp[s]);
      const PRec B = expand_record(recp[pp ? t : s]);
      eval_pair<R, kTangent>(cd, A, kin[s], B, pp ? &kin[t] : nullptr, pp,
                             pp ? 0 : -1 - t, o, h, status, iters,
                             pp && seedY ? seedY + 4 * (int64_t)w : nullptr, fb, nprev,
                             found, wu, nnew,
                             detail ? detail + (int64_t)kDetailWords * w : nullptr);
      if (warm_on && cd.warm_slots && status != 3) {
        warm.sup_val[e_sup] = make_float4((float)nnew[0], (float)nnew[1], (float)nnew[2],
                                          __int_as_float(tag));
      }
      if (cd.warm_ranges && (!kTangent || status != 3)) {
        // this call's value of the slot for the next call: the normal and
        // the pair's key, or -1 (no pair: the key of a pair is a xor of two
        // distinct non-negative indices) for a wall or a failed solve (the
        // tangent-sphere pass writes the slots it solves)
        const bool keep = warm_on && status != 3;
        warm.cur_val[w] = make_float4((float)nnew[0], (float)nnew[1], (float)nnew[2],
                                      __int_as_float(keep ? key : -1));
      }
      out[w] = o;
      out_h[w] = h;
      out_status[w] = (int8_t)status;
      out_iters[w] = (uint8_t)(iters > 255 ? 255 : iters);
      if (!kTangent && status == 3 && t >= 0 && cd.model != LUB_MODEL_LADD) {
        // deferred to the tangent-sphere pass, which counts it
        fail_list[atomicAdd(&cnt->failed, 1)] = w;
        status = -1;
        iters = fb = wu = 0;
      }
    }
    const int bucket = on && status >= 0 ? (iters < 31 ? iters : 31) : -1;
    n_iters += iters;
    max_it = max(max_it, iters);
    n_active += __popcll(__ballot(status == 0));
    n_overlap += __popcll(__ballot(status == 0 && h <= 0.0));
    n_unres += __popcll(__ballot(status == 2));
    n_uncon += __popcll(__ballot(status == 3));
    n_fb += __popcll(__ballot(fb != 0));
    n_warm += __popcll(__ballot(wu != 0));
    // histogram over the buckets present in this pass
    int lo = bucket >= 0 ? bucket : 32, hi = bucket;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    for (int b = lo; b <= hi; ++b) {
      const int64_t c = __popcll(__ballot(bucket == b));
      if (lane == b) my_hist += c;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    n_iters += __shfl_xor(n_iters, o, 64);
    max_it = max(max_it, __shfl_xor(max_it, o, 64));
  }
  int64_t* row = stat_pair + (int64_t)kStatPairWords *
                                 (blockIdx.x + (kTangent ? kMaxPairBlocks : 0));
  const int64_t v = lane == 0 ? n_iters
                  : lane == 1 ? n_active
                  : lane == 2 ? n_overlap
                  : lane == 3 ? n_unres
                  : lane == 4 ? n_uncon
                  : lane == 5 ? n_fb
                  : lane == 6 ? (int64_t)max_it
                              : n_warm;
  if (lane < 8) row[lane] = v;
  if (lane < 32) row[8 + lane] = my_hist;
}

// seed features of the particle-particle slots
__global__ void k_seed_features(CallDesc cd, const PRec* __restrict__ rec,
                                const int32_t* __restrict__ work_s,
                                const int32_t* __restrict__ work_t,
                                float* __restrict__ X, const Counters* cnt) {
  const int nwork = cnt->error == 0 ? min(cnt->work, cd.cap_work) : 0;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nwork;
       w += gridDim.x * blockDim.x) {
    const int s = work_s[w], t = work_t[w];
    float x[10] = {0, 0, 0, 1, 0, 0, 0, 1, 1, 1};
    if (t >= 0) {
      const PRec& A = rec[s];
      const PRec& B = rec[t];
      double d[3];
      pair_image(cd, A.r, B.r, d);
      seed_features(d, A, B, x);
    }
    for (int k = 0; k < 10; ++k) X[10 * (int64_t)w + k] = x[k];
  }
}

}  // namespace

void launch_seed_features(const CallDesc& d, const PRec* rec,
                          const int32_t* work_s, const int32_t* work_t,
                          float* X, Counters* cnt, hipStream_t s) {
  int blocks = (d.cap_work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_seed_features, dim3(blocks), dim3(256), 0, s, d, rec,
                     work_s, work_t, X, cnt);
}

int pair_grid(const CallDesc& d) {
  int blocks = (d.cap_work + kPairBlock - 1) / kPairBlock;
  if (blocks > kMaxPairBlocks) blocks = kMaxPairBlocks;  // grid-stride beyond
  return blocks < 1 ? 1 : blocks;
}

void launch_pairs(const CallDesc& d, const PRecP* recp, const KRec* kin,
                  const int32_t* work_s, const int32_t* work_t, const float* seedY,
                  void* out, double* out_h, int8_t* out_status, uint8_t* out_iters,
                  WarmTables warm, int32_t* fail_list, int64_t* stat_pair, Counters* cnt,
                  hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, double* detail) {
  const int blocks = pair_grid(d);
  // the events (may be null) take the main pass's own start and end stamps
  if (d.precision == LUB_MIXED) {
    hipExtLaunchKernelGGL(k_pairs<float, false>, dim3(blocks), dim3(kPairBlock), 0, s,
                          ev_start, ev_stop, 0, d, recp, kin, work_s, work_t, seedY,
                          (PairOut<float>*)out, out_h, out_status, out_iters, warm,
                          fail_list, stat_pair, cnt, detail);
    hipLaunchKernelGGL((k_pairs<float, true>), dim3(kTangentBlocks), dim3(kPairBlock), 0, s,
                       d, recp, kin, work_s, work_t, seedY, (PairOut<float>*)out, out_h,
                       out_status, out_iters, warm, fail_list, stat_pair, cnt, detail);
  } else {
    hipExtLaunchKernelGGL(k_pairs<double, false>, dim3(blocks), dim3(kPairBlock), 0, s,
                          ev_start, ev_stop, 0, d, recp, kin, work_s, work_t, seedY,
                          (PairOut<double>*)out, out_h, out_status, out_iters, warm,
                          fail_list, stat_pair, cnt, detail);
    hipLaunchKernelGGL((k_pairs<double, true>), dim3(kTangentBlocks), dim3(kPairBlock), 0,
                       s, d, recp, kin, work_s, work_t, seedY, (PairOut<double>*)out,
                       out_h, out_status, out_iters, warm, fail_list, stat_pair, cnt, detail);
  }
}

}  // namespace lub
