/*
 * lubref.c -- plain FP64 CPU oracle (test infrastructure only; see
 * lubref.h for scope, conventions and the paper passages it follows).
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 * No fast-math, no contraction: the centre test must be reproducible bit
 * for bit, and every other expression is evaluated as written.
 */
#include "lubref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static void scale3(double a[3], double s) {
  a[0] *= s;
  a[1] *= s;
  a[2] *= s;
}
static void matvec3(const double M[9], const double x[3], double y[3]) {
  for (int r = 0; r < 3; ++r)
    y[r] = M[3 * r] * x[0] + M[3 * r + 1] * x[1] + M[3 * r + 2] * x[2];
}
static void mattvec3(const double M[9], const double x[3], double y[3]) {
  for (int c = 0; c < 3; ++c)
    y[c] = M[c] * x[0] + M[3 + c] * x[1] + M[6 + c] * x[2];
}

/* ------------------------------------------------------------------ */
/* particle description                                                */
/* ------------------------------------------------------------------ */
void ref_quat_to_matrix(const double qin[4], double Q[9]) {
  double nq = sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] +
                   qin[3] * qin[3]);
  double w = qin[0] / nq, x = qin[1] / nq, y = qin[2] / nq, z = qin[3] / nq;
  Q[0] = 1.0 - 2.0 * (y * y + z * z);
  Q[1] = 2.0 * (x * y - w * z);
  Q[2] = 2.0 * (x * z + w * y);
  Q[3] = 2.0 * (x * y + w * z);
  Q[4] = 1.0 - 2.0 * (x * x + z * z);
  Q[5] = 2.0 * (y * z - w * x);
  Q[6] = 2.0 * (x * z - w * y);
  Q[7] = 2.0 * (y * z + w * x);
  Q[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* A spheroid with centre c (world frame), rotation Q, semi-axes
 * D = diag(R_perp, R_perp, R_par) in the body frame (Eq. lub:spheroid). */
typedef struct {
  double c[3];
  double Q[9];
  double Rpar, Rperp;
  double D[3];
  double M[9]; /* Q D^2 Q^T: support function h(n) = sqrt(n.M n) */
} body;

static void body_init(body* b, const double c[3], const double q[4],
                      const double semi[2]) {
  memcpy(b->c, c, sizeof(b->c));
  ref_quat_to_matrix(q, b->Q);
  b->Rpar = semi[0];
  b->Rperp = semi[1];
  b->D[0] = semi[1];
  b->D[1] = semi[1];
  b->D[2] = semi[0];
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        acc += b->Q[3 * r + k] * b->D[k] * b->D[k] * b->Q[3 * s + k];
      b->M[3 * r + s] = acc;
    }
}

static void to_body(const body* b, const double x[3], double xb[3]) {
  double d[3] = {x[0] - b->c[0], x[1] - b->c[1], x[2] - b->c[2]};
  mattvec3(b->Q, d, xb);
}

/* implicit function f(x) = sum (xb_k / D_k)^2 - 1 (negative inside) */
static double body_implicit(const body* b, const double x[3]) {
  double xb[3];
  to_body(b, x, xb);
  double acc = 0.0;
  for (int k = 0; k < 3; ++k) acc += (xb[k] / b->D[k]) * (xb[k] / b->D[k]);
  return acc - 1.0;
}

/* outward unit normal at a surface point y (gradient of the implicit
 * function of the spheroid) */
static void body_normal(const body* b, const double y[3], double n[3]) {
  double yb[3], nb[3];
  to_body(b, y, yb);
  for (int k = 0; k < 3; ++k) nb[k] = yb[k] / (b->D[k] * b->D[k]);
  matvec3(b->Q, nb, n);
  scale3(n, 1.0 / norm3(n));
}

/* point where the line a + t u leaves the spheroid in direction u (the
 * larger root t).  a normally lies inside; with the enlarged local radius
 * of the first Lin-Han phase it may lie behind the body, which is fine as
 * long as the line crosses the surface ahead of a.  Returns 0 on success. */
static int ray_exit(const body* b, const double a[3], const double u[3],
                    double y[3]) {
  double ab[3], ub[3];
  to_body(b, a, ab);
  mattvec3(b->Q, u, ub);
  double A = 0.0, B = 0.0, C = -1.0;
  for (int k = 0; k < 3; ++k) {
    double inv = 1.0 / (b->D[k] * b->D[k]);
    A += ub[k] * ub[k] * inv;
    B += ab[k] * ub[k] * inv;
    C += ab[k] * ab[k] * inv;
  }
  double disc = B * B - A * C;
  if (!(A > 0.0) || !(disc >= 0.0)) return 1;
  double t = (-B + sqrt(disc)) / A;
  if (!(t > 0.0)) return 1;
  for (int k = 0; k < 3; ++k) y[k] = a[k] + t * u[k];
  return 0;
}

/* parametric latitude p and longitude q (Eq. lub:spheroid) of a surface
 * point given in the body frame: sin p = y3/R_par, cos p = rho/R_perp */
static void surface_params(const body* b, const double yb[3], double* sp,
                           double* cp, double* sq, double* cq) {
  double rho = sqrt(yb[0] * yb[0] + yb[1] * yb[1]);
  double s = yb[2] / b->Rpar, c = rho / b->Rperp;
  double nrm = sqrt(s * s + c * c);
  *sp = s / nrm;
  *cp = c / nrm;
  double qq = atan2(yb[1], yb[0]);
  *sq = sin(qq);
  *cq = cos(qq);
}

/* principal radii (Eq. lub:curvature-radii) and cubic coefficients
 * Gamma_0, Gamma_2 (Sec. III.B) at parametric latitude p */
static void surface_coeffs(const body* b, double sp, double cp, double* S1,
                           double* S2, double* G0, double* G2) {
  double Rpa = b->Rpar, Rpe = b->Rperp;
  double s1 = sqrt(Rpe * Rpe * sp * sp + Rpa * Rpa * cp * cp);
  *S1 = s1 * s1 * s1 / (Rpa * Rpe);
  *S2 = Rpe * s1 / Rpa;
  double s1_4 = s1 * s1 * s1 * s1;
  double s1_6 = s1_4 * s1 * s1;
  *G0 = (Rpa * Rpa - Rpe * Rpe) * Rpa * Rpe * sp * cp / (2.0 * s1_6);
  *G2 = (Rpa * Rpa - Rpe * Rpe) * Rpa * sp * cp / (2.0 * Rpe * s1_4);
}

/* conservative tangent-sphere radius, Eq. lub:minimum-radius */
static double conservative_radius(const body* b) {
  if (b->Rpar < b->Rperp) return b->Rpar * b->Rpar / b->Rperp;
  if (b->Rpar > b->Rperp) return b->Rperp * b->Rperp / b->Rpar;
  return b->Rpar;
}

/* local tangent-sphere radius of the two-fold strategy: the smaller local
 * principal radius at the current tangent point */
static double local_radius(const body* b, const double y[3]) {
  double yb[3], sp, cp, sq, cq, S1, S2, G0, G2;
  to_body(b, y, yb);
  surface_params(b, yb, &sp, &cp, &sq, &cq);
  surface_coeffs(b, sp, cp, &S1, &S2, &G0, &G2);
  return S1 < S2 ? S1 : S2;
}

/* support function h(n) = max over the body of n.(x - c) and the support
 * point offset M n / h(n) (n need not be unit) */
static double support(const body* b, const double n[3], double off[3]) {
  double Mn[3];
  matvec3(b->M, n, Mn);
  double h = sqrt(dot3(n, Mn));
  if (off) {
    off[0] = Mn[0] / h;
    off[1] = Mn[1] / h;
    off[2] = Mn[2] / h;
  }
  return h;
}

/* ------------------------------------------------------------------ */
/* closest points                                                      */
/* ------------------------------------------------------------------ */

/* Lin-Han tangent-sphere iteration (Sec. III.A).  Start on the centre
 * line; tangent spheres of radius Sbar placed inside each surface at the
 * current tangent points; new tangent points are the exits of both
 * surfaces on the line joining the sphere centres; stop when both normals
 * are within the angle criterion of Eq. lub:convergence.
 * mode 0: local radius min(S1,S2) (first phase), mode 1: conservative
 * radius of Eq. lub:minimum-radius.  Returns 0 when converged. */
static int lin_han_phase(const body* bi, const body* bj, int mode, int nmax,
                         double eps, double yi[3], double yj[3], double zhat[3],
                         double* gap, int* iters) {
  double u[3], d[3];
  for (int k = 0; k < 3; ++k) d[k] = bj->c[k] - bi->c[k];
  double dn = norm3(d);
  for (int k = 0; k < 3; ++k) u[k] = d[k] / dn;
  if (ray_exit(bi, bi->c, u, yi)) return 1;
  double mu_[3] = {-u[0], -u[1], -u[2]};
  if (ray_exit(bj, bj->c, mu_, yj)) return 1;
  double Sbi = conservative_radius(bi), Sbj = conservative_radius(bj);
  for (int it = 0; it <= nmax; ++it) {
    double ni[3], nj[3], zi[3], zj[3], zij[3];
    body_normal(bi, yi, ni);
    body_normal(bj, yj, nj);
    if (mode == 0) {
      Sbi = local_radius(bi, yi);
      Sbj = local_radius(bj, yj);
    }
    for (int k = 0; k < 3; ++k) {
      zi[k] = yi[k] - Sbi * ni[k];
      zj[k] = yj[k] - Sbj * nj[k];
      zij[k] = zi[k] - zj[k];
    }
    double zl = norm3(zij);
    double zh[3] = {zij[0] / zl, zij[1] / zl, zij[2] / zl};
    double cos_i = -dot3(ni, zh);
    double cos_j = dot3(nj, zh);
    if (cos_i > 1.0 - eps && cos_j > 1.0 - eps) {
      /* gap direction from i to j and scalar gap (reading Q4) */
      for (int k = 0; k < 3; ++k) zhat[k] = -zh[k];
      *gap = zl - Sbi - Sbj;
      return 0;
    }
    if (it == nmax) break;
    *iters += 1;
    double dirj[3] = {-zh[0], -zh[1], -zh[2]}; /* from z_i towards z_j */
    if (ray_exit(bi, zi, dirj, yi)) return 1;
    if (ray_exit(bj, zj, zh, yj)) return 1;
  }
  return 1;
}

/* The paper's two-fold strategy: up to N1 iterations with the local radius,
 * consistency checks on convergence, otherwise restart from the centre line
 * with the conservative radius for up to N2 iterations. */
static int lin_han(const body* bi, const body* bj, double n0[3], int* iters,
                   int* fallback) {
  const int N1 = 10, N2 = 1000;
  const double eps = 1e-6;
  double yi[3], yj[3], zh[3], gap;
  double rij[3];
  for (int k = 0; k < 3; ++k) rij[k] = bi->c[k] - bj->c[k];
  *iters = 0;
  *fallback = 0;
  if (lin_han_phase(bi, bj, 0, N1, eps, yi, yj, zh, &gap, iters) == 0) {
    double ni[3], nj[3];
    body_normal(bi, yi, ni);
    body_normal(bj, yj, nj);
    int ok = dot3(nj, rij) > 0.0 && dot3(ni, rij) < 0.0;
    if (ok && gap < 0.0)
      ok = body_implicit(bj, yi) < 0.0 && body_implicit(bi, yj) < 0.0;
    if (ok) {
      memcpy(n0, zh, sizeof(zh));
      return 0;
    }
  }
  *fallback = 1;
  if (lin_han_phase(bi, bj, 1, N2, eps, yi, yj, zh, &gap, iters) == 0) {
    memcpy(n0, zh, sizeof(zh));
    return 0;
  }
  return 1;
}

/* 4x4 Gaussian elimination with partial pivoting; returns 0 on success */
static int solve4(double A[4][4], double b[4], double x[4]) {
  int piv[4] = {0, 1, 2, 3};
  for (int c = 0; c < 4; ++c) {
    int best = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[piv[r]][c]) > fabs(A[piv[best]][c])) best = r;
    int tmp = piv[c];
    piv[c] = piv[best];
    piv[best] = tmp;
    double p = A[piv[c]][c];
    if (p == 0.0) return 1;
    for (int r = c + 1; r < 4; ++r) {
      double f = A[piv[r]][c] / p;
      for (int k = c; k < 4; ++k) A[piv[r]][k] -= f * A[piv[c]][k];
      b[piv[r]] -= f * b[piv[c]];
    }
  }
  for (int c = 3; c >= 0; --c) {
    double acc = b[piv[c]];
    for (int k = c + 1; k < 4; ++k) acc -= A[piv[c]][k] * x[k];
    x[c] = acc / A[piv[c]][c];
  }
  return 0;
}

/* Polish of the Lin-Han fixed point to round-off.  At the fixed point the
 * two outward normals are antiparallel and along the line joining the
 * tangent points; with y_i and y_j written as the support points of i in
 * direction n and of j in direction -n, that is the stationarity of
 *   g(n) = n.d - h_i(n) - h_j(n)
 * on the unit sphere (d = r_j - r_i), and g(n) is then the signed gap.
 * Newton on the Lagrange conditions grad g - nu n = 0, n.n = 1 (bordered
 * 4x4 system). */
static int polish(const body* bi, const body* bj, const double d[3],
                  double n[3], int* iters) {
  double nu = 0.0;
  int first = 1;
  *iters = 0;
  for (int it = 0; it < 60; ++it) {
    double oi[3], oj[3];
    double hi = support(bi, n, oi), hj = support(bj, n, oj);
    double grad[3];
    for (int k = 0; k < 3; ++k) grad[k] = d[k] - oi[k] - oj[k];
    if (first) {
      nu = dot3(grad, n) / dot3(n, n);
      first = 0;
    }
    /* Hessian of g: -sum_k (M_k / h_k - (M_k n)(M_k n)^T / h_k^3) */
    double H[3][3];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s)
        H[r][s] = -(bi->M[3 * r + s] / hi - oi[r] * oi[s] / hi) -
                  (bj->M[3 * r + s] / hj - oj[r] * oj[s] / hj);
    double A[4][4], b[4], x[4];
    for (int r = 0; r < 3; ++r) {
      for (int s = 0; s < 3; ++s) A[r][s] = H[r][s] - (r == s ? nu : 0.0);
      A[r][3] = -n[r];
      b[r] = -(grad[r] - nu * n[r]);
      A[3][r] = n[r];
    }
    A[3][3] = 0.0;
    b[3] = -0.5 * (dot3(n, n) - 1.0);
    if (solve4(A, b, x)) return 1;
    double step = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double damp = step > 0.25 ? 0.25 / step : 1.0;
    for (int k = 0; k < 3; ++k) n[k] += damp * x[k];
    nu += damp * x[3];
    *iters += 1;
    if (step < 1e-15) break;
  }
  double nn = norm3(n);
  scale3(n, 1.0 / nn);
  /* final stationarity residual: tangential part of grad g */
  double oi[3], oj[3], grad[3];
  support(bi, n, oi);
  support(bj, n, oj);
  for (int k = 0; k < 3; ++k) grad[k] = d[k] - oi[k] - oj[k];
  double gn = dot3(grad, n);
  double res = 0.0;
  for (int k = 0; k < 3; ++k) res += (grad[k] - gn * n[k]) * (grad[k] - gn * n[k]);
  double scale = norm3(d) + bi->Rpar + bi->Rperp + bj->Rpar + bj->Rperp;
  return sqrt(res) <= 1e-11 * scale ? 0 : 1;
}

/* closest points of two spheroids with centres 0 and d */
static int closest_pp(const body* bi, const body* bj, const double d[3],
                      ref_pair_result* o) {
  double n[3];
  int it_lh = 0, fb = 0, it_p = 0;
  o->iters_lh = 0;
  o->iters_polish = 0;
  o->fallback = 0;
  int lh = lin_han(bi, bj, n, &it_lh, &fb);
  o->iters_lh = it_lh;
  o->fallback = fb;
  if (lh) {
    /* no converged tangent points: start the polish from the centre line */
    double dn = norm3(d);
    for (int k = 0; k < 3; ++k) n[k] = d[k] / dn;
  }
  if (polish(bi, bj, d, n, &it_p)) {
    o->iters_polish = it_p;
    return 1;
  }
  o->iters_polish = it_p;
  double oi[3], oj[3];
  double hi = support(bi, n, oi), hj = support(bj, n, oj);
  o->h = dot3(n, d) - hi - hj;
  for (int k = 0; k < 3; ++k) {
    o->n[k] = n[k];
    o->yi[k] = oi[k];   /* y_i - r_i */
    o->yj[k] = -oj[k];  /* y_j - r_j */
  }
  double sep[3];
  for (int k = 0; k < 3; ++k) sep[k] = d[k] + o->yj[k] - o->yi[k];
  o->certificate = o->h > 0.0 ? norm3(sep) - o->h : 0.0;
  return 0;
}

/* ------------------------------------------------------------------ */
/* resistance (Appendix)                                               */
/* ------------------------------------------------------------------ */

/* cubic coefficients m_i(alpha, a) of the Appendix: a cubic given in axes
 * rotated by +alpha expressed in the unrotated axes */
static void cubic_rotate(double ca, double sa, const double a[4], double m[4]) {
  double c2 = ca * ca, s2 = sa * sa;
  m[0] = a[0] * c2 * ca - a[1] * sa * c2 + a[2] * s2 * ca - a[3] * s2 * sa;
  m[1] = a[0] * 3.0 * sa * c2 + a[1] * (c2 * ca - 2.0 * s2 * ca) +
         a[2] * (s2 * sa - 2.0 * sa * c2) + a[3] * 3.0 * s2 * ca;
  m[2] = a[0] * 3.0 * ca * s2 + a[1] * (2.0 * c2 * sa - s2 * sa) +
         a[2] * (c2 * ca - 2.0 * ca * s2) - a[3] * (3.0 * c2 * sa);
  m[3] = a[0] * s2 * sa + a[1] * ca * s2 + a[2] * c2 * sa + a[3] * c2 * ca;
}

void ref_K_coeffs(double S1, double S2, double invS1p, double invS2p,
                  const double G[4], const double Gp[4], double cphi,
                  double sphi, double C[6][6], double aux[8]) {
  /* curvature matrix of the quadratic gap (Appendix) */
  double m11 = 1.0 / (2.0 * S1) + cphi * cphi * invS1p / 2.0 +
               sphi * sphi * invS2p / 2.0;
  double m12 = sphi * cphi / 2.0 * (invS1p - invS2p);
  double m22 = 1.0 / (2.0 * S2) + sphi * sphi * invS1p / 2.0 +
               cphi * cphi * invS2p / 2.0;
  /* eigenvalues lambda1 >= lambda2; eigenvector of lambda2 is
   * l2 = (sin chi, cos chi), that of lambda1 is l1 = (cos chi, -sin chi) */
  double tr = m11 + m22;
  double rad = sqrt((m11 - m22) * (m11 - m22) / 4.0 + m12 * m12);
  double l1 = tr / 2.0 + rad, l2 = tr / 2.0 - rad;
  double cchi = 1.0, schi = 0.0;
  if (rad > 0.0) {
    /* (M - l2 I) v = 0: v is orthogonal to both rows of M - l2 I; take the
     * row of larger norm */
    double ra0 = m11 - l2, ra1 = m12, rb0 = m12, rb1 = m22 - l2;
    double v0, v1;
    if (ra0 * ra0 + ra1 * ra1 >= rb0 * rb0 + rb1 * rb1) {
      v0 = -ra1;
      v1 = ra0;
    } else {
      v0 = -rb1;
      v1 = rb0;
    }
    double vn = sqrt(v0 * v0 + v1 * v1);
    schi = v0 / vn;
    cchi = v1 / vn;
  }
  /* beta = m(phi, Gamma'), k = Gamma + beta, kappa = m(chi, k) rescaled */
  double beta[4], kk[4], mk[4], kap[4];
  cubic_rotate(cphi, sphi, Gp, beta);
  for (int i = 0; i < 4; ++i) kk[i] = G[i] + beta[i];
  cubic_rotate(cchi, schi, kk, mk);
  double sl1 = sqrt(l1), sl2 = sqrt(l2);
  for (int i = 0; i < 4; ++i)
    kap[i] = mk[i] / (pow(sl1, 3 - i) * pow(sl2, i));

  double c = cchi, s = schi;
  double sl = sqrt(l1 * l2);
  double A = 3.0 * l1 + 2.0 * l2, B = 2.0 * l1 + 3.0 * l2;
  double G0 = G[0], G1 = G[1], G2 = G[2], G3 = G[3];
  memset(C, 0, 36 * sizeof(double));

  /* K11 .. K55 with ln h factored out; K33 with 1/h factored out */
  C[0][0] = -PI / (sl * S1 * S1) *
            (3.0 * c * c * (1.0 - l1 * S1) * (1.0 - l1 * S1) / (A * l1) +
             3.0 * s * s * (1.0 - l2 * S1) * (1.0 - l2 * S1) / (B * l2) +
             S1 * S1);
  C[0][1] = 3.0 * PI / (sl * S1 * S2) * s * c *
            ((1.0 - l1 * S1) * (1.0 - l1 * S2) / (A * l1) -
             (1.0 - l2 * S1) * (1.0 - l2 * S2) / (B * l2));
  {
    double t1 = (2.0 * sl1 * (3.0 * kap[0] * l1 + kap[2] * l2) -
                 3.0 / (2.0 * S1 * sl1) *
                     ((7.0 * l1 + 2.0 * l2) * kap[0] +
                      (l1 + 2.0 * l2) * kap[2])) *
                c / A;
    double t2 = (2.0 * sl2 * (kap[1] * l1 + 3.0 * kap[3] * l2) -
                 3.0 / (2.0 * S1 * sl2) *
                     ((2.0 * l1 + l2) * kap[1] +
                      (2.0 * l1 + 7.0 * l2) * kap[3])) *
                s / B;
    double t3 = 3.0 * G0 * (c * c / l1 + s * s / l2) +
                2.0 * G1 * s * c * (1.0 / l2 - 1.0 / l1) +
                G2 * (s * s / l1 + c * c / l2);
    C[0][2] = -3.0 * PI / (2.0 * sl * (l1 + l2)) * (t1 + t2 + t3);
  }
  C[0][3] = 3.0 * PI / (sl * S1) * s * c *
            ((1.0 - l1 * S1) / (A * l1) - (1.0 - l2 * S1) / (B * l2));
  C[0][4] = 3.0 * PI / (sl * S1) *
            (c * c * (1.0 - l1 * S1) / (A * l1) +
             s * s * (1.0 - l2 * S1) / (B * l2));
  C[1][1] = -PI / (sl * S2 * S2) *
            (3.0 * s * s * (1.0 - l1 * S2) * (1.0 - l1 * S2) / (A * l1) +
             3.0 * c * c * (1.0 - l2 * S2) * (1.0 - l2 * S2) / (B * l2) +
             S2 * S2);
  {
    double t1 = (-2.0 * sl1 * (3.0 * kap[0] * l1 + kap[2] * l2) +
                 3.0 / (2.0 * S2 * sl1) *
                     ((7.0 * l1 + 2.0 * l2) * kap[0] +
                      (l1 + 2.0 * l2) * kap[2])) *
                s / A;
    double t2 = (2.0 * sl2 * (kap[1] * l1 + 3.0 * kap[3] * l2) -
                 3.0 / (2.0 * S2 * sl2) *
                     ((2.0 * l1 + l2) * kap[1] +
                      (2.0 * l1 + 7.0 * l2) * kap[3])) *
                c / B;
    double t3 = 3.0 * G3 * (s * s / l1 + c * c / l2) +
                2.0 * G2 * s * c * (1.0 / l2 - 1.0 / l1) +
                G1 * (c * c / l1 + s * s / l2);
    C[1][2] = -3.0 * PI / (2.0 * sl * (l1 + l2)) * (t1 + t2 + t3);
  }
  C[1][3] = -3.0 * PI / (sl * S2) *
            (s * s * (1.0 - l1 * S2) / (A * l1) +
             c * c * (1.0 - l2 * S2) / (B * l2));
  C[1][4] = 3.0 * PI / (sl * S2) * s * c *
            (-(1.0 - l1 * S2) / (A * l1) + (1.0 - l2 * S2) / (B * l2));
  C[2][2] = 3.0 * PI / (sl * (l1 + l2));
  {
    double P = ((2.0 * l1 + l2) * kap[1] + (2.0 * l1 + 7.0 * l2) * kap[3]) /
               (sl2 * B);
    double R = ((l1 + 2.0 * l2) * kap[2] + (7.0 * l1 + 2.0 * l2) * kap[0]) /
               (sl1 * A);
    C[2][3] = 9.0 * PI / (4.0 * sl * (l1 + l2)) * (P * c - R * s);
    C[2][4] = -9.0 * PI / (4.0 * sl * (l1 + l2)) * (R * c + P * s);
  }
  C[2][5] = -3.0 * PI / (2.0 * sl * (l1 + l2)) * s * c * (1.0 / S1 - 1.0 / S2) *
            (1.0 / l1 - 1.0 / l2);
  C[3][3] = -3.0 * PI / sl * (s * s / (A * l1) + c * c / (B * l2));
  C[3][4] = 3.0 * PI / sl * s * c * (-1.0 / (A * l1) + 1.0 / (B * l2));
  C[4][4] = -3.0 * PI / sl * (c * c / (A * l1) + s * s / (B * l2));
  /* symmetry of K (Sec. III.B) */
  for (int r = 0; r < 6; ++r)
    for (int q = 0; q < r; ++q) C[r][q] = C[q][r];
  if (aux) {
    aux[0] = l1;
    aux[1] = l2;
    aux[2] = cchi;
    aux[3] = schi;
    for (int i = 0; i < 4; ++i) aux[4 + i] = kap[i];
  }
}

/* cut-off of element (r,c), Eq. lub:resistance-correction */
static double cutoff(int r, int c, const ref_params* p) {
  if (r == 2 && c == 2) return p->delta_n;
  if ((r == 3 || r == 4) && (c == 3 || c == 4)) return p->delta_r;
  return p->delta_t;
}

static double max_cutoff(const ref_params* p) {
  if (p->model == REF_MODEL_CONTACT) return p->h_c;   /* the repulsion's range */
  /* link-wise: a site of i within two links (2 sqrt 2) of a site of j */
  if (p->model == REF_MODEL_LINK || p->model == REF_MODEL_LINK_NAVG) return 2.0 * sqrt(2.0);
  if (p->model != REF_MODEL_FULL) return p->delta_n;  /* only the normal element */
  double m = p->delta_n;
  if (p->delta_t > m) m = p->delta_t;
  if (p->delta_r > m) m = p->delta_r;
  return m;
}

/* Local frame, geometry, K~ and the contact model for a solved pair.
 * bj == NULL: wall (infinite radii, zero cubic terms) with velocity
 * vwall.  o->n, o->yi, o->yj, o->h must be set. */
static void resistance_and_transfer(const body* bi, const body* bj,
                                    const double vi[3], const double wi[3],
                                    const double vj[3], const double wj[3],
                                    const ref_params* prm, ref_pair_result* o) {
  double hmax = max_cutoff(prm);
  double h = o->h;
  double heff = h > prm->h_c ? h : prm->h_c;
  memset(o->F, 0, sizeof(o->F));
  memset(o->Ti, 0, sizeof(o->Ti));
  memset(o->Tj, 0, sizeof(o->Tj));
  memset(o->Kt, 0, sizeof(o->Kt));
  memset(o->C, 0, sizeof(o->C));
  memset(o->Fbar, 0, sizeof(o->Fbar));
  if (heff >= hmax && h > prm->h_c) {
    o->status = REFP_INACTIVE;
    return;
  }
  if (!(heff > 0.0)) {
    o->status = REFP_UNRESOLVED;
    return;
  }
  o->status = REFP_ACTIVE;

  /* surface i: parameters of the closest point, principal direction
   * x1 = d y / d p (Eq. lub:curvature-directions), x3 along h */
  double e1[3], e2[3], e3[3];
  memcpy(e3, o->n, sizeof(e3));
  {
    double yb[3], sp, cp, sq, cq;
    mattvec3(bi->Q, o->yi, yb);
    surface_params(bi, yb, &sp, &cp, &sq, &cq);
    double s1b[3] = {-bi->Rperp * sp * cq, -bi->Rperp * sp * sq,
                     bi->Rpar * cp};
    matvec3(bi->Q, s1b, e1);
    double pr = dot3(e1, e3);
    for (int k = 0; k < 3; ++k) e1[k] -= pr * e3[k];
    scale3(e1, 1.0 / norm3(e1));
    cross3(e3, e1, e2);
    surface_coeffs(bi, sp, cp, &o->S1, &o->S2, &o->G[0], &o->G[2]);
    o->G[1] = 0.0;
    o->G[3] = 0.0;
  }
  /* surface j: its own principal direction x1', both x3 axes along h */
  if (bj) {
    double yb[3], sp, cp, sq, cq, S1p, S2p, e1p[3];
    mattvec3(bj->Q, o->yj, yb);
    surface_params(bj, yb, &sp, &cp, &sq, &cq);
    double s1b[3] = {-bj->Rperp * sp * cq, -bj->Rperp * sp * sq,
                     bj->Rpar * cp};
    matvec3(bj->Q, s1b, e1p);
    double pr = dot3(e1p, e3);
    for (int k = 0; k < 3; ++k) e1p[k] -= pr * e3[k];
    scale3(e1p, 1.0 / norm3(e1p));
    surface_coeffs(bj, sp, cp, &S1p, &S2p, &o->Gp[0], &o->Gp[2]);
    o->Gp[1] = 0.0;
    o->Gp[3] = 0.0;
    o->invS1p = 1.0 / S1p;
    o->invS2p = 1.0 / S2p;
    o->cphi = dot3(e1p, e1);
    o->sphi = dot3(e1p, e2);
  } else {
    o->invS1p = 0.0;
    o->invS2p = 0.0;
    memset(o->Gp, 0, sizeof(o->Gp));
    o->cphi = 1.0;
    o->sphi = 0.0;
  }
  for (int k = 0; k < 3; ++k) {
    o->e[0][k] = e1[k];
    o->e[1][k] = e2[k];
    o->e[2][k] = e3[k];
  }
  double aux[8];
  ref_K_coeffs(o->S1, o->S2, o->invS1p, o->invS2p, o->G, o->Gp, o->cphi,
               o->sphi, o->C, aux);
  o->lam1 = aux[0];
  o->lam2 = aux[1];
  o->cchi = aux[2];
  o->schi = aux[3];
  for (int i = 0; i < 4; ++i) o->kappa[i] = aux[4 + i];

  /* corrective matrix, Eq. lub:resistance-correction, gap clipped at h_c;
   * the "normal only" model keeps K33 alone */
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      double D = cutoff(r, c, prm);
      if (!(heff < D)) continue;
      if (prm->model == REF_MODEL_NORMAL && !(r == 2 && c == 2)) continue;
      if (prm->model == REF_MODEL_CONTACT) continue;
      if (r == 2 && c == 2)
        o->Kt[r][c] = o->C[r][c] * (1.0 / heff - 1.0 / D);
      else
        o->Kt[r][c] = o->C[r][c] * (log(heff) - log(D));
    }

  /* surface velocities at the closest points (rigid body) */
  double Vi[3], Vj[3], tmp[3];
  cross3(wi, o->yi, tmp);
  for (int k = 0; k < 3; ++k) Vi[k] = vi[k] + tmp[k];
  if (bj) {
    cross3(wj, o->yj, tmp);
    for (int k = 0; k < 3; ++k) Vj[k] = vj[k] + tmp[k];
  } else {
    for (int k = 0; k < 3; ++k) Vj[k] = vj[k];
  }
  double dU[6];
  double dV[3] = {Vj[0] - Vi[0], Vj[1] - Vi[1], Vj[2] - Vi[2]};
  double dW[3] = {wj[0] - wi[0], wj[1] - wi[1], wj[2] - wi[2]};
  dU[0] = dot3(e1, dV);
  dU[1] = dot3(e2, dV);
  dU[2] = dot3(e3, dV);
  dU[3] = dot3(e1, dW);
  dU[4] = dot3(e2, dW);
  dU[5] = dot3(e3, dW);
  /* Eq. lub:model */
  for (int r = 0; r < 6; ++r) {
    double acc = 0.0;
    for (int c = 0; c < 6; ++c) acc += o->Kt[r][c] * dU[c];
    o->Fbar[r] = prm->mu * acc;
  }
  if (h <= prm->h_c) {
    double Fr = h > 0.0 ? prm->eps_c * (prm->h_c - h) : prm->eps_c * prm->h_c;
    o->Fbar[2] -= Fr;
  }
  /* back to the world frame; torques about the particle centres */
  double T[3];
  for (int k = 0; k < 3; ++k) {
    o->F[k] = o->Fbar[0] * e1[k] + o->Fbar[1] * e2[k] + o->Fbar[2] * e3[k];
    T[k] = o->Fbar[3] * e1[k] + o->Fbar[4] * e2[k] + o->Fbar[5] * e3[k];
  }
  cross3(o->yi, o->F, tmp);
  for (int k = 0; k < 3; ++k) o->Ti[k] = T[k] + tmp[k];
  cross3(o->yj, o->F, tmp);
  for (int k = 0; k < 3; ++k) o->Tj[k] = -T[k] - tmp[k];
}

int ref_closest_points(const double d[3], const double qi[4],
                       const double semii[2], const double qj[4],
                       const double semij[2], ref_pair_result* out) {
  memset(out, 0, sizeof(*out));
  double zero[3] = {0, 0, 0};
  body bi, bj;
  body_init(&bi, zero, qi, semii);
  body_init(&bj, d, qj, semij);
  if (closest_pp(&bi, &bj, d, out)) {
    out->status = REFP_FAILED;
    return 0;
  }
  out->status = REFP_ACTIVE;
  return 0;
}

/* Ladd's normal law, Eq. methods:llub, for spheres of radii a and b (b = 0:
 * a wall): force on i along the unit n from i to j,
 *   mu 6 pi (a b / (a + b))^2 [n.(v_j - v_i)] (1/h - 1/Delta_n) n,
 * which is 3 pi mu R^2 / 2 for equal spheres and 6 pi mu a^2 against a
 * wall; the gap is clipped at h_c and the contact force of Eq. lub:frep
 * added, as in the contact-based model.  No torque: the force passes
 * through both centres. */
static void ladd_eval(const double n[3], double h, double a, double b,
                      const double vi[3], const double vj[3],
                      const ref_params* prm, ref_pair_result* o) {
  o->h = h;
  memcpy(o->n, n, 3 * sizeof(double));
  for (int k = 0; k < 3; ++k) {
    o->yi[k] = a * n[k];
    o->yj[k] = -b * n[k];
  }
  double heff = h > prm->h_c ? h : prm->h_c;
  if (heff >= prm->delta_n) {
    o->status = REFP_INACTIVE;
    return;
  }
  if (!(heff > 0.0)) {
    o->status = REFP_UNRESOLVED;
    return;
  }
  o->status = REFP_ACTIVE;
  double g = b > 0.0 ? a * b / (a + b) : a;
  o->C[2][2] = 6.0 * PI * g * g;
  o->Kt[2][2] = o->C[2][2] * (1.0 / heff - 1.0 / prm->delta_n);
  double dv[3] = {vj[0] - vi[0], vj[1] - vi[1], vj[2] - vi[2]};
  double fn = prm->mu * o->Kt[2][2] * dot3(n, dv);
  if (h <= prm->h_c) fn -= h > 0.0 ? prm->eps_c * (prm->h_c - h) : prm->eps_c * prm->h_c;
  o->Fbar[2] = fn;
  for (int k = 0; k < 3; ++k) o->F[k] = fn * n[k];
}

int ref_pair_eval(const double d[3], const double qi[4], const double semii[2],
                  const double vi[3], const double wi[3], const double qj[4],
                  const double semij[2], const double vj[3], const double wj[3],
                  const ref_params* prm, ref_pair_result* out) {
  memset(out, 0, sizeof(*out));
  if (prm->model == REF_MODEL_LADD) {
    if (semii[0] != semii[1] || semij[0] != semij[1]) {
      out->status = REFP_FAILED;  /* Ladd's law is for spheres */
      return 0;
    }
    double dn = norm3(d);
    double n[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
    ladd_eval(n, dn - semii[0] - semij[0], semii[0], semij[0], vi, vj, prm, out);
    return 0;
  }
  double zero[3] = {0, 0, 0};
  body bi, bj;
  body_init(&bi, zero, qi, semii);
  body_init(&bj, d, qj, semij);
  if (closest_pp(&bi, &bj, d, out)) {
    out->status = REFP_FAILED;
    return 0;
  }
  resistance_and_transfer(&bi, &bj, vi, wi, vj, wj, prm, out);
  return 0;
}

/* ------------------------------------------------------------------ */
/* link-wise law (Sec. II.D, Eq. methods:dlub)                         */
/* ------------------------------------------------------------------ */

/* the 18 non-zero velocities of the D3Q19 lattice */
static const int kD3Q19[18][3] = {
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
    {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* a lattice site belongs to a particle when it lies inside or on its
 * surface */
static int site_in(const body* b, const double x[3]) { return body_implicit(b, x) <= 0.0; }

/* parameters s_lo <= s_hi where the line x - s u (u unit) crosses the
 * surface: roots of A s^2 - 2 B s + C = 0 with q(x - s u) = 1 + that */
static int line_roots(const body* b, const double x[3], const double u[3], double* s_lo,
                      double* s_hi) {
  double xb[3], ub[3];
  to_body(b, x, xb);
  mattvec3(b->Q, u, ub);
  double A = 0.0, B = 0.0, C = -1.0;
  for (int k = 0; k < 3; ++k) {
    double inv = 1.0 / (b->D[k] * b->D[k]);
    A += ub[k] * ub[k] * inv;
    B += xb[k] * ub[k] * inv;
    C += xb[k] * xb[k] * inv;
  }
  double disc = B * B - A * C;
  if (!(disc >= 0.0) || !(A > 0.0)) return 1;
  double sq = sqrt(disc);
  *s_lo = (B - sq) / A;
  *s_hi = (B + sq) / A;
  return 0;
}

/* mean curvature (1/S1 + 1/S2) / 2 at the surface point y (Eq.
 * lub:curvature-radii) */
static double mean_curvature(const body* b, const double y[3]) {
  double yb[3], sp, cp, sq, cq, S1, S2, G0, G2;
  to_body(b, y, yb);
  surface_params(b, yb, &sp, &cp, &sq, &cq);
  surface_coeffs(b, sp, cp, &S1, &S2, &G0, &G2);
  return 0.5 * (1.0 / S1 + 1.0 / S2);
}

/* Every lattice link that ends on a site of i and starts on a site of j,
 * or on a fluid site halfway along two links from a site of j, each
 * undirected link once.  Its gap h* runs from where the link leaves the
 * surface of i to where it enters the surface of j; links with h* < |c_r|
 * carry the force of Eq. methods:dlub on i (minus it on j), at the
 * crossing points, with lambda* the mean of the two surfaces' mean
 * curvatures there, the gap clipped at h_c and the link-wise repulsion of
 * Eq. lub:frep below h_c.  Averaged-normal variant: velocity difference,
 * gap and force along the normalised difference of the two outward
 * normals (pointing from j to i). */
int ref_link_eval(const double ri[3], const double d[3], const double qi[4],
                  const double semii[2], const double vi[3], const double wi[3],
                  const double qj[4], const double semij[2], const double vj[3],
                  const double wj[3], const ref_params* prm, ref_pair_result* out) {
  memset(out, 0, sizeof(*out));
  double rj[3] = {ri[0] + d[0], ri[1] + d[1], ri[2] + d[2]};
  body bi, bj;
  body_init(&bi, ri, qi, semii);
  body_init(&bj, rj, qj, semij);
  const int navg = prm->model == REF_MODEL_LINK_NAVG;
  int lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    double e = sqrt(bi.M[4 * k]);
    lo[k] = (int)floor(ri[k] - e);
    hi[k] = (int)ceil(ri[k] + e);
  }
  double hmin = INFINITY;
  int links = 0;
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x) {
        double xb[3] = {(double)x, (double)y, (double)z};
        if (!site_in(&bi, xb) || site_in(&bj, xb)) continue;
        for (int r = 0; r < 18; ++r) {
          const int* c = kD3Q19[r];
          double cl = sqrt((double)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
          double x1[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
          if (site_in(&bi, x1)) continue;
          if (!site_in(&bj, x1)) {
            /* a fluid site: the pair of links from a site of j */
            double x2[3] = {xb[0] - 2 * c[0], xb[1] - 2 * c[1], xb[2] - 2 * c[2]};
            if (!site_in(&bj, x2) || site_in(&bi, x2)) continue;
          }
          double u[3] = {c[0] / cl, c[1] / cl, c[2] / cl}; /* from j's side to i */
          double a0, a1, b0, b1;
          if (line_roots(&bi, xb, u, &a0, &a1) || line_roots(&bj, xb, u, &b0, &b1)) continue;
          double hs = b0 - a1;
          if (!(hs < cl)) continue;
          ++links;
          if (hs < hmin) hmin = hs;
          double pi[3], pj[3], Vi[3], Vj[3], tmp[3], ai[3], aj[3];
          for (int k = 0; k < 3; ++k) {
            pi[k] = xb[k] - a1 * u[k];
            pj[k] = xb[k] - b0 * u[k];
            ai[k] = pi[k] - ri[k];
            aj[k] = pj[k] - rj[k];
          }
          cross3(wi, ai, tmp);
          for (int k = 0; k < 3; ++k) Vi[k] = vi[k] + tmp[k];
          cross3(wj, aj, tmp);
          for (int k = 0; k < 3; ++k) Vj[k] = vj[k] + tmp[k];
          double lam = 0.5 * (mean_curvature(&bi, pi) + mean_curvature(&bj, pj));
          double dir[3], gap;
          if (navg) {
            double ni[3], nj[3];
            body_normal(&bi, pi, ni);
            body_normal(&bj, pj, nj);
            for (int k = 0; k < 3; ++k) dir[k] = nj[k] - ni[k];
            scale3(dir, 1.0 / norm3(dir));
            gap = hs * dot3(u, dir);
          } else {
            memcpy(dir, u, sizeof(dir));
            gap = hs;
          }
          double heff = gap > prm->h_c ? gap : prm->h_c;
          double dvn = dot3(dir, Vi) - dot3(dir, Vj);
          double f = 0.0;
          if (heff > 0.0)
            f = -3.0 * prm->q_bar * prm->mu / (2.0 * cl * cl * lam) * dvn *
                (1.0 / (heff * heff) - 1.0 / (cl * cl));
          if (gap <= prm->h_c) f += gap > 0.0 ? prm->eps_c * (prm->h_c - gap) : prm->eps_c * prm->h_c;
          double Fl[3] = {f * dir[0], f * dir[1], f * dir[2]};
          for (int k = 0; k < 3; ++k) out->F[k] += Fl[k];
          cross3(ai, Fl, tmp);
          for (int k = 0; k < 3; ++k) out->Ti[k] += tmp[k];
          cross3(aj, Fl, tmp);
          for (int k = 0; k < 3; ++k) out->Tj[k] -= tmp[k];
        }
      }
  out->links = links;
  out->h = links ? hmin : 0.0;
  out->status = links ? REFP_ACTIVE : REFP_INACTIVE;
  return 0;
}

/* particle-wall: the wall is the second surface with infinite radii
 * (Appendix, wall remark); closest point on the particle is its support
 * point towards the wall */
int ref_wall_eval(const double ri[3], const double qi[4], const double semii[2],
                  const double vi[3], const double wi[3], int side,
                  const ref_domain* dom, const ref_params* prm,
                  ref_pair_result* out) {
  memset(out, 0, sizeof(*out));
  double n[3] = {0.0, 0.0, side == 0 ? -1.0 : 1.0};
  if (prm->model == REF_MODEL_LADD) {
    if (semii[0] != semii[1]) {
      out->status = REFP_FAILED;
      return 0;
    }
    double dist = side == 0 ? ri[2] : dom->L[2] - ri[2];
    ladd_eval(n, dist - semii[0], semii[0], 0.0, vi, dom->wall_vel[side], prm, out);
    return 0;
  }
  body bi;
  double zero[3] = {0, 0, 0};
  body_init(&bi, zero, qi, semii);
  double off[3];
  double hs = support(&bi, n, off);
  out->h = side == 0 ? ri[2] - hs : dom->L[2] - ri[2] - hs;
  memcpy(out->n, n, sizeof(n));
  memcpy(out->yi, off, sizeof(off));
  out->yj[0] = off[0];
  out->yj[1] = off[1];
  out->yj[2] = off[2] + out->h * n[2];
  double wzero[3] = {0, 0, 0};
  resistance_and_transfer(&bi, NULL, vi, wi, dom->wall_vel[side], wzero, prm,
                          out);
  return 0;
}

/* ------------------------------------------------------------------ */
/* pair sets and per-particle sums                                     */
/* ------------------------------------------------------------------ */

static double min_image(double dx, double L, int periodic) {
  if (periodic) dx = dx - L * nearbyint(dx / L);
  return dx;
}

/* Offset from i to the nearest image of j.  With Lees-Edwards images the
 * z image is chosen first; taking m boxes down in z moves the image by
 * -m le_offset in x (and its velocity by -m le_velocity), and x is then
 * wrapped as usual.  The offset is used modulo L_x, in [0, L_x).  Returns m
 * (0 without Lees-Edwards images). */
static int pair_image(const double ri[3], const double rj[3], const ref_domain* dom,
                      double d[3]) {
  int m = 0;
  double dx = rj[0] - ri[0];
  double dz = rj[2] - ri[2];
  if (dom->lees_edwards) {
    double c = nearbyint(dz / dom->L[2]);
    m = (int)c;
    dz = dz - dom->L[2] * c;
    double off = fmod(dom->le_offset, dom->L[0]);
    if (off < 0.0) off = off + dom->L[0];
    double shift = c * off;
    dx = dx - shift;
  } else {
    dz = min_image(dz, dom->L[2], dom->periodic[2]);
  }
  d[0] = min_image(dx, dom->L[0], dom->periodic[0]);
  d[1] = min_image(rj[1] - ri[1], dom->L[1], dom->periodic[1]);
  d[2] = dz;
  return m;
}

int ref_centre_test(const double ri[3], const double rj[3], double rmax_i,
                    double rmax_j, double dmax, const ref_domain* dom) {
  double d[3];
  pair_image(ri, rj, dom, d);
  double dx = d[0], dy = d[1], dz = d[2];
  double d2 = dx * dx + dy * dy + dz * dz;
  double s = (rmax_i + rmax_j) + dmax;
  return d2 < s * s;
}

static double rmax_of(const double* semi, int64_t i) {
  return semi[2 * i] > semi[2 * i + 1] ? semi[2 * i] : semi[2 * i + 1];
}

/* wall candidate test: centre-to-wall distance minus the bounding radius
 * below the largest cut-off */
static int wall_test(const double* r, const double* semi, int64_t i, int side,
                     const ref_domain* dom, double dmax) {
  double dist = side == 0 ? r[3 * i + 2] : dom->L[2] - r[3 * i + 2];
  return (dist - rmax_of(semi, i)) < dmax;
}

int ref_candidates(int64_t n, const double* r, const double* semi,
                   const ref_domain* dom, const ref_params* prm, int64_t cap,
                   int32_t* ij, int64_t* n_pairs, int64_t wcap, int32_t* wall,
                   int64_t* n_wall) {
  double dmax = max_cutoff(prm);
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0;
    for (int64_t j = i + 1; j < n; ++j)
      c += ref_centre_test(&r[3 * i], &r[3 * j], rmax_of(semi, i),
                           rmax_of(semi, j), dmax, dom);
    cnt[i + 1] = c;
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  *n_pairs = cnt[n];
  int rc = REF_OK;
  if (cnt[n] > cap) rc = REF_ECAPACITY;
  if (rc == REF_OK && ij) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      int64_t o = cnt[i];
      for (int64_t j = i + 1; j < n; ++j)
        if (ref_centre_test(&r[3 * i], &r[3 * j], rmax_of(semi, i),
                            rmax_of(semi, j), dmax, dom)) {
          ij[2 * o] = (int32_t)i;
          ij[2 * o + 1] = (int32_t)j;
          ++o;
        }
    }
  }
  free(cnt);
  int64_t nw = 0;
  if (dom->n_walls == 2) {
    for (int64_t i = 0; i < n; ++i)
      for (int side = 0; side < 2; ++side)
        if (wall_test(r, semi, i, side, dom, dmax)) {
          if (nw < wcap && wall) {
            wall[2 * nw] = (int32_t)i;
            wall[2 * nw + 1] = side;
          }
          ++nw;
        }
  }
  *n_wall = nw;
  if (nw > wcap) rc = REF_ECAPACITY;
  return rc;
}

int ref_partners_subset(int64_t n, const double* r, const double* semi,
                        const ref_domain* dom, const ref_params* prm, int64_t m,
                        const int64_t* idx, int64_t cap, int32_t* partners,
                        int64_t* counts) {
  double dmax = max_cutoff(prm);
  int rc = REF_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m; ++s) {
    const int64_t k = idx[s];
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == k) continue;
      if (!ref_centre_test(&r[3 * k], &r[3 * j], rmax_of(semi, k), rmax_of(semi, j),
                           dmax, dom))
        continue;
      if (c < cap) partners[s * cap + c] = (int32_t)j;
      ++c;
    }
    counts[s] = c;
    if (c > cap) {
#pragma omp critical
      rc = REF_ECAPACITY;
    }
  }
  return rc;
}


static void eval_one(int64_t n, const double* r, const double* q,
                     const double* semi, const double* v, const double* w,
                     const ref_domain* dom, const ref_params* prm, int32_t i,
                     int32_t j, ref_pair_result* o) {
  (void)n;
  if (j >= 0) {
    double d[3];
    const int m = pair_image(&r[3 * i], &r[3 * j], dom, d);
    /* velocity of the image of j that d points to */
    double vj[3] = {v[3 * j] - m * dom->le_velocity, v[3 * j + 1], v[3 * j + 2]};
    if (prm->model == REF_MODEL_LINK || prm->model == REF_MODEL_LINK_NAVG)
      ref_link_eval(&r[3 * i], d, &q[4 * i], &semi[2 * i], &v[3 * i], &w[3 * i], &q[4 * j],
                    &semi[2 * j], vj, &w[3 * j], prm, o);
    else
      ref_pair_eval(d, &q[4 * i], &semi[2 * i], &v[3 * i], &w[3 * i], &q[4 * j],
                    &semi[2 * j], vj, &w[3 * j], prm, o);
  } else {
    ref_wall_eval(&r[3 * i], &q[4 * i], &semi[2 * i], &v[3 * i], &w[3 * i],
                  -j - 1, dom, prm, o);
  }
}

static void tally(ref_stats* st, const ref_pair_result* o) {
  if (!st) return;
  if (o->status == REFP_ACTIVE) {
    st->active++;
    if (o->h <= 0.0) st->overlaps++;
  }
  if (o->status == REFP_UNRESOLVED) st->unresolved++;
  if (o->status == REFP_FAILED) st->failed++;
  st->fallbacks += o->fallback;
  st->iters_lh_total += o->iters_lh;
  if (o->iters_lh > st->iters_lh_max) st->iters_lh_max = o->iters_lh;
  st->iters_polish_total += o->iters_polish;
}

static int valid_inputs(int64_t n, const double* r, const double* q,
                        const double* semi, const double* v, const double* w,
                        const ref_domain* dom, const ref_params* prm) {
  if (n < 0 || !dom || !prm) return 0;
  if (n > 0 && (!r || !q || !semi || !v || !w)) return 0;
  if (dom->lees_edwards &&
      (!dom->periodic[0] || !dom->periodic[1] || !dom->periodic[2] || dom->n_walls ||
       !isfinite(dom->le_offset) || !isfinite(dom->le_velocity)))
    return 0;
  if (prm->model == REF_MODEL_LINK || prm->model == REF_MODEL_LINK_NAVG) {
    /* lattice images of the sites: integer periodic lengths, no walls */
    if (dom->n_walls || dom->lees_edwards || !(prm->q_bar > 0.0)) return 0;
    for (int k = 0; k < 3; ++k)
      if (dom->periodic[k] && dom->L[k] != floor(dom->L[k])) return 0;
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k)
      if (!isfinite(r[3 * i + k]) || !isfinite(v[3 * i + k]) ||
          !isfinite(w[3 * i + k]))
        return 0;
    double qq = 0.0;
    for (int k = 0; k < 4; ++k) {
      if (!isfinite(q[4 * i + k])) return 0;
      qq += q[4 * i + k] * q[4 * i + k];
    }
    if (fabs(sqrt(qq) - 1.0) > 1e-6) return 0;
    if (!(semi[2 * i] > 0.0) || !(semi[2 * i + 1] > 0.0)) return 0;
  }
  return 1;
}

int ref_compute(int64_t n, const double* r, const double* q,
                const double* semi, const double* v, const double* w,
                const ref_domain* dom, const ref_params* prm, int nthreads,
                double* f, double* t, ref_stats* st) {
  if (!valid_inputs(n, r, q, semi, v, w, dom, prm)) return REF_EINVAL;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  if (st) memset(st, 0, sizeof(*st));
  int64_t np = 0, nw = 0;
  ref_candidates(n, r, semi, dom, prm, 0, NULL, &np, 0, NULL, &nw);
  int32_t* ij = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(np + nw + 1));
  int64_t np2 = 0, nw2 = 0;
  ref_candidates(n, r, semi, dom, prm, np, ij, &np2, nw, ij + 2 * np, &nw2);
  for (int64_t k = 0; k < nw; ++k) /* wall side s -> j = -(s+1) */
    ij[2 * (np + k) + 1] = -(ij[2 * (np + k) + 1] + 1);
  int64_t tot = np + nw;
  double* out = (double*)malloc(sizeof(double) * 9 * (size_t)(tot + 1));
  int32_t* stat = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tot + 1));
  ref_pair_result* tmp = NULL;
  int used = 1;
#pragma omp parallel
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
    ref_pair_result o;
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < tot; ++p) {
      eval_one(n, r, q, semi, v, w, dom, prm, ij[2 * p], ij[2 * p + 1], &o);
      memcpy(&out[9 * p], o.F, 3 * sizeof(double));
      memcpy(&out[9 * p + 3], o.Ti, 3 * sizeof(double));
      memcpy(&out[9 * p + 6], o.Tj, 3 * sizeof(double));
      stat[p] = o.status;
#pragma omp critical
      tally(st, &o);
    }
  }
  (void)tmp;
  memset(f, 0, sizeof(double) * 3 * (size_t)n);
  memset(t, 0, sizeof(double) * 3 * (size_t)n);
  for (int64_t p = 0; p < tot; ++p) {
    if (stat[p] != REFP_ACTIVE) continue;
    int32_t i = ij[2 * p], j = ij[2 * p + 1];
    for (int k = 0; k < 3; ++k) {
      f[3 * i + k] += out[9 * p + k];
      t[3 * i + k] += out[9 * p + 3 + k];
      if (j >= 0) {
        f[3 * j + k] -= out[9 * p + k];
        t[3 * j + k] += out[9 * p + 6 + k];
      }
    }
  }
  if (st) {
    st->candidates = np;
    st->wall_candidates = nw;
    st->threads = used;
  }
  free(ij);
  free(out);
  free(stat);
  return REF_OK;
}

int ref_compute_subset(int64_t n, const double* r, const double* q,
                       const double* semi, const double* v, const double* w,
                       const ref_domain* dom, const ref_params* prm,
                       int64_t m, const int64_t* idx, int nthreads, double* f,
                       double* t, ref_stats* st) {
  if (!valid_inputs(n, r, q, semi, v, w, dom, prm)) return REF_EINVAL;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  if (st) memset(st, 0, sizeof(*st));
  double dmax = max_cutoff(prm);
  int used = 1;
#pragma omp parallel
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; ++s) {
      int64_t k = idx[s];
      double fk[3] = {0, 0, 0}, tk[3] = {0, 0, 0};
      ref_pair_result o;
      /* ascending partner order: pairs (j,k) with j<k, then (k,j) with
       * j>k -- the order in which the sorted pair list visits k */
      for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        if (!ref_centre_test(&r[3 * k], &r[3 * j], rmax_of(semi, k),
                             rmax_of(semi, j), dmax, dom))
          continue;
        int32_t a = (int32_t)(j < k ? j : k), b = (int32_t)(j < k ? k : j);
        eval_one(n, r, q, semi, v, w, dom, prm, a, b, &o);
        if (st) {
#pragma omp critical
          {
            st->candidates++;
            tally(st, &o);
          }
        }
        if (o.status != REFP_ACTIVE) continue;
        for (int c = 0; c < 3; ++c) {
          if (a == k) {
            fk[c] += o.F[c];
            tk[c] += o.Ti[c];
          } else {
            fk[c] -= o.F[c];
            tk[c] += o.Tj[c];
          }
        }
      }
      if (dom->n_walls == 2)
        for (int side = 0; side < 2; ++side) {
          if (!wall_test(r, semi, k, side, dom, dmax)) continue;
          eval_one(n, r, q, semi, v, w, dom, prm, (int32_t)k, -(side + 1), &o);
          if (st) {
#pragma omp critical
            {
              st->wall_candidates++;
              tally(st, &o);
            }
          }
          if (o.status != REFP_ACTIVE) continue;
          for (int c = 0; c < 3; ++c) {
            fk[c] += o.F[c];
            tk[c] += o.Ti[c];
          }
        }
      memcpy(&f[3 * s], fk, sizeof(fk));
      memcpy(&t[3 * s], tk, sizeof(tk));
    }
  }
  if (st) st->threads = used;
  return REF_OK;
}

int ref_eval_pairs(int64_t n, const double* r, const double* q,
                   const double* semi, const double* v, const double* w,
                   const ref_domain* dom, const ref_params* prm, int64_t np,
                   const int32_t* ij, int nthreads, double* F, double* Ti,
                   double* Tj, double* h, int32_t* status, int32_t* links) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < np; ++p) {
    ref_pair_result o;
    eval_one(n, r, q, semi, v, w, dom, prm, ij[2 * p], ij[2 * p + 1], &o);
    for (int k = 0; k < 3; ++k) {
      F[3 * p + k] = o.F[k];
      Ti[3 * p + k] = o.Ti[k];
      Tj[3 * p + k] = o.Tj[k];
    }
    h[p] = o.h;
    status[p] = o.status;
    if (links) links[p] = o.links;
  }
  return REF_OK;
}

int ref_eval_pairs_detail(int64_t n, const double* r, const double* q,
                          const double* semi, const double* v, const double* w,
                          const ref_domain* dom, const ref_params* prm,
                          int64_t np, const int32_t* ij, int nthreads,
                          double* F, double* Ti, double* Tj, double* h,
                          int32_t* status, double* nrm, double* yi, double* yj,
                          double* e1, double* Kt, int32_t* iters_lh,
                          int32_t* iters_polish) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < np; ++p) {
    ref_pair_result o;
    eval_one(n, r, q, semi, v, w, dom, prm, ij[2 * p], ij[2 * p + 1], &o);
    for (int k = 0; k < 3; ++k) {
      if (F) F[3 * p + k] = o.F[k];
      if (Ti) Ti[3 * p + k] = o.Ti[k];
      if (Tj) Tj[3 * p + k] = o.Tj[k];
      if (nrm) nrm[3 * p + k] = o.n[k];
      if (yi) yi[3 * p + k] = o.yi[k];
      if (yj) yj[3 * p + k] = o.yj[k];
      if (e1) e1[3 * p + k] = o.e[0][k];
    }
    if (Kt)
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) Kt[36 * p + 6 * a + b] = o.Kt[a][b];
    if (h) h[p] = o.h;
    if (status) status[p] = o.status;
    if (iters_lh) iters_lh[p] = o.iters_lh;
    if (iters_polish) iters_polish[p] = o.iters_polish;
  }
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* pairs at a prescribed gap (learned-seed data)                       */
/* ------------------------------------------------------------------ */

int ref_place_pairs(int64_t m, const double* u, const double* target,
                    const double* qi, const double* semii, const double* qj,
                    const double* semij, int nthreads, double* s, double* h,
                    double* n, double* yi, double* yj, int32_t* iters_lh,
                    int32_t* status) {
  if (m < 0) return REF_EINVAL;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < m; ++k) {
    const double* uk = u + 3 * k;
    const double g = target[k];
    const double rmi = semii[2 * k] > semii[2 * k + 1] ? semii[2 * k] : semii[2 * k + 1];
    const double rmj = semij[2 * k] > semij[2 * k + 1] ? semij[2 * k] : semij[2 * k + 1];
    double sk = rmi + rmj + g;  /* the gap here is >= g */
    ref_pair_result o;
    int st = 3;
    for (int it = 0; it < 60; ++it) {
      const double d[3] = {sk * uk[0], sk * uk[1], sk * uk[2]};
      ref_closest_points(d, qi + 4 * k, semii + 2 * k, qj + 4 * k, semij + 2 * k, &o);
      if (o.status != REFP_ACTIVE) break;
      const double diff = o.h - g;
      if (fabs(diff) <= 1e-12 * (1.0 + g)) {
        st = 0;
        break;
      }
      const double slope = dot3(o.n, uk);
      if (!(slope > 1e-12)) break;
      sk -= diff / slope;
    }
    s[k] = sk;
    h[k] = o.h;
    for (int a = 0; a < 3; ++a) {
      n[3 * k + a] = o.n[a];
      yi[3 * k + a] = o.yi[a];
      yj[3 * k + a] = o.yj[a];
    }
    iters_lh[k] = o.iters_lh;
    status[k] = st;
  }
  return 0;
}
