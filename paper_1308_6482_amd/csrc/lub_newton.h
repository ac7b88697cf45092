// lub_newton.h -- closest points of two spheroids by Newton's method on the
// common normal (Sec. III.A), shared by the pair kernels.  Host and device
// code: a host build of this header checks the solver's branches on the CPU.
//
// The paper's fixed point -- outward normals antiparallel and along the line
// joining the tangent points -- is, with the tangent points written as
// support points y_i = r_i + M_i n / h_i(n), y_j = r_j - M_j n / h_j(n)
// (h_k(n) = sqrt(n.M_k n)), the stationary point of
// g(n) = n.d - h_i(n) - h_j(n) on the unit sphere; g there is the signed gap
// (negative for a small overlap).  Newton's method in the tangent plane of n
// (two unknowns), FP64, with the Hessian shifted to stay negative definite
// far from the solution and Armijo backtracking.
#pragma once

#include <math.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#define __forceinline__ inline
#endif

// 1 / sqrt(x): on the device the reciprocal square root, one correctly
// refined sequence instead of a square root and a division; the host build
// of the header divides.
__host__ __device__ __forceinline__ double inv_sqrt(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  return rsqrt(x);
#else
  return 1.0 / sqrt(x);
#endif
}
__host__ __device__ __forceinline__ float inv_sqrt(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return rsqrtf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// backtracking trials and sufficient-increase constant of the line search
// (a host test build overrides them to force an exhausted search)
#ifndef LUB_LINE_SEARCH_TRIALS
#define LUB_LINE_SEARCH_TRIALS 30
#endif
#ifndef LUB_ARMIJO
#define LUB_ARMIJO 1e-4
#endif

namespace lub {

__host__ __device__ __forceinline__ void symv(const double* M, const double x[3],
                                     double y[3]) {
  y[0] = M[0] * x[0] + M[1] * x[1] + M[2] * x[2];
  y[1] = M[1] * x[0] + M[3] * x[1] + M[4] * x[2];
  y[2] = M[2] * x[0] + M[4] * x[1] + M[5] * x[2];
}

template <typename T>
__host__ __device__ __forceinline__ T dot3(const T a[3], const T b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <typename T>
__host__ __device__ __forceinline__ void cross3(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// any unit vector orthogonal to the unit vector n
__host__ __device__ __forceinline__ void perp(const double n[3], double t[3]) {
  double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
  if (ax <= ay && ax <= az) {
    t[0] = 0.0;
    t[1] = n[2];
    t[2] = -n[1];
  } else if (ay <= az) {
    t[0] = -n[2];
    t[1] = 0.0;
    t[2] = n[0];
  } else {
    t[0] = n[1];
    t[1] = -n[0];
    t[2] = 0.0;
  }
  double inv = inv_sqrt(dot3(t, t));
  t[0] *= inv;
  t[1] *= inv;
  t[2] *= inv;
}

struct Solve {
  double n[3];   // unit gap direction i -> j
  double ai[3];  // y_i - r_i
  double bj[3];  // r_j - y_j
  double h;
  int iters;
  bool ok;
};

// The plain start: the line of centres mapped by (M_i + M_j)^-1, the
// normal at d of the ellipsoid with matrix M_i + M_j, which stands in for
// the Minkowski sum of the two bodies (whose normal at d - h n is the
// answer).  Exact for spheres and for aligned bodies of one shape; for the
// others about one Newton iteration closer than the line of centres.
// Formed with the adjugate (S is positive definite: only the direction
// counts), falling back to the line of centres for a degenerate d.
__host__ __device__ __forceinline__ void plain_start(const double d[3], const double* Mi,
                                                     const double* Mj, double n[3]) {
  const double a = Mi[0] + Mj[0], b = Mi[1] + Mj[1], c = Mi[2] + Mj[2];
  const double e = Mi[3] + Mj[3], f = Mi[4] + Mj[4], g = Mi[5] + Mj[5];
  // adj(S) d for S = [a b c; b e f; c f g]
  const double m0 = (e * g - f * f) * d[0] + (c * f - b * g) * d[1] + (b * f - c * e) * d[2];
  const double m1 = (c * f - b * g) * d[0] + (a * g - c * c) * d[1] + (b * c - a * f) * d[2];
  const double m2 = (b * f - c * e) * d[0] + (b * c - a * f) * d[1] + (a * e - b * b) * d[2];
  const double mn2 = m0 * m0 + m1 * m1 + m2 * m2;
  if (mn2 > 0.0 && m0 * d[0] + m1 * d[1] + m2 * d[2] > 0.0) {
    const double im = inv_sqrt(mn2);
    n[0] = m0 * im;
    n[1] = m1 * im;
    n[2] = m2 * im;
  } else {
    const double id = inv_sqrt(dot3(d, d));
    n[0] = d[0] * id;
    n[1] = d[1] * id;
    n[2] = d[2] * id;
  }
}

// Newton iteration for the stationary point of g(n) on the unit sphere,
// started from n0 (unit) when use_n0, else from the plain start above (the
// start is selected by value: no pointer to a local escapes to memory);
// converged when the tangential residual is below rel_tol (h_i + h_j)
__host__ __device__ __forceinline__ Solve closest_points(const double d[3],
                                                const double* Mi,
                                                const double* Mj, int maxit,
                                                const double (&n0)[3], bool use_n0,
                                                double rel_tol = 1e-14) {
  Solve o;
  double n[3];
  plain_start(d, Mi, Mj, n);
  for (int k = 0; k < 3; ++k) n[k] = use_n0 ? n0[k] : n[k];
  double prev2 = 1.0;  // squared length of the last step
  bool last_full = false;
  o.ok = false;
  int it = 0;
  double hi = 0, hj = 0, ai[3], bj[3];
  for (;; ++it) {
    double a[3], b[3];
    symv(Mi, n, a);
    symv(Mj, n, b);
    // h = q / sqrt(q): one reciprocal square root per body
    const double qi = dot3(n, a), qj = dot3(n, b);
    const double ih = inv_sqrt(qi), jh = inv_sqrt(qj);
    hi = qi * ih;
    hj = qj * jh;
    for (int k = 0; k < 3; ++k) {
      ai[k] = a[k] * ih;
      bj[k] = b[k] * jh;
    }
    double g[3] = {d[0] - ai[0] - bj[0], d[1] - ai[1] - bj[1],
                   d[2] - ai[2] - bj[2]};
    double t1[3], t2[3];
    perp(n, t1);
    cross3(n, t1, t2);
    double r1 = dot3(g, t1), r2 = dot3(g, t2);
    double tol = rel_tol * (hi + hj);
    // converged: the tangential residual at round-off, or a full Newton step
    // below 1e-8 (quadratic convergence leaves an error of its square); a
    // step shortened by the line search says nothing about convergence
    if ((prev2 < 1e-16 && last_full) || r1 * r1 + r2 * r2 <= tol * tol) {
      o.ok = true;
      break;
    }
    if (it >= maxit) break;
    double gn = dot3(g, n);
    double u1[3], u2[3], w1[3], w2[3];
    symv(Mi, t1, u1);
    symv(Mi, t2, u2);
    symv(Mj, t1, w1);
    symv(Mj, t2, w2);
    double at1 = dot3(ai, t1), at2 = dot3(ai, t2);
    double bt1 = dot3(bj, t1), bt2 = dot3(bj, t2);
    double H11 = -(dot3(t1, u1) - at1 * at1) * ih - (dot3(t1, w1) - bt1 * bt1) * jh - gn;
    double H12 = -(dot3(t1, u2) - at1 * at2) * ih - (dot3(t1, w2) - bt1 * bt2) * jh;
    double H22 = -(dot3(t2, u2) - at2 * at2) * ih - (dot3(t2, w2) - bt2 * bt2) * jh - gn;
    // keep the (maximisation) Hessian negative definite
    double mid = 0.5 * (H11 + H22), dif = 0.5 * (H11 - H22);
    double lmax = mid + sqrt(dif * dif + H12 * H12);
    double floor_ = 1e-3 * (hi + hj);
    if (lmax > -floor_) {
      H11 -= lmax + floor_;
      H22 -= lmax + floor_;
    }
    const double idet = 1.0 / (H11 * H22 - H12 * H12);
    double s1 = -(H22 * r1 - H12 * r2) * idet;
    double s2 = -(H11 * r2 - H12 * r1) * idet;
    // the step's length is compared squared: a square root only to shorten it
    double len2 = s1 * s1 + s2 * s2;
    if (len2 > 0.25) {
      const double f = 0.5 * inv_sqrt(len2);
      s1 *= f;
      s2 *= f;
      len2 = 0.25;
    }
    // Armijo backtracking on g along the (ascent) direction; skipped in the
    // quadratic basin where the full step is always taken
    double alpha = 1.0;
    if (len2 > 1e-6) {
      const double g0 = gn;  // g(n) = n.d - h_i - h_j
      const double slope = r1 * s1 + r2 * s2;
      bool ascent = false;
      for (int ls = 0; ls < LUB_LINE_SEARCH_TRIALS; ++ls) {
        double m[3];
        for (int k = 0; k < 3; ++k) m[k] = n[k] + alpha * (s1 * t1[k] + s2 * t2[k]);
        double inv = 1.0 / sqrt(dot3(m, m));
        for (int k = 0; k < 3; ++k) m[k] *= inv;
        double a2[3], b2[3];
        symv(Mi, m, a2);
        symv(Mj, m, b2);
        double gt = dot3(m, d) - sqrt(dot3(m, a2)) - sqrt(dot3(m, b2));
        if (gt >= g0 + LUB_ARMIJO * alpha * slope) {
          ascent = true;
          break;
        }
        alpha *= 0.5;
      }
      // no ascent step along the direction: the solve fails (the caller
      // starts again from another seed or takes the tangent-sphere pass)
      if (!ascent) break;
    }
    prev2 = alpha * alpha * len2;
    last_full = alpha == 1.0;
    double m[3];
    for (int k = 0; k < 3; ++k) m[k] = n[k] + alpha * (s1 * t1[k] + s2 * t2[k]);
    const double inv = inv_sqrt(dot3(m, m));
    for (int k = 0; k < 3; ++k) n[k] = m[k] * inv;
  }
  for (int k = 0; k < 3; ++k) {
    o.n[k] = n[k];
    o.ai[k] = ai[k];
    o.bj[k] = bj[k];
  }
  o.h = dot3(n, d) - hi - hj;
  o.iters = it;
  return o;
}

}  // namespace lub
