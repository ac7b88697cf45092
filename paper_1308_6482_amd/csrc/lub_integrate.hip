// Particle update of the sub-stepped integrator (Sec. II: the particle time
// step is a fraction of the fluid's, with the lubrication forces evaluated
// again at every sub-step) and the size ramp of the packing generator's
// growth stage (Sec. IV.C).
//
// One thread per particle, FP64 throughout.  The update is semi-implicit
// Euler with the angular momentum carried in the world frame:
//   v <- v + dt (F / m - damping v)
//   L = I(q) w;  L <- L + dt (T - damping L)
//   q <- exp(dt I(q)^-1 L / 2) q          (rotation quaternion, world frame)
//   r <- r + dt v;  w <- I(q)^-1 L
// For a spheroid with unit symmetry axis a, mass m and inertias I_par (about
// a) and I_perp (across it), I = I_perp 1 + (I_par - I_perp) a a^T and
// I^-1 = (1 / I_perp) 1 + (1 / I_par - 1 / I_perp) a a^T.
#include <hip/hip_runtime.h>

#include "lub_internal.h"

namespace lub {
namespace {

constexpr double kPi = 3.14159265358979323846;

// symmetry axis Q(q) e_z of the unit quaternion (w, x, y, z)
__device__ __forceinline__ void body_axis(const double* q, double a[3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  a[0] = 2.0 * (x * z + w * y);
  a[1] = 2.0 * (y * z - w * x);
  a[2] = 1.0 - 2.0 * (x * x + y * y);
}

__global__ void k_integrate(StepDesc s, double* __restrict__ r, double* __restrict__ q,
                            const double* __restrict__ semi,
                            double* __restrict__ v, double* __restrict__ w,
                            const double* __restrict__ f_ext,
                            const double* __restrict__ t_ext,
                            const double* __restrict__ f, const double* __restrict__ t) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const double Rpa = semi[2 * i], Rpe = semi[2 * i + 1];
  const double m = s.density * (4.0 / 3.0 * kPi) * Rpa * Rpe * Rpe;
  const double Ipa = 0.4 * m * Rpe * Rpe;
  const double Ipe = 0.2 * m * (Rpa * Rpa + Rpe * Rpe);
  const double dt = s.dt, damp = s.damping;
  double F[3], T[3], vi[3], wi[3], ri[3], qi[4];
  for (int k = 0; k < 3; ++k) {
    F[k] = f[3 * i + k];
    T[k] = t[3 * i + k];
    if (f_ext) F[k] = F[k] + f_ext[3 * i + k];
    if (t_ext) T[k] = T[k] + t_ext[3 * i + k];
    vi[k] = v[3 * i + k];
    wi[k] = w[3 * i + k];
    ri[k] = r[3 * i + k];
  }
  for (int k = 0; k < 4; ++k) qi[k] = q[4 * i + k];
  // translation
  for (int k = 0; k < 3; ++k) vi[k] = vi[k] + dt * (F[k] / m - damp * vi[k]);
  // angular momentum in the world frame
  double a[3];
  body_axis(qi, a);
  const double aw = a[0] * wi[0] + a[1] * wi[1] + a[2] * wi[2];
  double L[3];
  for (int k = 0; k < 3; ++k) L[k] = Ipe * wi[k] + (Ipa - Ipe) * aw * a[k];
  for (int k = 0; k < 3; ++k) L[k] = L[k] + dt * (T[k] - damp * L[k]);
  // rotation by the angular velocity of the current orientation
  const double cI = 1.0 / Ipa - 1.0 / Ipe;
  double aL = a[0] * L[0] + a[1] * L[1] + a[2] * L[2];
  double om[3];
  for (int k = 0; k < 3; ++k) om[k] = L[k] / Ipe + cI * aL * a[k];
  const double on = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
  if (on > 0.0) {
    const double half = 0.5 * on * dt;
    const double c = cos(half), sn = sin(half) / on;
    const double p0 = c, p1 = sn * om[0], p2 = sn * om[1], p3 = sn * om[2];
    // p (x) q
    const double q0 = p0 * qi[0] - p1 * qi[1] - p2 * qi[2] - p3 * qi[3];
    const double q1 = p0 * qi[1] + p1 * qi[0] + p2 * qi[3] - p3 * qi[2];
    const double q2 = p0 * qi[2] - p1 * qi[3] + p2 * qi[0] + p3 * qi[1];
    const double q3 = p0 * qi[3] + p1 * qi[2] - p2 * qi[1] + p3 * qi[0];
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    qi[0] = q0 / qn;
    qi[1] = q1 / qn;
    qi[2] = q2 / qn;
    qi[3] = q3 / qn;
  }
  // angular velocity of the new orientation
  body_axis(qi, a);
  aL = a[0] * L[0] + a[1] * L[1] + a[2] * L[2];
  for (int k = 0; k < 3; ++k) wi[k] = L[k] / Ipe + cI * aL * a[k];
  // position, then back into the box
  for (int k = 0; k < 3; ++k) ri[k] = ri[k] + dt * vi[k];
  if (s.le) {
    // through the top (bottom): shifted by -offset (+offset) in x, x
    // velocity lowered (raised) by the image velocity
    const double c = floor(ri[2] / s.L[2]);
    if (c != 0.0) {
      ri[2] = ri[2] - c * s.L[2];
      ri[0] = ri[0] - c * s.le_offset;
      vi[0] = vi[0] - c * s.le_vel;
    }
  }
  for (int k = 0; k < 3; ++k)
    if (s.periodic[k] && !(s.le && k == 2)) ri[k] = ri[k] - s.L[k] * floor(ri[k] / s.L[k]);
  for (int k = 0; k < 3; ++k) {
    r[3 * i + k] = ri[k];
    v[3 * i + k] = vi[k];
    w[3 * i + k] = wi[k];
  }
  for (int k = 0; k < 4; ++k) q[4 * i + k] = qi[k];
}

// Kinematic advance: the particles follow their given velocities, with no
// forces: r <- r + dt v, and the first-order orientation step
// q <- normalise(q + dt/2 (0, w) q) with (0, w) q the quaternion product
// (a rotation by 2 atan(dt |w| / 2) about w).  One thread per particle,
// FP64, the terms in a fixed order.
__global__ void k_advance(int n, double dt, double* __restrict__ r, double* __restrict__ q,
                          const double* __restrict__ v, const double* __restrict__ w) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) r[3 * i + k] = r[3 * i + k] + dt * v[3 * i + k];
  const double q0 = q[4 * i], q1 = q[4 * i + 1], q2 = q[4 * i + 2], q3 = q[4 * i + 3];
  const double w0 = w[3 * i], w1 = w[3 * i + 1], w2 = w[3 * i + 2];
  const double h = 0.5 * dt;
  // (0, w) q = (-w . q_v, q_0 w + w x q_v)
  const double p0 = q0 + h * -(w0 * q1 + w1 * q2 + w2 * q3);
  const double p1 = q1 + h * (q0 * w0 + (w1 * q3 - w2 * q2));
  const double p2 = q2 + h * (q0 * w1 + (w2 * q1 - w0 * q3));
  const double p3 = q3 + h * (q0 * w2 + (w0 * q2 - w1 * q1));
  const double pn = sqrt(p0 * p0 + p1 * p1 + p2 * p2 + p3 * p3);
  q[4 * i] = p0 / pn;
  q[4 * i + 1] = p1 / pn;
  q[4 * i + 2] = p2 / pn;
  q[4 * i + 3] = p3 / pn;
}

__global__ void k_scale(int n, const double* __restrict__ semi, double scale,
                        double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * n) out[i] = semi[i] * scale;
}

}  // namespace

void launch_integrate(const StepDesc& s, double* r, double* q, const double* semi,
                      double* v, double* w, const double* f_ext, const double* t_ext,
                      const double* f, const double* t, hipStream_t st) {
  if (s.n <= 0) return;
  hipLaunchKernelGGL(k_integrate, dim3((s.n + 255) / 256), dim3(256), 0, st, s, r, q, semi,
                     v, w, f_ext, t_ext, f, t);
}

void launch_advance(int n, double dt, double* r, double* q, const double* v, const double* w,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, st, n, dt, r, q, v, w);
}

void launch_scale(int n, const double* semi, double scale, double* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale, dim3((2 * n + 255) / 256), dim3(256), 0, st, n, semi, scale,
                     out);
}

}  // namespace lub
