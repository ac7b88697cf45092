// Link-wise lubrication laws (Sec. II.D): the correction of Ding and Aidun,
// Eq. methods:dlub, summed over the lattice links that connect two
// particles, and Clausen's variant along the averaged surface normal.
//
// The lattice sites are the integer points; a site belongs to a particle
// when it lies inside or on its surface.  For a candidate pair (i, j) every
// D3Q19 link c ending on a site x_b of i (not of j) counts when it starts
// on a site of j, or on a fluid site x_b - c halfway along two links from
// the site x_b - 2c of j; each undirected link once.  Along the link the
// gap h* runs from where it leaves the surface of i to where it enters the
// surface of j; links with h* < |c| carry
//   f = -3 q_bar mu / (2 |c|^2 lambda*) (e . (V_i - V_j)) (1/h_eff^2 - 1/|c|^2)
// along e (the link direction from j to i; in the averaged-normal variant
// the normalised difference of the two outward normals, with the gap
// projected on it), h_eff = max(gap, h_c), lambda* the mean of the two
// surfaces' mean curvatures at the crossing points, V the rigid-body
// surface velocities there, plus the repulsion of Eq. lub:frep below h_c.
// The force acts on i at its crossing point and the opposite force on j at
// its crossing point.
//
// One wavefront per pair over the box where sites of i can be linked to
// sites of j (the bounding box of i cut to that of j widened by three
// lattice units, more than the two-link reach 2 sqrt 2), 64 sites at a time:
// each lane tests a site, the sites of i within the reach of j are
// compacted, and their (site, direction) items are spread over the lanes.
// Per-lane sums are combined by a fixed butterfly.  FP64 throughout.
#include <hip/hip_runtime.h>

#include "lub_internal.h"

namespace lub {
namespace {

constexpr int kLinkWaves = 8;              // wavefronts per block
constexpr int kLinkSlots = 64;             // slots per block (one stats row)

__device__ __forceinline__ double dot3d(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3d(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// value of the spheroid's quadratic form at x (relative to the centre):
// (|x|^2 - (a.x)^2) / R_perp^2 + (a.x)^2 / R_par^2
__device__ __forceinline__ double quad_form(const PRec& P, const double x[3]) {
  const double ax = dot3d(P.ax, x);
  return (dot3d(x, x) - ax * ax) / (P.Rperp * P.Rperp) + ax * ax / (P.Rpar * P.Rpar);
}

__device__ __forceinline__ bool site_in(const PRec& P, const double c[3], const double x[3]) {
  const double y[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  return quad_form(P, y) <= 1.0;
}

// parameters s_lo <= s_hi where the line x - s u (u unit) crosses the
// surface of P centred at c
__device__ __forceinline__ bool line_roots(const PRec& P, const double c[3], const double x[3],
                                           const double u[3], double* s_lo, double* s_hi) {
  const double y[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  const double ip = 1.0 / (P.Rperp * P.Rperp), ia = 1.0 / (P.Rpar * P.Rpar);
  const double ay = dot3d(P.ax, y), au = dot3d(P.ax, u);
  const double A = (1.0 - au * au) * ip + au * au * ia;
  const double B = (dot3d(y, u) - ay * au) * ip + ay * au * ia;
  const double C = (dot3d(y, y) - ay * ay) * ip + ay * ay * ia - 1.0;
  const double disc = B * B - A * C;
  if (!(disc >= 0.0) || !(A > 0.0)) return false;
  const double sq = sqrt(disc);
  *s_lo = (B - sq) / A;
  *s_hi = (B + sq) / A;
  return true;
}

// mean curvature (1/S1 + 1/S2) / 2 at the surface point y (relative to the
// centre), with the principal radii of Eq. lub:curvature-radii at the
// parametric latitude of y
__device__ __forceinline__ double mean_curvature(const PRec& P, const double y[3]) {
  const double ay = dot3d(P.ax, y);
  double sp = ay / P.Rpar;
  double cp = sqrt(fmax(dot3d(y, y) - ay * ay, 0.0)) / P.Rperp;
  const double l = sqrt(sp * sp + cp * cp);
  sp /= l;
  cp /= l;
  const double s1 = sqrt(P.Rperp * P.Rperp * sp * sp + P.Rpar * P.Rpar * cp * cp);
  const double S1 = s1 * s1 * s1 / (P.Rpar * P.Rperp);
  const double S2 = P.Rperp * s1 / P.Rpar;
  return 0.5 * (1.0 / S1 + 1.0 / S2);
}

// outward unit normal at the surface point y (relative to the centre)
__device__ __forceinline__ void outward_normal(const PRec& P, const double y[3], double n[3]) {
  const double ay = dot3d(P.ax, y);
  const double ip = 1.0 / (P.Rperp * P.Rperp), ia = 1.0 / (P.Rpar * P.Rpar);
  for (int k = 0; k < 3; ++k) n[k] = (y[k] - ay * P.ax[k]) * ip + ay * P.ax[k] * ia;
  const double l = sqrt(dot3d(n, n));
  for (int k = 0; k < 3; ++k) n[k] /= l;
}

// the 18 non-zero velocities of the D3Q19 lattice
__constant__ int kD3Q19[18][3] = {
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
    {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

__global__ void __launch_bounds__(64 * kLinkWaves)
    k_links(CallDesc cd, const PRec* __restrict__ rec, const KRec* __restrict__ kin,
            const int32_t* __restrict__ work_s, const int32_t* __restrict__ work_t,
            PairOut<double>* __restrict__ out, double* __restrict__ out_h,
            int8_t* __restrict__ out_status, int32_t* __restrict__ out_links,
            int64_t* __restrict__ stat_pair, const Counters* cnt) {
#pragma clang fp contract(off)
  __shared__ int64_t s_stat[kLinkWaves][4];
  __shared__ int32_t s_list[kLinkWaves][64];   // per wavefront: the kept sites
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nwork = cnt->error == 0 ? min(cnt->work, cd.cap_work) : 0;
  if ((int)(blockIdx.x * kLinkSlots) >= nwork) return;
  const bool navg = cd.model == LUB_MODEL_LINK_NAVG;
  int64_t n_links = 0, n_active = 0, n_overlap = 0, max_links = 0;
  for (int c0 = blockIdx.x * kLinkSlots; c0 < nwork; c0 += gridDim.x * kLinkSlots) {
    for (int w = c0 + wv; w < min(c0 + kLinkSlots, nwork); w += kLinkWaves) {
      const int s = work_s[w], t = work_t[w];
      const PRec& A = rec[s];
      double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      int links = 0;
      double hmin = 1e300;
      if (t >= 0) {
        const PRec& B = rec[t];
        const KRec& KA = kin[s];
        const KRec& KB = kin[t];
        double d[3];
        pair_image(cd, A.r, B.r, d);
        const double ri[3] = {A.r[0], A.r[1], A.r[2]};
        const double rj[3] = {ri[0] + d[0], ri[1] + d[1], ri[2] + d[2]};
        int lo[3], n3[3];
        for (int k = 0; k < 3; ++k) {
          const double ei = sqrt(A.M[k == 0 ? 0 : (k == 1 ? 3 : 5)]);
          const double ej = sqrt(B.M[k == 0 ? 0 : (k == 1 ? 3 : 5)]);
          const int l0 = max((int)floor(ri[k] - ei), (int)floor(rj[k] - ej) - 3);
          const int h0 = min((int)ceil(ri[k] + ei), (int)ceil(rj[k] + ej) + 3);
          lo[k] = l0;
          n3[k] = max(0, h0 - l0 + 1);
        }
        const int nsites = n3[0] * n3[1] * n3[2];
        // a site farther than the two-link reach 2 sqrt 2 from j carries no
        // link: the body scaled by s = sqrt(q_j) lies at least
        // (s - 1) min(R_par, R_perp) outside it
        const double reach = (2.0 * sqrt(2.0)) * (1.0 + 1e-9) + 1e-9;
        const double rminB = fmin(B.Rpar, B.Rperp);
        for (int base = 0; base < nsites; base += 64) {
          // phase 1: each lane tests one site; the sites of i within the
          // two-link reach of j are compacted into the wavefront's list
          const int idx = base + lane;
          bool keep = false;
          if (idx < nsites) {
            const double xb[3] = {(double)(lo[0] + idx % n3[0]),
                                  (double)(lo[1] + (idx / n3[0]) % n3[1]),
                                  (double)(lo[2] + idx / (n3[0] * n3[1]))};
            if (site_in(A, ri, xb)) {
              const double yj[3] = {xb[0] - rj[0], xb[1] - rj[1], xb[2] - rj[2]};
              const double qj = quad_form(B, yj);
              keep = qj > 1.0 && !((sqrt(qj) - 1.0) * rminB > reach);
            }
          }
          const unsigned long long m = __ballot(keep);
          if (keep) s_list[wv][__popcll(m & ((1ull << lane) - 1ull))] = idx;
          __builtin_amdgcn_wave_barrier();
          const int nk = __popcll(m);
          // phase 2: the (site, direction) items spread over the lanes
          for (int it = lane; it < 18 * nk; it += 64) {
            const int sidx = s_list[wv][it / 18];
            const int r = it % 18;
            const double xb[3] = {(double)(lo[0] + sidx % n3[0]),
                                  (double)(lo[1] + (sidx / n3[0]) % n3[1]),
                                  (double)(lo[2] + sidx / (n3[0] * n3[1]))};
            const int c[3] = {kD3Q19[r][0], kD3Q19[r][1], kD3Q19[r][2]};
            const double cl = sqrt((double)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
            const double x1[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
            if (site_in(A, ri, x1)) continue;
            if (!site_in(B, rj, x1)) {
              const double x2[3] = {xb[0] - 2 * c[0], xb[1] - 2 * c[1], xb[2] - 2 * c[2]};
              if (!site_in(B, rj, x2) || site_in(A, ri, x2)) continue;
            }
            const double u[3] = {c[0] / cl, c[1] / cl, c[2] / cl};
            double a0, a1, b0, b1;
            if (!line_roots(A, ri, xb, u, &a0, &a1) || !line_roots(B, rj, xb, u, &b0, &b1))
              continue;
            const double hs = b0 - a1;
            if (!(hs < cl)) continue;
            ++links;
            hmin = fmin(hmin, hs);
            double ai[3], aj[3], Vi[3], Vj[3], tmp[3];
            for (int k = 0; k < 3; ++k) {
              ai[k] = xb[k] - a1 * u[k] - ri[k];
              aj[k] = xb[k] - b0 * u[k] - rj[k];
            }
            cross3d(KA.w, ai, tmp);
            for (int k = 0; k < 3; ++k) Vi[k] = KA.v[k] + tmp[k];
            cross3d(KB.w, aj, tmp);
            for (int k = 0; k < 3; ++k) Vj[k] = KB.v[k] + tmp[k];
            const double lam = 0.5 * (mean_curvature(A, ai) + mean_curvature(B, aj));
            double dir[3], gap;
            if (navg) {
              double ni[3], nj[3];
              outward_normal(A, ai, ni);
              outward_normal(B, aj, nj);
              for (int k = 0; k < 3; ++k) dir[k] = nj[k] - ni[k];
              const double l = sqrt(dot3d(dir, dir));
              for (int k = 0; k < 3; ++k) dir[k] /= l;
              gap = hs * dot3d(u, dir);
            } else {
              for (int k = 0; k < 3; ++k) dir[k] = u[k];
              gap = hs;
            }
            const double heff = gap > cd.h_c ? gap : cd.h_c;
            const double dvn = dot3d(dir, Vi) - dot3d(dir, Vj);
            double f = 0.0;
            if (heff > 0.0)
              f = -3.0 * cd.q_bar * cd.mu / (2.0 * cl * cl * lam) * dvn *
                  (1.0 / (heff * heff) - 1.0 / (cl * cl));
            if (gap <= cd.h_c) f += gap > 0.0 ? cd.eps_c * (cd.h_c - gap) : cd.eps_c * cd.h_c;
            const double Fl[3] = {f * dir[0], f * dir[1], f * dir[2]};
            for (int k = 0; k < 3; ++k) acc[k] += Fl[k];
            cross3d(ai, Fl, tmp);
            for (int k = 0; k < 3; ++k) acc[3 + k] += tmp[k];
            cross3d(aj, Fl, tmp);
            for (int k = 0; k < 3; ++k) acc[6 + k] -= tmp[k];
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
      // fixed butterfly over the wavefront
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        for (int k = 0; k < 9; ++k) acc[k] += __shfl_xor(acc[k], o, 64);
        links += __shfl_xor(links, o, 64);
        hmin = fmin(hmin, __shfl_xor(hmin, o, 64));
      }
      if (lane == 0) {
        PairOut<double> po;
        for (int k = 0; k < 3; ++k) {
          po.F[k] = acc[k];
          po.Ti[k] = acc[3 + k];
          po.Tj[k] = acc[6 + k];
        }
        out[w] = po;
        out_h[w] = links ? hmin : 0.0;
        out_status[w] = links ? 0 : 1;
        out_links[w] = links;
      }
      n_links += links;
      n_active += links > 0;
      n_overlap += links > 0 && hmin <= 0.0;
      max_links = max(max_links, (int64_t)links);
    }
  }
  // one statistics row per block (the pair kernel's layout: [0] links,
  // [1] active pairs, [2] pairs with a link gap <= 0, [6] most links of a
  // pair; the other words zero)
  if (lane == 0) {
    s_stat[wv][0] = n_links;
    s_stat[wv][1] = n_active;
    s_stat[wv][2] = n_overlap;
    s_stat[wv][3] = max_links;
  }
  __syncthreads();
  if (threadIdx.x < kStatPairWords) {
    int64_t v = 0;
    const int word = threadIdx.x;
    for (int k = 0; k < kLinkWaves; ++k) {
      if (word == 0) v += s_stat[k][0];
      if (word == 1) v += s_stat[k][1];
      if (word == 2) v += s_stat[k][2];
      if (word == 6) v = max(v, s_stat[k][3]);
    }
    stat_pair[(int64_t)kStatPairWords * blockIdx.x + word] = v;
  }
}

}  // namespace

int link_grid(const CallDesc& d) {
  int blocks = (d.cap_work + kLinkSlots - 1) / kLinkSlots;
  if (blocks > kMaxPairBlocks) blocks = kMaxPairBlocks;
  return blocks < 1 ? 1 : blocks;
}

void launch_links(const CallDesc& d, const PRec* rec, const KRec* kin, const int32_t* work_s,
                  const int32_t* work_t, void* out, double* out_h, int8_t* out_status,
                  int32_t* out_links, int64_t* stat_pair, Counters* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_links, dim3(link_grid(d)), dim3(64 * kLinkWaves), 0, s, d, rec, kin,
                     work_s, work_t, (PairOut<double>*)out, out_h, out_status, out_links,
                     stat_pair, cnt);
}

}  // namespace lub
