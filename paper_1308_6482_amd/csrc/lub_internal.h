// lub_internal.h -- device data layout and launch wrappers shared by the
// HIP sources of the gfx950 lubrication library.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lub.h"

namespace lub {

// Per-particle geometry record, 128 B (one cache line), in cell order.
// M = Q diag(Rperp^2, Rperp^2, Rpar^2) Q^T stored as xx xy xz yy yz zz; the
// support function of the particle is h(n) = sqrt(n.M n) and the support
// point in direction n is r + M n / h(n).
struct alignas(128) PRec {
  double r[3];
  double M[6];
  double ax[3];  // symmetry axis (body z) in the world frame
  double Rpar, Rperp, Rmax;
  double pad;
};

// Per-particle kinematics, 64 B, in cell order.
struct alignas(64) KRec {
  double v[3];
  double w[3];
  double pad[2];
};

// Device-side counters of one call.
struct Counters {
  int32_t work;          // evaluated pair slots (particle + wall)
  int32_t error;         // LUB_E* found on the device
  int32_t newton_max;
  int32_t pad0;
  int64_t candidates;
  int64_t wall_candidates;
  int64_t active;
  int64_t overlaps;
  int64_t unresolved;
  int64_t unconverged;
  int64_t fallbacks;
  int64_t newton_iters;
  int64_t total_entries;  // neighbour-list entries (both directions)
  int64_t iter_hist[32];
};

// Constant description of one call.
struct CallDesc {
  int32_t n;
  int32_t nc[3];         // cells per axis
  double cell[3];        // cell edge per axis
  double L[3];
  int32_t periodic[3];
  int32_t n_walls;
  double wall_vel[2][3];
  double rmax_bound;
  double dmax;           // largest cut-off
  double mu, delta_n, delta_t, delta_r, h_c, eps_c;
  int32_t max_iter;
  int32_t max_nbr;       // neighbour-segment stride (entries per particle)
  int32_t cap_entries;
  int32_t cap_work;
  int32_t precision;
};

// Pair output record: force on i, torque on i and torque on j about the
// particle centres.
template <typename R>
struct PairOut {
  R F[3], Ti[3], Tj[3];
};

// ---- launch wrappers (lub_neighbors.hip) --------------------------------
void launch_reset(Counters* c, int32_t* cell_count, int32_t* cell_fill,
                  int ncell, hipStream_t s);
void launch_stage_bin(const CallDesc& d, const double* r, const double* q,
                      const double* semi, int32_t* cell_id, int32_t* cell_count,
                      Counters* cnt, hipStream_t s);
void launch_scan(const int32_t* in, int32_t* out, int n, int32_t* block_sums,
                 int64_t* total, hipStream_t s);
void launch_cell_scatter(const CallDesc& d, const int32_t* cell_id,
                         const int32_t* cell_start, int32_t* cell_fill,
                         int32_t* sorted, hipStream_t s);
void launch_cell_sort(int ncell, const int32_t* cell_start, int32_t* sorted,
                      hipStream_t s);
void launch_build_records(const CallDesc& d, const int32_t* sorted,
                          const int32_t* cell_id, const double* r,
                          const double* q, const double* semi, const double* v,
                          const double* w, PRec* rec, KRec* kin,
                          int32_t* cell_sorted, hipStream_t s);
void launch_neighbors_wave(const CallDesc& d, const PRec* rec,
                           const int32_t* orig, const int32_t* cell_sorted,
                           const int32_t* cell_start, int32_t* deg,
                           int32_t* nbr, int32_t* slot, int32_t* wall_slot,
                           int32_t* work_s, int32_t* work_t, Counters* cnt,
                           hipStream_t s);

// ---- pair kernel (lub_pair.hip) -------------------------------------------
void launch_pairs(const CallDesc& d, const PRec* rec, const KRec* kin,
                  const int32_t* work_s, const int32_t* work_t, void* out,
                  double* out_h, int8_t* out_status, uint8_t* out_iters,
                  Counters* cnt, hipStream_t s);

// ---- per-particle reduction (lub_gather.hip) ------------------------------
void launch_gather(const CallDesc& d, const int32_t* orig, const int32_t* deg,
                   const int32_t* nbr, const int32_t* slot,
                   const int32_t* wall_slot, const void* out,
                   const Counters* cnt, double* f, double* t, hipStream_t s);

}  // namespace lub
