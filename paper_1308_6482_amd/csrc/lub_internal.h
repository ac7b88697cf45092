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

// The pair kernels' copy of the geometry, 64 B, in cell order: the full
// record is formed from it in registers (support_matrix gives the M of the
// staging), which halves the bytes a pair gathers.
struct alignas(64) PRecP {
  double r[3];
  double ax[3];
  double Rpar, Rperp;
};

// M = Rperp^2 I + (Rpar^2 - Rperp^2) a a^T as xx xy xz yy yz zz, in a fixed
// order without contraction: the staging and the pair kernels form the same
// bits.
__host__ __device__ inline void support_matrix(const double a[3], double Rpa, double Rpe,
                                               double M[6]) {
#pragma clang fp contract(off)
  const double p2 = Rpe * Rpe, dd = Rpa * Rpa - p2;
  M[0] = p2 + dd * a[0] * a[0];
  M[1] = dd * a[0] * a[1];
  M[2] = dd * a[0] * a[2];
  M[3] = p2 + dd * a[1] * a[1];
  M[4] = dd * a[1] * a[2];
  M[5] = p2 + dd * a[2] * a[2];
}

__host__ __device__ inline PRec expand_record(const PRecP& c) {
  PRec o;
  for (int k = 0; k < 3; ++k) {
    o.r[k] = c.r[k];
    o.ax[k] = c.ax[k];
  }
  o.Rpar = c.Rpar;
  o.Rperp = c.Rperp;
  o.Rmax = c.Rpar > c.Rperp ? c.Rpar : c.Rperp;
  o.pad = 0.0;
  support_matrix(o.ax, o.Rpar, o.Rperp, o.M);
  return o;
}

// Per-particle kinematics, 64 B, in cell order.
struct alignas(64) KRec {
  double v[3];
  double w[3];
  double pad[2];
};

// A particle's two cell-order copies, formed where its inputs are read in
// input order: one 128-B line, which the record build moves into cell order
// instead of gathering the five input arrays from random places.
struct alignas(128) RecStage {
  PRecP p;
  KRec k;
};

// Device-side counters of one call.
struct Counters {
  int32_t work;          // evaluated pair slots (particle + wall)
  int32_t error;         // LUB_E* found on the device
  int32_t newton_max;
  int32_t failed;        // slots whose Newton solve failed from every start
  int64_t candidates;
  int64_t wall_candidates;
  int64_t active;
  int64_t overlaps;
  int64_t unresolved;
  int64_t unconverged;
  int64_t fallbacks;
  int64_t newton_iters;
  int64_t total_entries;  // neighbour-list entries (both directions)
  int64_t warm_seeded;    // pairs started from the previous call's normal
  int64_t max_degree;     // largest number of candidates of one particle
  int64_t iter_hist[32];
  // reused neighbour lists: this call's decision (1: search)
  int32_t rebuild;
  int32_t pad_list;
};

// Reused neighbour lists, kept on the device across calls: the epoch of the
// lists in the superset buffers (-1: none) and the number of searches.
struct ListState {
  int32_t epoch;
  int32_t pad;
  int64_t builds;
  double le_offset;  // Lees-Edwards offset at the search
};

// The buffers of reused neighbour lists: the superset segments and their
// lengths (cell order of the search), each particle's position and R_max at
// the search and its place in the search's cell order (input order), one
// displacement maximum per block of the measuring kernel, and the state.
struct ListBufs {
  int32_t* sup_nbr;
  int32_t* sup_deg;
  double4* ref_pos;
  int32_t* inv;
  double* disp_blk;
  ListState* state;
  int32_t* work_sup;  // per evaluation slot: its superset entry (warm start)
  int2* warm_range;   // warm start: this call's slot range per input index
};

// Per-block partial statistics, written with plain stores and summed only
// when the host asks for the counters.
//   pair kernel rows (the main pass's blocks, then from row kMaxPairBlocks
//   the tangent-sphere pass's blocks; a pair is counted by the pass that
//   finished it): [0] Newton iterations, [1] active, [2] overlaps,
//   [3] unresolved, [4] unconverged, [5] fallbacks, [6] max iterations,
//   [7] warm-seeded pairs, [8..39] iteration histogram
//   neighbour kernel rows: [0] candidate pairs, [1] wall candidates,
//   [2] largest number of candidates of one particle
constexpr int kStatPairWords = 40;
constexpr int kStatNbrWords = 3;
constexpr int kMaxPairBlocks = 16384;  // larger slot counts: grid-stride loop
constexpr int kTangentBlocks = 8;      // grid of the tangent-sphere pass

// Constant description of one call.
struct CallDesc {
  int32_t n;
  int32_t nc[3];         // cells per axis
  double cell[3];        // cell edge per axis
  double L[3];
  double invL[3];       // 1 / L
  int32_t reach_max;    // cells searched on each side at most (cells are at
                        // least 1/reach_max of the largest pair bound)
  int32_t model;        // LUB_MODEL_*
  double r_small;       // size classes: R_max <= r_small is small (own cells)
  int32_t warm_ranges;  // warm start from the previous call's slot ranges
  int32_t periodic[3];
  int32_t n_walls;
  double wall_vel[2][3];
  double skin;           // reused neighbour lists: superset margin (0: off)
  int32_t list_epoch;    // lists searched under another epoch are not reused
  int32_t warm_slots;    // warm start stored per superset entry (reused lists)
  int32_t le;            // Lees-Edwards images (all axes periodic, no walls)
  double le_offset;      // x offset of the image one box up, in [0, L_x)
  double le_vel;         // x velocity of the image one box up
  double rmax_bound;
  double dmax;           // largest cut-off
  double mu, delta_n, delta_t, delta_r, h_c, eps_c;
  double q_bar;          // weight of the link-wise laws
  double ln_delta_t, ln_delta_r;  // log of the cut-offs (host-evaluated once)
  double inv_delta_n;             // 1 / Delta_n (host-evaluated once)
  int32_t max_iter;
  int32_t max_nbr;       // neighbour-segment stride (entries per particle)
  double newton_tol;     // relative tangential residual of the Newton solve
  int32_t cap_entries;
  int32_t cap_work;
  int32_t precision;
  int32_t partner_codes;  // kPartner*: how a particle's sum finds the
                          // results of the pairs its partners evaluate
};

// How the gather finds a pair's result from the particle that does not
// evaluate it.  With segments (both directions of every pair, sorted by
// partner): by a binary search of the partner's segment (small systems), or
// through the code -3 - slot written into its own entry by a kernel beside
// the pair pass (large systems).  After the forward search no segments are
// built (kPartnerRanges): each pair has a slot in the range of the particle
// that found it, and the other particle reads it through its backward list
// (finder, rank of the pair among the finder's kept pairs).
constexpr int kPartnerSearch = 0;
constexpr int kPartnerSide = 1;
constexpr int kPartnerRanges = 2;

// The forward search's entries carry two flags above the partner index
// (cell order): this entry's particle evaluates the pair (the smaller input
// index), and the support-function bound lets the pair through.
constexpr int32_t kOwnBit = 1 << 29;
constexpr int32_t kKeepBit = 1 << 30;
constexpr int32_t kIndexMask = kOwnBit - 1;

// Pair output record: force on i, torque on i and torque on j about the
// particle centres.
template <typename R>
struct PairOut {
  R F[3], Ti[3], Tj[3];
};

// ---- learned seed network: flat FP32 parameter layout ---------------------
// W1 (10 x 128, input-major), b1, W2 (128 x 128), b2, W3 (128 x 128), b3,
// W4 (128 x 4), b4
constexpr int kOffW1 = 0, kOffB1 = 1280, kOffW2 = 1408, kOffB2 = 17792;
constexpr int kOffW3 = 17920, kOffB3 = 34304, kOffW4 = 34432, kOffB4 = 34944;
constexpr int kNParams = 34948;
// packed BF16 copies: forward (output-major, padded) and backward
constexpr int kWt1 = 128 * 32, kWt2 = 128 * 128;
constexpr int kWtTotal = kWt1 + 2 * kWt2 + 16 * 128;
constexpr int kWbTotal = 2 * kWt2 + 128 * 32;

// ---- launch wrappers (lub_neighbors.hip) --------------------------------
void launch_reset(Counters* c, int32_t* cell_count, int ncell, hipStream_t s);
// The cell-build launchers take `gate`: null, or this call's counters, whose
// `rebuild` flag (set on the device) turns the kernels into no-ops when the
// neighbour lists are reused.  The binning writes each particle's cell, its
// ticket in the cell (a distinct place among the cell's members) and its
// staged record copies (input order), counts the cells, and zeroes `bcount`
// (2 n entries) when given.
void launch_stage_bin(const CallDesc& d, const double* r, const double* q,
                      const double* semi, const double* v, const double* w,
                      int32_t* cell_id, int32_t* ticket, RecStage* staged,
                      int32_t* cell_count, Counters* cnt, const Counters* gate,
                      hipStream_t s, int32_t* bcount = nullptr);
void launch_scan(const int32_t* in, int32_t* out, int n, int32_t* block_sums,
                 int64_t* total, hipStream_t s);
// scatter into the cells' ranges (at the binning's tickets), with the cell
// of each cell-order place into cell_sorted; zeroes cell_count
void launch_cell_scatter(const CallDesc& d, const int32_t* cell_id, const int32_t* ticket,
                         const int32_t* cell_start, int32_t* unsorted, int32_t* cell_sorted,
                         int32_t* cell_count, int ncell, const Counters* gate,
                         hipStream_t s);
// in-cell placement by input index and the records, from the staged copies
void launch_build_records(const CallDesc& d, const int32_t* unsorted,
                          const int32_t* cell_sorted, const int32_t* cell_start,
                          const RecStage* staged, int32_t* sorted, PRec* rec,
                          PRecP* recp, double4* pos, KRec* kin, const Counters* gate,
                          hipStream_t s);
// the whole cell build in one workgroup, when n and the grid are small enough
bool cells_small_fits(const CallDesc& d);
void launch_cells_small(const CallDesc& d, const double* r, const double* q,
                        const double* semi, const double* v, const double* w,
                        int32_t* cell_start, int32_t* sorted, PRec* rec, PRecP* recp,
                        double4* pos,
                        KRec* kin, int32_t* cell_sorted, Counters* cnt, const Counters* gate,
                        hipStream_t s);
void launch_neighbors_wave(const CallDesc& d, const PRec* rec, const PRecP* recp,
                           const double4* pos, const int32_t* orig, const int32_t* cell_sorted,
                           const int32_t* cell_start, int32_t* deg,
                           int32_t* nbr, int32_t* slot, int32_t* wall_slot,
                           int32_t* work_s, int32_t* work_t, int64_t* stat_nbr,
                           Counters* cnt, hipStream_t s, int mode = 0,
                           const ListBufs* lists = nullptr, int32_t* bcount = nullptr,
                           int32_t* block_sums = nullptr, int2* bstage = nullptr,
                           hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// whether the full search runs as forward search + evaluation list (then
// the 128-B records are not read by the search)
bool nbr_forward(const CallDesc& d, const int32_t* bcount, const int32_t* block_sums,
                 const int2* bstage);
// (bcount: 2 n + 2 ints, the first 2 n zeroed by the binning of this call,
// block_sums, scan scratch for n entries, and bstage, one int2 per segment
// entry; given, the full search of large systems runs as a forward search, a
// scan of the kept counts and the evaluation list, and leaves the layout
// kPartnerRanges: deg and the slot rows hold each particle's forward list
// (partners with the flags), bcount[n ..] the slot offsets, and the first n
// words of bcount the number of its partners' kept pairs, whose slot codes
// (slot, or -1 - slot where the partner evaluates) its nbr row holds in
// increasing finder index; the events, when given, take
// the search kernel's own start and end stamps: the full search, the
// forward walk or the filter of reused lists)
// reused neighbour lists: the displacement plus growth since the search
// (skipped unless the lists are of this epoch), then the decision (a
// search if the lists are of another epoch or the measure exceeds half the
// skin), and the records of the current inputs in the search's cell order
// (a no-op when searching)
void launch_disp(const CallDesc& d, const double* r, const double* q, const double* semi,
                 const ListBufs& lists, Counters* cnt, hipStream_t s);
void launch_refresh(const CallDesc& d, const double* r, const double* q, const double* semi,
                    const double* v, const double* w, const ListBufs& lists, PRec* rec,
                    PRecP* recp,
                    double4* pos, KRec* kin, const Counters* cnt, hipStream_t s);

// ---- pair kernel (lub_pair.hip) -------------------------------------------
// seedY: network outputs per slot (p_i, q_i, p_j, q_j) or null for the
// line-of-centres start
// Warm start: the search assigns evaluation slots particle by particle (to
// the particle that evaluates a pair, or, in the forward search, to the one
// that found it), so every particle's slots are one contiguous range.  Each
// call records, per input index, that range, and per slot the converged
// normal with the xor of the pair's input indices; the next call finds a
// pair's previous normal by scanning the previous ranges of its two
// particles (a few consecutive slots each).  Two sets, swapped between
// calls.
constexpr int kWarmScan = 520;  // longest range scanned (segment + 2 walls)
struct WarmTables {
  const int2* prev_range;    // read: [first, end) slot of each input index
  const float4* prev_val;    // read: (normal, xor of the pair's input indices)
  float4* cur_val;           // written: this call's values per slot
  const int32_t* orig;       // cell order -> input index
  // with reused lists (CallDesc::warm_slots): the last normal of each
  // superset entry, tagged with the search that made the superset
  const int32_t* slot_sup;   // evaluation slot -> superset entry
  float4* sup_val;           // normal (x, y, z), tag in w (int bits)
  const ListState* state;    // the current search count (the tag)
  const int2* cur_range;     // read: this call's [first, end) slot of each input index
};

// detail (may be null): kDetailWords doubles per evaluation slot, the
// unit gap direction n, y_i - r_i, y_j - r_j, the frame axis x1 of surface i
// and the 16 corrective elements K~ (order 11 12 13 14 15 22 23 24 25 33 34
// 35 36 44 45 55, without the viscosity)
constexpr int kDetailWords = 28;
void launch_pairs(const CallDesc& d, const PRecP* recp, const KRec* kin,
                  const int32_t* work_s, const int32_t* work_t, const float* seedY,
                  void* out, double* out_h, int8_t* out_status, uint8_t* out_iters,
                  WarmTables warm, int32_t* fail_list, int64_t* stat_pair,
                  Counters* cnt, hipStream_t s, hipEvent_t ev_start = nullptr,
                  hipEvent_t ev_stop = nullptr, double* detail = nullptr);

// seed features of every particle-particle evaluation slot (m x 10, FP32)
void launch_seed_features(const CallDesc& d, const PRec* rec,
                          const int32_t* work_s, const int32_t* work_t,
                          float* X, Counters* cnt, hipStream_t s);

// ---- learned seed network (lub_mlp.hip) -----------------------------------
void mlp_pack(const float* th, __bf16* wt, __bf16* wb, hipStream_t s);
void mlp_forward(int64_t m, const float* X, float* Y, const __bf16* wt,
                 const float* th, hipStream_t s);
int mlp_train_step(int64_t m, int64_t off, int B, const float* X, const float* T,
                   const __bf16* wt, const __bf16* wb, float* th, __bf16* aT,
                   __bf16* dT, float* grad, float* m1, float* m2, float* loss_parts,
                   float lr, float beta1, float beta2, float eps, int step,
                   float* loss_out, bool update, hipStream_t s);
// network output for the evaluation slots of the last lub_compute: the
// forward pass over the seed features, sized by the device work count
void mlp_forward_slots(const Counters* cnt, int cap, const float* X, float* Y,
                       const __bf16* wt, const float* th, hipStream_t s);

// per-particle sums; also zeroes `next_cnt`, the counters of the next call
// the partner's slot code in every non-owned entry of an evaluated pair
void launch_partner_slots(const CallDesc& d, const int32_t* work_s, const int32_t* work_t,
                          const int32_t* deg, const int32_t* nbr, int32_t* slot,
                          const Counters* cnt, hipStream_t s);
// (bcount, work_s: read in the layout kPartnerRanges, with the nbr rows,
// where deg, slot and wall_slot are not)
void launch_gather(const CallDesc& d, const int32_t* orig, const int32_t* deg,
                   const int32_t* nbr, const int32_t* slot,
                   const int32_t* wall_slot, const void* out,
                   const Counters* cnt, Counters* next_cnt, double* f, double* t,
                   hipStream_t s, const int32_t* bcount = nullptr,
                   const int32_t* work_s = nullptr);

// ---- link-wise laws (lub_link.hip) ------------------------------------------
int link_grid(const CallDesc& d);
void launch_links(const CallDesc& d, const PRec* rec, const KRec* kin, const int32_t* work_s,
                  const int32_t* work_t, void* out, double* out_h, int8_t* out_status,
                  int32_t* out_links, int64_t* stat_pair, Counters* cnt, hipStream_t s);

// ---- integrator (lub_integrate.hip) ---------------------------------------
struct StepDesc {
  int32_t n;
  int32_t periodic[3];
  int32_t le;           // Lees-Edwards images
  double L[3];
  double le_offset;     // offset after this sub-step, in [0, L_x)
  double le_vel;
  double dt, density, damping;
};
void launch_integrate(const StepDesc& s, double* r, double* q, const double* semi,
                      double* v, double* w, const double* f_ext, const double* t_ext,
                      const double* f, const double* t, hipStream_t st);
// out = scale * semi (n x 2)
void launch_scale(int n, const double* semi, double scale, double* out, hipStream_t st);
// r <- r + dt v, q <- normalise(q + dt/2 (0, w) q)
void launch_advance(int n, double dt, double* r, double* q, const double* v, const double* w,
                    hipStream_t st);

// grid of the pair kernel for a given slot capacity
int pair_grid(const CallDesc& d);
// neighbour kernel: lanes per particle, blocks of a call, and the most
// blocks n particles can need
int nbr_group(const CallDesc& d);
int nbr_blocks(const CallDesc& d);
int nbr_blocks_max(int n);
// sum the per-block partial statistics of the last call into `cnt`
void launch_stats_reduce(const CallDesc& d, Counters* cnt, const int64_t* stat_pair,
                         const int64_t* stat_nbr, hipStream_t s);

#ifdef __HIPCC__
// LDS written by lanes of this wavefront is visible to its other lanes
// after this point (no workgroup barrier: that would also wait for every
// global load in flight)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Minimum-image displacement along a periodic axis, dx - L rint(dx / L),
// with the quotient taken as dx (1/L): the two round to different integers
// only next to a half-integer, and there the division itself decides.
// No contraction, so the result equals the plain expression bit for bit.
__device__ __forceinline__ double image_count(double dx, double L, double invL) {
#pragma clang fp contract(off)
  const double x = dx * invL;
  double k = rint(x);
  if (fabs(fabs(x - k) - 0.5) < 1e-9) k = rint(dx / L);
  return k;
}

__device__ __forceinline__ double min_image(double dx, double L, double invL) {
#pragma clang fp contract(off)
  return dx - L * image_count(dx, L, invL);
}

// Offset from centre ri to the nearest image of centre rj.  With
// Lees-Edwards images the z image is taken first: m boxes down in z moves
// the image by -m le_offset in x (and its velocity by -m le_velocity); x and
// y are then wrapped as usual.  Returns m (0 without Lees-Edwards images).
// Fixed order, no contraction: equal to the plain expressions bit for bit.
__device__ __forceinline__ int pair_image(const CallDesc& d, const double* ri,
                                          const double* rj, double* out) {
#pragma clang fp contract(off)
  double dx = rj[0] - ri[0];
  double dy = rj[1] - ri[1];
  double dz = rj[2] - ri[2];
  int m = 0;
  if (d.le) {
    const double c = image_count(dz, d.L[2], d.invL[2]);
    m = (int)c;
    dz = dz - d.L[2] * c;
    const double shift = c * d.le_offset;
    dx = dx - shift;
  } else if (d.periodic[2]) {
    dz = min_image(dz, d.L[2], d.invL[2]);
  }
  if (d.periodic[0]) dx = min_image(dx, d.L[0], d.invL[0]);
  if (d.periodic[1]) dy = min_image(dy, d.L[1], d.invL[1]);
  out[0] = dx;
  out[1] = dy;
  out[2] = dz;
  return m;
}
#endif

}  // namespace lub
