// lub_neighbors.hip -- staging, cell list and neighbour lists (gfx950).
//
// Candidate pairs follow the pruning of Sec. III.A of the paper: a pair is a
// candidate when its minimum-image centre distance is below
// R_max,i + R_max,j + (largest cut-off).  That test is evaluated in IEEE
// double with FP contraction switched off so that it is reproducible bit for
// bit.  A second, exact reject (a lower bound of the gap from the support
// functions along the line of centres) removes candidates that can never be
// lubrication-active before the closest-point solve.
//
// Layout: particles are binned into a uniform grid (cell edge >= 2 R_max +
// largest cut-off) with a counting sort; every per-particle record is stored
// in cell order so that neighbour loads of a wavefront hit few cache lines.
// The neighbour list holds both directions of every pair, one fixed-stride
// segment per particle (cell-order indices), each segment sorted by partner
// index; the pair (i, j) is evaluated once, from the entry whose owner has
// the smaller input index.
//
// Reused lists (a skin): a search keeps every pair within the bound + skin;
// later calls measure how far the particles moved and grew since, decide on
// the device whether to search again, and otherwise refresh the records in
// the old cell order and filter the kept pairs with the exact centre test.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lub_internal.h"

namespace lub {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 8;                             // per thread and chunk
constexpr int kScanChunk = kScanThreads * kScanItems;     // staged through LDS
constexpr int kScanTile = kScanChunk;                     // one block per tile

// A coordinate wrapped into the box along a periodic axis.  The binning and
// the neighbour search take the same expression, so that a centre's cell
// and its place in that cell agree.
__device__ __forceinline__ double wrap_coord(double x, double L, double invL) {
  return x - L * floor(x * invL);
}

// Cell along one axis (inv_edge = 1 / cell edge; the grid's margin is far
// above the rounding of the product).
__device__ __forceinline__ int cell_coord(double x, double L, double invL, int periodic,
                                          double inv_edge, int nc) {
  if (periodic) x = wrap_coord(x, L, invL);
  int c = (int)floor(x * inv_edge);
  c = c < 0 ? 0 : c;
  c = c >= nc ? nc - 1 : c;
  return c;
}

__device__ __forceinline__ void set_error(Counters* cnt, int code) {
  atomicCAS(&cnt->error, 0, code);
}

// Exact centre test: minimum-image squared distance below the squared
// pruning bound, evaluated in a fixed order without contraction.
// `extra` widens the bound (the skin of a reused list); with extra = 0 the
// bound is (rmi + rmj) + dmax exactly.
__device__ __forceinline__ bool centre_test(const double* ri, const double* rj,
                                            double rmi, double rmj,
                                            const CallDesc& d, double extra) {
#pragma clang fp contract(off)
  double o[3];
  pair_image(d, ri, rj, o);
  const double dx = o[0], dy = o[1], dz = o[2];
  double d2 = dx * dx + dy * dy;
  d2 = d2 + dz * dz;
  double sb = (rmi + rmj) + (d.dmax + extra);
  return d2 < sb * sb;
}

// Inclusive scan of one int per thread across a block of up to 1024 threads.
__device__ int block_inclusive_scan(int x, int* lds, int* total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63 || threadIdx.x == blockDim.x - 1) lds[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int v = lane < nw ? lds[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(v, o, 64);
      if (lane >= o) v += y;
    }
    if (lane < nw) lds[lane] = v;
  }
  __syncthreads();
  int res = x + (wid > 0 ? lds[wid - 1] : 0);
  *total = lds[nw - 1];
  __syncthreads();
  return res;
}

__global__ void k_reset(Counters* c, int32_t* cell_count, int ncell) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncell) cell_count[i] = 0;
  if (i < (int)(sizeof(Counters) / sizeof(int32_t)))
    reinterpret_cast<int32_t*>(c)[i] = 0;
}

// One particle's input, loaded at once.
struct PIn {
  double x, y, z, qw, qx, qy, qz, a, b;
};

__device__ __forceinline__ PIn load_input(const double* __restrict__ r,
                                          const double* __restrict__ q,
                                          const double* __restrict__ semi, int p) {
  return PIn{r[3 * p],     r[3 * p + 1], r[3 * p + 2], q[4 * p],        q[4 * p + 1],
             q[4 * p + 2], q[4 * p + 3], semi[2 * p],  semi[2 * p + 1]};
}

// checks of one particle's input: bit 0 an invalid value (EINVAL), bit 1 a
// centre beyond a wall by more than the particle's size (EDOMAIN)
__device__ __forceinline__ int input_faults(const CallDesc& d, const PIn& u) {
  bool ok = isfinite(u.x) && isfinite(u.y) && isfinite(u.z) && isfinite(u.qw) &&
            isfinite(u.qx) && isfinite(u.qy) && isfinite(u.qz) && u.a > 0.0 && u.b > 0.0 &&
            isfinite(u.a) && isfinite(u.b);
  double qn = sqrt(u.qw * u.qw + u.qx * u.qx + u.qy * u.qy + u.qz * u.qz);
  ok = ok && fabs(qn - 1.0) <= 1e-6 && fmax(u.a, u.b) <= d.rmax_bound;
  ok = ok && (d.model != LUB_MODEL_LADD || u.a == u.b);  // Ladd's law is for spheres
  double rm = fmax(u.a, u.b);
  const bool wall = d.n_walls && (u.z < -rm || u.z > d.L[2] + rm);
  return (ok ? 0 : 1) | (wall ? 2 : 0);
}

__device__ __forceinline__ int input_faults(const CallDesc& d, const double* __restrict__ r,
                                            const double* __restrict__ q,
                                            const double* __restrict__ semi, int p) {
  return input_faults(d, load_input(r, q, semi, p));
}

// validate one particle's input (EINVAL, EDOMAIN) and return its cell
// (inv_cell: 1 / cell edge per axis)
__device__ int validate_bin(const CallDesc& d, const PIn& u, const double inv_cell[3],
                            Counters* cnt) {
  const int faults = input_faults(d, u);
  const bool ok = !(faults & 1);
  if (!ok) set_error(cnt, LUB_EINVAL);
  double rm = fmax(u.a, u.b);
  if (faults & 2) set_error(cnt, LUB_EDOMAIN);
  int cx = cell_coord(u.x, d.L[0], d.invL[0], d.periodic[0], inv_cell[0], d.nc[0]);
  int cy = cell_coord(u.y, d.L[1], d.invL[1], d.periodic[1], inv_cell[1], d.nc[1]);
  int cz = cell_coord(u.z, d.L[2], d.invL[2], d.periodic[2], inv_cell[2], d.nc[2]);
  if (!ok) cx = cy = cz = 0;
  // the large particles' cells follow the small particles' cells
  const int big = rm > d.r_small ? d.nc[0] * d.nc[1] * d.nc[2] : 0;
  return (cz * d.nc[1] + cy) * d.nc[0] + cx + big;
}

// Exclusive scan of in[0, n) into out[0, n) (the two may be the same
// array) by one block of kScanThreads, chunk by chunk: coalesced loads into
// LDS, kScanItems consecutive elements per thread, block scan, coalesced
// stores.  Returns the total to every thread.
__device__ int block_scan_range(const int32_t* in, int32_t* out, int n, int* chunk,
                                int* lds_scan) {
  int carry = 0;
  for (int c0 = 0; c0 < n; c0 += kScanChunk) {
    const int m = min(kScanChunk, n - c0);
    for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads)
      chunk[k] = k < m ? in[c0 + k] : 0;
    __syncthreads();
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = chunk[threadIdx.x * kScanItems + k];
      sum += v[k];
    }
    int tot;
    const int incl = block_inclusive_scan(sum, lds_scan, &tot);
    int run = carry + incl - sum;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      chunk[threadIdx.x * kScanItems + k] = run;
      run += v[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += kScanThreads) out[c0 + k] = chunk[k];
    carry += tot;
    __syncthreads();  // the next chunk reuses the LDS
  }
  return carry;
}

// exclusive scan, tile level; the single-tile case writes the total directly
__global__ void __launch_bounds__(kScanThreads)
k_scan_tile(const int32_t* __restrict__ in, int32_t* __restrict__ out, int n,
            int32_t* __restrict__ block_sums, int64_t* total) {
  __shared__ int chunk[kScanChunk];
  __shared__ int lds[16];
  const int base = blockIdx.x * kScanTile;
  const int m = min(kScanTile, n - base);
  const int tot = block_scan_range(in + base, out + base, m, chunk, lds);
  if (threadIdx.x == 0) {
    block_sums[blockIdx.x] = tot;
    if (gridDim.x == 1) {
      out[n] = tot;
      if (total) *total = tot;
    }
  }
}

// Each tile plus the sum of the tile totals before it: every block sums
// those totals itself (a few hundred, from L2) instead of waiting for a
// separate scan of them; the last block, which sums them all, writes the
// grand total.
constexpr int kAddThreads = 256;

__global__ void __launch_bounds__(kAddThreads)
k_scan_add(int32_t* out, int n, const int32_t* block_sums, int nb, int64_t* total) {
  __shared__ int lds[kAddThreads / 64];
  const int b = blockIdx.x;
  const bool last = b == nb - 1;
  int part = 0;
  for (int k = threadIdx.x; k < (last ? nb : b); k += kAddThreads) part += block_sums[k];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = part;
  __syncthreads();
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kAddThreads / 64; ++k) sum += lds[k];
  const int add = last ? sum - block_sums[b] : sum;
  if (last && threadIdx.x == 0) {
    out[n] = sum;
    if (total) *total = sum;
  }
  const int base = b * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kAddThreads) {
    const int idx = base + k;
    if (idx < n) out[idx] += add;
  }
}

// Particles into their cells' ranges in arbitrary order (the binning's
// tickets), with the cell of each place of the range (every place of a
// cell's range holds one of its particles, whatever the order: the cell of
// each cell-order place).  The counts have been consumed by the scan: they
// are zeroed here for the next call.
__global__ void k_cell_scatter(CallDesc d, const int32_t* __restrict__ cell_id,
                               const int32_t* __restrict__ ticket,
                               const int32_t* __restrict__ cell_start,
                               int32_t* __restrict__ unsorted,
                               int32_t* __restrict__ cell_sorted,
                               int32_t* __restrict__ cell_count, int ncell,
                               const Counters* gate) {
  if (gate && !gate->rebuild) return;  // reused lists: the counts stayed zero
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int c = i; c < ncell; c += gridDim.x * blockDim.x) cell_count[c] = 0;
  if (i >= d.n) return;
  const int c = cell_id[i];
  const int at = cell_start[c] + ticket[i];
  unsorted[at] = i;
  cell_sorted[at] = c;
}

// One particle's inputs for its records, loaded at once.
struct RecIn {
  PIn u;
  double v[3], w[3];
};

__device__ __forceinline__ RecIn load_record_input(const double* __restrict__ r,
                                                   const double* __restrict__ q,
                                                   const double* __restrict__ semi,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ w, int p) {
  RecIn in;
  in.u = load_input(r, q, semi, p);
  for (int k = 0; k < 3; ++k) {
    in.v[k] = v[3 * p + k];
    in.w[k] = w[3 * p + k];
  }
  return in;
}

// One particle's 64-B geometry copy and kinematics from its inputs: the
// symmetry axis a is the third column of the rotation of the normalised q.
__device__ __forceinline__ RecStage stage_record(const RecIn& in) {
  double qw = in.u.qw, qx = in.u.qx, qy = in.u.qy, qz = in.u.qz;
  double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= inv;
  qx *= inv;
  qy *= inv;
  qz *= inv;
  double ax = 2.0 * (qx * qz + qw * qy);
  double ay = 2.0 * (qy * qz - qw * qx);
  double az = 1.0 - 2.0 * (qx * qx + qy * qy);
  RecStage o;
  o.p.r[0] = in.u.x;
  o.p.r[1] = in.u.y;
  o.p.r[2] = in.u.z;
  o.p.ax[0] = ax;
  o.p.ax[1] = ay;
  o.p.ax[2] = az;
  o.p.Rpar = in.u.a;
  o.p.Rperp = in.u.b;
  for (int m = 0; m < 3; ++m) {
    o.k.v[m] = in.v[m];
    o.k.w[m] = in.w[m];
  }
  o.k.pad[0] = o.k.pad[1] = 0.0;
  return o;
}

// Per-particle records of place s in cell order.  M = Rperp^2 I + (Rpar^2 -
// Rperp^2) a a^T; the 128-B record only when rec is given (the forward
// search of large systems reads the 64-B copy).
__device__ __forceinline__ void store_record(int s, const RecStage& st,
                                             PRec* __restrict__ rec, PRecP* __restrict__ recp,
                                             double4* __restrict__ pos,
                                             KRec* __restrict__ kin) {
  recp[s] = st.p;
  const PRec o = expand_record(st.p);
  if (rec) rec[s] = o;
  pos[s] = make_double4(o.r[0], o.r[1], o.r[2], o.Rmax);
  kin[s] = st.k;
}

__device__ void make_record(int s, int p, const double* __restrict__ r,
                            const double* __restrict__ q, const double* __restrict__ semi,
                            const double* __restrict__ v, const double* __restrict__ w,
                            PRec* __restrict__ rec, PRecP* __restrict__ recp,
                            double4* __restrict__ pos, KRec* __restrict__ kin) {
  store_record(s, stage_record(load_record_input(r, q, semi, v, w, p)), rec, recp, pos, kin);
}

// Each particle's cell, its ticket in that cell (the count of the cell
// before its own increment: distinct within the cell, in arbitrary order)
// and its staged record copies, in input order.  The copies go out through
// LDS, so that the block's stores are contiguous 16-B pieces rather than
// one 128-B record per lane (a store instruction would touch 64 lines).
constexpr int kBinThreads = 256;
constexpr int kStagePieces = (int)(sizeof(RecStage) / 16);  // 16-B pieces of a copy
constexpr int kStageStride = kStagePieces + 1;  // LDS stride: no bank conflicts
static_assert(sizeof(RecStage) == 128, "staged copy: 16 doubles");

__global__ void __launch_bounds__(kBinThreads)
k_stage_bin(CallDesc d, const double* __restrict__ r, const double* __restrict__ q,
            const double* __restrict__ semi, const double* __restrict__ v,
            const double* __restrict__ w, int32_t* __restrict__ cell_id,
            int32_t* __restrict__ ticket, RecStage* __restrict__ staged,
            int32_t* __restrict__ cell_count, Counters* cnt, const Counters* gate,
            int32_t* __restrict__ bcount) {
  if (gate && !gate->rebuild) return;  // reused lists: nothing to bin (uniform)
  __shared__ double2 lds[kBinThreads * kStageStride];
  const int p0 = blockIdx.x * kBinThreads;
  const int p = p0 + threadIdx.x;
  if (p < d.n) {
    if (bcount) {  // backward counts and kept pairs of the forward search
      bcount[p] = 0;
      bcount[d.n + p] = 0;
    }
    const double inv_cell[3] = {1.0 / d.cell[0], 1.0 / d.cell[1], 1.0 / d.cell[2]};
    const RecIn in = load_record_input(r, q, semi, v, w, p);
    const int c = validate_bin(d, in.u, inv_cell, cnt);
    cell_id[p] = c;
    ticket[p] = atomicAdd(&cell_count[c], 1);
    // the copy in its memory order: r, ax, Rpar, Rperp, then v, w, pad
    const RecStage st = stage_record(in);
    double2* row = lds + threadIdx.x * kStageStride;
    row[0] = make_double2(st.p.r[0], st.p.r[1]);
    row[1] = make_double2(st.p.r[2], st.p.ax[0]);
    row[2] = make_double2(st.p.ax[1], st.p.ax[2]);
    row[3] = make_double2(st.p.Rpar, st.p.Rperp);
    row[4] = make_double2(st.k.v[0], st.k.v[1]);
    row[5] = make_double2(st.k.v[2], st.k.w[0]);
    row[6] = make_double2(st.k.w[1], st.k.w[2]);
    row[7] = make_double2(st.k.pad[0], st.k.pad[1]);
  }
  __syncthreads();
  const int pieces = min(kBinThreads, d.n - p0) * kStagePieces;
  double2* out = reinterpret_cast<double2*>(staged + p0);
  for (int m = threadIdx.x; m < pieces; m += kBinThreads)
    out[m] = lds[(m / kStagePieces) * kStageStride + m % kStagePieces];
}

// Each cell's members in increasing input index (the position of a particle
// is its cell's start plus the number of members with a smaller index), so
// that every later step is deterministic, and their records, moved from the
// binning's staged copies (one line per particle).  The cell of each place
// comes from the scatter, beside the particle: no dependent look-up of the
// particle's cell.  A particle's position s lies in its cell's range, which
// holds its own place: almost always inside the block's places, whose 64-B
// and 32-B copies then go out through LDS as contiguous 16-B pieces (one
// copy per lane would make each store touch up to 64 lines); a particle
// whose position lies outside (a cell across the block's edge) is written
// directly, and its place left out of the block's stores.
constexpr int kBuildThreads = 256;
constexpr int kBuildPieces = 10;  // 16-B pieces: the 64-B copy, kinematics, position
constexpr int kBuildStride = kBuildPieces + 1;  // LDS stride: no bank conflicts

__global__ void __launch_bounds__(kBuildThreads)
k_build_records(CallDesc d, const int32_t* __restrict__ unsorted,
                const int32_t* __restrict__ cell_sorted, const int32_t* __restrict__ cell_start,
                const RecStage* __restrict__ staged, int32_t* __restrict__ sorted,
                PRec* __restrict__ rec, PRecP* __restrict__ recp, double4* __restrict__ pos,
                KRec* __restrict__ kin, const Counters* gate) {
  if (gate && !gate->rebuild) return;  // reused lists: nothing to build (uniform)
  __shared__ double2 lds[kBuildThreads * kBuildStride];
  __shared__ int filled[kBuildThreads];
  const int p0 = blockIdx.x * kBuildThreads;
  const int nrec = min(kBuildThreads, d.n - p0);
  const int i = p0 + threadIdx.x;
  filled[threadIdx.x] = 0;
  __syncthreads();
  if (i < d.n) {
    const int p = unsorted[i];
    const int c = cell_sorted[i];  // the cell of place i is the cell of place s
    // the staged copy is fetched while the rank within the cell is counted
    const RecStage st = staged[p];
    const int b = cell_start[c], e = cell_start[c + 1];
    int rank = 0;
    for (int k = b; k < e; ++k) rank += unsorted[k] < p;
    const int s = b + rank;
    sorted[s] = p;
    const int row = s - p0;
    if (row >= 0 && row < nrec) {
      const PRec o = expand_record(st.p);
      if (rec) rec[s] = o;
      double2* q = lds + row * kBuildStride;
      q[0] = make_double2(st.p.r[0], st.p.r[1]);
      q[1] = make_double2(st.p.r[2], st.p.ax[0]);
      q[2] = make_double2(st.p.ax[1], st.p.ax[2]);
      q[3] = make_double2(st.p.Rpar, st.p.Rperp);
      q[4] = make_double2(st.k.v[0], st.k.v[1]);
      q[5] = make_double2(st.k.v[2], st.k.w[0]);
      q[6] = make_double2(st.k.w[1], st.k.w[2]);
      q[7] = make_double2(st.k.pad[0], st.k.pad[1]);
      q[8] = make_double2(o.r[0], o.r[1]);
      q[9] = make_double2(o.r[2], o.Rmax);
      filled[row] = 1;
    } else {
      store_record(s, st, rec, recp, pos, kin);
    }
  }
  __syncthreads();
  // the block's places, array by array: 64-B copies, kinematics, positions
  double2* out_p = reinterpret_cast<double2*>(recp + p0);
  for (int m = threadIdx.x; m < 4 * nrec; m += kBuildThreads)
    if (filled[m >> 2]) out_p[m] = lds[(m >> 2) * kBuildStride + (m & 3)];
  double2* out_k = reinterpret_cast<double2*>(kin + p0);
  for (int m = threadIdx.x; m < 4 * nrec; m += kBuildThreads)
    if (filled[m >> 2]) out_k[m] = lds[(m >> 2) * kBuildStride + 4 + (m & 3)];
  double2* out_q = reinterpret_cast<double2*>(pos + p0);
  for (int m = threadIdx.x; m < 2 * nrec; m += kBuildThreads)
    if (filled[m >> 1]) out_q[m] = lds[(m >> 1) * kBuildStride + 8 + (m & 1)];
}

// neighbour offsets along one axis: distinct cells only (a periodic axis
// with fewer than three cells would otherwise visit a cell twice)
// The cells along one axis within `reach` cells of cell c: first cell
// (possibly negative or past the end on a periodic axis, to be wrapped) and
// count.  A periodic axis shorter than the stencil is taken whole, once.
__device__ __forceinline__ void axis_stencil(int c, int nc, int periodic, int reach,
                                             int* first, int* count) {
  if (periodic) {
    if (2 * reach + 1 >= nc) {
      *first = 0;
      *count = nc;
    } else {
      *first = c - reach;
      *count = 2 * reach + 1;
    }
  } else {
    const int lo = max(0, c - reach), hi = min(nc - 1, c + reach);
    *first = lo;
    *count = hi - lo + 1;
  }
}

// Lower bound of the distance along one axis from a point at offset f from
// the lower face of its cell to the cell `o` cells away, shrunk by a relative
// margin far above rounding (the bound only prunes).
__device__ __forceinline__ double axis_gap(int o, double f, double cell) {
  const double g = o > 0 ? o * cell - f : (o < 0 ? f - (o + 1) * cell : 0.0);
  return fmax(0.0, g * (1.0 - 1e-9) - 1e-9 * cell);
}

__device__ __forceinline__ int wrap_cell(int c, int nc) {
  return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

__device__ __forceinline__ double support(const double* M, double nx, double ny,
                                          double nz) {
  double mx = M[0] * nx + M[1] * ny + M[2] * nz;
  double my = M[1] * nx + M[3] * ny + M[4] * nz;
  double mz = M[2] * nx + M[4] * ny + M[5] * nz;
  return sqrt(nx * mx + ny * my + nz * mz);
}

// Whole cell build in one workgroup for small systems (all per-particle and
// per-cell arrays in LDS, 16-bit where the values fit): validation and
// binning, counts, exclusive scan, scatter, placement in increasing input
// index within each cell, and up to kSmallRecN particles the cell-order
// records (beyond, k_records_sorted writes them with the whole chip).
// Replaces four launches.  The counters were zeroed by the previous call.
constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxN = 4096;
constexpr int kSmallMaxCells = 4096;
constexpr int kSmallRecN = 1024;
constexpr int kSmallPer = kSmallMaxN / kSmallThreads;

__global__ void __launch_bounds__(kSmallThreads)
k_cells_small(CallDesc d, const double* __restrict__ r, const double* __restrict__ q,
              const double* __restrict__ semi, const double* __restrict__ v,
              const double* __restrict__ w, int32_t* __restrict__ cell_start,
              int32_t* __restrict__ sorted, PRec* __restrict__ rec,
              PRecP* __restrict__ recp, double4* __restrict__ pos, KRec* __restrict__ kin,
              int32_t* __restrict__ cell_sorted, Counters* cnt, const Counters* gate) {
  if (gate && !gate->rebuild) return;  // reused lists (uniform: one block)
  __shared__ int32_t cnt_l[kSmallMaxCells];        // counts, then cursors
  __shared__ int16_t start_l[kSmallMaxCells + 1];
  __shared__ int16_t cid_l[kSmallMaxN];            // cell of each input index
  __shared__ int16_t scat_l[kSmallMaxN];           // scatter output
  __shared__ int lds_scan[16];
  const int ncell = 2 * d.nc[0] * d.nc[1] * d.nc[2];  // bins: two size classes
  const int tid = threadIdx.x;
  for (int c = tid; c < ncell; c += kSmallThreads) cnt_l[c] = 0;
  __syncthreads();
  // all loads first: one memory round trip for the thread's particles
  PIn in[kSmallPer];
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int p = tid + k * kSmallThreads;
    if (p < d.n) in[k] = load_input(r, q, semi, p);
  }
  const double inv_cell[3] = {1.0 / d.cell[0], 1.0 / d.cell[1], 1.0 / d.cell[2]};
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int p = tid + k * kSmallThreads;
    if (p < d.n) {
      const int c = validate_bin(d, in[k], inv_cell, cnt);
      cid_l[p] = (int16_t)c;
      atomicAdd(&cnt_l[c], 1);
    }
  }
  __syncthreads();
  // exclusive scan of the counts, `per` consecutive cells per thread
  const int per = (ncell + kSmallThreads - 1) / kSmallThreads;
  int run = 0;
  for (int k = 0; k < per; ++k) {
    const int c = tid * per + k;
    run += c < ncell ? cnt_l[c] : 0;
  }
  int tot;
  const int incl = block_inclusive_scan(run, lds_scan, &tot);
  int acc = incl - run;
  for (int k = 0; k < per; ++k) {
    const int c = tid * per + k;
    if (c < ncell) {
      start_l[c] = (int16_t)acc;
      cell_start[c] = acc;
      acc += cnt_l[c];
      cnt_l[c] = 0;
    }
  }
  if (tid == 0) {
    start_l[ncell] = (int16_t)tot;
    cell_start[ncell] = tot;
  }
  __syncthreads();
  for (int p = tid; p < d.n; p += kSmallThreads) {
    const int c = cid_l[p];
    scat_l[start_l[c] + atomicAdd(&cnt_l[c], 1)] = (int16_t)p;
  }
  __syncthreads();
  for (int i = tid; i < d.n; i += kSmallThreads) {
    const int p = scat_l[i];
    const int c = cid_l[p];
    const int b = start_l[c], e = start_l[c + 1];
    int rank = 0;
    for (int k = b; k < e; ++k) rank += scat_l[k] < p;
    const int s = b + rank;
    sorted[s] = p;
    cell_sorted[s] = c;
    if (d.n <= kSmallRecN)
      make_record(s, p, r, q, semi, v, w, rec, recp, pos, kin);
  }
}

// the cell-order records of a small system's larger part: particle sorted[s]
// into place s
__global__ void k_records_sorted(CallDesc d, const int32_t* __restrict__ sorted,
                                 const double* __restrict__ r, const double* __restrict__ q,
                                 const double* __restrict__ semi,
                                 const double* __restrict__ v, const double* __restrict__ w,
                                 PRec* __restrict__ rec, PRecP* __restrict__ recp,
                                 double4* __restrict__ pos, KRec* __restrict__ kin,
                                 const Counters* gate) {
  if (gate && !gate->rebuild) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= d.n) return;
  make_record(s, sorted[s], r, q, semi, v, w, rec, recp, pos, kin);
}

// A group of G lanes per particle (G = 64: one wavefront; G = 32 or 16: two
// or four particles per wavefront): candidate test over the rows of its stencil
// (lanes over the flattened row members, G rows at a time), compaction with
// a ballot, rank sort of the segment by partner index, the support-function
// reject for the entries this particle owns (smaller input index), slot
// assignment (one atomic per block) and the wall candidates.  Segments have
// a fixed stride of d.max_nbr entries, at most 8 G.
// Wavefronts per block (template W): 8 below 16,384 particles, 4 from
// there, where more, smaller blocks fit beside each other on a CU
// (measured: a million particles 2.19 -> 1.97 ms, 65,536 106 -> 101 us;
// 8 is faster at 4096 and for the kernels of reused lists).
constexpr int kWavesSmall = 8;
constexpr int kWavesLarge = 4;
constexpr int kMaxPerLane = 8;  // segment entries per lane after the sort

__device__ __forceinline__ int lane_prefix(unsigned long long mask, int lane) {
  return __popcll(mask & ((1ull << lane) - 1ull));
}

// kMode 0: the full search.  kMode 1: the superset of a reused list (bound
// widened by the skin), only in calls that search: writes the sorted
// segments into nbr, their lengths into deg (minus the count when a segment
// overflows), and per input index the position and size at the search
// (lb.ref_pos) and the place in its cell order (lb.inv); an overflow or an
// earlier input error discards the lists (state epoch -1).  kMode 2: the
// reused superset lb.sup_nbr / lb.sup_deg filtered by the exact centre test
// on the current positions, then as the full search.
template <int G, int kMode, int kWavesPerBlock>
__global__ void __launch_bounds__(64 * kWavesPerBlock)
k_neighbors(CallDesc d, const PRec* __restrict__ rec, const double4* __restrict__ pos,
            const int32_t* __restrict__ orig, const int32_t* __restrict__ cell_sorted,
            const int32_t* __restrict__ cell_start, int32_t* __restrict__ deg,
            int32_t* __restrict__ nbr, int32_t* __restrict__ slot,
            int32_t* __restrict__ wall_slot, int32_t* __restrict__ work_s,
            int32_t* __restrict__ work_t, int64_t* __restrict__ stat_nbr, Counters* cnt,
            ListBufs lb) {
  if (kMode == 1 && !cnt->rebuild) return;  // the lists are reused
  constexpr int kPer = 64 / G;                 // particles per wavefront
  constexpr int kSteps = G == 64 ? 6 : (G == 32 ? 5 : 4);  // log2 G
  constexpr unsigned long long kGroupMask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
  // kWavesPerBlock * kPer * max_nbr partner keys; mode 2 with a warm start
  // then as many superset positions
  extern __shared__ int32_t lds_keys[];
  __shared__ int s_keep[kWavesPerBlock];
  __shared__ int s_upper[kWavesPerBlock];
  __shared__ int s_wallc[kWavesPerBlock];
  __shared__ int s_base[kWavesPerBlock];
  __shared__ int s_deg[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int grp = lane / G;                    // particle of the wavefront
  const int gl = lane % G;                     // lane within its group
  const int gbase = grp * G;
  const int s = (blockIdx.x * kWavesPerBlock + wv) * kPer + grp;
  const int maxn = d.max_nbr;
  int32_t* keys = lds_keys + (wv * kPer + grp) * maxn;
  // mode 2 with a warm start: the superset position of each kept key
  int32_t* keys_e = keys + kWavesPerBlock * kPer * maxn;
  const bool want_e = kMode == 2 && lb.work_sup != nullptr;
  const bool live = s < d.n;

  int count = 0;
  int nkeep = 0, nupper = 0, nwallc = 0;
  // entries held by this lane after the sort: entry gl + G k
  int my_key[kMaxPerLane];
  int my_keep[kMaxPerLane];
  int wall_keep = 0;
  const double extra = kMode == 1 ? d.skin : 0.0;
  int sup_need = 0;  // mode 2: the superset's length (its need if it overflowed)
  if (live && kMode == 2) {
    // the superset of the last build (sorted), filtered in order
    const double4 pi = pos[s];
    const double ri[3] = {pi.x, pi.y, pi.z};
    const int ns_raw = lb.sup_deg[s];
    const int ns = ns_raw > 0 ? ns_raw : 0;
    sup_need = ns_raw >= 0 ? ns_raw : -ns_raw;
    const int32_t* seg = lb.sup_nbr + (size_t)s * maxn;
    for (int base = 0; base < ns; base += G) {
      const int e = base + gl;
      bool acc = false;
      int t = -1;
      if (e < ns) {
        t = seg[e];
        const double4 pj = pos[t];
        const double rj[3] = {pj.x, pj.y, pj.z};
        acc = centre_test(ri, rj, pi.w, pj.w, d, 0.0);
      }
      const unsigned long long m = (__ballot(acc) >> gbase) & kGroupMask;
      if (acc) {
        const int at = count + lane_prefix(m, gl);
        if (at < maxn) {
          keys[at] = t;
          if (want_e) keys_e[at] = e;
        }
      }
      count += __popcll(m);
    }
  }
  if (live && kMode != 2) {
    const double4 pi = pos[s];
    const double ri[3] = {pi.x, pi.y, pi.z};
    const double rmi = pi.w;
    // bins: the cells of the small particles (R_max <= r_small), then those
    // of the large ones
    const int ngeo = d.nc[0] * d.nc[1] * d.nc[2];
    const int c = cell_sorted[s] % ngeo;
    const int cx = c % d.nc[0];
    const int cy = (c / d.nc[0]) % d.nc[1];
    const int cz = c / (d.nc[0] * d.nc[1]);
    // this centre relative to the lower corner of its cell (the wrap of the
    // binning on periodic axes)
    double f3[3];
    const int c3[3] = {cx, cy, cz};
    for (int k = 0; k < 3; ++k) {
      double x = ri[k];
      if (d.periodic[k]) x = wrap_coord(x, d.L[k], d.invL[k]);
      f3[k] = x - c3[k] * d.cell[k];
    }
    const double inv_cx = 1.0 / d.cell[0];
    for (int cls = 0; cls < 2; ++cls) {
      const int32_t* cs_cls = cell_start + cls * ngeo;
      if (cs_cls[ngeo] == cs_cls[0]) continue;  // no particle of this class
      // every partner of the class lies within rho of this centre along each
      // axis: at most `reach` cells away (cells are at least 1/reach_max of
      // the largest rho)
      const double rho = rmi + (cls == 0 ? d.r_small : d.rmax_bound) + d.dmax + extra;
      int reach[3], first[3], cnt3[3];
      for (int k = 0; k < 3; ++k)
        reach[k] = min(d.reach_max, max(1, (int)ceil(rho / d.cell[k])));
      axis_stencil(cx, d.nc[0], d.periodic[0], reach[0], &first[0], &cnt3[0]);
      axis_stencil(cy, d.nc[1], d.periodic[1], reach[1], &first[1], &cnt3[1]);
      axis_stencil(cz, d.nc[2], d.periodic[2], reach[2], &first[2], &cnt3[2]);
      const int nrows = cnt3[1] * cnt3[2];
      // an axis taken whole (periodic, shorter than the stencil) is not pruned
      bool whole[3];
      for (int k = 0; k < 3; ++k) whole[k] = d.periodic[k] && cnt3[k] == d.nc[k];
      // Lees-Edwards images: a row reached across the z boundary holds
      // partners whose nearest image is shifted by the offset in x, so its
      // x window is moved by that offset.  With z taken whole a row's image
      // is not known from the row: then x is taken whole too
      if (d.le && whole[2]) {
        whole[0] = true;
        first[0] = 0;
        cnt3[0] = d.nc[0];
      }
      for (int row0 = 0; row0 < nrows; row0 += G) {
        // lane gl owns row row0 + gl of the stencil (cells (y, z)).  Rows
        // farther than rho from the centre hold no candidate; in the others
        // the cells along x are cut to the chord of the sphere of radius
        // rho.  What is left is one contiguous range of cell-ordered
        // particles, or two when it wraps around a periodic axis
        const int row = row0 + gl;
        int s0 = 0, n0 = 0, s1 = 0, n1 = 0;
        if (row < nrows) {
          const int oy = first[1] + row % cnt3[1] - cy;  // offsets from this cell
          const int oz = first[2] + row / cnt3[1] - cz;
          const double gy = whole[1] ? 0.0 : axis_gap(oy, f3[1], d.cell[1]);
          const double gz = whole[2] ? 0.0 : axis_gap(oz, f3[2], d.cell[2]);
          const double rem = rho * rho - gy * gy - gz * gz;
          int a0 = first[0], a1 = first[0] + cnt3[0] - 1;  // cells a0..a1 along x
          if (!whole[0]) {
            const double wx = sqrt(fmax(rem, 0.0)) * (1.0 + 1e-9) + 1e-9 * d.cell[0];
            int cxr = cx;
            double fx = f3[0];
            const int zr = cz + oz;
            if (d.le && (zr < 0 || zr >= d.nc[2])) {
              // partners across the top sit at x - offset, across the bottom
              // at x + offset (stored coordinates of the nearest image)
              double xs = fx + cx * d.cell[0] + (zr < 0 ? d.le_offset : -d.le_offset);
              xs = xs - d.L[0] * floor(xs / d.L[0]);
              cxr = min(d.nc[0] - 1, max(0, (int)floor(xs / d.cell[0])));
              fx = xs - cxr * d.cell[0];
              a0 = cxr - reach[0];
              a1 = cxr + reach[0];
            }
            // (products with 1 / cell: the chord's margin is far above
            // their rounding)
            a0 = max(a0, cxr + (int)floor((fx - wx) * inv_cx));
            a1 = min(a1, cxr + (int)floor((fx + wx) * inv_cx));
          }
          if (rem > 0.0 && a1 >= a0) {
            const int ry = wrap_cell(cy + oy, d.nc[1]);
            const int rz = wrap_cell(cz + oz, d.nc[2]);
            const int rowbase = (rz * d.nc[1] + ry) * d.nc[0];
            // the part inside [0, nc) and the part wrapped around (the range
            // is shorter than the axis, so at most one side wraps)
            const int nx = d.nc[0];
            const int p0 = max(a0, 0), p1 = min(a1, nx - 1);
            int b0 = 0, b1 = -1;
            if (a0 < 0) {
              b0 = a0 + nx;
              b1 = min(a1, -1) + nx;
            } else if (a1 >= nx) {
              b0 = max(a0, nx) - nx;
              b1 = a1 - nx;
            }
            if (p1 >= p0) {
              s0 = cs_cls[rowbase + p0];
              n0 = cs_cls[rowbase + p1 + 1] - s0;
            }
            if (b1 >= b0) {
              s1 = cs_cls[rowbase + b0];
              n1 = cs_cls[rowbase + b1 + 1] - s1;
            }
          }
        }
        const int cn = n0 + n1;
        int incl = cn;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
          int y = __shfl_up(incl, o, G);
          if (gl >= o) incl += y;
        }
        const int total = __shfl(incl, gbase + G - 1, 64);
        const int excl = incl - cn;
        const int nlanes = min(G, nrows - row0);
        for (int base = 0; base < total; base += G) {
          const int idx = base + gl;
          bool acc = false;
          int t = -1;
          // the row holding flattened index idx: binary search over the
          // group's exclusive prefixes, every lane of the group taking part
          int lo = 0, hi = nlanes - 1;
          for (int step = 0; step < kSteps; ++step) {
            int mid = (lo + hi + 1) >> 1;
            int em = __shfl(excl, gbase + mid, 64);
            bool up = lo < hi && em <= idx;
            bool down = lo < hi && !(em <= idx);
            lo = up ? mid : lo;
            hi = down ? mid - 1 : hi;
          }
          const int r0 = __shfl(s0, gbase + lo, 64);
          const int rn0 = __shfl(n0, gbase + lo, 64);
          const int r1 = __shfl(s1, gbase + lo, 64);
          const int ex = __shfl(excl, gbase + lo, 64);
          if (idx < total) {
            const int off = idx - ex;
            t = off < rn0 ? r0 + off : r1 + (off - rn0);
            const double4 pj = pos[t];
            const double rj[3] = {pj.x, pj.y, pj.z};
            acc = t != s && centre_test(ri, rj, rmi, pj.w, d, extra);
          }
          const unsigned long long m = (__ballot(acc) >> gbase) & kGroupMask;
          if (acc) {
            const int at = count + lane_prefix(m, gl);
            if (at < maxn) keys[at] = t;
          }
          count += __popcll(m);
        }
      }
    }
  }
  __syncthreads();
  const bool overflow = live && count > maxn;
  if (overflow && gl == 0) set_error(cnt, LUB_ECAPACITY);
  const int nent = (live && !overflow) ? count : 0;
  // rank sort: keys are distinct partner indices (mode 2 keeps the order of
  // the sorted superset: the rank is the position)
  const int me = live ? orig[s] : 0;
  const double* Mi = live ? rec[s].M : nullptr;
  double rs[3] = {0, 0, 0};
  if (live) {
    rs[0] = rec[s].r[0];
    rs[1] = rec[s].r[1];
    rs[2] = rec[s].r[2];
  }
  for (int k = 0; k < kMaxPerLane; ++k) {
    my_key[k] = -1;
    my_keep[k] = 0;
    const int e = gl + G * k;
    if (e >= nent) continue;
    const int key = keys[e];
    int rank = 0;
    if (kMode == 2)
      rank = e;
    else
      for (int m2 = 0; m2 < nent; ++m2) rank += keys[m2] < key;
    nbr[(size_t)s * maxn + rank] = key;
    my_key[k] = key;
    if (kMode == 1) continue;  // the superset: segments only
    // owned entries (smaller input index) are evaluated unless the support
    // functions along the line of centres already bound the gap above every
    // cut-off
    if (orig[key] > me) {
      ++nupper;
      double dv[3];
      pair_image(d, rs, rec[key].r, dv);
      const double dx = dv[0], dy = dv[1], dz = dv[2];
      double dn = sqrt(dx * dx + dy * dy + dz * dz);
      bool keep = true;
      if (dn > 0.0) {
        const double idn = 1.0 / dn;
        double ux = dx * idn, uy = dy * idn, uz = dz * idn;
        double g = dn - support(Mi, ux, uy, uz) - support(rec[key].M, ux, uy, uz);
        keep = g < d.dmax;
      }
      slot[(size_t)s * maxn + rank] = -1;
      if (keep) {
        my_keep[k] = 1 + rank;  // remember the rank for the slot write
        ++nkeep;
      }
    } else {
      slot[(size_t)s * maxn + rank] = -2;
    }
  }
  if (kMode == 1) {
    if (live && gl == 0) {
      deg[s] = overflow ? -count : nent;
      lb.ref_pos[me] = pos[s];
      lb.inv[me] = s;
      if (overflow) lb.state->epoch = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt->error) lb.state->epoch = -1;
    return;
  }
  if (live && d.n_walls && gl < 2) {
    const int side = gl;
    double dist = side == 0 ? rs[2] : d.L[2] - rs[2];
    bool cand = (dist - rec[s].Rmax) < d.dmax;
    bool keep = cand && (dist - sqrt(Mi[5])) < d.dmax;
    nwallc += cand;
    wall_keep = keep;
    nkeep += keep;
    // -3: candidate beyond every cut-off, -1: no candidate
    wall_slot[2 * s + side] = keep ? 0 : (cand ? -3 : -1);
  }
  if (live && gl == 0) deg[s] = nent;
  // wave totals -> block total -> one atomic per block
  int wkeep = nkeep, wup = nupper, wwall = nwallc;
  int wdeg = live ? max(count, sup_need) : 0;  // uniform in each group
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    wkeep += __shfl_xor(wkeep, o, 64);
    wup += __shfl_xor(wup, o, 64);
    wwall += __shfl_xor(wwall, o, 64);
    wdeg = max(wdeg, __shfl_xor(wdeg, o, 64));
  }
  if (lane == 0) {
    s_keep[wv] = wkeep;
    s_upper[wv] = wup;
    s_wallc[wv] = wwall;
    s_deg[wv] = wdeg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0, up = 0, wc = 0, dg = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) {
      s_base[k] = tot;
      tot += s_keep[k];
      up += s_upper[k];
      wc += s_wallc[k];
      dg = max(dg, s_deg[k]);
    }
    int b = tot ? atomicAdd(&cnt->work, tot) : 0;
    if (b + tot > d.cap_work) set_error(cnt, LUB_ECAPACITY);
    for (int k = 0; k < kWavesPerBlock; ++k) s_base[k] += b;
    stat_nbr[kStatNbrWords * blockIdx.x] = up;
    stat_nbr[kStatNbrWords * blockIdx.x + 1] = wc;
    stat_nbr[kStatNbrWords * blockIdx.x + 2] = dg;
    s_keep[0] = b + tot <= d.cap_work;
  }
  __syncthreads();
  const bool fits = s_keep[0] != 0;
  // slots in lane order: exclusive prefix of nkeep across the wave
  int incl2 = nkeep;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(incl2, o, 64);
    if (lane >= o) incl2 += y;
  }
  // warm start: this particle's slot range (its lanes' slots are
  // consecutive), by input index
  if (lb.warm_range) {
    const int start = s_base[wv] + incl2 - nkeep;
    int gsum = nkeep;
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) gsum += __shfl_xor(gsum, o, G);
    const int first = __shfl(start, gbase, 64);
    if (live && gl == 0)
      lb.warm_range[me] = fits ? make_int2(first, first + gsum) : make_int2(0, 0);
  }
  if (!live || !fits) return;
  int next = s_base[wv] + incl2 - nkeep;
  for (int k = 0; k < kMaxPerLane; ++k) {
    if (my_keep[k] <= 0) continue;
    const int rank = my_keep[k] - 1;
    slot[(size_t)s * maxn + rank] = next;
    work_s[next] = s;
    work_t[next] = my_key[k];
    if (want_e) lb.work_sup[next] = s * maxn + keys_e[rank];
    ++next;
  }
  if (d.n_walls && gl < 2 && wall_keep) {
    wall_slot[2 * s + gl] = next;
    work_s[next] = s;
    work_t[next] = -1 - gl;
    ++next;
  }
}

// The search without Lees-Edwards images, flattened through LDS (kMode 0:
// the full search; kMode 1: the superset of reused lists, bound widened by
// the skin).  G lanes share a particle.  Its stencil rows are visited in
// increasing cell order (a periodic axis's window from its smallest wrapped
// cell, the two x parts of a row in increasing order too), so that the
// candidates, and with them the accepted partners, come out sorted by cell
// order: no sort.  Per chunk of G rows each lane cuts its row to the chord
// of the sphere of radius rho and appends the particle indices of that range
// to the group's LDS buffer; the group then tests the buffer G entries at a
// time with the exact centre test, one candidate per lane, and writes the
// accepted ones straight into the segment.  Owned entries then get the
// support-function reject and their evaluation slots (one atomic per block).
// kMode kFwd, the forward search of large systems: each pair is tested once:
// a pair of one size class by the particle that comes first in cell order
// (its own class's rows from its own row on, the ranges cut to later
// indices), a small-large pair by the large particle (the small class
// whole); the particle is appended to each partner's backward list through
// an atomic count.  After a scan of the kept counts, k_nbr_emit writes the
// evaluation list; no segments are built (the gather reads each particle's
// slot range and backward list).  About half the centre tests of the full
// search, and the small particles (most of them) walk no rows of the sparse
// large class.
constexpr int kFlatG = 16;
constexpr int kFlatWaves = 4;
constexpr int kFlatBuf = 256;  // candidate indices per group
constexpr int kFlushK = 4;  // candidates per lane and round of the test
constexpr int kFwd = 3;        // mode of the forward search (partners later in cell order)
// the forward search from this many particles, with at most kFwdMaxNbr
// entries per particle (the gather's LDS: 2 x 4 B per entry and particle)
constexpr int kFwdMinN = 1 << 15;
constexpr int kFwdMaxNbr = 256;

// Workgroups are dealt to the eight XCDs in turn.  Renumbered so that each
// XCD takes runs of kXcdRun consecutive blocks (particles close in cell
// order share most stencil rows, so their candidates stay in the L2 of the
// XCD that tests them) and the runs go round the XCDs (the work per block
// changes along the cell order: the large particles come last).  Blocks past
// the last whole round keep their number.
constexpr int kXcds = 8;
constexpr int kXcdRun = 128;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int full = nb / (kXcds * kXcdRun) * (kXcds * kXcdRun);
  if (b >= full) return b;
  const int x = b % kXcds, k = b / kXcds;
  return ((k / kXcdRun) * kXcds + x) * kXcdRun + k % kXcdRun;
}

// Row range of a stencil row along one axis, in FP32 with margins far above
// its rounding (a row or cell too many is harmless: the exact FP64 centre
// test decides): the distance from the centre (f from its cell's lower
// corner) to cells o away, under-estimated.
__device__ __forceinline__ float axis_gap_f(int o, float f, float cell) {
  const float g = o > 0 ? (float)o * cell - f : (o < 0 ? f - (float)(o + 1) * cell : 0.0f);
  return fmaxf(0.0f, g * (1.0f - 1e-5f) - 1e-5f * cell);
}

// x / m and x % m for 0 <= x < 2^20 and m >= 1: a float estimate (off by at
// most one) and one correction
__device__ __forceinline__ int small_divmod(int x, int m, int* rem) {
  int q = (int)((float)x * __builtin_amdgcn_rcpf((float)m));
  int r = x - q * m;
  if (r < 0) {
    --q;
    r += m;
  } else if (r >= m) {
    ++q;
    r -= m;
  }
  *rem = r;
  return q;
}

// the visiting order of an axis window [first, first + count): the offset
// into the window at which the wrapped cell index is smallest
__device__ __forceinline__ int axis_rotation(int first, int count, int nc) {
  if (first < 0) return -first;
  if (first + count > nc) return nc - first;
  return 0;
}

// The end of the full search: owned entries (smaller input index) are
// evaluated unless the support functions along the line of centres bound
// the gap above every cut-off; wall candidates; the block's statistics row
// and one atomic per block for its evaluation slots, assigned in lane order.
// keys: the particle's segment (nent entries); need: its length before an
// overflow cut it.  Every thread of the block calls it.
__device__ __forceinline__ void evaluation_slots(
    const CallDesc& d, const PRec* __restrict__ rec, const int32_t* __restrict__ orig,
    int blk, int s, bool live, int need, int nent, const int32_t* keys,
    int32_t* __restrict__ deg, int32_t* __restrict__ slot, int32_t* __restrict__ wall_slot,
    int32_t* __restrict__ work_s, int32_t* __restrict__ work_t,
    int64_t* __restrict__ stat_nbr, Counters* cnt, int* s_keep, int* s_upper, int* s_wallc,
    int* s_base, int* s_deg, int2* __restrict__ warm_range) {
  constexpr int G = kFlatG;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int gl = lane % G;
  const int maxn = d.max_nbr;
  const int me = live ? orig[s] : 0;
  // bit k of `kept`: entry gl + G k is kept
  int nkeep = 0, nupper = 0, nwallc = 0, wall_keep = 0;
  unsigned kept = 0u;
  double rs[3] = {0, 0, 0};
  const double* Mi = live ? rec[s].M : nullptr;
  if (live) {
    for (int k = 0; k < 3; ++k) rs[k] = rec[s].r[k];
  }
  int32_t* sl = slot + (size_t)(live ? s : 0) * maxn;
  for (int k = 0, e = gl; e < nent; ++k, e += G) {
    const int key = keys[e];
    if (orig[key] > me) {
      ++nupper;
      const PRec& B = rec[key];
      double dv[3];
      pair_image(d, rs, B.r, dv);
      const double dx = dv[0], dy = dv[1], dz = dv[2];
      const double dn = sqrt(dx * dx + dy * dy + dz * dz);
      bool keep = true;
      if (dn > 0.0) {
        const double idn = 1.0 / dn;
        const double ux = dx * idn, uy = dy * idn, uz = dz * idn;
        const double g = dn - support(Mi, ux, uy, uz) - support(B.M, ux, uy, uz);
        keep = g < d.dmax;
      }
      sl[e] = -1;
      if (keep) {
        kept |= 1u << k;
        ++nkeep;
      }
    } else {
      sl[e] = -2;
    }
  }
  if (live && d.n_walls && gl < 2) {
    const int side = gl;
    const double dist = side == 0 ? rs[2] : d.L[2] - rs[2];
    const bool cand_w = (dist - rec[s].Rmax) < d.dmax;
    const bool keep = cand_w && (dist - sqrt(Mi[5])) < d.dmax;
    nwallc += cand_w;
    wall_keep = keep;
    nkeep += keep;
    // -3: candidate beyond every cut-off, -1: no candidate
    wall_slot[2 * s + side] = keep ? 0 : (cand_w ? -3 : -1);
  }
  if (live && gl == 0) deg[s] = nent;
  // wave totals -> block total -> one atomic per block
  int wkeep = nkeep, wup = nupper, wwall = nwallc;
  int wdeg = live ? need : 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    wkeep += __shfl_xor(wkeep, o, 64);
    wup += __shfl_xor(wup, o, 64);
    wwall += __shfl_xor(wwall, o, 64);
    wdeg = max(wdeg, __shfl_xor(wdeg, o, 64));
  }
  if (lane == 0) {
    s_keep[wv] = wkeep;
    s_upper[wv] = wup;
    s_wallc[wv] = wwall;
    s_deg[wv] = wdeg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0, up = 0, wc = 0, dg = 0;
    for (int k = 0; k < kFlatWaves; ++k) {
      s_base[k] = tot;
      tot += s_keep[k];
      up += s_upper[k];
      wc += s_wallc[k];
      dg = max(dg, s_deg[k]);
    }
    const int b = tot ? atomicAdd(&cnt->work, tot) : 0;
    if (b + tot > d.cap_work) set_error(cnt, LUB_ECAPACITY);
    for (int k = 0; k < kFlatWaves; ++k) s_base[k] += b;
    stat_nbr[kStatNbrWords * blk] = up;
    stat_nbr[kStatNbrWords * blk + 1] = wc;
    stat_nbr[kStatNbrWords * blk + 2] = dg;
    s_keep[0] = b + tot <= d.cap_work;
  }
  __syncthreads();
  const bool fits = s_keep[0] != 0;
  // slots in lane order: exclusive prefix of nkeep across the wave
  int incl2 = nkeep;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl2, o, 64);
    if (lane >= o) incl2 += y;
  }
  // warm start: this particle's slot range (its lanes' slots are
  // consecutive), by input index
  if (warm_range) {
    const int start = s_base[wv] + incl2 - nkeep;
    int gsum = nkeep;
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) gsum += __shfl_xor(gsum, o, G);
    const int first = __shfl(start, lane - gl, 64);
    if (live && gl == 0)
      warm_range[me] = fits ? make_int2(first, first + gsum) : make_int2(0, 0);
  }
  if (!live || !fits) return;
  int next = s_base[wv] + incl2 - nkeep;
  for (int k = 0, e = gl; e < nent; ++k, e += G) {
    if (!((kept >> k) & 1u)) continue;
    sl[e] = next;
    work_s[next] = s;
    work_t[next] = keys[e];
    ++next;
  }
  if (d.n_walls && gl < 2 && wall_keep) {
    wall_slot[2 * s + gl] = next;
    work_s[next] = s;
    work_t[next] = -1 - gl;
    ++next;
  }
}

template <int kMode>
__global__ void __launch_bounds__(64 * kFlatWaves)
k_neighbors_flat(CallDesc d, const PRec* __restrict__ rec, const PRecP* __restrict__ recp,
                 const double4* __restrict__ pos,
                 const int32_t* __restrict__ orig, const int32_t* __restrict__ cell_sorted,
                 const int32_t* __restrict__ cell_start, int32_t* __restrict__ deg,
                 int32_t* __restrict__ nbr, int32_t* __restrict__ slot,
                 int32_t* __restrict__ wall_slot, int32_t* __restrict__ work_s,
                 int32_t* __restrict__ work_t, int64_t* __restrict__ stat_nbr, Counters* cnt,
                 ListBufs lb, int32_t* __restrict__ bcount, int2* __restrict__ bstage) {
  if (kMode == 1 && !cnt->rebuild) return;  // the lists are reused
  constexpr int G = kFlatG;
  constexpr int kPer = 64 / G;
  constexpr unsigned long long kGroupMask = (1ull << G) - 1ull;
  __shared__ int32_t s_cand[kFlatWaves * kPer][kFlatBuf];
  // the forward search keeps its accepted partners here (max_nbr per group)
  extern __shared__ int32_t s_fwd[];
  __shared__ int s_keep[kFlatWaves], s_upper[kFlatWaves], s_wallc[kFlatWaves];
  __shared__ int s_base[kFlatWaves], s_deg[kFlatWaves];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int grp = lane / G;
  const int gl = lane % G;
  const int gbase = grp * G;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int s = (blk * kFlatWaves + wv) * kPer + grp;
  const bool live = s < d.n;
  const int maxn = d.max_nbr;
  int32_t* cand = s_cand[wv * kPer + grp];
  int32_t* seg = kMode == kFwd ? s_fwd + (size_t)(wv * kPer + grp) * maxn
                               : nbr + (size_t)(live ? s : 0) * maxn;
  const double extra = kMode == 1 ? d.skin : 0.0;
  int count = 0;
  if (live) {
    const double4 pi = pos[s];
    const double ri[3] = {pi.x, pi.y, pi.z};
    const double rmi = pi.w;
    const int ngeo = d.nc[0] * d.nc[1] * d.nc[2];
    const int c = cell_sorted[s] % ngeo;
    const int c3[3] = {c % d.nc[0], (c / d.nc[0]) % d.nc[1], c / (d.nc[0] * d.nc[1])};
    double f3[3];
    for (int k = 0; k < 3; ++k) {
      double x = ri[k];
      if (d.periodic[k]) x = wrap_coord(x, d.L[k], d.invL[k]);
      f3[k] = x - c3[k] * d.cell[k];
    }
    // the chord cut in FP32 (see axis_gap_f)
    const float fx = (float)f3[0], fy = (float)f3[1], fz = (float)f3[2];
    const float cellx = (float)d.cell[0], celly = (float)d.cell[1], cellz = (float)d.cell[2];
    const float inv_cx = 1.0f / cellx;
    int nbuf = 0;  // entries in the buffer (uniform in the group)
    // test the buffer's entries [0, m): accepted partners go to the segment
    auto flush = [&](int m) {
      // kFlushK candidates per lane and round: their positions are loaded
      // together (the walk waits on these loads)
      for (int base = 0; base < m; base += kFlushK * G) {
        int tk[kFlushK];
        double4 pk[kFlushK];
#pragma unroll
        for (int u = 0; u < kFlushK; ++u) {
          const int e = base + u * G + gl;
          tk[u] = e < m ? cand[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < kFlushK; ++u)
          pk[u] = tk[u] >= 0 ? pos[tk[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
        for (int u = 0; u < kFlushK; ++u) {
          bool acc = false;
          if (tk[u] >= 0) {
            const double rj[3] = {pk[u].x, pk[u].y, pk[u].z};
            acc = tk[u] != s && centre_test(ri, rj, rmi, pk[u].w, d, extra);
          }
          const unsigned long long mk = (__ballot(acc) >> gbase) & kGroupMask;
          if (acc) {
            const int at = count + lane_prefix(mk, gl);
            if (at < maxn) seg[at] = tk[u];
          }
          count += __popcll(mk);
        }
      }
    };
    // the forward search: a small particle searches its own class only,
    // from its own row on; a large one the small class whole and its own
    // class from its own row on (each small-large pair is found by the
    // large particle: the small class is the dense one)
    const int cls_s = s >= cell_start[ngeo] ? 1 : 0;
    const int cls_end = kMode == kFwd && cls_s == 0 ? 1 : 2;
    for (int cls = 0; cls < cls_end; ++cls) {
      const int32_t* cs_cls = cell_start + cls * ngeo;
      if (cs_cls[ngeo] == cs_cls[0]) continue;  // no particle of this class
      const double rho = rmi + (cls == 0 ? d.r_small : d.rmax_bound) + d.dmax + extra;
      int first[3], cnt3[3], rot[3];
      bool whole[3];
      for (int k = 0; k < 3; ++k) {
        const int reach = min(d.reach_max, max(1, (int)ceil(rho / d.cell[k])));
        axis_stencil(c3[k], d.nc[k], d.periodic[k], reach, &first[k], &cnt3[k]);
        whole[k] = d.periodic[k] && cnt3[k] == d.nc[k];
        rot[k] = axis_rotation(first[k], cnt3[k], d.nc[k]);
      }
      const float rhof = (float)rho * (1.0f + 1e-5f) + 1e-5f * cellx;
      const int nrows = cnt3[1] * cnt3[2];
      // the forward search in this particle's own class starts at its own
      // row: the rows before it (in increasing cell order) hold smaller
      // indices only, the rows after it larger ones, and in its own row
      // the ranges are cut to indices above s
      const bool own = kMode == kFwd && cls == cls_s;
      // (c3 - first and rot both lie in [0, cnt): their difference in
      // (-cnt, cnt))
      int py = 0, pz = 0;
      if (own) {
        py = c3[1] - first[1] - rot[1];
        pz = c3[2] - first[2] - rot[2];
        py += py < 0 ? cnt3[1] : 0;
        pz += pz < 0 ? cnt3[2] : 0;
      }
      const int row_start = pz * cnt3[1] + py;
      // lane gl's row (iy, iz) = row0 + gl, advanced by G rows per chunk
      int step_y, iy;
      const int step_z = small_divmod(G, cnt3[1], &step_y);
      const int iz0 = small_divmod(py + gl, cnt3[1], &iy);
      int iz = pz + iz0;
      for (int row0 = row_start; row0 < nrows; row0 += G) {
        // lane gl's row: its cell range along x cut to the chord, as one or
        // two index ranges in increasing order
        int lo0 = 0, n0 = 0, lo1 = 0, n1 = 0;
        if (row0 + gl < nrows) {
          int ry = iy + rot[1], rz = iz + rot[2];
          ry = ry >= cnt3[1] ? ry - cnt3[1] : ry;
          rz = rz >= cnt3[2] ? rz - cnt3[2] : rz;
          const int uy = first[1] + ry, uz = first[2] + rz;  // unwrapped cells
          const float gy = whole[1] ? 0.0f : axis_gap_f(uy - c3[1], fy, celly);
          const float gz = whole[2] ? 0.0f : axis_gap_f(uz - c3[2], fz, cellz);
          const float rem = rhof * rhof - gy * gy - gz * gz;
          int a0 = first[0], a1 = first[0] + cnt3[0] - 1;
          if (!whole[0]) {
            const float wx = sqrtf(fmaxf(rem, 0.0f)) * (1.0f + 1e-5f) + 1e-5f * cellx;
            a0 = max(a0, c3[0] + (int)floorf((fx - wx) * inv_cx));
            a1 = min(a1, c3[0] + (int)floorf((fx + wx) * inv_cx));
          }
          if (rem > 0.0f && a1 >= a0) {
            const int nx = d.nc[0];
            const int rowbase = (wrap_cell(uz, d.nc[2]) * d.nc[1] + wrap_cell(uy, d.nc[1])) * nx;
            // the part wrapped to the start (smaller cells) first, then the
            // part inside [0, nx), then the part wrapped to the end
            int b0 = 0, b1 = -1, e0 = 0, e1 = -1;
            const int p0 = max(a0, 0), p1 = min(a1, nx - 1);
            if (a1 >= nx) {
              b0 = max(a0, nx) - nx;
              b1 = a1 - nx;
            }
            if (a0 < 0) {
              e0 = a0 + nx;
              e1 = min(a1, -1) + nx;
            }
            if (b1 >= b0) {
              lo0 = cs_cls[rowbase + b0];
              n0 = cs_cls[rowbase + b1 + 1] - lo0;
            }
            if (p1 >= p0) {
              const int l = cs_cls[rowbase + p0], h = cs_cls[rowbase + p1 + 1];
              if (n0 == 0) {
                lo0 = l;
                n0 = h - l;
              } else {
                lo1 = l;
                n1 = h - l;
              }
            }
            if (e1 >= e0) {
              lo1 = cs_cls[rowbase + e0];
              n1 = cs_cls[rowbase + e1 + 1] - lo1;
            }
          }
        }
        if (own) {
          int h = lo0 + n0;
          lo0 = max(lo0, s + 1);
          n0 = max(0, h - lo0);
          h = lo1 + n1;
          lo1 = max(lo1, s + 1);
          n1 = max(0, h - lo1);
        }
        iy += step_y;
        iz += step_z;
        if (iy >= cnt3[1]) {
          iy -= cnt3[1];
          ++iz;
        }
        const int cn = n0 + n1;
        int incl = cn;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
          const int y = __shfl_up(incl, o, G);
          if (gl >= o) incl += y;
        }
        const int total = __shfl(incl, gbase + G - 1, 64);
        const int excl = incl - cn;
        if (nbuf + total > kFlatBuf) {
          flush(nbuf);
          nbuf = 0;
        }
        if (total <= kFlatBuf) {
          // append
          int at = nbuf + excl;
          for (int j = 0; j < n0; ++j) cand[at + j] = lo0 + j;
          at += n0;
          for (int j = 0; j < n1; ++j) cand[at + j] = lo1 + j;
          nbuf += total;
        } else {
          // a chunk longer than the buffer goes through it in windows (the
          // buffer was flushed above)
          for (int win = 0; win < total; win += kFlatBuf) {
            const int lim = min(total - win, kFlatBuf);
            for (int j = 0; j < cn; ++j) {
              const int q = excl + j - win;
              if (q >= 0 && q < lim) cand[q] = j < n0 ? lo0 + j : lo1 + (j - n0);
            }
            flush(lim);
          }
        }
      }
    }
    flush(nbuf);
  }
  const bool overflow = live && count > maxn;
  if (overflow && gl == 0) set_error(cnt, LUB_ECAPACITY);
  const int nent = (live && !overflow) ? count : 0;
  if (kMode == kFwd) {
    // Each pair once, by the particle that found it (the finder): which side
    // evaluates it (smaller input index) and the support-function bound
    // along the line of centres, taken as the evaluating side would take it
    // (same operands, same order).  The kept pairs get evaluation slots in
    // the finder's range, in the order of its forward list, then its kept
    // walls: slot = fbase[finder] + kk with fbase the scan of kcnt.  The
    // forward partners go to this particle's slot row (read by the
    // evaluation-list kernel), and this particle, with the flags and its kk,
    // to each partner's row of bstage
    // at a place counted by bcount (the backward partners, in no particular
    // order; one 8-B store per pair).
    if (live) {
      int32_t* kcnt = bcount + d.n;
      if (gl == 0) deg[s] = count;
      const int nf = min(count, maxn);
      const int me = orig[s];
      // the 64-B geometry copies, M formed with the staging's expression
      const PRecP A = recp[s];
      int32_t* srow = slot + (size_t)s * maxn;
      int kept = 0;  // kept forward pairs so far (uniform in the group)
      double ma[6];
      support_matrix(A.ax, A.Rpar, A.Rperp, ma);
      const double* ra = A.r;
      for (int k0 = 0; k0 < nf; k0 += G) {
        const int k = k0 + gl;
        const bool on = k < nf;
        bool keep = false, own = false;
        int t = 0, q = 0;
        if (on) {
          t = seg[k];
          // the partner's data first, the atomic after it: its return is
          // needed last (vector memory operations complete in order)
          const int ot = orig[t];
          const PRecP B = recp[t];
          q = atomicAdd(&bcount[t], 1);
          double mb[6];
          support_matrix(B.ax, B.Rpar, B.Rperp, mb);
          const double* rb = B.r;
          own = me < ot;
          double dv[3];
          if (own)
            pair_image(d, ra, rb, dv);
          else
            pair_image(d, rb, ra, dv);
          const double dx = dv[0], dy = dv[1], dz = dv[2];
          const double dn = sqrt(dx * dx + dy * dy + dz * dz);
          keep = true;
          if (dn > 0.0) {
            const double idn = 1.0 / dn;
            const double ux = dx * idn, uy = dy * idn, uz = dz * idn;
            const double* M1 = own ? ma : mb;
            const double* M2 = own ? mb : ma;
            const double g = dn - support(M1, ux, uy, uz) - support(M2, ux, uy, uz);
            keep = g < d.dmax;
          }
        }
        const unsigned long long mk = (__ballot(keep) >> gbase) & kGroupMask;
        if (on) {
          const int32_t fk = keep ? kKeepBit : 0;
          srow[k] = t | (own ? kOwnBit : 0) | fk;
          if (q < maxn)
            bstage[(size_t)t * maxn + q] =
                make_int2(s | (own ? 0 : kOwnBit) | fk, keep ? kept + lane_prefix(mk, gl) : 0);
        }
        kept += __popcll(mk);
      }
      int walls = 0;
      if (d.n_walls && gl < 2) {
        // -3: candidate beyond every cut-off, -1: no candidate, 0: kept
        const double dist = gl == 0 ? ra[2] : d.L[2] - ra[2];
        const bool cand_w = (dist - (A.Rpar > A.Rperp ? A.Rpar : A.Rperp)) < d.dmax;
        const bool keep = cand_w && (dist - sqrt(ma[5])) < d.dmax;
        wall_slot[2 * s + gl] = keep ? 0 : (cand_w ? -3 : -1);
        walls = keep;
      }
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) walls += __shfl_xor(walls, o, G);
      if (gl == 0) kcnt[s] = kept + walls;
    }
    return;
  }
  if (kMode == 1) {
    const int me = live ? orig[s] : 0;
    if (live && gl == 0) {
      deg[s] = overflow ? -count : nent;
      lb.ref_pos[me] = pos[s];
      lb.inv[me] = s;
      if (overflow) lb.state->epoch = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt->error) lb.state->epoch = -1;
    return;
  }
  evaluation_slots(d, rec, orig, blk, s, live, live ? count : 0, nent, seg, deg, slot,
                   wall_slot, work_s, work_t, stat_nbr, cnt, s_keep, s_upper, s_wallc, s_base,
                   s_deg, lb.warm_range);
}

// The evaluation list of the forward search, from the scan of the kept
// counts: each particle's range [fbase[s], fbase[s + 1]) holds its kept
// forward pairs in the order of its forward list (the evaluating side
// first), then its kept walls.  Also the wall codes, the range by input
// index for the next call's warm start, the number of slots and the
// statistics row; and, for the gather, the slot codes of the kept pairs its
// partners found (fbase[finder] + kk; -1 - slot where the partner
// evaluates) in increasing finder index in its nbr row, with their number
// in bcount[s]: the backward rows are in the order of the search's atomics,
// the sums must not be.  No atomics; nothing depends on the schedule.
// kEmitG lanes per particle, four entries each (a forward list holds about
// ten entries, a handful of them kept; a backward list about as many, a few
// dozen next to large particles), the backward entries ranked in registers.
// No LDS.  bcount: [n] backward counts, [n] slot offsets,
// the int64 total.
constexpr int kEmitG = 4;
constexpr int kEmitWaves = 4;
constexpr int kEmitPerBlock = kEmitWaves * 64 / kEmitG;

__global__ void __launch_bounds__(64 * kEmitWaves)
k_nbr_emit(CallDesc d, int32_t* __restrict__ bcount, const int32_t* __restrict__ deg,
           const int32_t* __restrict__ slot, const int2* __restrict__ bstage,
           int32_t* __restrict__ nbr, int32_t* __restrict__ wall_slot,
           int32_t* __restrict__ work_s, int32_t* __restrict__ work_t,
           int64_t* __restrict__ stat_nbr, Counters* cnt, const int32_t* __restrict__ orig,
           int2* __restrict__ warm_range) {
  constexpr int G = kEmitG;
  __shared__ int s_cand[kEmitWaves], s_wallc[kEmitWaves], s_deg[kEmitWaves];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int gl = lane % G;
  const int gbase = lane - gl;
  const int s = blockIdx.x * kEmitPerBlock + (int)(threadIdx.x / G);
  const bool live = s < d.n;
  const int maxn = d.max_nbr;
  const int32_t* kbase = bcount + d.n;
  const int64_t total = *reinterpret_cast<const int64_t*>(bcount + 2 * (size_t)d.n);
  // every per-particle word up front, with this lane's first four forward
  // entries (one 16-B load; rows hold max_nbr >= 64 entries, a multiple of
  // 64)
  const size_t rbase = (size_t)(live ? s : 0) * maxn;
  const int nb = live ? bcount[s] : 0;
  const int nf = live ? deg[s] : 0;  // the walk's count (beyond max_nbr: overflow)
  const int base = live ? kbase[s] : 0;
  const int64_t next = live ? (s + 1 < d.n ? (int64_t)kbase[s + 1] : total) : 0;
  const int w0 = live && d.n_walls ? wall_slot[2 * s] : -1;
  const int w1 = live && d.n_walls ? wall_slot[2 * s + 1] : -1;
  const int32_t* sl = slot + rbase;
  const int4 e_first = live ? *reinterpret_cast<const int4*>(sl + 4 * gl) : make_int4(0, 0, 0, 0);
  // and its first four backward entries (two 16-B loads; a bstage row holds
  // max_nbr entries, 16-B aligned)
  const int4 bA = live ? *reinterpret_cast<const int4*>(bstage + rbase + 4 * gl)
                       : make_int4(0, 0, 0, 0);
  const int4 bB = live ? *reinterpret_cast<const int4*>(bstage + rbase + 4 * gl + 2)
                       : make_int4(0, 0, 0, 0);
  const int me = live && warm_range ? orig[s] : 0;
  const int need = (nb < 0 || nf < 0) ? maxn + 1 : nb + nf;
  const bool overflow = live && need > maxn;
  if (overflow && gl == 0) set_error(cnt, LUB_ECAPACITY);
  // the kept forward pairs (the walk counted them over these entries), in
  // chunks of 4 G: four consecutive entries per lane
  const int nfk = live ? min(max(nf, 0), maxn) : 0;
  int at = base;
  for (int k0 = 0; k0 < nfk; k0 += 4 * G) {
    const int kl = k0 + 4 * gl;
    const int4 e4 = k0 == 0 ? e_first : *reinterpret_cast<const int4*>(sl + kl);
    const int ev[4] = {e4.x, e4.y, e4.z, e4.w};
    bool kp[4];
    int c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      kp[j] = kl + j < nfk && (ev[j] & kKeepBit);
      c += kp[j];
    }
    // exclusive prefix of the kept counts over the group's lanes
    int incl = c;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int y = __shfl_up(incl, o, G);
      if (gl >= o) incl += y;
    }
    const int tot = __shfl(incl, gbase + G - 1, 64);
    int sid = at + incl - c;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (kp[j]) {
        if (sid < d.cap_work) {
          const bool own = ev[j] & kOwnBit;
          const int key = ev[j] & kIndexMask;
          work_s[sid] = own ? s : key;
          work_t[sid] = own ? key : s;
        }
        ++sid;
      }
    }
    at += tot;
  }
  int ncand = 0, nwallc = 0;
  if (live) {
    // the kept walls after the kept forward pairs
    if (d.n_walls) {
      if (gl == 0 && !overflow) nwallc = (w0 != -1) + (w1 != -1);
      if (gl < 2 && (gl == 0 ? w0 : w1) == 0) {
        const int code = at + (gl == 1 && w0 == 0 ? 1 : 0);
        if (code < d.cap_work) {
          work_s[code] = s;
          work_t[code] = -1 - gl;
        }
        wall_slot[2 * s + gl] = code;
      }
      at += (w0 == 0) + (w1 == 0);
    }
    // the range holds exactly these (the walk counted the same flags);
    // anything left would get harmless particle-wall slots
    for (int64_t k = at + gl; k < next; k += G)
      if (k < d.cap_work) {
        work_s[k] = s;
        work_t[k] = -1;
      }
    // warm start: this particle's slot range, by input index
    if (warm_range && gl == 0) warm_range[me] = make_int2(base, (int)next);
    if (s == d.n - 1 && gl == 0) {
      cnt->work = (int32_t)min<int64_t>(total, INT32_MAX);
      if (total > d.cap_work) set_error(cnt, LUB_ECAPACITY);
    }
    // each pair is in the forward list of exactly one of its particles
    if (gl == 0 && !overflow) ncand = nf;
  }
  // the partners' kept pairs: each kept entry's rank by finder index among
  // the kept ones (the finders are distinct) is where its slot code goes.
  // Chunks of 4 G entries, four consecutive ones per lane, compared chunk
  // against chunk through shuffles within the group; the first chunk comes
  // with the per-particle words, its finders' slot offsets loaded together.
  const int nbk = live && !overflow ? nb : 0;
  int key0[4], y0[4], kb0[4];  // key: INT32_MAX for a dropped or absent entry
  bool own0[4];
  {
    const int ex[4] = {bA.x, bA.z, bB.x, bB.z};
    const int ey[4] = {bA.y, bA.w, bB.y, bB.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool kp = 4 * gl + j < nbk && (ex[j] & kKeepBit);
      key0[j] = kp ? (ex[j] & kIndexMask) : INT32_MAX;
      kb0[j] = kp ? kbase[key0[j]] : 0;
      y0[j] = ey[j];
      own0[j] = ex[j] & kOwnBit;
    }
  }
  int nkept = 0;
  for (int c1 = 0; c1 < nbk; c1 += 4 * G) {
    int key1[4], y1[4], kb1[4];
    bool own1[4];
    if (c1 == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        key1[j] = key0[j];
        y1[j] = y0[j];
        kb1[j] = kb0[j];
        own1[j] = own0[j];
      }
    } else {
      const int4 u = *reinterpret_cast<const int4*>(bstage + rbase + c1 + 4 * gl);
      const int4 v = *reinterpret_cast<const int4*>(bstage + rbase + c1 + 4 * gl + 2);
      const int ex[4] = {u.x, u.z, v.x, v.z};
      const int ey[4] = {u.y, u.w, v.y, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool kp = c1 + 4 * gl + j < nbk && (ex[j] & kKeepBit);
        key1[j] = kp ? (ex[j] & kIndexMask) : INT32_MAX;
        kb1[j] = kp ? kbase[key1[j]] : 0;
        y1[j] = ey[j];
        own1[j] = ex[j] & kOwnBit;
      }
    }
    int r[4] = {0, 0, 0, 0};
    for (int c2 = 0; c2 < nbk; c2 += 4 * G) {
      int key2[4];
      if (c2 == c1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) key2[j] = key1[j];
      } else if (c2 == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) key2[j] = key0[j];
      } else {
        const int4 u = *reinterpret_cast<const int4*>(bstage + rbase + c2 + 4 * gl);
        const int4 v = *reinterpret_cast<const int4*>(bstage + rbase + c2 + 4 * gl + 2);
        const int ex[4] = {u.x, u.z, v.x, v.z};
#pragma unroll
        for (int j = 0; j < 4; ++j)
          key2[j] = c2 + 4 * gl + j < nbk && (ex[j] & kKeepBit) ? (ex[j] & kIndexMask)
                                                                : INT32_MAX;
      }
      // only the lanes that hold entries of this chunk (a list holds about
      // ten: most chunks end after three lanes)
      const int lanes = min(G, (nbk - c2 + 3) >> 2);
      for (int l = 0; l < lanes; ++l)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int kk = __shfl(key2[jj], gbase + l, 64);
#pragma unroll
          for (int j = 0; j < 4; ++j) r[j] += kk < key1[j];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (key1[j] != INT32_MAX) {
        const int sid = kb1[j] + y1[j];
        nbr[rbase + r[j]] = own1[j] ? sid : -1 - sid;
        ++nkept;
      }
  }
#pragma unroll
  for (int o = 1; o < G; o <<= 1) nkept += __shfl_xor(nkept, o, G);
  if (live && gl == 0) bcount[s] = nkept;
  // the block's statistics row: candidate pairs, wall candidates, the
  // largest number of entries of one particle
  int wc = ncand, ww = nwallc, wd = live && gl == 0 ? need : 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    wc += __shfl_xor(wc, o, 64);
    ww += __shfl_xor(ww, o, 64);
    wd = max(wd, __shfl_xor(wd, o, 64));
  }
  if (lane == 0) {
    s_cand[wv] = wc;
    s_wallc[wv] = ww;
    s_deg[wv] = wd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, w = 0, dg = 0;
    for (int k = 0; k < kEmitWaves; ++k) {
      c += s_cand[k];
      w += s_wallc[k];
      dg = max(dg, s_deg[k]);
    }
    stat_nbr[kStatNbrWords * blockIdx.x] = c;
    stat_nbr[kStatNbrWords * blockIdx.x + 1] = w;
    stat_nbr[kStatNbrWords * blockIdx.x + 2] = dg;
  }
}

}  // namespace

void launch_reset(Counters* c, int32_t* cell_count, int ncell, hipStream_t s) {
  int n = ncell > 128 ? ncell : 128;
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, c,
                     cell_count, ncell);
}

void launch_stage_bin(const CallDesc& d, const double* r, const double* q,
                      const double* semi, const double* v, const double* w,
                      int32_t* cell_id, int32_t* ticket, RecStage* staged,
                      int32_t* cell_count, Counters* cnt, const Counters* gate,
                      hipStream_t s, int32_t* bcount) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_stage_bin, dim3((d.n + kBinThreads - 1) / kBinThreads),
                     dim3(kBinThreads), 0, s, d,
                     r, q, semi, v, w, cell_id, ticket, staged, cell_count, cnt, gate,
                     bcount);
}

void launch_scan(const int32_t* in, int32_t* out, int n, int32_t* block_sums,
                 int64_t* total, hipStream_t s) {
  int nb = (n + kScanTile - 1) / kScanTile;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(kScanThreads), 0, s, in, out,
                     n, block_sums, total);
  if (nb > 1)
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kAddThreads), 0, s, out, n, block_sums,
                       nb, total);
}

void launch_cell_scatter(const CallDesc& d, const int32_t* cell_id, const int32_t* ticket,
                         const int32_t* cell_start, int32_t* unsorted, int32_t* cell_sorted,
                         int32_t* cell_count, int ncell, const Counters* gate,
                         hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_cell_scatter, dim3((d.n + 255) / 256), dim3(256), 0, s,
                     d, cell_id, ticket, cell_start, unsorted, cell_sorted, cell_count,
                     ncell, gate);
}

void launch_build_records(const CallDesc& d, const int32_t* unsorted,
                          const int32_t* cell_sorted, const int32_t* cell_start,
                          const RecStage* staged, int32_t* sorted, PRec* rec,
                          PRecP* recp, double4* pos, KRec* kin, const Counters* gate,
                          hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_build_records, dim3((d.n + kBuildThreads - 1) / kBuildThreads),
                     dim3(kBuildThreads), 0, s,
                     d, unsorted, cell_sorted, cell_start, staged, sorted, rec, recp, pos,
                     kin, gate);
}

bool cells_small_fits(const CallDesc& d) {
  const int64_t nbins = 2 * (int64_t)d.nc[0] * d.nc[1] * d.nc[2];
  return d.n <= kSmallMaxN && nbins <= kSmallMaxCells;
}

void launch_cells_small(const CallDesc& d, const double* r, const double* q,
                        const double* semi, const double* v, const double* w,
                        int32_t* cell_start, int32_t* sorted, PRec* rec, PRecP* recp,
                        double4* pos,
                        KRec* kin, int32_t* cell_sorted, Counters* cnt, const Counters* gate,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_cells_small, dim3(1), dim3(kSmallThreads), 0, s, d, r, q, semi,
                     v, w, cell_start, sorted, rec, recp, pos, kin, cell_sorted, cnt, gate);
  if (d.n > kSmallRecN)
    hipLaunchKernelGGL(k_records_sorted, dim3((d.n + 255) / 256), dim3(256), 0, s, d, sorted,
                       r, q, semi, v, w, rec, recp, pos, kin, gate);
}

int nbr_waves(const CallDesc& d);  // wavefronts per block of the neighbour kernel
int nbr_blocks_group(const CallDesc& d);
bool nbr_flat(const CallDesc& d);
bool nbr_forward(const CallDesc& d, const int32_t* bcount, const int32_t* block_sums,
                 const int2* bstage);
int nbr_blocks_flat(const CallDesc& d);

template <int G, int W>
void launch_nbr_mode(int mode, dim3 grid, size_t lds, hipStream_t s, const CallDesc& d,
                     const PRec* rec, const double4* pos, const int32_t* orig,
                     const int32_t* cell_sorted, const int32_t* cell_start, int32_t* deg,
                     int32_t* nbr, int32_t* slot, int32_t* wall_slot, int32_t* work_s,
                     int32_t* work_t, int64_t* stat_nbr, Counters* cnt, const ListBufs& lb) {
  if (mode == 0)
    hipLaunchKernelGGL((k_neighbors<G, 0, W>), grid, dim3(64 * W), lds, s, d, rec, pos, orig,
                       cell_sorted, cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                       stat_nbr, cnt, lb);
  else if (mode == 1)
    hipLaunchKernelGGL((k_neighbors<G, 1, W>), grid, dim3(64 * W), lds, s, d, rec, pos, orig,
                       cell_sorted, cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                       stat_nbr, cnt, lb);
  else
    hipLaunchKernelGGL((k_neighbors<G, 2, W>), grid, dim3(64 * W), lds, s, d, rec, pos, orig,
                       cell_sorted, cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                       stat_nbr, cnt, lb);
}

template <int G>
void launch_nbr_waves(int mode, dim3 grid, size_t lds, hipStream_t s, const CallDesc& d,
                      const PRec* rec, const double4* pos, const int32_t* orig,
                      const int32_t* cell_sorted, const int32_t* cell_start, int32_t* deg,
                      int32_t* nbr, int32_t* slot, int32_t* wall_slot, int32_t* work_s,
                      int32_t* work_t, int64_t* stat_nbr, Counters* cnt, const ListBufs& lb) {
  if (nbr_waves(d) == kWavesLarge)
    launch_nbr_mode<G, kWavesLarge>(mode, grid, lds, s, d, rec, pos, orig, cell_sorted,
                                    cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                                    stat_nbr, cnt, lb);
  else
    launch_nbr_mode<G, kWavesSmall>(mode, grid, lds, s, d, rec, pos, orig, cell_sorted,
                                    cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                                    stat_nbr, cnt, lb);
}

void launch_neighbors_wave(const CallDesc& d, const PRec* rec, const PRecP* recp,
                           const double4* pos, const int32_t* orig, const int32_t* cell_sorted,
                           const int32_t* cell_start, int32_t* deg,
                           int32_t* nbr, int32_t* slot, int32_t* wall_slot,
                           int32_t* work_s, int32_t* work_t, int64_t* stat_nbr,
                           Counters* cnt, hipStream_t s, int mode, const ListBufs* lists,
                           int32_t* bcount, int32_t* block_sums, int2* bstage,
                           hipEvent_t ev_start, hipEvent_t ev_stop) {
  const ListBufs lb = lists ? *lists : ListBufs{};
  if (d.n == 0) return;
  if (mode != 2 && nbr_flat(d)) {
    const dim3 grid_f(nbr_blocks_flat(d)), block_f(64 * kFlatWaves);
    if (mode == 0 && nbr_forward(d, bcount, block_sums, bstage)) {
      const size_t lds_f = sizeof(int32_t) * kFlatWaves * (64 / kFlatG) * (size_t)d.max_nbr;
      hipExtLaunchKernelGGL(k_neighbors_flat<kFwd>, grid_f, block_f, lds_f, s, ev_start,
                            ev_stop, 0, d, rec, recp, pos, orig, cell_sorted, cell_start, deg,
                            nbr, slot, wall_slot, work_s, work_t, stat_nbr, cnt, lb, bcount,
                            bstage);
      int32_t* kcnt = bcount + d.n;
      launch_scan(kcnt, kcnt, d.n, block_sums,
                  reinterpret_cast<int64_t*>(bcount + 2 * (size_t)d.n), s);
      hipLaunchKernelGGL(k_nbr_emit, dim3((d.n + kEmitPerBlock - 1) / kEmitPerBlock),
                         dim3(64 * kEmitWaves), 0, s, d, bcount, deg, slot, bstage, nbr,
                         wall_slot, work_s, work_t, stat_nbr, cnt, orig, lb.warm_range);
    } else if (mode == 0) {
      hipExtLaunchKernelGGL(k_neighbors_flat<0>, grid_f, block_f, 0, s, ev_start, ev_stop, 0,
                            d, rec, recp, pos, orig, cell_sorted, cell_start, deg, nbr, slot,
                            wall_slot, work_s, work_t, stat_nbr, cnt, lb, nullptr, nullptr);
    } else {
      hipLaunchKernelGGL(k_neighbors_flat<1>, grid_f, block_f, 0, s, d, rec, recp, pos, orig,
                         cell_sorted, cell_start, deg, nbr, slot, wall_slot, work_s, work_t,
                         stat_nbr, cnt, lb, nullptr, nullptr);
    }
    return;
  }
  dim3 grid(nbr_blocks_group(d));
  size_t lds = sizeof(int32_t) * 64 * nbr_waves(d) / nbr_group(d) * (size_t)d.max_nbr;
  if (mode == 2 && lists && lists->work_sup) lds *= 2;  // the superset positions too
  // (the lane-group kernels take stream-ordered stamps around their launch)
  if (ev_start) (void)hipEventRecord(ev_start, s);  // timing only
  if (nbr_group(d) == 16)
    launch_nbr_waves<16>(mode, grid, lds, s, d, rec, pos, orig, cell_sorted, cell_start, deg,
                        nbr, slot, wall_slot, work_s, work_t, stat_nbr, cnt, lb);
  else if (nbr_group(d) == 32)
    launch_nbr_waves<32>(mode, grid, lds, s, d, rec, pos, orig, cell_sorted, cell_start, deg,
                        nbr, slot, wall_slot, work_s, work_t, stat_nbr, cnt, lb);
  else
    launch_nbr_waves<64>(mode, grid, lds, s, d, rec, pos, orig, cell_sorted, cell_start, deg,
                        nbr, slot, wall_slot, work_s, work_t, stat_nbr, cnt, lb);
  if (ev_stop) (void)hipEventRecord(ev_stop, s);
}

namespace {

constexpr int kDispThreads = 256;

// Reused neighbour lists: the largest of |displacement since the search|
// (the nearest image of the current centre seen from the centre at the
// search, with the current Lees-Edwards offset) + growth of R_max since the
// search, per block of particles in input order, into lb.disp_blk.  An input that the search
// would reject counts as infinite, so that the search runs and reports it.
// Lists of another epoch (or none) are not measured.
__global__ void __launch_bounds__(kDispThreads)
k_disp(CallDesc d, const double* __restrict__ r, const double* __restrict__ q,
       const double* __restrict__ semi, ListBufs lb) {
  __shared__ double s_max[kDispThreads / 64];
  if (lb.state->epoch != d.list_epoch) return;
  const int p = blockIdx.x * kDispThreads + threadIdx.x;
  double m = 0.0;
  if (p < d.n) {
    const double4 o = lb.ref_pos[p];
    const double r0[3] = {o.x, o.y, o.z};
    const double r1[3] = {r[3 * p], r[3 * p + 1], r[3 * p + 2]};
    double u[3];
    pair_image(d, r0, r1, u);
    const double grow = fmax(semi[2 * p], semi[2 * p + 1]) - o.w;
    m = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + (grow > 0.0 ? grow : 0.0);
    if (!isfinite(m) || input_faults(d, r, q, semi, p) != 0) m = INFINITY;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = s_max[0];
    for (int k = 1; k < kDispThreads / 64; ++k) b = fmax(b, s_max[k]);
    lb.disp_blk[blockIdx.x] = b;
  }
}

// The call's decision: search when the lists are of another epoch or when
// 2 (largest displacement + growth) + |change of the Lees-Edwards offset
// since the search| exceeds the skin (the margin keeps a rounding of the
// measure from deciding).  Every pair within the bound now was then within
// the bound + skin at the search: writing each centre as its centre at the
// search plus its displacement plus a lattice vector of the current images,
// the pair's image vector differs from one at the search by the two
// displacements and at most one box's change of offset (the images in
// question are the nearest in z), and the bound grew by at most the two
// growths.  One block.
__global__ void __launch_bounds__(kDispThreads)
k_decide(CallDesc d, ListBufs lb, Counters* cnt) {
  __shared__ double s_max[kDispThreads / 64];
  const bool same = lb.state->epoch == d.list_epoch;
  double m = 0.0;
  if (same) {
    const int nb = (d.n + kDispThreads - 1) / kDispThreads;
    for (int k = threadIdx.x; k < nb; k += kDispThreads) m = fmax(m, lb.disp_blk[k]);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < kDispThreads / 64; ++k) m = fmax(m, s_max[k]);
  double shear = 0.0;
  if (d.le && same)
    shear = fabs(min_image(d.le_offset - lb.state->le_offset, d.L[0], d.invL[0]));
  const bool search = !same || !(2.0 * m + shear <= d.skin * (1.0 - 1e-12));
  cnt->rebuild = search ? 1 : 0;
  if (search) {
    lb.state->epoch = d.list_epoch;
    lb.state->builds += 1;
    lb.state->le_offset = d.le_offset;
  }
}

// records of the current inputs in the cell order of the last search (calls
// that reuse the lists only): read in input order, written to their places
__global__ void k_refresh(CallDesc d, const double* __restrict__ r,
                          const double* __restrict__ q, const double* __restrict__ semi,
                          const double* __restrict__ v, const double* __restrict__ w,
                          ListBufs lb, PRec* __restrict__ rec, PRecP* __restrict__ recp,
                          double4* __restrict__ pos,
                          KRec* __restrict__ kin, const Counters* cnt) {
  if (cnt->rebuild) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.n) return;
  make_record(lb.inv[p], p, r, q, semi, v, w, rec, recp, pos, kin);
}

}  // namespace

void launch_disp(const CallDesc& d, const double* r, const double* q, const double* semi,
                 const ListBufs& lists, Counters* cnt, hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_disp, dim3((d.n + kDispThreads - 1) / kDispThreads), dim3(kDispThreads),
                     0, s, d, r, q, semi, lists);
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDispThreads), 0, s, d, lists, cnt);
}

void launch_refresh(const CallDesc& d, const double* r, const double* q, const double* semi,
                    const double* v, const double* w, const ListBufs& lists, PRec* rec,
                    PRecP* recp, double4* pos, KRec* kin, const Counters* cnt, hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_refresh, dim3((d.n + 255) / 256), dim3(256), 0, s, d, r, q, semi, v, w,
                     lists, rec, recp, pos, kin, cnt);
}

// lanes per particle: the smallest group whose lanes hold the segment at 8
// entries per lane (more lanes for small systems measured slower)
int nbr_group(const CallDesc& d) {
  return d.max_nbr <= 8 * 16 ? 16 : (d.max_nbr <= 8 * 32 ? 32 : 64);
}

// (the superset search and filter of reused lists measured faster with 8)
int nbr_waves(const CallDesc& d) {
  return d.n >= (1 << 14) && !(d.skin > 0.0) ? kWavesLarge : kWavesSmall;
}

// blocks of the lane-group kernel (the filter of reused lists, Lees-Edwards
// images)
int nbr_blocks_group(const CallDesc& d) {
  const int per_block = nbr_waves(d) * 64 / nbr_group(d);
  return (d.n + per_block - 1) / per_block;
}

// blocks of the flattened search
int nbr_blocks_flat(const CallDesc& d) {
  constexpr int per_block = kFlatWaves * 64 / kFlatG;
  return (d.n + per_block - 1) / per_block;
}

// the search and the superset of reused lists without Lees-Edwards images
// go through the flattened kernel
bool nbr_flat(const CallDesc& d) { return !d.le; }

// the full search of large systems as forward search + evaluation list
// (needs the backward counts, zeroed by the binning kernel)
bool nbr_forward(const CallDesc& d, const int32_t* bcount, const int32_t* block_sums,
                 const int2* bstage) {
  return bcount != nullptr && block_sums != nullptr && bstage != nullptr && !d.le &&
         d.n >= kFwdMinN &&
         d.n <= kIndexMask &&
         d.max_nbr <= kFwdMaxNbr;
}

// blocks of the kernel that writes a call's statistics rows: the filter of
// reused lists, the Lees-Edwards search, the evaluation list of the forward
// search, else the flattened search
int nbr_blocks(const CallDesc& d) {
  if (d.partner_codes == kPartnerRanges) return (d.n + kEmitPerBlock - 1) / kEmitPerBlock;
  return d.skin > 0.0 || !nbr_flat(d) ? nbr_blocks_group(d) : nbr_blocks_flat(d);
}

// at least one particle per wavefront, at most kWavesLarge wavefronts
int nbr_blocks_max(int n) { return (n + kWavesLarge - 1) / kWavesLarge; }

}  // namespace lub
