// lub_gather.hip -- per-particle sums of the pair forces and torques
// (gfx950).  Sec. III.B: particle i receives f_i = F and t_i = T + (y_i -
// r_i) x F from every pair, particle j the opposite force and -T + ... about
// its own centre.
//
// No atomics: a group of 16 (large systems: 8) lanes per particle, lanes
// over the entries of its neighbour segment (both directions of each of its
// pairs).  A pair's result sits in the slot of the entry owned by its
// smaller-index particle; the other particle reads it through the slot code
// written into its own entry beside the pair kernel (large systems) or finds
// that entry by binary search in its partner's sorted segment.  After the
// forward search there are no segments: each particle sums its own slot
// range and then, in increasing finder index, the pairs its partners found.
// The group then reduces the six components with a fixed butterfly in FP64,
// so the sums are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include "lub_internal.h"

namespace lub {

namespace {

#ifndef LUB_GATHER_WAVES
#define LUB_GATHER_WAVES 4
#endif
constexpr int kWaves = LUB_GATHER_WAVES;

__device__ __forceinline__ int find_entry(const int32_t* __restrict__ seg, int n,
                                          int key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int v = seg[mid];
    if (v == key) return mid;
    if (v < key)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// lanes per particle (template G): the segments hold about ten to twenty
// entries in dense suspensions.  16 lanes (four particles per wavefront)
// for small systems, where the launch is latency-bound; 8 from about a
// quarter million particles, where two entries per lane keep more loads in
// flight per wavefront (measured: 220 -> 180 us at a million particles,
// slower below)
constexpr int kGroupLarge = 8;
constexpr int kGroupSmall = 16;

// For every evaluated particle pair (slot w, owner s, partner t): the
// position of s in t's sorted segment, where the entry's code becomes
// -3 - w, so that the gather reads the partner's result without a search.
// Entries of pairs the owner did not evaluate keep -2.  Runs beside the
// pair kernel (it reads only the neighbour kernel's output).
__global__ void k_partner_slots(CallDesc d, const int32_t* __restrict__ work_s,
                                const int32_t* __restrict__ work_t,
                                const int32_t* __restrict__ deg,
                                const int32_t* __restrict__ nbr, int32_t* __restrict__ slot,
                                const Counters* cnt) {
  const int nwork = cnt->error == 0 ? min(cnt->work, d.cap_work) : 0;
  const size_t stride = (size_t)d.max_nbr;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nwork;
       w += gridDim.x * blockDim.x) {
    const int t = work_t[w];
    if (t < 0) continue;  // wall slot
    const int s = work_s[w];
    const int kk = find_entry(nbr + (size_t)t * stride, deg[t], s);
    if (kk >= 0) slot[(size_t)t * stride + kk] = -3 - w;
  }
}

// One pair's terms for one of its particles: +F and T_i for the first
// (evaluating) particle, -F and T_j for the other.  The whole record is
// loaded before the side is chosen, so that its loads go out together.
template <typename R>
__device__ __forceinline__ void add_pair(double* acc, const PairOut<R>& o, bool first) {
  R F[3], Ti[3], Tj[3];
  for (int c = 0; c < 3; ++c) {
    F[c] = o.F[c];
    Ti[c] = o.Ti[c];
    Tj[c] = o.Tj[c];
  }
  for (int c = 0; c < 3; ++c) {
    const double fc = (double)F[c];
    acc[c] += first ? fc : -fc;
    acc[3 + c] += (double)(first ? Ti[c] : Tj[c]);
  }
}

template <typename R, int kGroup>
__global__ void __launch_bounds__(64 * kWaves) k_gather(
    CallDesc d, const int32_t* __restrict__ orig, const int32_t* __restrict__ deg,
    const int32_t* __restrict__ nbr, const int32_t* __restrict__ slot,
    const int32_t* __restrict__ wall_slot, const PairOut<R>* __restrict__ out,
    const Counters* cnt, Counters* __restrict__ next_cnt, double* __restrict__ f,
    double* __restrict__ t) {
  constexpr int kPerWave = 64 / kGroup;
  const int lane = threadIdx.x & 63;
  const int g = lane % kGroup;  // lane within the particle's group
  const int s = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * kPerWave + lane / kGroup;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < (int)(sizeof(Counters) / sizeof(int32_t));
         i += blockDim.x)
      reinterpret_cast<int32_t*>(next_cnt)[i] = 0;
  const bool live = s < d.n;
  const size_t stride = (size_t)d.max_nbr;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  // this lane's first slot code and wall slot, loaded beside the count
  // (a segment row holds max_nbr >= kGroup entries): one dependent load less
  const int sl_first = live ? slot[(size_t)s * stride + g] : 0;
  const int ws = live && d.n_walls && g >= kGroup - 2 ? wall_slot[2 * s + (g - (kGroup - 2))]
                                                      : -1;
  if (live && cnt->error == 0) {
    const int ns = deg[s];
    for (int k = g; k < ns; k += kGroup) {
      const size_t e = (size_t)s * stride + k;
      const int sl = k == g ? sl_first : slot[e];
      // this particle's own slot, or the partner's (its slot code written
      // by k_partner_slots, or found in the partner's sorted segment)
      int w = sl;
      if (sl <= -3) {
        w = -3 - sl;
      } else if (sl == -2 && d.partner_codes == kPartnerSearch) {
        const int p = nbr[e];
        const int kk = find_entry(nbr + (size_t)p * stride, deg[p], s);
        w = kk >= 0 ? slot[(size_t)p * stride + kk] : -1;
      }
      if (w >= 0) add_pair(acc, out[w], sl >= 0);
    }
    if (d.n_walls && g >= kGroup - 2 && ws >= 0) add_pair(acc, out[ws], true);
  }
  // fixed butterfly within each group of kGroup lanes
#pragma unroll
  for (int o = kGroup / 2; o >= 1; o >>= 1)
    for (int c = 0; c < 6; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
  if (live && g == 0) {
    const int p = orig[s];
    for (int c = 0; c < 3; ++c) {
      f[3 * p + c] = acc[c];
      t[3 * p + c] = acc[3 + c];
    }
  }
}

// After the forward search (large systems): a particle's evaluation slots
// [fbase[s], fbase[s + 1]) hold the pairs its forward search found (work_s
// names the evaluating side) and its walls; the slot codes of the pairs its
// partners found (slot where this particle evaluates, else -1 - slot) are
// in its nbr row in increasing finder index, bcount[s] of them.  A group
// sums the own range in slot order, then those codes in row order: sums
// that do not depend on the search's schedule.
constexpr int kRangeGroup = 8;
constexpr int kRangeWaves = 4;
constexpr int kRangePerBlock = kRangeWaves * 64 / kRangeGroup;

template <typename R>
__global__ void __launch_bounds__(64 * kRangeWaves) k_gather_ranges(
    CallDesc d, const int32_t* __restrict__ orig, const int32_t* __restrict__ bcount,
    const int32_t* __restrict__ nbr, const int32_t* __restrict__ work_s,
    const PairOut<R>* __restrict__ out, const Counters* cnt,
    Counters* __restrict__ next_cnt, double* __restrict__ f, double* __restrict__ t) {
  constexpr int G = kRangeGroup;
  const int lane = threadIdx.x & 63;
  const int g = lane % G;
  const int s = blockIdx.x * kRangePerBlock + (int)(threadIdx.x / G);
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < (int)(sizeof(Counters) / sizeof(int32_t));
         i += blockDim.x)
      reinterpret_cast<int32_t*>(next_cnt)[i] = 0;
  const bool live = s < d.n;
  // without an error every slot lies below the capacity (the search checked)
  const bool ok = live && cnt->error == 0;
  const int maxn = d.max_nbr;
  const int32_t* kbase = bcount + d.n;
  // the per-particle words and this lane's first two codes up front (a row
  // holds max_nbr >= 2 kRangeGroup entries; those past the count are not
  // used): one round of loads, then one for the records
  const size_t rbase = (size_t)(ok ? s : 0) * maxn;
  const int nk = ok ? bcount[s] : 0;
  const int base = ok ? kbase[s] : 0;
  const int next =
      ok ? (s + 1 < d.n ? kbase[s + 1]
                        : (int)*reinterpret_cast<const int64_t*>(bcount + 2 * (size_t)d.n))
         : 0;
  const int p = live ? orig[s] : 0;
  const int c0 = ok ? nbr[rbase + g] : 0;
  const int c1 = ok ? nbr[rbase + g + G] : 0;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  // the own range: pairs this particle found (either side evaluates) and
  // its walls; the evaluating side of each is work_s (s itself for a wall)
  for (int w = base + g; w < next; w += G) add_pair(acc, out[w], work_s[w] == s);
  // the pairs its partners found
  for (int r = g; r < nk; r += G) {
    const int c = r < G ? c0 : r < 2 * G ? c1 : nbr[rbase + r];
    const int w = c >= 0 ? c : -1 - c;
    if (w < d.cap_work) add_pair(acc, out[w], c >= 0);
  }
  // fixed butterfly within each group
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1)
    for (int c = 0; c < 6; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
  if (live && g == 0) {
    for (int c = 0; c < 3; ++c) {
      f[3 * p + c] = acc[c];
      t[3 * p + c] = acc[3 + c];
    }
  }
}

}  // namespace

void launch_partner_slots(const CallDesc& d, const int32_t* work_s, const int32_t* work_t,
                          const int32_t* deg, const int32_t* nbr, int32_t* slot,
                          const Counters* cnt, hipStream_t s) {
  int blocks = (d.cap_work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_partner_slots, dim3(blocks), dim3(256), 0, s, d, work_s, work_t, deg,
                     nbr, slot, cnt);
}

void launch_gather(const CallDesc& d, const int32_t* orig, const int32_t* deg,
                   const int32_t* nbr, const int32_t* slot,
                   const int32_t* wall_slot, const void* out,
                   const Counters* cnt, Counters* next_cnt, double* f, double* t,
                   hipStream_t s, const int32_t* bcount, const int32_t* work_s) {
  if (d.n == 0) return;
  if (d.partner_codes == kPartnerRanges) {
    const dim3 grid((d.n + kRangePerBlock - 1) / kRangePerBlock), block(64 * kRangeWaves);
    if (d.precision == LUB_MIXED)
      hipLaunchKernelGGL(k_gather_ranges<float>, grid, block, 0, s, d, orig, bcount, nbr,
                         work_s, (const PairOut<float>*)out, cnt, next_cnt, f, t);
    else
      hipLaunchKernelGGL(k_gather_ranges<double>, grid, block, 0, s, d, orig, bcount, nbr,
                         work_s, (const PairOut<double>*)out, cnt, next_cnt, f, t);
    return;
  }
  const bool large = d.n >= (1 << 18);
  const int per_block = kWaves * (64 / (large ? kGroupLarge : kGroupSmall));
  dim3 grid((d.n + per_block - 1) / per_block);
  const dim3 block(64 * kWaves);
  if (d.precision == LUB_MIXED) {
    const PairOut<float>* o = (const PairOut<float>*)out;
    if (large)
      hipLaunchKernelGGL((k_gather<float, kGroupLarge>), grid, block, 0, s, d, orig, deg, nbr,
                         slot, wall_slot, o, cnt, next_cnt, f, t);
    else
      hipLaunchKernelGGL((k_gather<float, kGroupSmall>), grid, block, 0, s, d, orig, deg, nbr,
                         slot, wall_slot, o, cnt, next_cnt, f, t);
  } else {
    const PairOut<double>* o = (const PairOut<double>*)out;
    if (large)
      hipLaunchKernelGGL((k_gather<double, kGroupLarge>), grid, block, 0, s, d, orig, deg, nbr,
                         slot, wall_slot, o, cnt, next_cnt, f, t);
    else
      hipLaunchKernelGGL((k_gather<double, kGroupSmall>), grid, block, 0, s, d, orig, deg, nbr,
                         slot, wall_slot, o, cnt, next_cnt, f, t);
  }
}

namespace {

// One block per statistic: the sum (or, for the largest iteration count,
// the maximum) of that word over the rows the last call's blocks wrote.
// Each thread keeps four loads in flight (the rows are strided, so the
// block is bound by the latency of its loads, not by their bytes).
constexpr int kReduceThreads = 1024;
constexpr int kReduceUnroll = 4;

__device__ __forceinline__ int64_t stat_combine(bool is_max, int64_t a, int64_t b) {
  return is_max ? max(a, b) : a + b;
}

__global__ void __launch_bounds__(kReduceThreads)
k_stats_reduce(Counters* cnt, const int64_t* __restrict__ stat_pair, int pair_blocks,
               const int64_t* __restrict__ stat_nbr, int nbr_rows, int cap_work) {
  __shared__ int64_t part[kReduceThreads / 64];
  const int word = blockIdx.x;
  int rows, stride;
  const int64_t* base;
  if (word < kStatPairWords) {
    const int nwork = cnt->error == 0 ? min(cnt->work, cap_work) : 0;
    rows = min(pair_blocks, (nwork + 63) / 64);
    base = stat_pair + word;
    stride = kStatPairWords;
  } else {
    rows = nbr_rows;
    base = stat_nbr + (word - kStatPairWords);
    stride = kStatNbrWords;
  }
  const bool is_max = word == 6 || word == kStatPairWords + 2;
  int64_t a[kReduceUnroll] = {};
  int r = threadIdx.x;
  for (; r + (kReduceUnroll - 1) * kReduceThreads < rows; r += kReduceUnroll * kReduceThreads) {
    int64_t v[kReduceUnroll];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u)
      v[u] = base[(int64_t)(r + u * kReduceThreads) * stride];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) a[u] = stat_combine(is_max, a[u], v[u]);
  }
  for (; r < rows; r += kReduceThreads) a[0] = stat_combine(is_max, a[0], base[(int64_t)r * stride]);
  int64_t acc = a[0];
#pragma unroll
  for (int u = 1; u < kReduceUnroll; ++u) acc = stat_combine(is_max, acc, a[u]);
  if (word < kStatPairWords) {
    // the rows of the tangent-sphere pass
    const int nfail = cnt->error == 0 ? min(cnt->failed, cap_work) : 0;
    const int trows = min(kTangentBlocks, (nfail + 63) / 64);
    for (int r = threadIdx.x; r < trows; r += kReduceThreads) {
      const int64_t v = base[(int64_t)(kMaxPairBlocks + r) * stride];
      acc = is_max ? max(acc, v) : acc + v;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t y = __shfl_xor(acc, o, 64);
    acc = is_max ? max(acc, y) : acc + y;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < kReduceThreads / 64; ++k) acc = is_max ? max(acc, part[k]) : acc + part[k];
  switch (word) {
    case 0: cnt->newton_iters = acc; break;
    case 1: cnt->active = acc; break;
    case 2: cnt->overlaps = acc; break;
    case 3: cnt->unresolved = acc; break;
    case 4: cnt->unconverged = acc; break;
    case 5: cnt->fallbacks = acc; break;
    case 6: cnt->newton_max = (int32_t)acc; break;
    case 7: cnt->warm_seeded = acc; break;
    case kStatPairWords: cnt->candidates = acc; break;
    case kStatPairWords + 1: cnt->wall_candidates = acc; break;
    case kStatPairWords + 2: cnt->max_degree = acc; break;
    default: cnt->iter_hist[word - 8] = acc; break;
  }
}

}  // namespace

void launch_stats_reduce(const CallDesc& d, Counters* cnt, const int64_t* stat_pair,
                         const int64_t* stat_nbr, hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_stats_reduce, dim3(kStatPairWords + kStatNbrWords),
                     dim3(kReduceThreads), 0, s, cnt, stat_pair, pair_grid(d), stat_nbr,
                     nbr_blocks(d), d.cap_work);
}

}  // namespace lub
