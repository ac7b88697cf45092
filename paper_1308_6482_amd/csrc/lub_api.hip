// lub_api.hip -- the C ABI declared in include/lub.h: handle, device
// workspace, the launch sequence of one evaluation, statistics and the
// diagnostic read-backs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lub_internal.h"

using namespace lub;

struct lub_ctx {
  int device = 0;
  lub_params_t prm{};
  lub_domain_t dom{};
  lub_opts_t opt{};
  hipStream_t last_stream = nullptr;
  CallDesc last{};
  bool have_last = false;
  // a second stream (default priority) for the partner-slot codes, forked
  // from the call's stream after the neighbour lists and joined before the
  // gather
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // reused neighbour lists (opts.skin > 0): the superset segments of the
  // last search in its cell order, the positions and sizes at the search,
  // the device-side state (epoch of the lists, searches), and the host's
  // epoch: any change that makes the lists unusable starts a new one
  int32_t* sup_nbr = nullptr;
  int32_t* sup_deg = nullptr;
  double4* ref_pos = nullptr;
  int32_t* inv = nullptr;
  double* disp_blk = nullptr;
  ListState* list_state = nullptr;
  // warm start with reused lists: per superset entry the last normal, per
  // evaluation slot its superset entry
  float4* sup_val = nullptr;
  int32_t* work_sup = nullptr;
  int32_t list_epoch = 0;
  int64_t epoch_n = -1;
  int32_t epoch_stride = 0;
  int64_t list_builds = 0;  // searches without reuse (counted on the host)

  // workspace
  int64_t cap_n = 0, cap_cells = 0, cap_entries = 0, cap_work = 0, cap_bs = 0;
  int32_t cur_nbr = 64;            // neighbour-segment stride in use
  int32_t* cell_id = nullptr;      // [n] by input index
  int32_t* cell_count = nullptr;   // [ncell]
  int32_t* cell_start = nullptr;   // [ncell + 1]
  int32_t* sorted = nullptr;       // [n] cell order -> input index
  int32_t* scat = nullptr;         // [n] scatter output (cell ranges, any order)
  int64_t* stat_nbr = nullptr;     // [neighbour blocks][kStatNbrWords]
  int64_t* stat_pair = nullptr;    // [kMaxPairBlocks][kStatPairWords]
  // warm start: two tables of (pair key, converged normal), the one of
  // counter set p written by calls using set p, read by the next call
  // warm start, two sets swapped between calls: per input index the slot
  // range of its pairs, per slot the normal and the partner's input index
  int2* warm_range[2] = {nullptr, nullptr};
  float4* warm_val[2] = {nullptr, nullptr};
  int32_t* cell_sorted = nullptr;  // [n] cell of each cell-order particle
  int32_t* deg = nullptr;          // [n] entries per segment
  int2* bstage = nullptr;          // [n * cur_nbr] forward search: backward entries
                                   // with their place in the finder's slot range
  int32_t* bcount = nullptr;       // [2n + 2] forward search: backward entries, slot
                                   // offsets, their int64 total
  int32_t* block_sums = nullptr;   // scan scratch
  int32_t* wall_slot = nullptr;    // [2n]
  PRec* rec = nullptr;             // [n]
  PRecP* recp = nullptr;           // [n] the pair kernels' copy
  double4* pos = nullptr;          // [n] centre and largest semi-axis (centre test)
  KRec* kin = nullptr;             // [n]
  RecStage* staged = nullptr;      // [n] record copies in input order (binning)
  int32_t* nbr = nullptr;          // [n * cur_nbr] partner (cell order)
  int32_t* slot = nullptr;         // [n * cur_nbr] evaluation slot, -1, -2
  int32_t* work_s = nullptr;       // [work]
  int32_t* fail_list = nullptr;    // [work] slots left to the tangent-sphere pass
  int32_t* out_links = nullptr;    // [work] link-wise laws: contributing links
  int32_t* work_t = nullptr;       // [work]
  void* out = nullptr;             // [work] PairOut<double> (or float)
  double* out_h = nullptr;         // [work]
  int8_t* out_status = nullptr;    // [work]
  uint8_t* out_iters = nullptr;    // [work]
  // Two sets of device counters, used by alternate calls: the last kernel
  // of a call zeroes the other set, and the scatter zeroes the cell counts,
  // so a call needs no reset launch when the previous one ran to the end
  // (`zeroed`).
  Counters* cnt_buf = nullptr;     // device [2]
  Counters* cnt = nullptr;         // the set of the current / last call
  int cnt_idx = 0;
  bool zeroed = false;
  Counters* host_cnt = nullptr;    // pinned

  // learned seed: FP32 master weights, Adam moments, gradient, packed BF16
  // operands, training scratch and the per-slot features / outputs
  float* th = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* grad = nullptr;
  __bf16* wt = nullptr;
  __bf16* wb = nullptr;
  float* dloss = nullptr;          // device loss accumulator(s)
  float* loss_parts = nullptr;
  int64_t cap_batch = 0;
  __bf16* aT = nullptr;
  __bf16* dT = nullptr;
  int64_t cap_seed = 0;
  float* seedX = nullptr;
  float* seedY = nullptr;
  // host-pointer mode: device copies of the inputs (15 n doubles: r, q,
  // semi, v, w) and of the outputs (6 n: f, t)
  double* detail = nullptr;        // [work][kDetailWords] with opts.record_detail
  double* stage_in = nullptr;
  double* stage_out = nullptr;
  int64_t cap_stage = 0;
  // growth stage: scaled semi-axes and the forces of each sub-step
  double* grow_semi = nullptr;
  double* grow_f = nullptr;
  double* grow_t = nullptr;
  int64_t cap_grow = 0;
  int adam_step = 0;

  // graph mode: the launch sequence of a call, captured once per counter set
  // (alternate calls use alternate sets) and replayed while the call's
  // arguments and the workspace stay the same
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    int64_t n = -1;
    const void* args[8] = {};
    CallDesc d{};
    std::vector<const void*> ws;
  };
  GraphSlot graphs[2];

  // stage timing: five stage events and the pair kernel's own start and
  // stop per timed call, resolved lazily
  std::vector<hipEvent_t> free_events;
  std::vector<std::vector<hipEvent_t>> pending;
  int64_t timed_calls = 0;
  double stage_ms[4] = {0, 0, 0, 0};
  double pair_kernel_ms = 0.0;
  double search_kernel_ms = 0.0;
};

namespace {

constexpr int32_t kMaxNbr = 512;  // largest neighbour segment (8 entries per lane)

int hip_err(hipError_t e) {
  if (e == hipSuccess) return LUB_OK;
  if (e == hipErrorOutOfMemory) return LUB_ENOMEM;
  return LUB_EDEVICE;
}

#define HIP_TRY(x)                        \
  do {                                    \
    int _rc = hip_err(x);                 \
    if (_rc != LUB_OK) return _rc;        \
  } while (0)

// Replace *p by a fresh allocation of `need` elements (contents dropped).
// Every buffer of a group that outgrew its capacity goes through this on
// its own: a capacity shared between buffers would let a later one keep its
// old, smaller allocation.
template <typename T>
int realloc_buf(T** p, int64_t need) {
  if (*p) HIP_TRY(hipFree(*p));
  *p = nullptr;
  HIP_TRY(hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(need, 1)));
  return LUB_OK;
}

template <typename T>
int grow(T** p, int64_t* cap, int64_t need) {
  if (*p && *cap >= need) return LUB_OK;
  if (*p) HIP_TRY(hipFree(*p));
  *p = nullptr;
  int64_t n = std::max<int64_t>(need, 1);
  HIP_TRY(hipMalloc((void**)p, sizeof(T) * (size_t)n));
  *cap = n;
  return LUB_OK;
}

bool is_link(int model) { return model == LUB_MODEL_LINK || model == LUB_MODEL_LINK_NAVG; }

// candidate and activity cut-off: the reduced models act below delta_n only
double max_cutoff(const lub_params_t& p) {
  if (p.model == LUB_MODEL_CONTACT) return p.h_c;
  // link-wise: a site of i within two links (2 sqrt 2) of a site of j
  if (is_link(p.model)) return 2.0 * std::sqrt(2.0);
  if (p.model != LUB_MODEL_FULL) return p.delta_n;
  return std::max(p.delta_n, std::max(p.delta_t, p.delta_r));
}

int check_params(const lub_params_t* p) {
  if (!p) return LUB_EINVAL;
  if (!(p->mu >= 0.0) || !(p->delta_n > 0.0) || !(p->delta_t > 0.0) ||
      !(p->delta_r > 0.0) || !(p->h_c >= 0.0) || !(p->eps_c >= 0.0))
    return LUB_EINVAL;
  if (p->model < LUB_MODEL_FULL || p->model > LUB_MODEL_LINK_NAVG || p->reserved != 0)
    return LUB_EINVAL;
  if (p->model == LUB_MODEL_CONTACT && !(p->h_c > 0.0)) return LUB_EINVAL;
  if (is_link(p->model) && !(p->q_bar > 0.0 && std::isfinite(p->q_bar))) return LUB_EINVAL;
  return LUB_OK;
}

int check_domain(const lub_domain_t* d) {
  if (!d) return LUB_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(d->L[k] > 0.0) || !std::isfinite(d->L[k])) return LUB_EINVAL;
  if (d->n_walls != 0 && d->n_walls != 2) return LUB_EINVAL;
  if (d->n_walls == 2 && d->periodic[2]) return LUB_EINVAL;
  if (d->lees_edwards != 0 && d->lees_edwards != 1) return LUB_EINVAL;
  if (d->reserved != 0) return LUB_EINVAL;
  if (d->lees_edwards &&
      (!d->periodic[0] || !d->periodic[1] || !d->periodic[2] || d->n_walls != 0 ||
       !std::isfinite(d->le_offset) || !std::isfinite(d->le_velocity)))
    return LUB_EINVAL;
  return LUB_OK;
}

// buffers sized by particle count
int ensure_particles(lub_ctx* c, int64_t n) {
  if (c->cap_n >= n && c->cell_id) return LUB_OK;
  int64_t need = std::max<int64_t>(n, 1);
  int rc;
  c->cap_n = 0;
  if ((rc = realloc_buf(&c->cell_id, need)) || (rc = realloc_buf(&c->sorted, need)) ||
      (rc = realloc_buf(&c->cell_sorted, need)) || (rc = realloc_buf(&c->deg, need)) ||
      (rc = realloc_buf(&c->bcount, 2 * need + 2)) ||
      (rc = realloc_buf(&c->rec, need)) || (rc = realloc_buf(&c->recp, need)) || (rc = realloc_buf(&c->kin, need)) ||
      (rc = realloc_buf(&c->staged, need)) ||
      (rc = realloc_buf(&c->pos, need)) ||
      (rc = realloc_buf(&c->scat, need)) ||
      (rc = realloc_buf(&c->stat_nbr, (int64_t)kStatNbrWords * nbr_blocks_max((int)need))) ||
      (rc = realloc_buf(&c->wall_slot, 2 * need)))
    return rc;
  if (c->opt.warm_start) {
    // new ranges are empty
    for (int k = 0; k < 2; ++k) {
      if ((rc = realloc_buf(&c->warm_range[k], need))) return rc;
      HIP_TRY(hipMemset(c->warm_range[k], 0, sizeof(int2) * need));
    }
    HIP_TRY(hipDeviceSynchronize());
  }
  if (c->opt.skin > 0.0 &&
      ((rc = realloc_buf(&c->sup_deg, need)) || (rc = realloc_buf(&c->ref_pos, need)) ||
       (rc = realloc_buf(&c->inv, need)) || (rc = realloc_buf(&c->disp_blk, (need + 255) / 256))))
    return rc;
  c->list_epoch++;
  c->cap_n = need;
  return LUB_OK;
}

int ensure_cells(lub_ctx* c, int64_t ncell) {
  if (c->cap_cells >= ncell && c->cell_count) return LUB_OK;
  int rc;
  c->cap_cells = 0;
  c->zeroed = false;
  if ((rc = realloc_buf(&c->cell_count, ncell)) || (rc = realloc_buf(&c->cell_start, ncell + 1)))
    return rc;
  c->cap_cells = ncell;
  return LUB_OK;
}

// neighbour segments of stride max_nbr for n particles, and the evaluation
// slots: at most half the entries (each pair appears in both segments) plus
// two wall pairs per particle
int ensure_entries(lub_ctx* c, int64_t n, int64_t max_nbr) {
  int64_t entries = std::max<int64_t>(n, 1) * max_nbr;
  int64_t work = entries / 2 + 2 * n + 64;
  int rc;
  if (c->cap_entries < entries || !c->nbr) {
    c->cap_entries = 0;
    if ((rc = realloc_buf(&c->nbr, entries)) || (rc = realloc_buf(&c->slot, entries)) ||
        (rc = realloc_buf(&c->bstage, entries)))
      return rc;
    if (c->opt.skin > 0.0 && (rc = realloc_buf(&c->sup_nbr, entries))) return rc;
    if (c->opt.skin > 0.0 && c->opt.warm_start) {
      // no stored normal yet: tag -1 matches no search
      if ((rc = realloc_buf(&c->sup_val, entries))) return rc;
      HIP_TRY(hipMemset(c->sup_val, 0xff, sizeof(float4) * entries));
      HIP_TRY(hipDeviceSynchronize());  // cleared before any stream uses it
    }
    c->list_epoch++;
    c->cap_entries = entries;
  }
  if (c->cap_work < work || !c->work_s) {
    c->cap_work = 0;
    if ((rc = realloc_buf(&c->work_s, work)) || (rc = realloc_buf(&c->work_t, work)) ||
        (rc = realloc_buf(&c->fail_list, work)) || (rc = realloc_buf(&c->out_links, work)) ||
        (rc = realloc_buf((PairOut<double>**)&c->out, work)) ||
        (rc = realloc_buf(&c->out_h, work)) || (rc = realloc_buf(&c->out_status, work)) ||
        (rc = realloc_buf(&c->out_iters, work)))
      return rc;
    if (c->opt.skin > 0.0 && c->opt.warm_start && (rc = realloc_buf(&c->work_sup, work)))
      return rc;
    if (c->opt.record_detail && (rc = realloc_buf(&c->detail, work * (int64_t)kDetailWords)))
      return rc;
    c->cap_work = work;
    if (c->opt.warm_start) {
      // new values hold no partner (-1): the seeds of earlier calls are
      // dropped
      for (int k = 0; k < 2; ++k) {
        if ((rc = realloc_buf(&c->warm_val[k], work))) return rc;
        HIP_TRY(hipMemset(c->warm_val[k], 0xff, sizeof(float4) * work));
      }
      HIP_TRY(hipDeviceSynchronize());  // cleared before any stream uses them
    }
  }
  return LUB_OK;
}

int build_desc(lub_ctx* c, int64_t n, CallDesc* d) {
  std::memset(d, 0, sizeof(*d));
  d->n = (int32_t)n;
  d->dmax = max_cutoff(c->prm);
  d->skin = c->opt.skin;
  // cells sized for the widest search: the pair bound plus the skin of
  // reused lists
  double edge = 2.0 * c->opt.rmax_bound + d->dmax + d->skin;
  for (int k = 0; k < 3; ++k) {
    d->L[k] = c->dom.L[k];
    d->invL[k] = 1.0 / c->dom.L[k];
    d->periodic[k] = c->dom.periodic[k];
    // minimum image must be unambiguous for the largest pair bound
    if (d->periodic[k] && d->L[k] < 2.0 * edge) return LUB_EDOMAIN;
  }
  // Cells of 1/sub of the largest pair bound, sub = 3, 2 or 1: the finest
  // grid with no more cells than particles (finer cells test fewer
  // candidates, but every cell costs scan and zeroing work).  A particle
  // searches up to `sub` cells on each side, fewer if it is small.  The
  // relative margin, far above rounding, keeps binning by floor(x / cell)
  // from putting a candidate more than `sub` cells away.
  for (int sub = 3; sub >= 1; --sub) {
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
      int64_t nc = (int64_t)std::floor(d->L[k] / (edge / sub * (1.0 + 1e-9)));
      nc = std::max<int64_t>(1, std::min<int64_t>(nc, 1024));
      d->nc[k] = (int32_t)nc;
      d->cell[k] = d->L[k] / (double)nc;
      ncell *= nc;
    }
    d->reach_max = sub;
    if (ncell <= std::max<int64_t>(n, 1)) break;
  }
  d->n_walls = c->dom.n_walls;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) d->wall_vel[s][k] = c->dom.wall_vel[s][k];
  d->le = c->dom.lees_edwards;
  if (d->le) {
    // the offset modulo L_x, in [0, L_x)
    double off = std::fmod(c->dom.le_offset, d->L[0]);
    if (off < 0.0) off = off + d->L[0];
    d->le_offset = off;
    d->le_vel = c->dom.le_velocity;
  }
  d->rmax_bound = c->opt.rmax_bound;
  d->mu = c->prm.mu;
  d->delta_n = c->prm.delta_n;
  d->delta_t = c->prm.delta_t;
  d->delta_r = c->prm.delta_r;
  d->h_c = c->prm.h_c;
  d->eps_c = c->prm.eps_c;
  d->max_iter = c->opt.newton_max_iter > 0 ? c->opt.newton_max_iter : 50;
  d->newton_tol = c->opt.newton_tol > 0.0 ? c->opt.newton_tol : 1e-14;
  d->max_nbr = c->cur_nbr;
  d->precision = c->opt.precision;
  d->model = c->prm.model;
  d->q_bar = c->prm.q_bar;
  d->ln_delta_t = std::log(c->prm.delta_t);
  d->ln_delta_r = std::log(c->prm.delta_r);
  d->inv_delta_n = 1.0 / c->prm.delta_n;
  if (is_link(d->model)) {
    // FP64 outputs; lattice images need integer periodic lengths
    d->precision = LUB_FP64;
    if (c->dom.n_walls || c->dom.lees_edwards) return LUB_EINVAL;
    for (int k = 0; k < 3; ++k)
      if (c->dom.periodic[k] && c->dom.L[k] != std::floor(c->dom.L[k])) return LUB_EINVAL;
  }
  // two size classes with cells of their own: a particle searches the small
  // ones within its own size + r_small + the cut-off only
  d->r_small = 0.5 * c->opt.rmax_bound;
  return LUB_OK;
}

hipEvent_t take_event(lub_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// resolve the events of finished timed calls into the stage totals
int resolve_timing(lub_ctx* c) {
  for (auto& ev : c->pending) {
    HIP_TRY(hipEventSynchronize(ev[4]));
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      c->stage_ms[k] += ms;
    }
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[5], ev[6]));
    c->pair_kernel_ms += ms;
    HIP_TRY(hipEventElapsedTime(&ms, ev[7], ev[8]));
    c->search_kernel_ms += ms;
    c->timed_calls++;
    for (hipEvent_t e : ev) c->free_events.push_back(e);
  }
  c->pending.clear();
  return LUB_OK;
}

int run_desc(lub_ctx* c, const CallDesc& d, const double* r, const double* q,
             const double* semi, const double* v, const double* w, double* f,
             double* t, hipStream_t s);

// the capacities of the current workspace, the warm-start table size and
// the epoch of reusable neighbour lists (a new one when n or the segment
// stride changed)
CallDesc finalize_desc(lub_ctx* c, const CallDesc& d0) {
  CallDesc d = d0;
  if (d.skin > 0.0 && (c->epoch_n != d.n || c->epoch_stride != d.max_nbr)) {
    c->list_epoch++;
    c->epoch_n = d.n;
    c->epoch_stride = d.max_nbr;
  }
  d.list_epoch = c->list_epoch;
  d.cap_entries = (int32_t)std::min<int64_t>(c->cap_entries, INT32_MAX);
  d.cap_work = (int32_t)std::min<int64_t>(c->cap_work, INT32_MAX);
  // the forward search leaves slot ranges and backward lists, no segments;
  // else, from about a quarter million particles, partner codes written
  // beside the pair kernel save the gather its searches (below, the fork
  // and join cost more than they save)
  d.partner_codes = d.skin == 0.0 && nbr_forward(d, c->bcount, c->block_sums, c->bstage)
                        ? kPartnerRanges
                        : (d.n >= (1 << 18) ? kPartnerSide : kPartnerSearch);
  // Ladd's law has no closest-point iteration to start.  With reused lists
  // the normals are kept per superset entry, else per slot with each
  // particle's slot range
  const bool warm = c->opt.warm_start && d.model != LUB_MODEL_LADD && !is_link(d.model);
  d.warm_slots = warm && d.skin > 0.0 && c->sup_val && c->work_sup &&
                 (int64_t)std::max<int64_t>(d.n, 1) * d.max_nbr <= INT32_MAX;
  d.warm_ranges = warm && !d.warm_slots && c->warm_range[0] && c->warm_val[0];
  return d;
}

int run(lub_ctx* c, const CallDesc& d0, const double* r, const double* q,
        const double* semi, const double* v, const double* w, double* f,
        double* t, hipStream_t s) {
  return run_desc(c, finalize_desc(c, d0), r, q, semi, v, w, f, t, s);
}

int run_desc(lub_ctx* c, const CallDesc& d, const double* r, const double* q,
             const double* semi, const double* v, const double* w, double* f,
             double* t, hipStream_t s) {
  const int ncell = 2 * d.nc[0] * d.nc[1] * d.nc[2];  // bins: two size classes
  std::vector<hipEvent_t> ev;
  const bool timing = c->opt.timing && d.n > 0;
  if (timing) {
    // bound the backlog of unresolved calls
    if (c->pending.size() >= 4096) {
      int rc = resolve_timing(c);
      if (rc) return rc;
    }
    // 0..4 stage marks, 5-6 the pair kernel, 7-8 the search kernel
    for (int k = 0; k < 9; ++k) {
      hipEvent_t e = take_event(c);
      if (!e) return LUB_EDEVICE;
      ev.push_back(e);
    }
  }
  auto mark = [&](int k) {
    if (timing) (void)hipEventRecord(ev[k], s);  // timing only: best effort
  };
  mark(0);
  // this call's counters: the set the previous call's last kernel zeroed
  c->cnt_idx ^= 1;
  c->cnt = c->cnt_buf + c->cnt_idx;
  Counters* next_cnt = c->cnt_buf + (c->cnt_idx ^ 1);
  const bool small = d.n > 0 && cells_small_fits(d);
  // warm-start sets of this call: written and read
  const int wc = c->cnt_idx, wp = c->cnt_idx ^ 1;
  if (!c->zeroed) launch_reset(c->cnt, c->cell_count, ncell, s);
  c->zeroed = false;
  // reused neighbour lists: the device decides whether this call searches
  // (every particle within half the skin of its place and size at the last
  // search: no); the cell build runs only if it does, the record refresh
  // only if it does not
  const bool reuse = d.n > 0 && d.skin > 0.0;
  const Counters* gate = reuse ? c->cnt : nullptr;
  const ListBufs lists{c->sup_nbr,    c->sup_deg,    c->ref_pos,
                       c->inv,        c->disp_blk,   c->list_state,
                       d.warm_slots ? c->work_sup : nullptr,
                       d.warm_ranges ? c->warm_range[wc] : nullptr};
  if (reuse) {
    launch_disp(d, r, q, semi, lists, c->cnt, s);
    launch_refresh(d, r, q, semi, v, w, lists, c->rec, c->recp, c->pos, c->kin, c->cnt, s);
  }
  if (d.n > 0) {
    if (small) {
      launch_cells_small(d, r, q, semi, v, w, c->cell_start, c->sorted, c->rec, c->recp, c->pos,
                         c->kin, c->cell_sorted, c->cnt, gate, s);
    } else {
      // the tickets are kept in `sorted` until the record build writes it
      launch_stage_bin(d, r, q, semi, v, w, c->cell_id, c->sorted, c->staged, c->cell_count,
                       c->cnt, gate, s, c->bcount);
      launch_scan(c->cell_count, c->cell_start, ncell, c->block_sums, nullptr, s);
      launch_cell_scatter(d, c->cell_id, c->sorted, c->cell_start, c->scat, c->cell_sorted,
                          c->cell_count, ncell, gate, s);
      // the 128-B records feed the lane-group search, the full search of
      // small systems, the learned seed's features and the link-wise laws
      const bool need_rec = !(d.skin == 0.0 && nbr_forward(d, c->bcount, c->block_sums,
                                                           c->bstage)) ||
                            is_link(d.model) || c->opt.seed_mode == LUB_SEED_MLP;
      launch_build_records(d, c->scat, c->cell_sorted, c->cell_start, c->staged, c->sorted,
                           need_rec ? c->rec : nullptr, c->recp, c->pos, c->kin, gate, s);
    }
  }
  if (d.n > 0) {
    mark(1);
    if (reuse) {
      // the superset (searched in calls that search), then the exact filter
      launch_neighbors_wave(d, c->rec, c->recp, c->pos, c->sorted, c->cell_sorted, c->cell_start,
                            c->sup_deg, c->sup_nbr, c->slot, c->wall_slot, c->work_s,
                            c->work_t, c->stat_nbr, c->cnt, s, 1, &lists);
      launch_neighbors_wave(d, c->rec, c->recp, c->pos, c->sorted, c->cell_sorted, c->cell_start,
                            c->deg, c->nbr, c->slot, c->wall_slot, c->work_s, c->work_t,
                            c->stat_nbr, c->cnt, s, 2, &lists, nullptr, nullptr, nullptr,
                            timing ? ev[7] : nullptr, timing ? ev[8] : nullptr);
    } else {
      launch_neighbors_wave(d, c->rec, c->recp, c->pos, c->sorted, c->cell_sorted, c->cell_start,
                            c->deg, c->nbr, c->slot, c->wall_slot, c->work_s,
                            c->work_t, c->stat_nbr, c->cnt, s, 0, &lists, c->bcount,
                            c->block_sums, c->bstage, timing ? ev[7] : nullptr,
                            timing ? ev[8] : nullptr);
      c->list_builds++;
    }
    mark(2);
    // the partner-slot codes beside the pair kernel
    const bool side = d.partner_codes == kPartnerSide;
    if (side) {
      HIP_TRY(hipEventRecord(c->ev_fork, s));
      HIP_TRY(hipStreamWaitEvent(c->side, c->ev_fork, 0));
      launch_partner_slots(d, c->work_s, c->work_t, c->deg, c->nbr, c->slot, c->cnt, c->side);
      HIP_TRY(hipEventRecord(c->ev_join, c->side));
    }
    const float* seeds = nullptr;
    if (c->opt.seed_mode == LUB_SEED_MLP && !is_link(d.model)) {
      launch_seed_features(d, c->rec, c->work_s, c->work_t, c->seedX, c->cnt, s);
      mlp_forward_slots(c->cnt, d.cap_work, c->seedX, c->seedY, c->wt, c->th, s);
      seeds = c->seedY;
    }
    WarmTables warm{c->warm_range[wp], c->warm_val[wp], c->warm_val[wc], c->sorted,
                    c->work_sup,       c->sup_val,      c->list_state, c->warm_range[wc]};
    if (is_link(d.model)) {
      launch_links(d, c->rec, c->kin, c->work_s, c->work_t, c->out, c->out_h, c->out_status,
                   c->out_links, c->stat_pair, c->cnt, s);
      if (timing) {  // no separate kernel stamps: the stage time
        (void)hipEventRecord(ev[5], s);
        (void)hipEventRecord(ev[6], s);
      }
    } else {
      launch_pairs(d, c->recp, c->kin, c->work_s, c->work_t, seeds, c->out,
                   c->out_h, c->out_status, c->out_iters, warm, c->fail_list, c->stat_pair,
                   c->cnt, s,
                   timing ? ev[5] : nullptr, timing ? ev[6] : nullptr, c->detail);
    }
    mark(3);
    if (side) HIP_TRY(hipStreamWaitEvent(s, c->ev_join, 0));
    launch_gather(d, c->sorted, c->deg, c->nbr, c->slot, c->wall_slot, c->out,
                  c->cnt, next_cnt, f, t, s, c->bcount, c->work_s);
    mark(4);
    if (timing) c->pending.push_back(ev);
  }
  HIP_TRY(hipGetLastError());
  c->zeroed = d.n > 0;
  c->last = d;
  c->have_last = true;
  c->last_stream = s;
  return LUB_OK;
}

int fetch_counters(lub_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  // the statistics are kept as per-block rows: sum them now
  if (c->have_last)
    launch_stats_reduce(c->last, c->cnt, c->stat_pair, c->stat_nbr, c->last_stream);
  HIP_TRY(hipMemcpyAsync(c->host_cnt, c->cnt, sizeof(Counters),
                         hipMemcpyDeviceToHost, c->last_stream));
  HIP_TRY(hipStreamSynchronize(c->last_stream));
  return LUB_OK;
}

// the device buffers a call's launch sequence uses
std::vector<const void*> workspace_signature(const lub_ctx* c) {
  return {c->cell_id, c->cell_count, c->cell_start, c->sorted, c->scat,
          c->cell_sorted, c->deg, c->bcount, c->bstage, c->block_sums, c->wall_slot, c->rec,
          c->recp,
          c->pos, c->kin, c->staged,
          c->nbr,
          c->slot, c->work_s, c->work_t, c->fail_list, c->out_links, c->out, c->out_h,
          c->out_status,
          c->out_iters, c->cnt_buf, c->stat_nbr, c->stat_pair, c->seedX, c->seedY, c->wt, c->th,
          c->warm_range[0], c->warm_range[1], c->warm_val[0], c->warm_val[1], c->sup_nbr,
          c->sup_deg, c->ref_pos, c->inv, c->disp_blk, c->list_state, c->sup_val, c->work_sup,
          c->detail};
}

void drop_graphs(lub_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) {
      // teardown: nothing to report an error to
      (void)hipStreamSynchronize((hipStream_t)g.args[7]);  // no replay in flight
      (void)hipGraphExecDestroy(g.exec);
    }
    g = lub_ctx::GraphSlot();
  }
}

// One call as a graph replay.  The first call (and any call after a failure)
// runs eagerly: it may need the reset launch, which a replay does not hold.
int run_graph(lub_ctx* c, const CallDesc& d0, const double* r, const double* q,
              const double* semi, const double* v, const double* w, double* f,
              double* t, hipStream_t s) {
  if (!c->zeroed || d0.n == 0) return run(c, d0, r, q, semi, v, w, f, t, s);
  const CallDesc d = finalize_desc(c, d0);
  const int par = c->cnt_idx ^ 1;  // the counter set this call uses
  lub_ctx::GraphSlot& g = c->graphs[par];
  const void* args[8] = {r, q, semi, v, w, f, t, s};
  const std::vector<const void*> ws = workspace_signature(c);
  const bool same = g.exec && g.n == d.n && std::memcmp(g.args, args, sizeof(args)) == 0 &&
                    std::memcmp(&g.d, &d, sizeof(d)) == 0 && g.ws == ws;
  if (!same) {
    if (g.exec) {
      HIP_TRY(hipStreamSynchronize((hipStream_t)g.args[7]));  // no replay in flight
      HIP_TRY(hipGraphExecDestroy(g.exec));
    }
    g = lub_ctx::GraphSlot();
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int rc = run_desc(c, d, r, q, semi, v, w, f, t, s);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    // the capture only recorded the launches: restore the state a replay sets
    c->zeroed = true;
    if (rc || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);  // the capture's error is returned
      c->zeroed = false;
      return rc ? rc : hip_err(e);
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);  // the instantiation's error is returned
    if (ei != hipSuccess) {
      g = lub_ctx::GraphSlot();
      c->zeroed = false;
      return hip_err(ei);
    }
    g.n = d.n;
    std::memcpy(g.args, args, sizeof(args));
    g.d = d;
    g.ws = ws;
  }
  c->cnt_idx = par;
  c->cnt = c->cnt_buf + par;
  HIP_TRY(hipGraphLaunch(g.exec, s));
  c->zeroed = true;
  c->last = d;
  c->have_last = true;
  c->last_stream = s;
  return LUB_OK;
}

int mlp_upload(lub_ctx* c, const std::vector<float>& th) {
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpy(c->th, th.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(c->m1, 0, sizeof(float) * kNParams));
  HIP_TRY(hipMemset(c->m2, 0, sizeof(float) * kNParams));
  c->adam_step = 0;
  mlp_pack(c->th, c->wt, c->wb, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  return LUB_OK;
}

int mlp_init_host(lub_ctx* c, uint64_t seed) {
  // uniform in [-sqrt(6/fan_in), sqrt(6/fan_in)], zero biases
  std::vector<float> th(kNParams, 0.0f);
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
  auto next = [&x]() {  // splitmix64
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int fan[4] = {10, 128, 128, 128}, outn[4] = {128, 128, 128, 4};
  const int off[4] = {kOffW1, kOffW2, kOffW3, kOffW4};
  for (int l = 0; l < 4; ++l) {
    const float lim = std::sqrt(6.0f / (float)fan[l]);
    for (int k = 0; k < fan[l] * outn[l]; ++k) {
      double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
      th[off[l] + k] = (float)((2.0 * u - 1.0) * lim);
    }
  }
  return mlp_upload(c, th);
}

int ensure_batch(lub_ctx* c, int64_t B) {
  if (c->cap_batch >= B && c->aT) return LUB_OK;
  int rc;
  c->cap_batch = 0;
  if ((rc = realloc_buf(&c->aT, 416 * B)) || (rc = realloc_buf(&c->dT, 400 * B)) ||
      (rc = realloc_buf(&c->loss_parts, B / 64 + 1)))
    return rc;
  c->cap_batch = B;
  return LUB_OK;
}

// seed features and outputs, one row per evaluation slot
int ensure_seed(lub_ctx* c) {
  int rc;
  c->cap_seed = 0;
  if ((rc = realloc_buf(&c->seedX, 10 * c->cap_work)) ||
      (rc = realloc_buf(&c->seedY, 4 * c->cap_work)))
    return rc;
  c->cap_seed = c->cap_work;
  return LUB_OK;
}

}  // namespace

// ---- allocation-free evaluation (lub_compute_static) -----------------------
// The workspace of one such call lives in this file-scope device array: each
// GPU that runs the call holds its own copy until the process ends.  Host
// code never uses the array's name as an address: its device address on each
// device is looked up once (hipGetSymbolAddress, with that device current)
// and kept per device.
static __device__ __align__(256) unsigned char scratch[LUB_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return LUB_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return LUB_EDEVICE;
    g_scratch_dev[device] = p;
  }
  *out = (unsigned char*)g_scratch_dev[device];
  return LUB_OK;
}

// Bump allocator over the scratch array (256-B aligned pieces).
struct Carve {
  unsigned char* base;
  size_t used = 0;
  bool ok = true;
  template <typename T>
  T* take(int64_t count) {
    const size_t bytes = (sizeof(T) * (size_t)std::max<int64_t>(count, 1) + 255) & ~(size_t)255;
    if (used + bytes > (size_t)LUB_STATIC_SCRATCH_BYTES) {
      ok = false;
      return nullptr;
    }
    T* p = (T*)(base + used);
    used += bytes;
    return p;
  }
};

}  // namespace

extern "C" {

int lub_create(lub_handle_t* out, const lub_domain_t* domain,
               const lub_params_t* params, const lub_opts_t* opts) {
  if (!out || !opts) return LUB_EINVAL;
  *out = nullptr;
  int rc;
  if ((rc = check_params(params))) return rc;
  if ((rc = check_domain(domain))) return rc;
  if (!(opts->rmax_bound > 0.0)) return LUB_EINVAL;
  if (opts->precision != LUB_FP64 && opts->precision != LUB_MIXED) return LUB_EINVAL;
  if (opts->seed_mode != LUB_SEED_PLAIN && opts->seed_mode != LUB_SEED_MLP)
    return LUB_EINVAL;
  if ((opts->graph != 0 && opts->graph != 1) || (opts->graph && opts->timing) ||
      (opts->warm_start != 0 && opts->warm_start != 1))
    return LUB_EINVAL;
  if (opts->reserved != 0 || !(opts->skin >= 0.0) || !std::isfinite(opts->skin))
    return LUB_EINVAL;
  if (!(opts->newton_tol < 1e-2) ||
      (opts->record_detail != 0 && opts->record_detail != 1) ||
      (opts->host_pointers != 0 && opts->host_pointers != 1) ||
      (opts->host_pointers && opts->graph))
    return LUB_EINVAL;
  lub_ctx* c = new (std::nothrow) lub_ctx();
  if (!c) return LUB_ENOMEM;
  c->device = opts->device;
  if (opts->max_neighbors > kMaxNbr) {
    delete c;
    return LUB_EINVAL;
  }
  c->cur_nbr = opts->max_neighbors > 0
                   ? (int32_t)((opts->max_neighbors + 63) / 64 * 64)
                   : 64;
  c->prm = *params;
  c->dom = *domain;
  c->opt = *opts;
  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return LUB_EDEVICE;
  }
  if (hipMalloc((void**)&c->cnt_buf, 2 * sizeof(Counters)) != hipSuccess ||
      hipHostMalloc((void**)&c->host_cnt, sizeof(Counters), 0) != hipSuccess) {
    lub_destroy(c);
    return LUB_ENOMEM;
  }
  std::memset(c->host_cnt, 0, sizeof(Counters));
  if (c->opt.skin > 0.0) {
    // no lists yet (epoch -1), no searches
    const ListState none{-1, 0, 0, 0.0};
    if (hipMalloc((void**)&c->list_state, sizeof(ListState)) != hipSuccess) {
      lub_destroy(c);
      return LUB_ENOMEM;
    }
    if (hipMemcpy(c->list_state, &none, sizeof(ListState), hipMemcpyHostToDevice) !=
        hipSuccess) {
      lub_destroy(c);
      return LUB_EDEVICE;
    }
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    lub_destroy(c);
    return LUB_EDEVICE;
  }
  c->cnt = c->cnt_buf;
  if (hipMemset(c->cnt_buf, 0, 2 * sizeof(Counters)) != hipSuccess) {
    lub_destroy(c);
    return LUB_EDEVICE;
  }
  {
    int rc2 = LUB_OK;
    if (!rc2) rc2 = realloc_buf(&c->th, kNParams);
    if (!rc2) rc2 = realloc_buf(&c->m1, kNParams);
    if (!rc2) rc2 = realloc_buf(&c->m2, kNParams);
    if (!rc2) rc2 = realloc_buf(&c->grad, kNParams);
    if (!rc2) rc2 = realloc_buf(&c->wt, kWtTotal);
    if (!rc2) rc2 = realloc_buf(&c->wb, kWbTotal);
    if (!rc2) rc2 = realloc_buf(&c->dloss, 64);
    if (!rc2) rc2 = realloc_buf(&c->stat_pair,
                                   (int64_t)kStatPairWords * (kMaxPairBlocks + kTangentBlocks));
    if (!rc2) rc2 = mlp_init_host(c, 0);
    if (rc2) {
      lub_destroy(c);
      return rc2;
    }
  }
  *out = c;
  return LUB_OK;
}

int lub_set_params(lub_handle_t h, const lub_params_t* params) {
  if (!h) return LUB_EINVAL;
  int rc = check_params(params);
  if (rc) return rc;
  h->prm = *params;
  h->list_epoch++;
  return LUB_OK;
}

int lub_set_domain(lub_handle_t h, const lub_domain_t* domain) {
  if (!h) return LUB_EINVAL;
  int rc = check_domain(domain);
  if (rc) return rc;
  // a new Lees-Edwards offset or velocity keeps reused lists (the offset's
  // change enters the decision); any other change discards them
  lub_domain_t a = h->dom, b = *domain;
  a.le_offset = b.le_offset = 0.0;
  a.le_velocity = b.le_velocity = 0.0;
  if (std::memcmp(&a, &b, sizeof(a)) != 0) h->list_epoch++;
  h->dom = *domain;
  return LUB_OK;
}

namespace {
int compute_device(lub_handle_t h, int64_t n, const double* r, const double* q,
                   const double* semi, const double* v, const double* w, double* f,
                   double* t, hipStream_t s);
}  // namespace

int lub_compute(lub_handle_t h, int64_t n, const double* r, const double* q,
                const double* semi, const double* v, const double* w,
                double* f, double* t, void* stream) {
  if (!h || n < 0 || n > (int64_t)1 << 30) return LUB_EINVAL;
  if (n > 0 && (!r || !q || !semi || !v || !w || !f || !t)) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  if (!h->opt.host_pointers || n == 0)
    return compute_device(h, n, r, q, semi, v, w, f, t, s);
  // host arrays: through the handle's staging buffers
  if (h->cap_stage < n || !h->stage_in) {
    h->cap_stage = 0;
    int rc;
    if ((rc = realloc_buf(&h->stage_in, 15 * n)) || (rc = realloc_buf(&h->stage_out, 6 * n)))
      return rc;
    h->cap_stage = n;
  }
  double* dr = h->stage_in;
  double* dq = dr + 3 * n;
  double* ds = dq + 4 * n;
  double* dv = ds + 2 * n;
  double* dw = dv + 3 * n;
  double* df = h->stage_out;
  double* dt = df + 3 * n;
  const size_t b = sizeof(double) * (size_t)n;
  HIP_TRY(hipMemcpyAsync(dr, r, 3 * b, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dq, q, 4 * b, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ds, semi, 2 * b, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dv, v, 3 * b, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dw, w, 3 * b, hipMemcpyHostToDevice, s));
  const int rc = compute_device(h, n, dr, dq, ds, dv, dw, df, dt, s);
  if (rc) {
    (void)hipStreamSynchronize(s);  // the call's own error is returned
    return rc;
  }
  HIP_TRY(hipMemcpyAsync(f, df, 3 * b, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(t, dt, 3 * b, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return LUB_OK;
}

namespace {
int compute_device(lub_handle_t h, int64_t n, const double* r, const double* q,
                   const double* semi, const double* v, const double* w, double* f,
                   double* t, hipStream_t s) {
  if (h->opt.graph && s == nullptr) return LUB_EINVAL;  // no capture on the null stream
  CallDesc d;
  int rc = build_desc(h, n, &d);
  if (rc) return rc;
  int64_t ncell = 2 * (int64_t)d.nc[0] * d.nc[1] * d.nc[2];  // bins: two size classes
  if ((rc = ensure_particles(h, n))) return rc;
  if ((rc = ensure_cells(h, ncell))) return rc;
  // scan scratch: one block sum per 8192 elements of the longer scan
  if ((rc = grow(&h->block_sums, &h->cap_bs, std::max<int64_t>(ncell, n) / 1024 + 64)))
    return rc;
  if ((rc = ensure_entries(h, n, h->cur_nbr))) return rc;
  if (h->opt.seed_mode == LUB_SEED_MLP && h->cap_seed < h->cap_work) {
    if ((rc = ensure_seed(h))) return rc;
  }
  if ((rc = h->opt.graph ? run_graph(h, d, r, q, semi, v, w, f, t, s)
                         : run(h, d, r, q, semi, v, w, f, t, s))) {
    h->list_epoch++;
    return rc;
  }
  if (!h->opt.sync) return LUB_OK;
  if ((rc = fetch_counters(h))) {
    h->list_epoch++;
    return rc;
  }
  // automatic limit: widen the segments and evaluate again
  while (h->host_cnt->error == LUB_ECAPACITY && h->opt.max_neighbors <= 0 &&
         h->cur_nbr < kMaxNbr) {
    h->cur_nbr = std::min(kMaxNbr, 2 * h->cur_nbr);
    if ((rc = build_desc(h, n, &d))) return rc;
    if ((rc = ensure_entries(h, n, h->cur_nbr))) return rc;
    if (h->opt.seed_mode == LUB_SEED_MLP && h->cap_seed < h->cap_work) {
      if ((rc = ensure_seed(h))) return rc;
    }
    if ((rc = run(h, d, r, q, semi, v, w, f, t, s)) || (rc = fetch_counters(h))) {
      h->list_epoch++;
      return rc;
    }
  }
  if (h->host_cnt->error) h->list_epoch++;
  return h->host_cnt->error;
}
}  // namespace


int lub_compute_static(const lub_domain_t* domain, const lub_params_t* params,
                       const lub_opts_t* opts, int64_t n, const double* r, const double* q,
                       const double* semi, const double* v, const double* w, double* f,
                       double* t, void* stream, lub_stats_t* stats) {
  if (!opts || n < 0 || n > LUB_STATIC_MAX_PARTICLES) return LUB_EINVAL;
  if (n > 0 && (!r || !q || !semi || !v || !w || !f || !t)) return LUB_EINVAL;
  int rc;
  if ((rc = check_params(params)) || (rc = check_domain(domain))) return rc;
  if (is_link(params->model)) return LUB_EINVAL;
  if (!(opts->rmax_bound > 0.0) || !std::isfinite(opts->rmax_bound)) return LUB_EINVAL;
  if (opts->precision != LUB_FP64 && opts->precision != LUB_MIXED) return LUB_EINVAL;
  if (opts->seed_mode != LUB_SEED_PLAIN || opts->warm_start || opts->graph || opts->timing ||
      opts->skin != 0.0 || opts->reserved != 0 || opts->host_pointers || opts->record_detail)
    return LUB_EINVAL;
  if (opts->max_neighbors > LUB_STATIC_MAX_NEIGHBORS) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(opts->device));
  unsigned char* base = nullptr;
  if ((rc = scratch_address(opts->device, &base))) return rc;
  // a handle on the stack whose workspace points into the scratch array
  lub_ctx c;
  c.device = opts->device;
  c.prm = *params;
  c.dom = *domain;
  c.opt = *opts;
  c.opt.sync = 0;
  c.cur_nbr = opts->max_neighbors > 0 ? (int32_t)((opts->max_neighbors + 63) / 64 * 64) : 64;
  CallDesc d;
  if ((rc = build_desc(&c, n, &d))) return rc;
  const int64_t ncell = 2 * (int64_t)d.nc[0] * d.nc[1] * d.nc[2];
  if (ncell > 4 * LUB_STATIC_MAX_PARTICLES + 64) return LUB_ECAPACITY;
  const int64_t np = std::max<int64_t>(n, 1);
  const int64_t entries = np * c.cur_nbr;
  const int64_t work = std::min<int64_t>(entries / 2 + 2 * np + 64, 8 * np + 64);
  Carve cv{base};
  c.cnt_buf = cv.take<Counters>(2);
  c.cell_id = cv.take<int32_t>(np);
  c.sorted = cv.take<int32_t>(np);
  c.cell_sorted = cv.take<int32_t>(np);
  c.deg = cv.take<int32_t>(np);
  c.scat = cv.take<int32_t>(np);
  c.wall_slot = cv.take<int32_t>(2 * np);
  c.rec = cv.take<PRec>(np);
  c.recp = cv.take<PRecP>(np);
  c.kin = cv.take<KRec>(np);
  c.staged = cv.take<RecStage>(np);
  c.pos = cv.take<double4>(np);
  c.stat_nbr = cv.take<int64_t>((int64_t)kStatNbrWords * nbr_blocks_max((int)np));
  c.stat_pair = cv.take<int64_t>((int64_t)kStatPairWords * (kMaxPairBlocks + kTangentBlocks));
  c.cell_count = cv.take<int32_t>(ncell);
  c.cell_start = cv.take<int32_t>(ncell + 1);
  c.block_sums = cv.take<int32_t>(std::max<int64_t>(ncell, np) / 1024 + 64);
  c.nbr = cv.take<int32_t>(entries);
  c.slot = cv.take<int32_t>(entries);
  c.work_s = cv.take<int32_t>(work);
  c.work_t = cv.take<int32_t>(work);
  c.fail_list = cv.take<int32_t>(work);
  c.out_links = cv.take<int32_t>(work);
  c.out = cv.take<PairOut<double>>(work);
  c.out_h = cv.take<double>(work);
  c.out_status = cv.take<int8_t>(work);
  c.out_iters = cv.take<uint8_t>(work);
  if (!cv.ok) return LUB_ECAPACITY;
  c.cap_n = np;
  c.cap_cells = ncell;
  c.cap_entries = entries;
  c.cap_work = work;
  c.cnt = c.cnt_buf;
  // the array keeps the last call's contents: the counters and the cell
  // counts are cleared by the reset kernel that starts the call
  c.zeroed = false;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = run(&c, d, r, q, semi, v, w, f, t, s))) return rc;
  if (!stats) return LUB_OK;
  // statistics: sum the per-block rows, copy them out, wait for the stream
  std::memset(stats, 0, sizeof(*stats));
  Counters host{};
  launch_stats_reduce(c.last, c.cnt, c.stat_pair, c.stat_nbr, s);
  HIP_TRY(hipMemcpyAsync(&host, c.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  stats->n = n;
  stats->candidates = host.candidates;
  stats->wall_candidates = host.wall_candidates;
  stats->evaluated = host.work;
  stats->active = host.active;
  stats->overlaps = host.overlaps;
  stats->unresolved = host.unresolved;
  stats->unconverged = host.unconverged;
  stats->fallbacks = host.fallbacks;
  stats->newton_iters = host.newton_iters;
  stats->newton_max = host.newton_max;
  stats->error = host.error;
  stats->max_degree = host.max_degree;
  for (int k = 0; k < 32; ++k) stats->iter_hist[k] = host.iter_hist[k];
  return host.error;
}

int lub_get_domain(lub_handle_t h, lub_domain_t* out) {
  if (!h || !out) return LUB_EINVAL;
  *out = h->dom;
  return LUB_OK;
}

namespace {

// One sub-step: the correction on the current state, then the particle
// update; the Lees-Edwards offset advances by le_velocity dt first, so the
// update re-enters particles with the offset of the new time.
int substep(lub_handle_t h, int64_t n, double* r, double* q, const double* semi,
            double* v, double* w, const double* f_ext, const double* t_ext, double* f,
            double* t, double dt, double density, double damping, hipStream_t s) {
  int rc = lub_compute(h, n, r, q, semi, v, w, f, t, s);
  if (rc) return rc;
  if (h->dom.lees_edwards) {
    double off = std::fmod(h->dom.le_offset + h->dom.le_velocity * dt, h->dom.L[0]);
    if (off < 0.0) off = off + h->dom.L[0];
    h->dom.le_offset = off;
  }
  StepDesc sd{};
  sd.n = (int32_t)n;
  for (int k = 0; k < 3; ++k) {
    sd.periodic[k] = h->dom.periodic[k];
    sd.L[k] = h->dom.L[k];
  }
  sd.le = h->dom.lees_edwards;
  sd.le_offset = h->dom.le_offset;
  sd.le_vel = h->dom.le_velocity;
  sd.dt = dt;
  sd.density = density;
  sd.damping = damping;
  launch_integrate(sd, r, q, semi, v, w, f_ext, t_ext, f, t, s);
  HIP_TRY(hipGetLastError());
  return LUB_OK;
}

}  // namespace

int lub_integrate(lub_handle_t h, int64_t n, double* r, double* q, const double* semi,
                  double* v, double* w, const double* f_ext, const double* t_ext,
                  double* f, double* t, const lub_step_t* step, void* stream) {
  if (!h || !step || n < 0 || n > (int64_t)1 << 30) return LUB_EINVAL;
  if (!(step->dt > 0.0) || !std::isfinite(step->dt) || step->n_sub < 1 ||
      step->reserved != 0 || !(step->density > 0.0) || !std::isfinite(step->density) ||
      !(step->damping >= 0.0) || !std::isfinite(step->damping))
    return LUB_EINVAL;
  if (n > 0 && (!r || !q || !semi || !v || !w || !f || !t)) return LUB_EINVAL;
  if (h->opt.host_pointers) return LUB_EINVAL;  // device arrays only
  HIP_TRY(hipSetDevice(h->device));
  for (int k = 0; k < step->n_sub; ++k) {
    int rc = substep(h, n, r, q, semi, v, w, f_ext, t_ext, f, t, step->dt, step->density,
                     step->damping, (hipStream_t)stream);
    if (rc) return rc;
  }
  return LUB_OK;
}

int lub_advance(lub_handle_t h, int64_t n, double* r, double* q, const double* v,
                const double* w, double dt, void* stream) {
  if (!h || n < 0 || n > (int64_t)1 << 30 || !std::isfinite(dt)) return LUB_EINVAL;
  if (n > 0 && (!r || !q || !v || !w)) return LUB_EINVAL;
  if (h->opt.host_pointers) return LUB_EINVAL;  // device arrays only
  HIP_TRY(hipSetDevice(h->device));
  launch_advance((int)n, dt, r, q, v, w, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return LUB_OK;
}

int lub_grow(lub_handle_t h, int64_t n, double* r, double* q, const double* semi,
             double* v, double* w, const lub_grow_t* cfg, void* stream) {
  if (!h || !cfg || n < 0 || n > (int64_t)1 << 30) return LUB_EINVAL;
  if (cfg->n_steps < 1 || cfg->reserved != 0 || !(cfg->scale0 > 0.0) ||
      !(cfg->scale1 >= cfg->scale0) || !std::isfinite(cfg->scale1) || !(cfg->dt > 0.0) ||
      !std::isfinite(cfg->dt) || !(cfg->density > 0.0) || !std::isfinite(cfg->density) ||
      !(cfg->damping >= 0.0) || !std::isfinite(cfg->damping) || !(cfg->h_c > 0.0) ||
      !(cfg->eps_c >= 0.0) || !std::isfinite(cfg->eps_c))
    return LUB_EINVAL;
  if (n > 0 && (!r || !q || !semi || !v || !w)) return LUB_EINVAL;
  if (h->opt.host_pointers) return LUB_EINVAL;  // device arrays only
  HIP_TRY(hipSetDevice(h->device));
  if (h->cap_grow < n || !h->grow_semi) {
    h->cap_grow = 0;
    int rc;
    if ((rc = realloc_buf(&h->grow_semi, 2 * n)) || (rc = realloc_buf(&h->grow_f, 3 * n)) ||
        (rc = realloc_buf(&h->grow_t, 3 * n)))
      return rc;
    h->cap_grow = n;
  }
  hipStream_t s = (hipStream_t)stream;
  // the contact repulsion alone for the call
  const lub_params_t saved = h->prm;
  // reused neighbour lists were built for the other law's cut-off
  h->list_epoch++;
  h->prm.model = LUB_MODEL_CONTACT;
  h->prm.h_c = cfg->h_c;
  h->prm.eps_c = cfg->eps_c;
  int rc = LUB_OK;
  for (int k = 0; k < cfg->n_steps && rc == LUB_OK; ++k) {
    const double sc =
        cfg->scale0 + (cfg->scale1 - cfg->scale0) * (double)(k + 1) / (double)cfg->n_steps;
    launch_scale((int)n, semi, sc, h->grow_semi, s);
    rc = hip_err(hipGetLastError());
    if (rc == LUB_OK)
      rc = substep(h, n, r, q, h->grow_semi, v, w, nullptr, nullptr, h->grow_f, h->grow_t,
                   cfg->dt, cfg->density, cfg->damping, s);
  }
  h->prm = saved;
  h->list_epoch++;
  return rc;
}

int lub_get_stats(lub_handle_t h, lub_stats_t* out) {
  if (!h || !out) return LUB_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (!h->have_last) return LUB_OK;
  int rc = fetch_counters(h);
  if (rc) return rc;
  const Counters& c = *h->host_cnt;
  out->n = h->last.n;
  out->candidates = c.candidates;
  out->warm_seeded = c.warm_seeded;
  out->max_degree = c.max_degree;
  out->wall_candidates = c.wall_candidates;
  out->evaluated = c.work;
  out->active = c.active;
  out->overlaps = c.overlaps;
  out->unresolved = c.unresolved;
  out->unconverged = c.unconverged;
  out->fallbacks = c.fallbacks;
  out->newton_iters = c.newton_iters;
  out->newton_max = c.newton_max;
  out->error = c.error;
  for (int k = 0; k < 32; ++k) out->iter_hist[k] = c.iter_hist[k];
  if ((rc = resolve_timing(h))) return rc;
  out->timed_calls = h->timed_calls;
  for (int k = 0; k < 4; ++k) out->stage_ms[k] = h->stage_ms[k];
  out->pair_kernel_ms = h->pair_kernel_ms;
  out->search_kernel_ms = h->search_kernel_ms;
  out->list_builds = h->list_builds;
  if (h->list_state) {
    // searches decided on the device
    ListState st{};
    if (h->have_last) HIP_TRY(hipStreamSynchronize(h->last_stream));
    HIP_TRY(hipMemcpy(&st, h->list_state, sizeof(ListState), hipMemcpyDeviceToHost));
    out->list_builds = st.builds;
  }
  return LUB_OK;
}

int lub_reset_timers(lub_handle_t h) {
  if (!h) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  int rc = resolve_timing(h);
  if (rc) return rc;
  h->timed_calls = 0;
  for (int k = 0; k < 4; ++k) h->stage_ms[k] = 0.0;
  h->pair_kernel_ms = 0.0;
  h->search_kernel_ms = 0.0;
  return LUB_OK;
}

int lub_get_pairs(lub_handle_t h, int64_t cap, int32_t* ij, int64_t* n_pairs,
                  int64_t wcap, int32_t* wall, int64_t* n_wall) {
  if (!h || !n_pairs || !n_wall) return LUB_EINVAL;
  *n_pairs = 0;
  *n_wall = 0;
  if (!h->have_last || h->last.n == 0) return LUB_OK;
  int rc = fetch_counters(h);
  if (rc) return rc;
  if (h->host_cnt->error) return h->host_cnt->error;
  const int n = h->last.n;
  const size_t stride = (size_t)h->last.max_nbr;
  std::vector<int32_t> deg(n), sorted(n), wall_slot(2 * n);
  HIP_TRY(hipMemcpy(deg.data(), h->deg, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sorted.data(), h->sorted, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  // segments hold each pair from both sides; after the forward search the
  // slot rows hold each pair once, in its finder's forward list (flagged)
  const bool ranges = h->last.partner_codes == kPartnerRanges;
  std::vector<int32_t> nbr(stride * n);
  HIP_TRY(hipMemcpy(nbr.data(), ranges ? h->slot : h->nbr, sizeof(int32_t) * stride * n,
                    hipMemcpyDeviceToHost));
  std::vector<std::pair<int32_t, int32_t>> pairs;
  for (int s = 0; s < n; ++s)
    for (int k = 0; k < std::min<int64_t>(deg[s], (int64_t)stride); ++k) {
      const int e = nbr[stride * s + k];
      int a = sorted[s], b = sorted[ranges ? (e & kIndexMask) : e];
      if (ranges && b < a) std::swap(a, b);
      if (a < b) pairs.emplace_back(a, b);
    }
  std::sort(pairs.begin(), pairs.end());
  *n_pairs = (int64_t)pairs.size();
  std::vector<std::pair<int32_t, int32_t>> walls;
  if (h->last.n_walls) {
    HIP_TRY(hipMemcpy(wall_slot.data(), h->wall_slot, sizeof(int32_t) * 2 * n,
                      hipMemcpyDeviceToHost));
    for (int s = 0; s < n; ++s)
      for (int side = 0; side < 2; ++side)
        if (wall_slot[2 * s + side] != -1) walls.emplace_back(sorted[s], side);
    std::sort(walls.begin(), walls.end());
  }
  *n_wall = (int64_t)walls.size();
  if ((int64_t)pairs.size() > cap || (int64_t)walls.size() > wcap) return LUB_ECAPACITY;
  for (size_t k = 0; k < pairs.size(); ++k) {
    ij[2 * k] = pairs[k].first;
    ij[2 * k + 1] = pairs[k].second;
  }
  for (size_t k = 0; k < walls.size(); ++k) {
    wall[2 * k] = walls[k].first;
    wall[2 * k + 1] = walls[k].second;
  }
  return LUB_OK;
}

int lub_get_pair_results(lub_handle_t h, int64_t cap, int32_t* ij, double* hgap,
                         double* F, double* Ti, double* Tj, int32_t* status,
                         int32_t* iters, int64_t* n_out) {
  if (!h || !n_out) return LUB_EINVAL;
  *n_out = 0;
  if (!h->have_last || h->last.n == 0) return LUB_OK;
  int rc = fetch_counters(h);
  if (rc) return rc;
  if (h->host_cnt->error) return h->host_cnt->error;
  const int n = h->last.n;
  const int m = h->host_cnt->work;
  *n_out = m;
  if (m > cap) return LUB_ECAPACITY;
  if (m == 0) return LUB_OK;
  std::vector<int32_t> sorted(n), ws(m), wt(m);
  std::vector<double> hh(m);
  std::vector<int8_t> st(m);
  std::vector<int32_t> it(m);
  HIP_TRY(hipMemcpy(sorted.data(), h->sorted, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ws.data(), h->work_s, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(wt.data(), h->work_t, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hh.data(), h->out_h, sizeof(double) * m, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(st.data(), h->out_status, m, hipMemcpyDeviceToHost));
  if (is_link(h->last.model)) {
    HIP_TRY(hipMemcpy(it.data(), h->out_links, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  } else {
    std::vector<uint8_t> it8(m);
    HIP_TRY(hipMemcpy(it8.data(), h->out_iters, m, hipMemcpyDeviceToHost));
    for (int k = 0; k < m; ++k) it[k] = it8[k];
  }
  const bool mixed = h->last.precision == LUB_MIXED;
  std::vector<double> od(9 * (size_t)m);
  if (mixed) {
    std::vector<float> of(9 * (size_t)m);
    HIP_TRY(hipMemcpy(of.data(), h->out, sizeof(float) * 9 * m, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < of.size(); ++k) od[k] = of[k];
  } else {
    HIP_TRY(hipMemcpy(od.data(), h->out, sizeof(double) * 9 * m, hipMemcpyDeviceToHost));
  }
  for (int k = 0; k < m; ++k) {
    if (ij) {
      ij[2 * k] = sorted[ws[k]];
      ij[2 * k + 1] = wt[k] >= 0 ? sorted[wt[k]] : wt[k];
    }
    if (hgap) hgap[k] = hh[k];
    for (int c = 0; c < 3; ++c) {
      if (F) F[3 * k + c] = od[9 * k + c];
      if (Ti) Ti[3 * k + c] = od[9 * k + 3 + c];
      if (Tj) Tj[3 * k + c] = od[9 * k + 6 + c];
    }
    if (status) status[k] = st[k];
    if (iters) iters[k] = it[k];
  }
  return LUB_OK;
}

int lub_get_pair_detail(lub_handle_t h, int64_t cap, double* n, double* yi, double* yj,
                        double* e1, double* Kt, int64_t* n_out) {
  if (!h || !n_out) return LUB_EINVAL;
  *n_out = 0;
  if (!h->opt.record_detail || is_link(h->last.model)) return LUB_EINVAL;
  if (!h->have_last || h->last.n == 0) return LUB_OK;
  int rc = fetch_counters(h);
  if (rc) return rc;
  if (h->host_cnt->error) return h->host_cnt->error;
  const int m = h->host_cnt->work;
  *n_out = m;
  if (m > cap) return LUB_ECAPACITY;
  if (m == 0) return LUB_OK;
  std::vector<double> det((size_t)m * kDetailWords);
  HIP_TRY(hipMemcpy(det.data(), h->detail, sizeof(double) * det.size(), hipMemcpyDeviceToHost));
  for (int k = 0; k < m; ++k) {
    const double* d = det.data() + (size_t)k * kDetailWords;
    for (int c = 0; c < 3; ++c) {
      if (n) n[3 * k + c] = d[c];
      if (yi) yi[3 * k + c] = d[3 + c];
      if (yj) yj[3 * k + c] = d[6 + c];
      if (e1) e1[3 * k + c] = d[9 + c];
    }
    if (Kt)
      for (int c = 0; c < 16; ++c) Kt[16 * k + c] = d[12 + c];
  }
  return LUB_OK;
}

int lub_mlp_set_weights(lub_handle_t h, const float* theta, int64_t n) {
  if (!h || !theta || n != kNParams) return LUB_EINVAL;
  std::vector<float> th(theta, theta + kNParams);
  for (float v : th)
    if (!std::isfinite(v)) return LUB_EINVAL;
  return mlp_upload(h, th);
}

int lub_mlp_get_weights(lub_handle_t h, float* theta, int64_t n) {
  if (!h || !theta || n != kNParams) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(theta, h->th, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  return LUB_OK;
}

int lub_mlp_save(lub_handle_t h, float* state, int64_t n) {
  if (!h || !state || n != 3 * (int64_t)kNParams + 1) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(state, h->th, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(state + kNParams, h->m1, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(state + 2 * kNParams, h->m2, sizeof(float) * kNParams,
                    hipMemcpyDeviceToHost));
  state[3 * kNParams] = (float)h->adam_step;
  return LUB_OK;
}

int lub_mlp_load(lub_handle_t h, const float* state, int64_t n) {
  if (!h || !state || n != 3 * (int64_t)kNParams + 1) return LUB_EINVAL;
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(state[k])) return LUB_EINVAL;
  const float st = state[3 * kNParams];
  if (!(st >= 0.f) || st > 16777216.f || st != std::floor(st)) return LUB_EINVAL;
  for (int k = 0; k < kNParams; ++k)
    if (state[2 * kNParams + k] < 0.f) return LUB_EINVAL;  // second moments
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(h->th, state, sizeof(float) * kNParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->m1, state + kNParams, sizeof(float) * kNParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->m2, state + 2 * kNParams, sizeof(float) * kNParams,
                    hipMemcpyHostToDevice));
  h->adam_step = (int)st;
  mlp_pack(h->th, h->wt, h->wb, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  return LUB_OK;
}

int lub_mlp_init(lub_handle_t h, uint64_t seed) {
  if (!h) return LUB_EINVAL;
  return mlp_init_host(h, seed);
}

int lub_mlp_forward(lub_handle_t h, int64_t m, const float* X, float* Y, void* stream) {
  if (!h || m < 0 || (m > 0 && (!X || !Y))) return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  mlp_forward(m, X, Y, h->wt, h->th, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return LUB_OK;
}

int lub_mlp_grad(lub_handle_t h, int64_t m, const float* X, const float* T,
                 float* loss, float* grad, void* stream) {
  if (!h || m <= 0 || m % 64 || m > (1 << 24) || !X || !T || !loss || !grad)
    return LUB_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_batch(h, m);
  if (rc) return rc;
  HIP_TRY(hipMemsetAsync(h->dloss, 0, sizeof(float), s));
  rc = mlp_train_step(m, 0, (int)m, X, T, h->wt, h->wb, h->th, h->aT, h->dT, h->grad,
                      h->m1, h->m2, h->loss_parts, 0.f, 0.9f, 0.999f, 1e-8f, 1, h->dloss,
                      false, s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(grad, h->grad, sizeof(float) * kNParams, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(loss, h->dloss, sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return LUB_OK;
}

int lub_mlp_train(lub_handle_t h, int64_t m, const float* X, const float* T,
                  const lub_train_cfg_t* cfg, float* epoch_loss, void* stream) {
  if (!h || !cfg || m <= 0 || !X || !T || cfg->epochs < 0 || cfg->epochs > 64)
    return LUB_EINVAL;
  const int B = cfg->batch > 0 ? cfg->batch : 2048;
  if (B % 64 || B > (1 << 20) || m < B || !(cfg->lr > 0.f)) return LUB_EINVAL;
  const float b1 = cfg->beta1 > 0.f ? cfg->beta1 : 0.9f;
  const float b2 = cfg->beta2 > 0.f ? cfg->beta2 : 0.999f;
  const float ep = cfg->eps > 0.f ? cfg->eps : 1e-8f;
  const float decay = cfg->lr_decay > 0.f ? cfg->lr_decay : 1.f;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_batch(h, B);
  if (rc) return rc;
  HIP_TRY(hipMemsetAsync(h->dloss, 0, sizeof(float) * 64, s));
  const int64_t steps = m / B;
  float lr = cfg->lr;
  for (int e = 0; e < cfg->epochs; ++e) {
    for (int64_t k = 0; k < steps; ++k) {
      h->adam_step += 1;
      rc = mlp_train_step(m, k * B, B, X, T, h->wt, h->wb, h->th, h->aT, h->dT, h->grad,
                          h->m1, h->m2, h->loss_parts, lr, b1, b2, ep, h->adam_step,
                          h->dloss + e, true, s);
      if (rc) return rc;
    }
    lr *= decay;
  }
  if (epoch_loss && cfg->epochs > 0) {
    std::vector<float> tot(cfg->epochs);
    HIP_TRY(hipMemcpyAsync(tot.data(), h->dloss, sizeof(float) * cfg->epochs,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int e = 0; e < cfg->epochs; ++e) epoch_loss[e] = tot[e] / (float)steps;
  } else {
    HIP_TRY(hipStreamSynchronize(s));
  }
  return LUB_OK;
}

void lub_destroy(lub_handle_t h) {
  if (!h) return;
  // teardown (no error to report): every release is attempted
  (void)hipSetDevice(h->device);
  drop_graphs(h);
  void* bufs[] = {h->cell_id, h->cell_count, h->cell_start,
                  h->sorted, h->cell_sorted, h->deg, h->bcount, h->bstage, h->block_sums,
                  h->wall_slot, h->rec, h->recp, h->kin, h->staged, h->nbr, h->slot, h->work_s,
                  h->fail_list, h->out_links,
                  h->work_t, h->out, h->out_h, h->out_status, h->out_iters,
                  h->cnt_buf, h->scat, h->pos, h->warm_range[0], h->warm_range[1],
                  h->warm_val[0], h->warm_val[1], h->stat_nbr, h->stat_pair, h->th, h->m1,
                  h->m2, h->grad, h->wt, h->wb, h->dloss,
                  h->loss_parts, h->aT, h->dT, h->seedX, h->seedY, h->grow_semi,
                  h->grow_f, h->grow_t, h->stage_in, h->stage_out, h->detail};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (h->host_cnt) (void)hipHostFree(h->host_cnt);
  for (void* p : {(void*)h->sup_nbr, (void*)h->sup_deg, (void*)h->ref_pos, (void*)h->inv,
                  (void*)h->disp_blk, (void*)h->list_state, (void*)h->sup_val,
                  (void*)h->work_sup})
    if (p) (void)hipFree(p);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (auto& ev : h->pending)
    for (hipEvent_t e : ev) h->free_events.push_back(e);
  for (hipEvent_t e : h->free_events) (void)hipEventDestroy(e);
  delete h;
}

const char* lub_strerror(int code) {
  switch (code) {
    case LUB_OK: return "ok";
    case LUB_EINVAL: return "invalid argument or input value";
    case LUB_EDOMAIN: return "domain too small for an unambiguous minimum image, or particle beyond a wall";
    case LUB_ECAPACITY: return "neighbour-list capacity exceeded";
    case LUB_ENOMEM: return "device allocation failed";
    case LUB_EDEVICE: return "HIP runtime error";
    default: return "unknown error";
  }
}

}  // extern "C"
