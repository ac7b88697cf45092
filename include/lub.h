/*
 * lub.h -- C ABI of the MI355X (gfx950) lubrication-correction library.
 *
 * The operation is the contact-based lubrication correction for spheres
 * and spheroids of Janoschek, Harting & Toschi (arXiv:1308.6482), Sec. III:
 * for every pair of particles whose centre distance is below the pruning
 * bound of Sec. III.A, and for every particle near one of two planar walls,
 *   1. the points of closest approach y_i*, y_j* and the signed gap h
 *      (Sec. III.A; negative h = small overlap),
 *   2. the local surface expansion at those points: principal directions
 *      and radii, cubic coefficients (Eqs. lub:curvature-directions,
 *      lub:curvature-radii, lub:surface-i, lub:surface-j, Sec. III.B),
 *   3. the singular resistance matrix K (Appendix, Eqs. app:first-element
 *      .. app:last-element), its cut-off correction (Eq.
 *      lub:resistance-correction) and the contact model (Eqs. lub:frep,
 *      lub:model),
 *   4. the rigid-body transfer to per-particle force and torque (last
 *      equations of Sec. III.B),
 * summed per particle.
 *
 * Conventions
 *   - Arrays are row-major float64 in DEVICE memory (HBM), e.g. the
 *     data_ptr() of contiguous torch.cuda tensors (lub_compute takes host
 *     arrays instead when lub_opts_t.host_pointers = 1); n may be 0.
 *   - r[n][3]     particle centres (any value; periodic axes are wrapped
 *                 by minimum image, wall axis z must lie in [0, L_z])
 *   - q[n][4]     unit quaternions (w, x, y, z); x_world = Q(q) x_body; the
 *                 body z axis is the symmetry axis (Eq. lub:spheroid)
 *   - semi[n][2]  semi-axes (R_par along the symmetry axis, R_perp)
 *   - v[n][3], w[n][3]  translational and angular velocities
 *   - f[n][3], t[n][3]  OUTPUT force and torque (about the centre) on each
 *                 particle; overwritten, not accumulated.
 *   - Pairs are oriented (i, j) with i < j in input order; i is the first
 *     surface (the gap vector points from i to j).  In a particle-wall pair
 *     the particle is the first surface.  Walls are the planes z = 0
 *     (side 0) and z = L_z (side 1).
 *   - stream: a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it; inputs must stay valid and unmodified until the
 *     stream has passed the call.
 *
 * Ownership: the caller owns every array it passes.  The handle owns its
 * device workspace (grown on demand) and keeps no caller pointer after the
 * call returns.  A handle is not thread-safe; distinct handles are
 * independent.
 *
 * Errors: every entry point returns LUB_OK (0) or a negative LUB_E* code;
 * lub_strerror() names it.  Overlapping pairs, pairs that fall back or do
 * not converge are not errors: they are counted in lub_stats_t.
 */
#ifndef LUB_H
#define LUB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LUB_OK 0
#define LUB_EINVAL -1     /* bad argument or input value (NaN, |q|!=1, semi<=0, ...) */
#define LUB_EDOMAIN -2    /* box too small for an unambiguous minimum image, */
                          /* or a particle beyond a wall by more than its size */
#define LUB_ECAPACITY -3  /* a particle has more candidates than max_neighbors */
#define LUB_ENOMEM -4     /* device allocation failed */
#define LUB_EDEVICE -5    /* HIP runtime error */

#define LUB_FP64 0        /* every step in double precision */
#define LUB_MIXED 1       /* FP64 closest-point solve, gap, surface geometry and */
                          /* ln h / 1/h terms; FP32 resistance coefficients, */
                          /* 6x6 product and transfer */

#define LUB_SEED_PLAIN 0  /* Newton started from the line of centres mapped by
                             (M_i + M_j)^-1, M the support matrices: no
                             learned input */
#define LUB_SEED_MLP 1    /* Newton started from the learned predictor */

/* Physical parameters (Sec. III.B-C). */
/* Resistance law (the models the paper compares in Sec. IV):
 *   LUB_MODEL_FULL    the contact-based correction of Sec. III, all sixteen
 *                     singular elements of K (Appendix);
 *   LUB_MODEL_NORMAL  the same with every non-normal element dropped (K33
 *                     alone, "normal only" in the paper's tables);
 *   LUB_MODEL_LADD    Ladd's normal law for spheres, Eq. methods:llub, with
 *                     coefficient 6 pi mu (a b / (a + b))^2 (6 pi mu a^2 at a
 *                     wall): force along the line of centres, no torque.
 *                     Every particle must be a sphere (R_par == R_perp),
 *                     else LUB_EINVAL.
 *   LUB_MODEL_CONTACT no lubrication: the Hookean repulsion of Eq. lub:frep
 *                     alone, acting for h <= h_c (needs h_c > 0).  The
 *                     interaction of the growth stage of the packing
 *                     generator (Sec. IV.C).
 *   LUB_MODEL_LINK    the link-wise law of Ding and Aidun (Sec. II.D, Eq.
 *                     methods:dlub) on the lattice of integer points: every
 *                     D3Q19 link from a site of j (or a fluid site halfway
 *                     along two links from a site of j) to a site of i with
 *                     link gap h* < |c| adds
 *                     -3 q_bar mu / (2 |c|^2 lambda*) e (e.(V_i - V_j))
 *                     (1/h_eff^2 - 1/|c|^2) on i at the crossing point of
 *                     its surface (minus that on j), e the link direction
 *                     from j to i, lambda* the mean of the two surfaces'
 *                     mean curvatures at the crossings, h_eff = max(h*, h_c),
 *                     plus the link-wise repulsion of Eq. lub:frep (h_c,
 *                     eps_c are then the link-wise h_c*, eps_c*).
 *   LUB_MODEL_LINK_NAVG the same with velocity difference, gap and force
 *                     projected on the average normal of the two surfaces
 *                     (Clausen's variant, Sec. II.D).
 *                     The link-wise laws run in FP64 whatever the precision,
 *                     need integer lengths on the periodic axes (lattice
 *                     images) and accept neither walls nor Lees-Edwards
 *                     images (LUB_EINVAL); lub_get_pair_results reports the
 *                     number of contributing links in iters[], the smallest
 *                     link gap in h.
 * The reduced models act below delta_n only; the first three clip the gap
 * at h_c and add the contact force of Eq. lub:frep. */
#define LUB_MODEL_FULL 0
#define LUB_MODEL_NORMAL 1
#define LUB_MODEL_LADD 2
#define LUB_MODEL_CONTACT 3
#define LUB_MODEL_LINK 4
#define LUB_MODEL_LINK_NAVG 5

typedef struct {
  double mu;       /* dynamic viscosity */
  double delta_n;  /* cut-off of K33 (normal) */
  double delta_t;  /* cut-off of all elements except K33 and K44,K45,K55 */
  double delta_r;  /* cut-off of K44, K45, K54, K55 (rotation) */
  double h_c;      /* clipping gap (Eq. lub:model); 0 disables clipping */
  double eps_c;    /* Hookean contact stiffness (Eq. lub:frep) */
  int32_t model;   /* LUB_MODEL_* */
  int32_t reserved;/* must be 0 */
  double q_bar;    /* empirical weight of the link-wise laws (Ding and Aidun: */
                   /* 0.6); must be > 0 for them, ignored by the others */
} lub_params_t;

/* Simulation box. */
typedef struct {
  double L[3];             /* box lengths */
  int32_t periodic[3];     /* 1: periodic (minimum image), 0: bounded */
  int32_t n_walls;         /* 0, or 2: planar walls z = 0 and z = L[2] (needs periodic[2] = 0) */
  double wall_vel[2][3];   /* translational velocity of each wall */
  /* Lees-Edwards images for a sheared periodic box (Sec. IV.C): with */
  /* lees_edwards = 1 the image one box up in z of a particle at r with */
  /* velocity v sits at r + (le_offset, 0, L_z) and moves with */
  /* v + (le_velocity, 0, 0); for a shear rate g at time t, le_velocity = */
  /* g L_z and le_offset = g L_z t (any value; taken modulo L_x).  Needs all */
  /* three axes periodic and no walls (else LUB_EINVAL).  The nearest image */
  /* is chosen in z first, then in x and y.  In graph mode a new offset */
  /* captures the launch sequence again. */
  int32_t lees_edwards;    /* 0 or 1 */
  int32_t reserved;        /* must be 0 */
  double le_offset;
  double le_velocity;
} lub_domain_t;

/* Library options. */
typedef struct {
  int32_t device;          /* HIP device ordinal */
  int32_t precision;       /* LUB_FP64 or LUB_MIXED */
  int32_t seed_mode;       /* LUB_SEED_PLAIN or LUB_SEED_MLP */
  int32_t newton_max_iter; /* iteration limit of the closest-point solve (<=0: 50); */
                           /* a pair whose Newton solve fails from every start */
                           /* falls back to the tangent-sphere iteration of */
                           /* Sec. III.A (N1 = 10 local, N2 = 1000 conservative) */
                           /* and a polish of max(limit, 8) Newton iterations */
  double rmax_bound;       /* upper bound of max(R_par, R_perp) over all particles; */
                           /* sizes the cell grid.  A larger particle is LUB_EINVAL */
  int32_t sync;            /* 1: lub_compute waits for the stream and reports input, */
                           /* domain and capacity errors (and regrows and reruns on */
                           /* capacity); 0: fully asynchronous, errors are reported */
                           /* by the next lub_get_stats() */
  int32_t timing;          /* 1: record HIP events around each pipeline stage on */
                           /* the call's stream; totals appear in lub_stats_t */
  int64_t max_neighbors;   /* neighbour-list entries per particle (candidate pairs */
                           /* it takes part in), rounded up to a multiple of 64, at */
                           /* most 512; <= 0: start at 64 and, with sync = 1, grow */
                           /* on demand.  More candidates than that: LUB_ECAPACITY */
  int32_t graph;           /* 1: replay the call's launch sequence as a HIP graph, */
                           /* captured on first use for the given n, array pointers */
                           /* and stream (two graphs, for alternate calls) and */
                           /* captured again when any of them or the workspace */
                           /* changes.  Needs a stream other than the null stream */
                           /* and timing = 0 (else LUB_EINVAL).  The arrays are read */
                           /* at replay time, so callers may update them in place */
  int32_t warm_start;      /* 1: start each pair's Newton iteration from the common */
                           /* normal it converged to in the previous call of this */
                           /* handle (pairs keyed by their input indices), the */
                           /* start of seed_mode judging it and taking over when it */
                           /* does not converge; pairs new to the call use */
                           /* seed_mode.  The paper's time-step continuation (Sec. */
                           /* III.A).  With skin > 0 the normals are kept per entry */
                           /* of the reused lists (16 B each; a call that searches */
                           /* again starts its pairs from seed_mode).  0: every call */
                           /* starts afresh */
  int32_t reserved;        /* must be 0 */
  double skin;             /* > 0: reuse the neighbour lists across calls.  A search */
                           /* keeps every pair within the pruning bound + skin; a */
                           /* call reuses the lists while 2 (largest displacement, */
                           /* nearest image, + growth of max(R_par, R_perp)) + the */
                           /* change of the Lees-Edwards offset since the search stays */
                           /* within the skin, re-applying the exact centre test to */
                           /* the kept pairs, and searches again otherwise (or when */
                           /* n, the parameters or the domain other than the */
                           /* Lees-Edwards offset and velocity changed, or a call */
                           /* failed).  The device takes the decision: calls stay */
                           /* asynchronous and may be captured (graph = 1).  The pair */
                           /* lists equal those of a fresh search.  The superset needs */
                           /* wider segments (max_neighbors, or the automatic growth */
                           /* with sync = 1).  Periodic lengths must hold twice */
                           /* 2 rmax_bound + cut-off + skin (else LUB_EDOMAIN). */
                           /* 0: search every call */
  double newton_tol;       /* convergence of the closest-point solve: tangential */
                           /* residual of the common normal below newton_tol */
                           /* (h_i(n) + h_j(n)), or a full Newton step below 1e-8 */
                           /* (<= 0: 1e-14) */
  int32_t host_pointers;   /* 1: the arrays of lub_compute are in HOST memory: the */
                           /* call copies r, q, semi, v, w to device staging buffers */
                           /* of the handle, evaluates, copies f and t back and */
                           /* waits for the stream (the results are in f and t when */
                           /* it returns).  Not with graph = 1; lub_integrate and */
                           /* lub_grow keep taking device arrays (LUB_EINVAL).  0: */
                           /* device arrays */
  int32_t record_detail;   /* 1: the pair kernel also stores, per evaluated pair, the */
                           /* closest points, the gap direction, the frame axis x1 */
                           /* and the 16 corrective resistance elements, for */
                           /* lub_get_pair_detail (validation: 224 B per evaluation */
                           /* slot of device memory and the stores); 0: not */
} lub_opts_t;

/* Per-call statistics of the last lub_compute. */
typedef struct {
  int64_t n;                /* particles */
  int64_t candidates;       /* particle pairs passing the centre test */
  int64_t wall_candidates;  /* particle-wall pairs passing the wall test */
  int64_t evaluated;        /* pairs whose closest points were solved */
  int64_t active;           /* pairs with a non-zero correction (incl. wall pairs) */
  int64_t overlaps;         /* active pairs with h <= 0 */
  int64_t unresolved;       /* h <= 0 with h_c = 0: skipped */
  int64_t unconverged;      /* closest-point solve failed: skipped */
  int64_t fallbacks;        /* pairs whose first start failed: a learned or previous- */
                            /* call seed rejected (plain start used), or the */
                            /* tangent-sphere fallback taken */
  int64_t newton_iters;     /* total Newton iterations */
  int32_t newton_max;       /* largest per-pair iteration count */
  int32_t error;            /* LUB_OK or the error found by the last call */
  int64_t iter_hist[32];    /* pairs per iteration count (last bin: >= 31) */
  /* with opts.timing: device time summed over the timed calls since the */
  /* handle was created or lub_reset_timers(), per stage: 0 staging and cell */
  /* list, 1 neighbour lists and evaluation slots, 2 pair kernel, */
  /* 3 per-particle reduction */
  int64_t timed_calls;
  double stage_ms[4];
  int64_t warm_seeded;      /* pairs started from the previous call's solution */
  int64_t max_degree;       /* most candidate partners of one particle (also when it */
                            /* exceeded max_neighbors: the value to set); with a */
                            /* skin, of the superset */
  double pair_kernel_ms;    /* with opts.timing: the pair kernel's own execution */
                            /* time (dispatch timestamps), summed like stage_ms */
  int64_t list_builds;      /* neighbour-list searches since the handle was created */
                            /* (one per call unless opts.skin > 0; with a skin, a */
                            /* search whose superset overflowed counts too) */
  double search_kernel_ms;  /* with opts.timing: the neighbour search's own */
                            /* execution time (dispatch timestamps; the forward walk */
                            /* of large systems, the filter of reused lists), summed */
                            /* like stage_ms */
} lub_stats_t;

typedef struct lub_ctx* lub_handle_t;

/* Create a handle on opts->device; copies the parameters. */
int lub_create(lub_handle_t* out, const lub_domain_t* domain,
               const lub_params_t* params, const lub_opts_t* opts);

/* ---- allocation-free evaluation -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * correction as lub_compute (same kernels, same results) without a handle:
 * the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); its workspace is a fixed device array of LUB_STATIC_SCRATCH_BYTES
 * inside the library, one per GPU, held until the process ends.
 *
 * domain, params: as for lub_create (link-wise laws excluded).  opts: device,
 * precision, newton_max_iter, rmax_bound and max_neighbors (<= 0: 64; at
 * most LUB_STATIC_MAX_NEIGHBORS) are used; seed_mode must be LUB_SEED_PLAIN
 * and warm_start, graph, timing, skin and reserved 0 (sync is ignored), else
 * LUB_EINVAL.  Arrays as for lub_compute (device memory, f and t
 * overwritten); n <= LUB_STATIC_MAX_PARTICLES (else LUB_EINVAL).  A call
 * whose workspace does not fit the array (a cell grid too fine for the box,
 * more than 8 evaluated pairs per particle) returns LUB_ECAPACITY before any
 * launch, or sets it on the device.
 *
 * stats: NULL, or a host struct that receives the call's statistics: the
 * call then waits for the stream and returns the error found on the device
 * (input errors, capacity); with NULL the call is fully asynchronous (and
 * may be captured into a graph) and device-side errors are not reported.
 * Every call on one GPU uses that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller. */
#define LUB_STATIC_MAX_PARTICLES 16384
#define LUB_STATIC_MAX_NEIGHBORS 128
#define LUB_STATIC_SCRATCH_BYTES (48u << 20)

int lub_compute_static(const lub_domain_t* domain, const lub_params_t* params,
                       const lub_opts_t* opts, int64_t n, const double* r,
                       const double* q, const double* semi, const double* v,
                       const double* w, double* f, double* t, void* stream,
                       lub_stats_t* stats);

/* Change parameters or domain between calls (no reallocation unless the
 * cell grid grows). */
int lub_set_params(lub_handle_t h, const lub_params_t* params);
int lub_set_domain(lub_handle_t h, const lub_domain_t* domain);

/* The correction: per-particle force f and torque t (device arrays, see
 * the conventions above). */
int lub_compute(lub_handle_t h, int64_t n, const double* r, const double* q,
                const double* semi, const double* v, const double* w,
                double* f, double* t, void* stream);

/* The handle's current domain (lub_integrate advances the Lees-Edwards
 * offset). */
int lub_get_domain(lub_handle_t h, lub_domain_t* out);

/* Sub-stepped explicit particle update (Sec. II): the particle time step is
 * decoupled from the fluid's and made a fraction of it (typically a tenth);
 * the hydrodynamic force from the fluid stays fixed over the fluid step
 * while the lubrication and contact forces are evaluated again at every
 * sub-step.  One call runs step->n_sub sub-steps of length step->dt; each
 * evaluates lub_compute on the current state and then, per particle (mass
 * m = density 4/3 pi R_par R_perp^2, body inertia I_par = 2/5 m R_perp^2 about
 * the axis and I_perp = 1/5 m (R_par^2 + R_perp^2) across it):
 *   F = f_ext + f,  T = t_ext + t
 *   v <- v + dt (F / m - damping v)
 *   L = I(q) w;  L <- L + dt (T - damping L)
 *   q <- rotation by the angle |I(q)^-1 L| dt about I(q)^-1 L, then q
 *   r <- r + dt v;  w <- I(q)^-1 L with the new q
 * (semi-implicit Euler, angular momentum in the world frame).  Periodic
 * axes are wrapped into [0, L); with Lees-Edwards images the offset
 * advances by le_velocity dt per sub-step and a particle leaving through
 * z = L_z (z = 0) re-enters shifted by -offset (+offset) in x with its x
 * velocity reduced (raised) by le_velocity.
 * r, q, v, w: device arrays updated in place.  f_ext, t_ext: device arrays
 * or NULL (zero).  f, t: device arrays receiving the last sub-step's
 * lubrication force and torque.  Errors as lub_compute (the state is left
 * after the last completed sub-step); LUB_EINVAL for dt <= 0, n_sub < 1,
 * density <= 0, damping < 0 or reserved != 0. */
typedef struct {
  double dt;        /* sub-step length */
  int32_t n_sub;    /* sub-steps per call */
  int32_t reserved; /* must be 0 */
  double density;   /* particle mass density */
  double damping;   /* velocity damping rate (1/time); 0 for plain dynamics */
} lub_step_t;

int lub_integrate(lub_handle_t h, int64_t n, double* r, double* q, const double* semi,
                  double* v, double* w, const double* f_ext, const double* t_ext,
                  double* f, double* t, const lub_step_t* step, void* stream);

/* Kinematic advance between evaluations: the particles follow their own
 * velocities with no forces (a prescribed flow such as simple shear moves
 * the suspension from one time step to the next, Sec. III.A), one step of
 * length dt:
 *   r <- r + dt v
 *   q <- normalise(q + dt/2 (0, w) q)   (quaternion product; a rotation by
 *                                         2 atan(dt |w| / 2) about w)
 * FP64.  r (n x 3), q (n x 4): device arrays updated in place; v, w (n x 3):
 * device arrays.  Periodic axes are not wrapped (evaluations take positions
 * outside the box by their images).  Asynchronous on `stream`.  LUB_EINVAL
 * for n < 0, non-finite dt, a null array with n > 0 or a handle with host
 * pointers. */
int lub_advance(lub_handle_t h, int64_t n, double* r, double* q, const double* v,
                const double* w, double dt, void* stream);

/* Growth stage of the packing generator (Sec. IV.C): particles placed
 * without overlap at a reduced size grow linearly from scale0 to scale1
 * times their semi-axes over n_steps sub-steps (scale1 slightly above 1
 * leaves a minimum separation once the size is reset), free to move and
 * turn, with the contact repulsion of Eq. lub:frep (stiffness eps_c, range
 * h_c) as the only interaction and velocities damped at rate damping.  The
 * handle's resistance law and clipping are set aside for the call (model
 * LUB_MODEL_CONTACT with the given h_c, eps_c) and restored afterwards.
 * r, q, v, w: device arrays updated in place; semi: the final semi-axes
 * (not modified).  Needs opts.rmax_bound >= scale1 max(R_par, R_perp). */
typedef struct {
  int32_t n_steps;
  int32_t reserved; /* must be 0 */
  double scale0, scale1;
  double dt, density, damping;
  double h_c, eps_c;
} lub_grow_t;

int lub_grow(lub_handle_t h, int64_t n, double* r, double* q, const double* semi,
             double* v, double* w, const lub_grow_t* cfg, void* stream);

/* Statistics of the last call (waits for the handle's last stream). */
int lub_get_stats(lub_handle_t h, lub_stats_t* out);

/* Zero the accumulated stage times (waits for the handle's last stream). */
int lub_reset_timers(lub_handle_t h);

/* Candidate lists of the last call, in input indices, written to HOST
 * memory: particle pairs ij[k] = (i, j), i < j, sorted by (i, j); wall
 * pairs wall[k] = (i, side) sorted.  *n_pairs / *n_wall receive the counts;
 * LUB_ECAPACITY if a capacity is too small (counts still set). */
int lub_get_pairs(lub_handle_t h, int64_t cap, int32_t* ij, int64_t* n_pairs,
                  int64_t wcap, int32_t* wall, int64_t* n_wall);

/* Per-pair results of the last call for every evaluated pair, HOST memory,
 * in no particular order: ij[k] = (i, j) with j = -1 / -2 for the walls
 * z = 0 / z = L; h[k] signed gap; F[k] force on i; Ti[k] torque on i about
 * its centre; Tj[k] torque on j about its centre (force on j = -F);
 * status[k]: 0 active, 1 inactive (h beyond the cut-offs), 2 unresolved
 * overlap, 3 unconverged; iters[k] Newton iterations. */
int lub_get_pair_results(lub_handle_t h, int64_t cap, int32_t* ij, double* hgap,
                         double* F, double* Ti, double* Tj, int32_t* status,
                         int32_t* iters, int64_t* n_out);

/* With opts.record_detail: per evaluated pair of the last call, in the order
 * of lub_get_pair_results, HOST arrays (each may be NULL): n[k] the unit gap
 * direction from i to j (3), yi[k] = y_i* - r_i and yj[k] = y_j* - r_j (3
 * each; 0 for a wall), e1[k] the principal direction x1 of surface i at its
 * closest point (3; Eq. lub:curvature-directions), Kt[k] the 16 corrective
 * elements of Eq. lub:resistance-correction at the clipped gap, without the
 * viscosity, in the order 11 12 13 14 15 22 23 24 25 33 34 35 36 44 45 55
 * (0 unless the pair is active; the "normal only" law keeps 33 alone).  A
 * pair whose solve failed reports zeros.  LUB_EINVAL without record_detail
 * or for the link-wise laws; LUB_ECAPACITY if cap is too small (*n_out
 * set). */
int lub_get_pair_detail(lub_handle_t h, int64_t cap, double* n, double* yi, double* yj,
                        double* e1, double* Kt, int64_t* n_out);

/* ---- learned Newton seed ------------------------------------------------
 * A 10-128-128-128-4 network with SiLU after the hidden layers predicts the
 * closest-approach parameters (p, q of Eq. lub:spheroid on each particle)
 * of a pair from 10 features in canonical pair frames (the relative centre,
 * the relative orientation as a unit quaternion, three shape ratios).  With
 * opts.seed_mode = LUB_SEED_MLP, lub_compute starts the closest-point Newton
 * iteration from the normal these parameters imply; the iteration always
 * runs to convergence from there, and a pair whose seeded iteration does not
 * converge is solved again from the plain start (counted in
 * lub_stats_t.fallbacks), so the results do not depend on the network.
 * Evaluation and training use BF16 MFMA with FP32 accumulation; the master
 * weights and the Adam moments are FP32.
 *
 * Parameters: LUB_MLP_PARAMS floats, W1 (10 x 128, input-major), b1 (128),
 * W2 (128 x 128), b2, W3 (128 x 128), b3, W4 (128 x 4), b4 (4).
 * Features X: m x 10 float; outputs Y: m x 4 float (p_i, q_i, p_j, q_j);
 * targets T: m x 6 float, the closest points in the canonical frames of i
 * and of j, in units of R_perp of particle i.  Loss: mean over the samples
 * of the squared distance between the surface points of the predicted
 * parameters and the targets. */
#define LUB_MLP_PARAMS 34948

typedef struct {
  int32_t epochs;    /* passes over the training set */
  int32_t batch;     /* samples per step, a multiple of 64 (<= 0: 2048) */
  float lr;          /* Adam step size */
  float beta1;       /* Adam moments (<= 0: 0.9, 0.999, 1e-8) */
  float beta2;
  float eps;
  float lr_decay;    /* step size factor per epoch (<= 0: 1) */
  int32_t reserved;
} lub_train_cfg_t;

/* Copy the FP32 parameters in (host array of n = LUB_MLP_PARAMS floats);
 * resets the Adam moments. */
int lub_mlp_set_weights(lub_handle_t h, const float* theta, int64_t n);
/* Copy the FP32 parameters out (host array). */
int lub_mlp_get_weights(lub_handle_t h, float* theta, int64_t n);
/* Training state for checkpoints: LUB_MLP_STATE floats, the parameters, the
 * Adam first and second moments (LUB_MLP_PARAMS each, in that order) and the
 * number of Adam steps taken (an integer below 2^24 held in a float).  A
 * state saved and loaded into any handle continues training bit for bit as
 * the saving handle would.  lub_mlp_save writes a host array (waits for the
 * device); lub_mlp_load reads one (LUB_EINVAL on a wrong size, a non-finite
 * value or a bad step count). */
#define LUB_MLP_STATE (3 * LUB_MLP_PARAMS + 1)
int lub_mlp_save(lub_handle_t h, float* state, int64_t n);
int lub_mlp_load(lub_handle_t h, const float* state, int64_t n);
/* Uniform initialisation with bound sqrt(6 / fan_in), zero biases, from a
 * seed; resets the Adam moments. */
int lub_mlp_init(lub_handle_t h, uint64_t seed);
/* Y = network(X) for m samples (device arrays). */
int lub_mlp_forward(lub_handle_t h, int64_t m, const float* X, float* Y,
                    void* stream);
/* Loss and gradient of the parameters over m samples (m a multiple of 64;
 * X, T device arrays; loss and grad host: 1 and LUB_MLP_PARAMS floats). */
int lub_mlp_grad(lub_handle_t h, int64_t m, const float* X, const float* T,
                 float* loss, float* grad, void* stream);
/* Adam training over m samples (device arrays), in order, whole batches
 * only (the samples are i.i.d. draws); the mean loss of every epoch is
 * written to epoch_loss (host, cfg->epochs floats, may be NULL). */
int lub_mlp_train(lub_handle_t h, int64_t m, const float* X, const float* T,
                  const lub_train_cfg_t* cfg, float* epoch_loss, void* stream);

void lub_destroy(lub_handle_t h);
const char* lub_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
