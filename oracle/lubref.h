/*
 * lubref.h -- plain FP64 CPU oracle of the contact-based lubrication
 * correction for spheroids (Janoschek, Harting, Toschi, "Accurate
 * lubrication corrections for spherical and non-spherical particles in
 * discretized fluid simulations", arXiv:1308.6482).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker the GPU path is
 * compared against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; the two are written independently
 * from the paper.
 *
 * Everything is IEEE double precision, compiled without FP contraction,
 * and evaluated in the order the paper states it:
 *   - pair set: all pairs whose centre distance is below the pruning bound
 *     (Sec. III.A, pruning paragraph), brute force over i<j;
 *   - closest points: the Lin-Han tangent-sphere iteration with the paper's
 *     two-fold radius strategy (Sec. III.A, Eqs. lub:minimum-radius and
 *     lub:convergence), then a Newton polish of the same fixed point to
 *     round-off (the paper's tolerance on cos theta leaves the angle at
 *     about 1e-3), then a duality certificate for separated pairs;
 *   - local geometry: Eq. lub:spheroid parametrisation, principal
 *     directions and radii (Eqs. lub:curvature-directions,
 *     lub:curvature-radii), cubic coefficients Gamma_0, Gamma_2 (Sec. III.B);
 *   - resistance: the 16 singular elements of K (Appendix, Eqs.
 *     app:first-element .. app:last-element) with lambda, chi, beta, k,
 *     kappa as defined there, the corrective matrix of Eq.
 *     lub:resistance-correction and the contact model of Eqs. lub:frep and
 *     lub:model;
 *   - rigid-body transfer of Sec. III.B (last equations of the section);
 *   - the comparison laws: normal only (K33 alone), Ladd's sphere law
 *     (Eq. methods:llub), the contact repulsion alone (growth stage of
 *     Sec. IV.C), and the link-wise laws of Sec. II.D (Eq. methods:dlub,
 *     Ding-Aidun and the averaged-normal variant) over the D3Q19 links
 *     between the lattice sites of the two particles;
 *   - Lees-Edwards images of a sheared periodic box (Sec. IV.C).
 *
 * Parity unpinned (no check independent of this code fixes them): the
 * absolute signs of K13/K23 and K34/K35 beyond the swap, relabel and
 * surface-fit consistency the tests verify; the Lin-Han iteration count
 * (a band around the paper's "almost 40" for aspect ratio 1/3); lambda* of
 * the link-wise law for non-spherical particles (the mean of the two
 * surfaces' mean curvatures; spheres are pinned in closed form).
 *
 * Conventions (the paper leaves them implicit):
 *   q = (w,x,y,z) unit quaternion, x_world = Q(q) x_body, body z axis =
 *   symmetry axis; semi = (R_par, R_perp).  n is the unit gap direction,
 *   the outward normal of the first surface i, pointing to j; the signed
 *   gap is h = n.(y_j - y_i).  Pairs are oriented i<j; in wall pairs the
 *   particle is the first surface.  Walls are the planes z=0 (side 0,
 *   fluid normal +z) and z=L[2] (side 1, fluid normal -z).
 */
#ifndef LUBREF_H
#define LUBREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REF_OK 0
#define REF_EINVAL 1
#define REF_ECAPACITY 2

/* pair status */
#define REFP_ACTIVE 0      /* h < max cut-off: contributes */
#define REFP_INACTIVE 1    /* h >= every cut-off and h > h_c: zero */
#define REFP_UNRESOLVED 2  /* h <= 0 with h_c == 0: K~ undefined, skipped */
#define REFP_FAILED 3      /* closest-point solve did not converge: skipped */

/* Resistance laws the paper compares (Sec. IV, the viscosity and
 * diffusion tables): the full contact-based model; the same with every
 * non-normal element dropped ("normal only"); Ladd's normal law for
 * spheres, Eq. methods:llub (force along the line of centres, no torque). */
#define REF_MODEL_FULL 0
#define REF_MODEL_NORMAL 1
#define REF_MODEL_LADD 2
#define REF_MODEL_CONTACT 3 /* no lubrication: the repulsion of Eq. lub:frep alone */
#define REF_MODEL_LINK 4    /* link-wise law of Ding and Aidun, Eq. methods:dlub */
#define REF_MODEL_LINK_NAVG 5 /* the same projected on the average normal (Clausen) */

typedef struct {
  double mu;       /* dynamic viscosity */
  double delta_n;  /* cut-off for K33 */
  double delta_t;  /* cut-off for all elements but K33 and the 44/45/55 block */
  double delta_r;  /* cut-off for K44, K45, K54, K55 */
  double h_c;      /* clipping gap of Eq. lub:model */
  double eps_c;    /* Hookean stiffness of Eq. lub:frep */
  int32_t model;   /* REF_MODEL_*; the reduced models are active below delta_n */
  int32_t reserved;
  double q_bar;    /* empirical weight of the link-wise law (0.6) */
} ref_params;

typedef struct {
  double L[3];
  int32_t periodic[3];
  int32_t n_walls;          /* 0 or 2 (planes z=0 and z=L[2]) */
  double wall_vel[2][3];    /* translational velocity of each wall */
  /* Lees-Edwards images (sheared periodic box, Sec. IV.C): the image one box
   * up in z of a particle at r with velocity v sits at r + (le_offset, 0, L_z)
   * and moves with v + (le_velocity, 0, 0).  Needs all axes periodic and no
   * walls. */
  int32_t lees_edwards;
  int32_t reserved;
  double le_offset;
  double le_velocity;
} ref_domain;

typedef struct {
  int32_t status;      /* REFP_* */
  int32_t fallback;    /* 1 if the conservative Lin-Han phase was needed */
  int32_t iters_lh;    /* Lin-Han iterations (both phases) */
  int32_t iters_polish;/* Newton polish iterations */
  double h;            /* signed gap */
  double n[3];         /* unit gap direction, i -> j */
  double yi[3];        /* closest point on i, relative to r_i */
  double yj[3];        /* closest point on j, relative to r_j (its image) */
  double certificate;  /* |y_j - y_i| - h for h > 0 (>= 0, ~0) */
  double e[3][3];      /* e1, e2, e3 of surface i (rows) */
  double S1, S2;       /* principal radii of i */
  double invS1p, invS2p; /* inverse principal radii of j (0 for a wall) */
  double G[4], Gp[4];  /* cubic coefficients Gamma_0..3 of i and j */
  double cphi, sphi;   /* angle between x1 and x1' */
  double lam1, lam2, cchi, schi;
  double kappa[4];
  double C[6][6];      /* K = C*ln(h) (C33/h for element 33) */
  double Kt[6][6];     /* corrective matrix at h_eff */
  double Fbar[6];      /* local force/torque on i (x1,x2,x3 frame) */
  double F[3];         /* force on i, world frame (force on j = -F) */
  double Ti[3];        /* torque on i about r_i */
  double Tj[3];        /* torque on j about r_j */
  int32_t links;       /* link-wise laws: contributing links (h* < |c_r|) */
  int32_t pad_;
} ref_pair_result;

typedef struct {
  int64_t candidates;       /* particle-particle pairs passing the centre test */
  int64_t wall_candidates;  /* particle-wall pairs passing the wall test */
  int64_t active;           /* pairs (incl. wall) that contribute */
  int64_t overlaps;         /* active pairs with h <= 0 */
  int64_t unresolved;
  int64_t failed;
  int64_t fallbacks;
  int64_t iters_lh_total;
  int64_t iters_lh_max;
  int64_t iters_polish_total;
  int32_t threads;          /* OpenMP threads actually used */
} ref_stats;

/* Quaternion (w,x,y,z), normalised internally, to the body->world matrix
 * (row-major 3x3). */
void ref_quat_to_matrix(const double q[4], double Q[9]);

/* Exact FP64 centre test of the pruning paragraph of Sec. III.A, with the
 * minimum image on periodic axes.  Written without FP contraction so the
 * GPU can reproduce it bit for bit. */
int ref_centre_test(const double ri[3], const double rj[3], double rmax_i,
                    double rmax_j, double dmax, const ref_domain* dom);

/* Brute-force candidate lists.  Particle pairs (i<j) sorted by (i,j);
 * wall pairs (i, side) sorted by (i, side).  Returns REF_ECAPACITY when a
 * capacity is too small (counts are still reported). */
int ref_candidates(int64_t n, const double* r, const double* semi,
                   const ref_domain* dom, const ref_params* prm,
                   int64_t cap, int32_t* ij, int64_t* n_pairs,
                   int64_t wcap, int32_t* wall, int64_t* n_wall);

/* Closest points, gap and full correction for one particle pair, given
 * both particles' data and the (image) centre offset d = r_j - r_i. */
int ref_pair_eval(const double d[3], const double qi[4], const double semii[2],
                  const double vi[3], const double wi[3], const double qj[4],
                  const double semij[2], const double vj[3], const double wj[3],
                  const ref_params* prm, ref_pair_result* out);

/* Link-wise laws (REF_MODEL_LINK, REF_MODEL_LINK_NAVG) for one particle
 * pair: ri is i's absolute centre (the lattice sites are the integer
 * points), d the offset of j's image.  out->h is the smallest link gap,
 * out->links the number of contributing links. */
int ref_link_eval(const double ri[3], const double d[3], const double qi[4],
                  const double semii[2], const double vi[3], const double wi[3],
                  const double qj[4], const double semij[2], const double vj[3],
                  const double wj[3], const ref_params* prm, ref_pair_result* out);

/* Same for a particle and a wall (side 0: z=0, side 1: z=L). */
int ref_wall_eval(const double ri[3], const double qi[4], const double semii[2],
                  const double vi[3], const double wi[3], int side,
                  const ref_domain* dom, const ref_params* prm,
                  ref_pair_result* out);

/* Closest points only (no resistance), for label generation. */
int ref_closest_points(const double d[3], const double qi[4],
                       const double semii[2], const double qj[4],
                       const double semij[2], ref_pair_result* out);

/* Singular coefficients C (K = C ln h, C33/h) from the local geometry,
 * general Gamma_0..3 on both surfaces.  aux receives lam1, lam2, cos chi,
 * sin chi, kappa0..3 (8 values). */
void ref_K_coeffs(double S1, double S2, double invS1p, double invS2p,
                  const double G[4], const double Gp[4], double cphi,
                  double sphi, double C[6][6], double aux[8]);

/* Full evaluation: per-particle force f (n x 3) and torque t (n x 3),
 * overwritten.  nthreads <= 0: OpenMP default.  Per-particle sums are in
 * FP64 and in a fixed order (pair list order, then wall pairs). */
int ref_compute(int64_t n, const double* r, const double* q,
                const double* semi, const double* v, const double* w,
                const ref_domain* dom, const ref_params* prm, int nthreads,
                double* f, double* t, ref_stats* st);

/* Per-particle force and torque for a subset of particles (brute-force
 * partner scan per sampled particle; same orientation and summation order
 * as ref_compute).  For large systems where the full oracle is too slow. */
/* The candidate partners (the centre test of ref_candidates) of each of
 * the m particles idx[s], in increasing index, into partners[s*cap ..]
 * (brute force over all particles); counts[s] their number.
 * REF_ECAPACITY if a particle has more than cap. */
int ref_partners_subset(int64_t n, const double* r, const double* semi,
                        const ref_domain* dom, const ref_params* prm, int64_t m,
                        const int64_t* idx, int64_t cap, int32_t* partners,
                        int64_t* counts);

int ref_compute_subset(int64_t n, const double* r, const double* q,
                       const double* semi, const double* v, const double* w,
                       const ref_domain* dom, const ref_params* prm,
                       int64_t m, const int64_t* idx, int nthreads,
                       double* f, double* t, ref_stats* st);

/* Evaluate a given list of particle pairs (and wall pairs): per-pair
 * F, Ti, Tj (each npairs x 3), h and status.  Used by parity tests on
 * sampled pairs. */
int ref_eval_pairs(int64_t n, const double* r, const double* q,
                   const double* semi, const double* v, const double* w,
                   const ref_domain* dom, const ref_params* prm,
                   int64_t np, const int32_t* ij, int nthreads,
                   double* F, double* Ti, double* Tj, double* h,
                   int32_t* status, int32_t* links);

/* As ref_eval_pairs, with the intermediate results of every pair: the unit
 * gap direction n, y_i - r_i, y_j - r_j (3 each), the frame axis e1 of
 * surface i (3), the corrective matrix K~ at the clipped gap (36, row-major,
 * without the viscosity), and the Lin-Han and polish iteration counts.  Any
 * output pointer may be NULL. */
int ref_eval_pairs_detail(int64_t n, const double* r, const double* q,
                          const double* semi, const double* v, const double* w,
                          const ref_domain* dom, const ref_params* prm,
                          int64_t np, const int32_t* ij, int nthreads,
                          double* F, double* Ti, double* Tj, double* h,
                          int32_t* status, double* nrm, double* yi, double* yj,
                          double* e1, double* Kt, int32_t* iters_lh,
                          int32_t* iters_polish);

/* Pairs at a prescribed gap along a prescribed direction (the learned
 * seed's training and held-out pairs): for each of the m pairs, the centre
 * separation s > 0 along the unit vector u[k] at which the gap of
 * ref_closest_points equals target[k] > 0, and the closest points there.
 * The gap along a ray, dist(s u, K_i - K_j), is convex and increasing in s
 * outside the bodies with slope n.u (n the unit gap direction), so Newton's
 * method started at the bounding-sphere distance R_max,i + R_max,j +
 * target converges monotonically from above; it stops when the gap is
 * within 1e-12 (1 + target) of the target.  Outputs per pair: s, the gap
 * h, n, y_i - r_i, y_j - r_j (each 3), the Lin-Han iterations of the last
 * solve, and a status (0 placed, 3 a solve failed or no convergence).
 * OpenMP over the pairs (nthreads <= 0: the default). */
int ref_place_pairs(int64_t m, const double* u, const double* target,
                    const double* qi, const double* semii, const double* qj,
                    const double* semij, int nthreads, double* s, double* h,
                    double* n, double* yi, double* yj, int32_t* iters_lh,
                    int32_t* status);

#ifdef __cplusplus
}
#endif
#endif
