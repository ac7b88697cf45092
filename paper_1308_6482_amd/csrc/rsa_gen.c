/*
 * rsa_gen.c -- random sequential addition of ellipsoids for the synthetic
 * input generators.  Not part of the lubrication path: it only decides
 * where particles go.  The overlap test is the Perram-Wertheim contact
 * function (max over l in [0,1] of l(1-l) d^T [(1-l) MA + l MB]^{-1} d < 1
 * means overlap), maximised by golden-section search, which never
 * over-estimates the maximum, so accepted pairs never overlap.
 *
 * The caller draws every random number (numpy PCG64) and hands trials in
 * chunks; this routine only accepts or rejects them in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n_target;   /* number of particles to place */
  int64_t placed;     /* placed so far */
  double L[3];
  int32_t periodic[3];
  double cell[3];
  int32_t nc[3];
  int32_t* head;      /* cell -> first particle, -1 terminated */
  int32_t* next;      /* particle -> next particle in its cell */
  double* r;          /* n_target x 3 */
  double* q;          /* n_target x 4 */
  double* M;          /* n_target x 9 (shape matrix Q D^2 Q^T) */
  const double* semi; /* n_target x 2, placement order */
  double rmax_glob;
  int32_t le;         /* Lees-Edwards images: one box up in z is shifted by */
  double le_offset;   /* le_offset in x */
} rsa_state;

static void quat_mat(const double* q, double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

static void shape_mat(const double* q, const double* semi, double M[9]) {
  double R[9], d2[3] = {semi[1] * semi[1], semi[1] * semi[1], semi[0] * semi[0]};
  quat_mat(q, R);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += R[3 * a + k] * d2[k] * R[3 * b + k];
      M[3 * a + b] = s;
    }
}

/* d^T C^{-1} d for symmetric positive definite C (adjugate formula) */
static double quad_inv(const double C[9], const double d[3]) {
  double a = C[0], b = C[1], c = C[2], e = C[4], f = C[5], i = C[8];
  double A = e * i - f * f, B = c * f - b * i, Cc = b * f - c * e;
  double E = a * i - c * c, F = b * c - a * f, I = a * e - b * b;
  double det = a * A + b * B + c * Cc;
  double v = d[0] * (A * d[0] + B * d[1] + Cc * d[2]) +
             d[1] * (B * d[0] + E * d[1] + F * d[2]) +
             d[2] * (Cc * d[0] + F * d[1] + I * d[2]);
  return v / det;
}

static double pw_value(const double MA[9], const double MB[9], const double d[3],
                       double lam) {
  double C[9];
  for (int k = 0; k < 9; ++k) C[k] = (1 - lam) * MA[k] + lam * MB[k];
  return lam * (1 - lam) * quad_inv(C, d);
}

static int pw_overlap(const double MA[9], const double MB[9], const double d[3]) {
  const double g = 0.6180339887498949;
  double a = 0.0, b = 1.0;
  for (int it = 0; it < 48; ++it) {
    double c1 = b - g * (b - a), c2 = a + g * (b - a);
    if (pw_value(MA, MB, d, c1) > pw_value(MA, MB, d, c2))
      b = c2;
    else
      a = c1;
  }
  return pw_value(MA, MB, d, 0.5 * (a + b)) < 1.0;
}

static int cell_of(const rsa_state* s, const double x[3], int c[3]) {
  for (int k = 0; k < 3; ++k) {
    int v = (int)floor(x[k] / s->cell[k]);
    if (v < 0) v = 0;
    if (v >= s->nc[k]) v = s->nc[k] - 1;
    c[k] = v;
  }
  return (c[2] * s->nc[1] + c[1]) * s->nc[0] + c[0];
}

/* does the trial at x (shape matrix Mi, semi-axes sem) overlap particle j's
 * nearest image? */
static int overlaps(const rsa_state* s, const double x[3], const double* Mi,
                    const double* sem, int32_t j) {
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = s->r[3 * j + k] - x[k];
  if (s->le) {
    double m = nearbyint(d[2] / s->L[2]);
    d[2] -= s->L[2] * m;
    d[0] -= m * s->le_offset;
  }
  for (int k = 0; k < 3; ++k)
    if (s->periodic[k] && !(s->le && k == 2)) d[k] -= s->L[k] * nearbyint(d[k] / s->L[k]);
  double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double* sj = &s->semi[2 * j];
  double rmi = sem[0] > sem[1] ? sem[0] : sem[1];
  double rni = sem[0] < sem[1] ? sem[0] : sem[1];
  double rmj = sj[0] > sj[1] ? sj[0] : sj[1];
  double rnj = sj[0] < sj[1] ? sj[0] : sj[1];
  if (dist >= rmi + rmj) return 0;
  if (dist < rni + rnj) return 1;
  return pw_overlap(Mi, &s->M[9 * j], d);
}

void* rsa_create(int64_t n_target, const double* semi, const double L[3],
                 const int32_t periodic[3]) {
  rsa_state* s = (rsa_state*)calloc(1, sizeof(rsa_state));
  s->n_target = n_target;
  s->semi = semi;
  double rm = 0.0;
  for (int64_t i = 0; i < n_target; ++i) {
    double m = semi[2 * i] > semi[2 * i + 1] ? semi[2 * i] : semi[2 * i + 1];
    if (m > rm) rm = m;
  }
  s->rmax_glob = rm;
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) {
    s->L[k] = L[k];
    s->periodic[k] = periodic[k];
    int nc = (int)floor(L[k] / (2.0 * rm));
    if (nc < 1) nc = 1;
    if (nc > 1024) nc = 1024;
    s->nc[k] = nc;
    s->cell[k] = L[k] / nc;
    ncell *= nc;
  }
  s->head = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
  for (int64_t c = 0; c < ncell; ++c) s->head[c] = -1;
  s->next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_target);
  s->r = (double*)malloc(sizeof(double) * 3 * (size_t)n_target);
  s->q = (double*)malloc(sizeof(double) * 4 * (size_t)n_target);
  s->M = (double*)malloc(sizeof(double) * 9 * (size_t)n_target);
  return s;
}

void rsa_destroy(void* p) {
  rsa_state* s = (rsa_state*)p;
  if (!s) return;
  free(s->head);
  free(s->next);
  free(s->r);
  free(s->q);
  free(s->M);
  free(s);
}

/* Process trials in order: pos (m x 3, in [0,1) units of L), quat (m x 4,
 * unit).  Returns the number of trials consumed (stops when all particles
 * are placed). */
int64_t rsa_run(void* p, int64_t m, const double* pos, const double* quat,
                double wall_margin) {
  rsa_state* s = (rsa_state*)p;
  int64_t t;
  for (t = 0; t < m && s->placed < s->n_target; ++t) {
    int64_t i = s->placed;
    const double* sem = &s->semi[2 * i];
    double x[3] = {pos[3 * t] * s->L[0], pos[3 * t + 1] * s->L[1],
                   pos[3 * t + 2] * s->L[2]};
    double Mi[9];
    shape_mat(&quat[4 * t], sem, Mi);
    int ok = 1;
    for (int k = 0; k < 3 && ok; ++k)
      if (!s->periodic[k]) {
        double ext = sqrt(Mi[4 * k]);
        if (x[k] - ext < wall_margin || x[k] + ext > s->L[k] - wall_margin)
          ok = 0;
      }
    if (!ok) continue;
    int c[3];
    cell_of(s, x, c);
    int visited[27];
    int nvis = 0;
    for (int dz = -1; dz <= 1 && ok; ++dz)
      for (int dy = -1; dy <= 1 && ok; ++dy)
        for (int dx = -1; dx <= 1 && ok; ++dx) {
          int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
          int skip = 0;
          /* Lees-Edwards: rows across the z boundary are searched whole
           * in x (from the dx = 0 pass) */
          const int zwrap = s->le && (cc[2] < 0 || cc[2] >= s->nc[2]);
          if (zwrap) {
            if (dx != 0) continue;
            int cy = ((cc[1] % s->nc[1]) + s->nc[1]) % s->nc[1];
            int cz = ((cc[2] % s->nc[2]) + s->nc[2]) % s->nc[2];
            if (cz == c[2]) continue; /* the own row is searched directly */
            for (int ax = 0; ax < s->nc[0] && ok; ++ax) {
              int id = (cz * s->nc[1] + cy) * s->nc[0] + ax;
              for (int32_t j = s->head[id]; j >= 0 && ok; j = s->next[j])
                if (overlaps(s, x, Mi, sem, j)) ok = 0;
            }
            continue;
          }
          for (int k = 0; k < 3; ++k) {
            if (s->periodic[k])
              cc[k] = ((cc[k] % s->nc[k]) + s->nc[k]) % s->nc[k];
            else if (cc[k] < 0 || cc[k] >= s->nc[k])
              skip = 1;
          }
          if (skip) continue;
          int id = (cc[2] * s->nc[1] + cc[1]) * s->nc[0] + cc[0];
          for (int v = 0; v < nvis; ++v)
            if (visited[v] == id) skip = 1;
          if (skip) continue;
          visited[nvis++] = id;
          for (int32_t j = s->head[id]; j >= 0 && ok; j = s->next[j])
            if (overlaps(s, x, Mi, sem, j)) ok = 0;
        }
    if (!ok) continue;
    memcpy(&s->r[3 * i], x, sizeof(x));
    memcpy(&s->q[4 * i], &quat[4 * t], 4 * sizeof(double));
    memcpy(&s->M[9 * i], Mi, sizeof(Mi));
    int id = cell_of(s, x, c);
    s->next[i] = s->head[id];
    s->head[id] = (int32_t)i;
    s->placed++;
  }
  return t;
}

int64_t rsa_placed(void* p) { return ((rsa_state*)p)->placed; }

/* Lees-Edwards images for the overlap test (all axes periodic): the image
 * one box up in z sits le_offset further in x. */
void rsa_set_lees_edwards(void* p, double le_offset) {
  rsa_state* s = (rsa_state*)p;
  s->le = 1;
  s->le_offset = le_offset;
}

void rsa_fetch(void* p, double* r, double* q) {
  rsa_state* s = (rsa_state*)p;
  memcpy(r, s->r, sizeof(double) * 3 * (size_t)s->placed);
  memcpy(q, s->q, sizeof(double) * 4 * (size_t)s->placed);
}
