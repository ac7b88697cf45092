// Host build of the library's closest-point solver (lub_newton.h) for the
// CPU tests: the same source the pair kernels compile for gfx950, here with
// g++ so that its branches can be exercised without a GPU.
#include "../../paper_1308_6482_amd/csrc/lub_newton.h"

extern "C" int newton_solve(const double* d, const double* Mi, const double* Mj, int maxit,
                            const double* n0, int use_n0, double* n_out, double* h_out,
                            int* iters) {
  const double dd[3] = {d[0], d[1], d[2]};
  double s[3] = {0.0, 0.0, 0.0};
  if (use_n0)
    for (int k = 0; k < 3; ++k) s[k] = n0[k];
  const lub::Solve o = lub::closest_points(dd, Mi, Mj, maxit, s, use_n0 != 0);
  for (int k = 0; k < 3; ++k) n_out[k] = o.n[k];
  *h_out = o.h;
  *iters = o.iters;
  return o.ok ? 1 : 0;
}
