// PCG solver (Algorithm 5) shared by krr_pcg_solve and krr_grad.
#pragma once

#include <vector>

#include "krr_internal.h"

namespace krr {

struct PcgResult {
  std::vector<int> iters;
  std::vector<double> relres;
  krr_solve_stats st{};
  int status = KRR_OK;
};

PcgResult pcg_solve(const double* X, int64_t n, int d, double eps, const double* Y, int R, const double* betas,
                    const krr_precond* P, double tol, int maxit, int replace_every, int prec, double* x,
                    bool timing, hipStream_t s);

}  // namespace krr
