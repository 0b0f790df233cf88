// The ID / Nystrom / Woodbury preconditioner handle (Sec. 3, Algorithms 1-4).
#pragma once

#include <vector>

#include "krr_internal.h"

struct krr_precond {
  int64_t n = 0;
  int d = 0, k = 0, l = 0, r = 0, kept = 0, prec = KRR_FP64;
  double eps = 0, tau = 0;
  std::vector<double> betas;
  std::vector<int64_t> S_host;        // anchors (first k pivots)
  std::vector<double> lam_host;       // eigenvalues of K_SS, ascending
  std::vector<double> rdiag_host;     // |R_jj| of the pivoted QR
  int jacobi_sweeps = 0;
  double t_build_ms[6] = {0, 0, 0, 0, 0, 0};   // sketch, qr, evd, factor, core, total
  krr::DevBuf<int64_t> S;
  krr::DevBuf<double> W64;            // n x kept, row-major: W = C V_kept diag(lam_kept)^{-1/2}
  krr::DevBuf<float> W32;             // FP32 copy (prec != FP64)
  krr::DevBuf<double> M64, M32;       // W^T W (kept x kept) for each copy of W
  std::vector<krr::DevBuf<double>> L64;   // per beta: Cholesky factor of beta I + M64 (column-major)
  std::vector<krr::DevBuf<double>> G64;   // per beta: (beta I + M64)^{-1} = L^{-T} L^{-1}
  std::vector<krr::DevBuf<double>> G32;   // per beta: (beta I + M32)^{-1}
  krr::DevBuf<double> Ysk;            // sketch n x l (KRR_KEEP_SKETCH)
};

namespace krr {

int beta_index(const krr_precond& P, double beta);   // -1 if absent

// out[:, c] = (x[:, c] - W z_c) / beta_c, z_c = G_{beta_c} W^T x[:, c]  (x, out: n x R row-major).
// bidx[c]: index of column c's beta in P.betas.  use32: use the FP32 copy of W.
void woodbury_apply(const krr_precond& P, const double* x, int R, const int* bidx_host, bool use32, double* out,
                    hipStream_t s);

// The buffers of the apply for one set of R columns and their betas, allocated and filled once by prepare();
// applies through it launch kernels only (no allocation, no host copy), so they can be captured in a graph.
struct WoodburyWork {
  int R = 0;
  std::vector<int> bidx_host;
  DevBuf<double> partial, t, z;           // one column: W^T x partial sums, t = W^T x, z = G t
  DevBuf<double> invb, T, Zall, Z, tn;    // several columns: 1 / beta, W^T X, G_b T for every beta, selection,
  DevBuf<int> bidx;                       // the row-split partial tiles of W^T X, beta index per column
  void prepare(const krr_precond& P, int R_, const int* bidx_host_, hipStream_t s);
};
void woodbury_apply(const krr_precond& P, const double* x, WoodburyWork& w, bool use32, double* out,
                    hipStream_t s);

}  // namespace krr
