// C ABI: krr_kernel_mv (the paper's FIG(targets, sources, h, V), Sec. 2.4, computed exactly).
#include "kmv.h"

namespace krr {

void validate_common(int64_t m, int64_t n, int32_t d, double eps) {
  KRR_REQUIRE(m >= 1 && n >= 1, "point counts must be >= 1");
  KRR_REQUIRE(d >= 1 && d <= KRR_MAX_D, "d must be in [1, KRR_MAX_D]");
  KRR_REQUIRE(eps > 0 && std::isfinite(eps), "eps must be positive and finite");
}

void validate_prec(int32_t prec) {
  KRR_REQUIRE(prec == KRR_FP64 || prec == KRR_FP32 || prec == KRR_MIXED, "unknown precision");
}

// Full MVM from raw FP64 inputs: stages both point sets (shared centre) and the vectors.
void kernel_mv_raw(const double* Xt, int64_t m, const double* Xs, int64_t n, int d, double eps, const double* V,
                   int R, const double* shift, int deriv, int prec, double* U, int64_t ldu, hipStream_t s) {
  const bool same = (Xt == Xs) && (m == n);
  const int dpad = padded_dim(d);
  DevBuf<double> center(dpad, s);
  point_mean(Xs, n, d, dpad, center.p, s);
  Staged S, T;
  // square one-column mixed products may be staged in spatial order for exact far-tile culling
  const bool sort = same && prec == KRR_MIXED && R == 1 && deriv == 0 && cull_wanted(Xs, n, d, eps, s);
  stage_points(S, Xs, n, d, eps, prec, center.p, same, true, s, sort);
  if (!same) stage_points(T, Xt, m, d, eps, prec, center.p, true, false, s);
  StagedVec SV;
  stage_vectors(SV, V, n, S.npad, R, prec, s, S.perm.p);
  kmv_launch(same ? S : T, S, SV, deriv, shift, V, prec, U, ldu, s);
}

}  // namespace krr

extern "C" int krr_kernel_mv(const double* Xt, int64_t m, const double* Xs, int64_t n, int32_t d, double eps,
                             const double* V, int32_t R, const double* shift, int32_t deriv, int32_t prec,
                             double* U, void* stream) {
  return krr::guarded([&] {
    krr::validate_common(m, n, d, eps);
    krr::validate_prec(prec);
    KRR_REQUIRE(Xt && Xs && V && U, "null pointer argument");
    KRR_REQUIRE(R >= 1 && R <= 256, "R must be in [1, 256]");
    KRR_REQUIRE(deriv >= 0 && deriv <= 2, "deriv must be 0, 1 or 2");
    KRR_REQUIRE(shift == nullptr || m == n, "shift requires targets == sources");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(Xt, m * (int64_t)d, "Xt", s);
    if (Xs != Xt) krr::check_finite_device(Xs, n * (int64_t)d, "Xs", s);
    krr::check_finite_device(V, n * (int64_t)R, "V", s);
    if (shift)
      for (int c = 0; c < R; ++c) KRR_REQUIRE(std::isfinite(shift[c]), "shift must be finite");
    const int64_t ldu = deriv == 2 ? 2 * (int64_t)R : R;
    krr::kernel_mv_raw(Xt, m, Xs, n, d, eps, V, R, shift, deriv, prec, U, ldu, s);
    return (int)KRR_OK;
  });
}
