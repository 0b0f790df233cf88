// Entry points not yet implemented in this build step: they report KRR_EINVAL.
#include "krr_internal.h"

#define KRR_NOT_YET(name) krr::guarded([&] { throw krr::Error{KRR_EINVAL, name " is not implemented yet"}; return 0; })
extern "C" {
int krr_sketch(const double*, int64_t, int32_t, double, const double*, const int64_t*, const double*, int32_t, int32_t,
               int32_t, double*, void*) { return KRR_NOT_YET("krr_sketch"); }
int krr_qrcp(const double*, int64_t, int32_t, int32_t, int32_t, int64_t*, double*, void*) { return KRR_NOT_YET("krr_qrcp"); }
int krr_build_precond(const double*, int64_t, int32_t, double, const double*, int32_t, int32_t, int32_t, const double*,
                      const int64_t*, const double*, int32_t, double, int32_t, int32_t, krr_precond**, void*) {
  return KRR_NOT_YET("krr_build_precond"); }
int krr_precond_info(const krr_precond*, int64_t*, int32_t*, double*, double*, int32_t*, int32_t*) { return KRR_NOT_YET("krr_precond_info"); }
int krr_precond_get(const krr_precond*, int32_t, int32_t, void*, size_t, void*) { return KRR_NOT_YET("krr_precond_get"); }
int krr_precond_apply(const krr_precond*, const double*, int32_t, const double*, int32_t, double*, void*) { return KRR_NOT_YET("krr_precond_apply"); }
void krr_precond_free(krr_precond*) {}
int krr_pcg_solve(const double*, int64_t, int32_t, double, const double*, int32_t, const double*, const krr_precond*,
                  double, int32_t, int32_t, int32_t, double*, int32_t*, double*, krr_solve_stats*, int32_t, void*) {
  return KRR_NOT_YET("krr_pcg_solve"); }
int krr_grad(const double*, int64_t, const double*, const double*, int64_t, const double*, int32_t, double, double,
             const krr_precond*, double, int32_t, int32_t, int32_t, double*, double*, double*, double*, double*, void*) {
  return KRR_NOT_YET("krr_grad"); }
int krr_autotune(int32_t, int32_t, int32_t, int64_t, int32_t*, void*) { return KRR_NOT_YET("krr_autotune"); }
int krr_autotune_save(const char*) { return KRR_NOT_YET("krr_autotune_save"); }
int krr_autotune_load(const char*) { return KRR_NOT_YET("krr_autotune_load"); }
int krr_set_variant(int32_t, int32_t, int32_t, int32_t) { return KRR_NOT_YET("krr_set_variant"); }
int krr_num_variants(int32_t, int32_t) { return 0; }
}
