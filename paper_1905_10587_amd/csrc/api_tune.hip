// C ABI: kernel-variant control and the autotuner of the kernel MVM's launch table (consulted by every kernel
// MVM launch).  The autotuner times the variants (tile shapes, fragments per wave, pipelining, LDS staging,
// symmetric form) and source splits / super-tile edges of (d, R, prec) at a problem size n with HIP events
// and keeps the fastest for that size class; the table can be saved and loaded as JSON.
#include <algorithm>
#include <fstream>
#include <sstream>
#include <vector>

#include "kmv.h"

namespace krr {

// splitmix64-based uniform numbers in [0, 1) (synthetic timing inputs only)
__global__ void k_fill_uniform(double* __restrict__ a, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  a[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace krr

extern "C" int krr_set_variant(int32_t d, int32_t R, int32_t prec, int32_t variant) {
  return krr::guarded([&] {
    KRR_REQUIRE(d >= 1 && d <= KRR_MAX_D, "d must be in [1, KRR_MAX_D]");
    KRR_REQUIRE(prec >= KRR_FP64 && prec <= KRR_MIXED, "unknown precision");
    KRR_REQUIRE(variant < krr::kmv_num_variants(prec, R), "variant out of range");
    krr::kmv_set_override(d, R, prec, variant);
    return (int)KRR_OK;
  });
}

extern "C" int krr_num_variants(int32_t prec, int32_t R) { return krr::kmv_num_variants(prec, R); }

extern "C" int krr_kmv_variant(int32_t d, int32_t R, int32_t deriv, int32_t prec, int32_t square, int64_t n,
                               int32_t* variant, int32_t* symmetric) {
  return krr::guarded([&] {
    KRR_REQUIRE(d >= 1 && d <= KRR_MAX_D, "d must be in [1, KRR_MAX_D]");
    KRR_REQUIRE(R >= 1 && R <= 256, "R must be in [1, 256]");
    KRR_REQUIRE(deriv >= 0 && deriv <= 2, "deriv must be 0, 1 or 2");
    KRR_REQUIRE(prec >= KRR_FP64 && prec <= KRR_MIXED, "unknown precision");
    KRR_REQUIRE(variant && symmetric, "null output pointer");
    const bool sq = square != 0 && deriv == 0;
    int v = krr::kmv_lookup(prec, d, R, n, sq).variant;
    if (v < 0) v = krr::kmv_default_variant(prec, d, R, n > 0 ? n : 0, n > 0 ? n : 0, sq);
    *variant = v;
    *symmetric = krr::kmv_is_symmetric(prec, d, R, deriv, square != 0, v) ? 1 : 0;
    return (int)KRR_OK;
  });
}

extern "C" int krr_kmv_last_launch(int32_t* variant, int32_t* split, int32_t* symmetric) {
  return krr::guarded([&] {
    KRR_REQUIRE(variant && split && symmetric, "null output pointer");
    const krr::KmvLaunchInfo li = krr::kmv_last_launch();
    *variant = li.variant;
    *split = li.split;
    *symmetric = li.symmetric;
    return (int)KRR_OK;
  });
}

// Search for square products K(X, X) V of n points (the solver's case): every variant at the launcher's own
// split, then the two fastest with the split halved and doubled (sources per block of the direct forms, the
// super-tile edge of the symmetric forms).  Each candidate: one warm-up launch, then up to three timed
// launches (stopped after one when it is already three times slower than the best).  The winner is recorded
// for (prec, d, shape class of R, floor(log2 n), square).
extern "C" int krr_autotune(int32_t d, int32_t R, int32_t prec, int64_t n, int32_t* best_variant, void* stream) {
  using namespace krr;
  return guarded([&] {
    KRR_REQUIRE(d >= 1 && d <= KRR_MAX_D, "d must be in [1, KRR_MAX_D]");
    KRR_REQUIRE(prec >= KRR_FP64 && prec <= KRR_MIXED, "unknown precision");
    KRR_REQUIRE(R >= 1 && R <= 256, "R must be in [1, 256]");
    KRR_REQUIRE(n >= 1024 && n <= (int64_t)1 << 26, "n must be in [1024, 2^26]");
    KRR_REQUIRE(best_variant != nullptr, "best_variant must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> X(n * d, s), V(n * R, s), U(n * R, s);
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)ceil_div(n * d, 256)), dim3(256), 0, s, X.p, n * d, 1234ull);
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, V.p, n * R, 99ull);
    KRR_LAUNCH_CHECK();
    const double eps = 0.05 * d;
    const int dpad = padded_dim(d);
    DevBuf<double> center(dpad, s);
    point_mean(X.p, n, d, dpad, center.p, s);
    Staged S;
    stage_points(S, X.p, n, d, eps, prec, center.p, true, true, s);
    StagedVec SV;
    stage_vectors(SV, V.p, n, S.npad, R, prec, s);
    DevBuf<double> ws;
    hipEvent_t e0, e1;
    KRR_CHECK_HIP(hipEventCreate(&e0));
    KRR_CHECK_HIP(hipEventCreate(&e1));
    struct EvGuard {
      hipEvent_t a, b;
      ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } guard{e0, e1};
    float best = 1e30f;
    auto time_one = [&](int v, int split, int* used_split) -> float {
      kmv_launch(S, S, SV, 0, nullptr, V.p, prec, U.p, R, s, v, &ws, nullptr, split);   // warm-up
      *used_split = kmv_last_launch().split;
      float tot = 0;
      int reps = 0;
      for (; reps < 3; ++reps) {
        KRR_CHECK_HIP(hipEventRecord(e0, s));
        kmv_launch(S, S, SV, 0, nullptr, V.p, prec, U.p, R, s, v, &ws, nullptr, split);
        KRR_CHECK_HIP(hipEventRecord(e1, s));
        KRR_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0;
        KRR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        tot += ms;
        if (ms > 3.0f * best) { ++reps; break; }
      }
      return tot / reps;
    };
    const int nv = kmv_num_variants(prec, R);
    std::vector<std::pair<float, std::pair<int, int>>> res;   // (ms, (variant, split))
    for (int v = 0; v < nv; ++v) {
      int used = 0;
      const float ms = time_one(v, 0, &used);
      res.push_back({ms, {v, used}});
      best = std::min(best, ms);
    }
    std::sort(res.begin(), res.end());
    KmvChoice win{res[0].second.first, 0};
    float win_ms = res[0].first;
    for (size_t t = 0; t < std::min<size_t>(2, res.size()); ++t) {
      const int v = res[t].second.first, sp0 = res[t].second.second;
      for (int sp : {sp0 / 2, sp0 * 2}) {
        if (sp < 1) continue;
        int used = 0;
        const float ms = time_one(v, sp, &used);
        if (used == sp0) continue;   // the launcher would not take this split: nothing new was timed
        if (ms < win_ms) { win_ms = ms; win = KmvChoice{v, used}; }
      }
    }
    kmv_set_tuned(prec, d, R, n, true, win);
    *best_variant = win.variant;
    return (int)KRR_OK;
  });
}

extern "C" int krr_autotune_save(const char* path) {
  return krr::guarded([&] {
    KRR_REQUIRE(path != nullptr, "path must not be NULL");
    std::ofstream f(path);
    KRR_REQUIRE(f.good(), std::string("cannot open ") + path);
    f << krr::kmv_table_json();
    return (int)KRR_OK;
  });
}

extern "C" int krr_autotune_load(const char* path) {
  return krr::guarded([&] {
    KRR_REQUIRE(path != nullptr, "path must not be NULL");
    std::ifstream f(path);
    KRR_REQUIRE(f.good(), std::string("cannot open ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    krr::kmv_table_from_json(ss.str());
    return (int)KRR_OK;
  });
}
