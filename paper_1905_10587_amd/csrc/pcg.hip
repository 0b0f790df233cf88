// Preconditioned conjugate gradient for (K + beta_c I) alpha_c = y_c, c = 0..R-1 (Algorithm 5, Sec. 3).
//
// All R recurrences advance in lockstep and share one kernel MVM of the whole block per iteration
// (multi-right-hand-side batching); every column keeps its own FP64 scalars (rho, gamma, beta) and is
// frozen once its true relative residual reaches tol.  Vectors x, r, z, p, q are FP64, n x R
// row-major.  The MVM runs in the working precision (FP64, FP32 or split-BF16 mixed); every
// `replace_every` iterations, and whenever a column's recursive residual claims convergence, the
// residual is recomputed as y - (K + beta I) x with the FP64 MVM (residual replacement).
// Whether a column's recursive residual claims convergence is decided on the device (in the final kernel
// of the residual-norm reduction); the host reads these claims with the norms and runs the true-residual
// check, the stopping rules and the safeguards.  Two drivers run the same kernels in the same order: a host
// loop with one synchronisation per iteration, and graph-captured cycles of `replace_every` iterations (one
// launch and one synchronisation per cycle) that halt on the device when a claim or a breakdown needs the host.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "kmv.h"
#include "pcg.h"
#include "precond.h"

namespace krr {

void validate_common(int64_t m, int64_t n, int32_t d, double eps);
void validate_prec(int32_t prec);

// ------------------------------------------------------------------ column reductions
// Block: 256 threads = CB columns x (256/CB) rows.  Deterministic two-stage sum:
// part[by * R + c] over row groups, then a fixed-order sum over by.
constexpr int kRedBlocks = 256;

// Halt gate of the graph-captured cycles.  *halt is 0, or u + 1 once the status of the cycle's iteration u
// has asked the host for a decision (a convergence claim or a breakdown); a gated kernel of stage `stage`
// does nothing when a status of an earlier stage has halted the cycle (kernels of iteration u up to its
// status have stage u + 1, the direction update after it u + 2).  halt == nullptr: never closed.
struct Gate {
  const int* halt = nullptr;
  int stage = 0;
  __device__ bool closed() const {
    if (!halt) return false;
    const int h = __hip_atomic_load(halt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return h != 0 && h < stage;
  }
};

template <int MODE>   // 0: sum a*b ; 1: sum a*a
__global__ __launch_bounds__(256) void k_coldot(const double* __restrict__ a, const double* __restrict__ b,
                                                int64_t n, int R, int CB, double* __restrict__ part, Gate gate) {
  if (gate.closed()) return;
  __shared__ double red[256];
  const int cl = threadIdx.x % CB;
  const int rl = threadIdx.x / CB;
  const int rows_per = 256 / CB;
  const int c = blockIdx.x * CB + cl;
  double s = 0;
  if (c < R) {
    for (int64_t i = (int64_t)blockIdx.y * rows_per + rl; i < n; i += (int64_t)gridDim.y * rows_per) {
      const double u = a[i * R + c];
      s = __builtin_fma(u, MODE == 1 ? u : b[i * R + c], s);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = rows_per / 2; w > 0; w >>= 1) {
    if (rl < w) red[threadIdx.x] += red[threadIdx.x + w * CB];
    __syncthreads();
  }
  if (rl == 0 && c < R) part[(int64_t)blockIdx.y * R + c] = red[threadIdx.x];
}

// x += gamma p ; r -= gamma q, and the partial sums of the new r^2 in the order of k_coldot<1> (the same
// grid, rows and tree), so the residual norms are those of the separate update and dot product.
__global__ __launch_bounds__(256) void k_axpy2_rr(double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ gamma, int64_t n, int R, int CB,
                                                  double* __restrict__ part, Gate gate) {
  if (gate.closed()) return;
  __shared__ double red[256];
  const int cl = threadIdx.x % CB;
  const int rl = threadIdx.x / CB;
  const int rows_per = 256 / CB;
  const int c = blockIdx.x * CB + cl;
  double s = 0;
  if (c < R) {
    const double g = gamma[c];
    for (int64_t i = (int64_t)blockIdx.y * rows_per + rl; i < n; i += (int64_t)gridDim.y * rows_per) {
      const int64_t t = i * R + c;
      x[t] = __builtin_fma(g, p[t], x[t]);
      const double u = __builtin_fma(-g, q[t], r[t]);
      r[t] = u;
      s = __builtin_fma(u, u, s);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = rows_per / 2; w > 0; w >>= 1) {
    if (rl < w) red[threadIdx.x] += red[threadIdx.x + w * CB];
    __syncthreads();
  }
  if (rl == 0 && c < R) part[(int64_t)blockIdx.y * R + c] = red[threadIdx.x];
}

// Scalar work done by the final reduction kernel on the column's sum v (saves a launch per scalar step):
//   kGamma:  gamma_c = rho_c / v for active columns (0 otherwise), breakdown flag if v <= 0 or not finite;
//   kBeta:   beta_c = v / rho_c for active columns (0 otherwise; v is the new r^T z);
//   kStatus: the status of iteration it for the host, stored into host-mapped memory,
//            hs = [rr = v (R) | gamma (R) | beta of the previous iteration (R) | claim (R) | flags (2)],
//            claim_c = 1 when column c is active, it >= next_check_c and sqrt(v) / ||y_c|| <= tol (its
//            recursive residual claims convergence); a claim or the breakdown flag closes the halt gate
//            (when there is one) at this kernel's stage;
//   kCheck:  the squared true residual norms of a check, also stored into hs (R).
// it = *it_base + it_off (it_base may be null: it = it_off).
struct DotEpilogue {
  enum Mode { kNone = 0, kGamma = 1, kBeta = 2, kStatus = 3, kCheck = 4 };
  int mode = kNone;
  const double* rho = nullptr;
  const int* active = nullptr;
  double* gamma = nullptr;
  double* beta = nullptr;
  int* flags = nullptr;
  double* hs = nullptr;
  const int* next_check = nullptr;
  const double* ynorm = nullptr;
  double tol = 0.0;
  const int* it_base = nullptr;
  int it_off = 0;
  int* halt = nullptr;
};

// The epilogue of column c's sum v (thread-level; out[c] = v first).  Returns gamma_c (kGamma) or beta_c
// (kBeta), 0 otherwise.
__device__ __forceinline__ double dot_epilogue(const DotEpilogue& e, const Gate& gate, int c, int R, double v,
                                               double* __restrict__ out) {
  out[c] = v;
  if (e.mode == DotEpilogue::kGamma) {
    double g = 0.0;
    if (e.active[c]) {
      if (!(v > 0.0) || !isfinite(v)) atomicOr(e.flags, 1);
      else g = e.rho[c] / v;
    }
    e.gamma[c] = g;
    return g;
  } else if (e.mode == DotEpilogue::kBeta) {
    double b = 0.0;
    if (e.active[c]) b = e.rho[c] != 0.0 ? v / e.rho[c] : 0.0;
    e.beta[c] = b;
    return b;
  } else if (e.mode == DotEpilogue::kStatus) {
    const int it = (e.it_base ? *e.it_base : 0) + e.it_off;
    const bool claim = e.active[c] && it >= e.next_check[c] && sqrt(v) / e.ynorm[c] <= e.tol;
    e.hs[c] = v;
    e.hs[R + c] = e.gamma[c];
    e.hs[2 * R + c] = e.beta[c];
    e.hs[3 * R + c] = claim ? 1.0 : 0.0;
    const int broke = c == 0 ? __hip_atomic_load(e.flags + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    if (c == 0) {
      e.hs[4 * R] = (double)e.flags[0];
      e.hs[4 * R + 1] = (double)broke;
    }
    if (e.halt && (claim || broke)) __hip_atomic_store(e.halt, gate.stage, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (e.mode == DotEpilogue::kCheck) {
    e.hs[c] = v;
  }
  return 0.0;
}

// out[c] = sum_by part[by, c]: one block per column, fixed-order LDS tree (nby <= 256), then the epilogue.
__global__ __launch_bounds__(256) void k_colsum_final(const double* __restrict__ part, int nby, int R,
                                                      double* __restrict__ out, DotEpilogue e, Gate gate) {
  if (gate.closed()) return;
  __shared__ double red[256];
  const int c = blockIdx.x;
  red[threadIdx.x] = (int)threadIdx.x < nby ? part[(int64_t)threadIdx.x * R + c] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) dot_epilogue(e, gate, c, R, red[0], out);
}

// ------------------------------------------------------------------ one-block forms for small problems
// For n * R <= kSmallElems one workgroup of 1024 threads does a whole reduction step, so that an iteration
// needs two launches besides the MVM and the preconditioner.  Threads: CB columns x (1024 / CB) rows per
// column group; per column a fixed-order LDS tree over the rows' partial sums.
constexpr int kSmallThreads = 1024;
constexpr int64_t kSmallElems = 16384;

// red: 1024 doubles; returns (at rl == 0) the sum over all threads of the column lane cl.  One column: a
// butterfly within each wave, then the 16 wave sums in order; several: a fixed-order LDS tree per column.
__device__ __forceinline__ double block_colsum(double* red, double s, int CB) {
  const int t = threadIdx.x;
  if (CB == 1) {
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kSmallThreads / 64; ++w) v += red[w];
    __syncthreads();
    return v;
  }
  const int rl = t / CB;
  red[t] = s;
  __syncthreads();
  for (int w = (kSmallThreads / CB) / 2; w > 0; w >>= 1) {
    if (rl < w) red[t] += red[t + w * CB];
    __syncthreads();
  }
  const double v = red[t];
  __syncthreads();
  return v;
}

// One iteration's update after its product q = A p: gamma = rho / p^T q (the kGamma epilogue, with the
// breakdown flag), x += gamma p, r -= gamma q, rr = r^T r, and the status (the kStatus epilogue ee).
__global__ __launch_bounds__(kSmallThreads) void k_step_small(double* __restrict__ x, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ q, int64_t n, int R,
                                                              int CB, double* __restrict__ pq,
                                                              double* __restrict__ rr, DotEpilogue eg,
                                                              DotEpilogue es, Gate gate) {
  if (gate.closed()) return;
  __shared__ double red[kSmallThreads];
  __shared__ double sg[256];   // gamma per column (R <= 256)
  const int cl = threadIdx.x % CB;
  const int rl = threadIdx.x / CB;
  const int rows = kSmallThreads / CB;
  for (int c0 = 0; c0 < R; c0 += CB) {
    const int c = c0 + cl;
    double s = 0.0;
    if (c < R)
      for (int64_t i = rl; i < n; i += rows) s = __builtin_fma(p[i * R + c], q[i * R + c], s);
    const double v = block_colsum(red, s, CB);
    if (rl == 0 && c < R) sg[c] = dot_epilogue(eg, gate, c, R, v, pq);
  }
  __syncthreads();   // every column's gamma and the breakdown flag are written
  for (int c0 = 0; c0 < R; c0 += CB) {
    const int c = c0 + cl;
    double s = 0.0;
    if (c < R) {
      const double g = sg[c];
      for (int64_t i = rl; i < n; i += rows) {
        const int64_t t = i * R + c;
        x[t] = __builtin_fma(g, p[t], x[t]);
        const double u = __builtin_fma(-g, q[t], r[t]);
        r[t] = u;
        s = __builtin_fma(u, u, s);
      }
    }
    const double v = block_colsum(red, s, CB);
    if (rl == 0 && c < R) dot_epilogue(es, gate, c, R, v, rr);
  }
}

// The next direction after z = M^{-1} r: rho_new = r^T z and beta = rho_new / rho (the kBeta epilogue eb),
// then pout = z + beta pin for active columns, pin for the others (pout may be pin).
__global__ __launch_bounds__(kSmallThreads) void k_dir_small(const double* __restrict__ r,
                                                             const double* __restrict__ z, const double* pin,
                                                             double* pout, const int* __restrict__ active,
                                                             int64_t n, int R, int CB, double* __restrict__ rho_new,
                                                             DotEpilogue eb, Gate gate) {
  if (gate.closed()) return;
  __shared__ double red[kSmallThreads];
  __shared__ double sb[256];   // beta per column (R <= 256)
  const int cl = threadIdx.x % CB;
  const int rl = threadIdx.x / CB;
  const int rows = kSmallThreads / CB;
  for (int c0 = 0; c0 < R; c0 += CB) {
    const int c = c0 + cl;
    double s = 0.0;
    if (c < R)
      for (int64_t i = rl; i < n; i += rows) s = __builtin_fma(r[i * R + c], z[i * R + c], s);
    const double v = block_colsum(red, s, CB);
    if (rl == 0 && c < R) sb[c] = dot_epilogue(eb, gate, c, R, v, rho_new);
  }
  __syncthreads();
  for (int c0 = 0; c0 < R; c0 += CB) {
    const int c = c0 + cl;
    if (c >= R) continue;
    const double b = sb[c];
    const bool act = active[c] != 0;
    for (int64_t i = rl; i < n; i += rows) {
      const int64_t t = i * R + c;
      pout[t] = act ? __builtin_fma(b, pin[t], z[t]) : pin[t];
    }
  }
}

struct ColReducer {
  DevBuf<double> part;
  int R = 0, CB = 1;
  void init(int R_, hipStream_t s) {
    R = R_;
    CB = 1;
    while (CB * 2 <= R && CB < 64) CB *= 2;
    part.alloc((size_t)kRedBlocks * R, s);
  }
  // out[c] = sum_i a[i,c] * b[i,c]  (b == nullptr: sum a^2), then the epilogue's scalar step
  void dot(const double* a, const double* b, int64_t n, double* out, hipStream_t s,
           const DotEpilogue& e = DotEpilogue(), Gate gate = Gate()) {
    dim3 grid((unsigned)ceil_div(R, CB), kRedBlocks);
    if (b) hipLaunchKernelGGL(k_coldot<0>, grid, dim3(256), 0, s, a, b, n, R, CB, part.p, gate);
    else hipLaunchKernelGGL(k_coldot<1>, grid, dim3(256), 0, s, a, a, n, R, CB, part.p, gate);
    hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)R), dim3(256), 0, s, part.p, kRedBlocks, R, out, e, gate);
    KRR_LAUNCH_CHECK();
  }
  // x += gamma p, r -= gamma q, rr = column sums of the new r^2 (as dot(r, nullptr) after the update)
  void axpy2_rr(double* x, double* r, const double* p, const double* q, const double* gamma, int64_t n,
                double* rr, hipStream_t s, const DotEpilogue& e, Gate gate = Gate()) {
    dim3 grid((unsigned)ceil_div(R, CB), kRedBlocks);
    hipLaunchKernelGGL(k_axpy2_rr, grid, dim3(256), 0, s, x, r, p, q, gamma, n, R, CB, part.p, gate);
    hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)R), dim3(256), 0, s, part.p, kRedBlocks, R, rr, e, gate);
    KRR_LAUNCH_CHECK();
  }
};

// ------------------------------------------------------------------ elementwise / scalar kernels
// r = y - q for active columns
__global__ void k_residual(double* __restrict__ r, const double* __restrict__ y, const double* __restrict__ q,
                           const int* __restrict__ active, int64_t n, int R, Gate gate) {
  if (gate.closed()) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  if (active[t % R]) r[t] = y[t] - q[t];
}

// Pinned, device-visible host buffer for the status store (one per thread, grown on demand, kept for the
// life of the process).
static double* status_buffer(size_t count) {
  thread_local double* buf = nullptr;
  thread_local size_t cap = 0;
  if (count > cap) {
    if (buf) KRR_CHECK_HIP(hipHostFree(buf));
    buf = nullptr;
    cap = 0;
    KRR_CHECK_HIP(hipHostMalloc((void**)&buf, count * sizeof(double), hipHostMallocDefault));
    cap = count;
  }
  return buf;
}

// p = z + beta p (active columns)
__global__ void k_update_p(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ beta,
                           const int* __restrict__ active, int64_t n, int R, Gate gate) {
  if (gate.closed()) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  const int c = (int)(t % R);
  if (active[c]) p[t] = __builtin_fma(beta[c], p[t], z[t]);
}

// out = z + beta p for active columns, p for the others (the look-ahead iteration writes a second buffer)
__global__ void k_update_p_to(double* __restrict__ out, const double* __restrict__ p, const double* __restrict__ z,
                              const double* __restrict__ beta, const int* __restrict__ active, int64_t n, int R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  const int c = (int)(t % R);
  out[t] = active[c] ? __builtin_fma(beta[c], p[t], z[t]) : p[t];
}

__global__ void k_copy_active(double* __restrict__ dst, const double* __restrict__ src,
                              const int* __restrict__ active, int64_t n, int R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  if (active[t % R]) dst[t] = src[t];
}

__global__ void k_absmax_flag(const double* __restrict__ a, int64_t cnt, int* __restrict__ flag) {
  int f = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    f |= a[i] != 0.0;
  if (f) atomicOr(flag, 1);
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) dst[t] = src[t];
}

// First and last node of a captured cycle: open the halt gate and take the cycle's starting iteration from
// the host-mapped control words ctrl = [iteration, halt]; report the gate's final state there.
__global__ void k_cycle_begin(int* __restrict__ halt, int* __restrict__ it_base, const double* __restrict__ ctrl) {
  if (threadIdx.x == 0) {
    *halt = 0;
    *it_base = (int)ctrl[0];
  }
}

// ... and copy the cycle's statuses and check (written to device memory during the cycle) to the host-mapped
// words in one pass, so that no iteration of the cycle waits on a store to host memory.
__global__ void k_cycle_end(const int* __restrict__ halt, double* __restrict__ ctrl, const double* __restrict__ src,
                            double* __restrict__ dst, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) ctrl[1] = (double)*halt;
}

static unsigned nb(int64_t n) { return (unsigned)ceil_div(n, 256); }

// ------------------------------------------------------------------ solver
struct EventTimer {
  bool on;
  hipStream_t s;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double* acc;
  EventTimer(bool on_, hipStream_t s_) : on(on_), s(s_), acc(nullptr) {}
  void start(double* where) {
    if (!on) return;
    hipEvent_t a, b;
    KRR_CHECK_HIP(hipEventCreate(&a));
    KRR_CHECK_HIP(hipEventCreate(&b));
    KRR_CHECK_HIP(hipEventRecord(a, s));
    open = ev.size();
    ev.push_back({a, b});
    acc = where;
    pending.push_back(where);
  }
  void stop() {   // ends the interval opened by the last start() (external pairs may follow it)
    if (!on) return;
    KRR_CHECK_HIP(hipEventRecord(ev[open].second, s));
  }
  size_t open = 0;
  // a pair of events that the callee records (around one kernel inside a library call); nullptr when off
  const hipEvent_t* external(double* where) {
    if (!on) return nullptr;
    hipEvent_t a, b;
    KRR_CHECK_HIP(hipEventCreate(&a));
    KRR_CHECK_HIP(hipEventCreate(&b));
    ev.push_back({a, b});
    pending.push_back(where);
    ext[0] = a;
    ext[1] = b;
    return ext;
  }
  hipEvent_t ext[2] = {nullptr, nullptr};
  // collect after a synchronise (the first `upto` intervals: those recorded before the point waited for)
  void collect(size_t upto = SIZE_MAX) {
    upto = std::min(upto, ev.size());
    for (size_t i = 0; i < upto; ++i) {
      float ms = 0;
      KRR_CHECK_HIP(hipEventElapsedTime(&ms, ev[i].first, ev[i].second));
      *pending[i] += ms;
      (void)hipEventDestroy(ev[i].first);
      (void)hipEventDestroy(ev[i].second);
    }
    ev.erase(ev.begin(), ev.begin() + upto);
    pending.erase(pending.begin(), pending.begin() + upto);
  }
  size_t marks() const { return ev.size(); }
  // intervals not collected yet are charged to `where` instead (work whose result was discarded)
  void retarget(double* where) {
    for (auto& w : pending) w = where;
  }
  std::vector<double*> pending;
  ~EventTimer() {
    for (auto& e : ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
};

// Staged operator (K + beta I) on one point set in one precision.
struct Operator {
  Staged S;
  StagedVec V;
  DevBuf<double> ws;
  int prec = KRR_FP64;
  const double* X = nullptr;
  int64_t n = 0;
  int R = 0;
  void init(const double* X_, int64_t n_, int d, double eps, int prec_, const double* center, int R_, hipStream_t s) {
    X = X_;
    n = n_;
    prec = prec_;
    R = R_;
    // one-column mixed operators may be staged in spatial order for exact far-tile culling
    const bool sort = prec == KRR_MIXED && R == 1 && cull_wanted(X, n, d, eps, s);
    stage_points(S, X, n, d, eps, prec, center, true, true, s, sort);
  }
  // out = (K + diag(shift)) v   (shift may be null).  cols (device, ncols entries): only those columns of v are
  // multiplied, into the same columns of out (shift then holds their ncols shifts); the others are not written.
  void apply(const double* v, const double* shift, double* out, hipStream_t s, const hipEvent_t* kev = nullptr,
             const int* cols = nullptr, int ncols = 0) {
    if (cols) stage_vectors(V, v, n, S.npad, ncols, prec, s, nullptr, cols, R);
    else stage_vectors(V, v, n, S.npad, R, prec, s, S.perm.p);
    kmv_launch(S, S, V, 0, shift, v, prec, out, R, s, -1, &ws, kev);
  }
};

// Driver selection (krr_set_pcg_mode): -1 automatic, 0 host loop, 1 graph-captured cycles.
static std::atomic<int> g_pcg_mode{-1};
void set_pcg_mode(int mode) { g_pcg_mode.store(mode); }

// Iterations per captured cycle without scheduled replacements.
constexpr int kGraphCycle = 16;

// Automatic choice: graph cycles where launches and synchronisations are a visible share of an iteration
// (products of at most 2^30 pair-columns: n <= 32768 for one column).  Above that the products that run after
// a halt cost more than the synchronisations saved (n = 1e5, R = 1: 501 ms against 491 ms for the host loop;
// n = 2000: 19 ms against 22 ms).  Cycles are replace_every iterations long (at most 64), or kGraphCycle
// without replacement.
static bool use_graph_cycles(int64_t n, int R, int replace_every, bool timing) {
  if (timing || replace_every > 64) return false;
  const int mode = g_pcg_mode.load();
  if (mode == 0) return false;
  if (mode == 1) return true;
  return (double)n * (double)n * (double)R <= 1073741824.0;
}

PcgResult pcg_solve(const double* X, int64_t n, int d, double eps, const double* Y, int R, const double* betas,
                    const krr_precond* P, double tol, int maxit, int replace_every, int prec, double* x,
                    bool timing, hipStream_t s) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  PcgResult res;
  res.iters.assign(R, 0);
  res.relres.assign(R, 0.0);
  std::vector<int> bidx(R, 0);
  if (P) {
    for (int c = 0; c < R; ++c) {
      bidx[c] = beta_index(*P, betas[c]);
      KRR_REQUIRE(bidx[c] >= 0, "a column's beta is not among the preconditioner's betas");
    }
    KRR_REQUIRE(P->n == n && P->d == d && P->eps == eps, "preconditioner was built for a different problem");
    KRR_REQUIRE(prec == KRR_FP64 || P->W32.p, "FP32/mixed solve needs a preconditioner built with FP32 factors");
  }
  const int64_t nR = n * R;
  const int dpad = padded_dim(d);
  DevBuf<double> center(dpad, s);
  point_mean(X, n, d, dpad, center.p, s);
  Operator Aw, A64;
  Aw.init(X, n, d, eps, prec, center.p, R, s);
  Operator* Atrue = &Aw;
  if (prec != KRR_FP64) {
    A64.init(X, n, d, eps, KRR_FP64, center.p, R, s);
    Atrue = &A64;
  }
  WoodburyWork ww;
  if (P) ww.prepare(*P, R, bidx.data(), s);
  DevBuf<double> r(nR, s), z(nR, s), p(nR, s), q(nR, s), p2(nR, s), q2(nR, s);
  for (double* b : {p.p, q.p, p2.p, q2.p}) KRR_CHECK_HIP(hipMemsetAsync(b, 0, sizeof(double) * nR, s));
  DevBuf<double> sc(8 * (size_t)R, s);   // rho (two buffers), pq, gamma, beta, rr, yy, ||y||
  // r^T z of the current iteration and of the next one; the host swaps the two when an iteration
  // advances, so a discarded look-ahead leaves rho as it was
  double* rho = sc.p;
  double* rho_new = sc.p + 5 * R;
  double* pq = sc.p + R;
  double* gamma = sc.p + 2 * R;
  double* beta = sc.p + 3 * R;
  double* rr = sc.p + 4 * R;
  double* yy = sc.p + 6 * R;
  double* ynorm_d = sc.p + 7 * R;
  // current search direction and its product; the look-ahead iteration writes the other pair
  double* pp = p.p;
  double* qq = q.p;
  double* pa = p2.p;
  double* qa = q2.p;
  DevBuf<int> active(R, s), flags(2, s);
  DevBuf<int> ictl(2 + (size_t)R, s);   // halt gate, cycle's first iteration, next_check (R)
  int* halt_d = ictl.p;
  int* it_base_d = ictl.p + 1;
  int* next_check_d = ictl.p + 2;
  ColReducer red;
  red.init(R, s);
  std::vector<int> act(R, 1);
  std::vector<double> h(3 * (size_t)R);
  EventTimer tm(timing, s);
  const bool graph_on = use_graph_cycles(n, R, replace_every, timing);
  const int B = !graph_on ? 1 : replace_every > 0 ? replace_every : kGraphCycle;   // iterations per cycle
  const bool cycle_check = replace_every > 0;   // a cycle ends with the scheduled check of its last iteration

  // ||y_c||
  red.dot(Y, nullptr, n, yy, s);
  std::vector<double> ynorm(R);
  KRR_CHECK_HIP(hipMemcpyAsync(h.data(), yy, sizeof(double) * R, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < R; ++c) {
    ynorm[c] = std::sqrt(h[c]);
    if (!(ynorm[c] > 0)) act[c] = 0;
  }
  std::vector<int> next_check(R, 0);
  // Products of a block with frozen columns form only the active ones (their columns gathered when staged,
  // scattered when finished); the frozen columns of q keep their last, finite values, which their zero step
  // lengths never use.
  std::vector<int> acols;
  std::vector<double> ashift;
  DevBuf<int> cols_d(R, s);
  const int* colsp = nullptr;   // device list of the active columns, nullptr when every column takes part
  int ncols = R;
  bool graphs_stale = false;    // captured cycles launch products of the previous active set
  // device copies of the mask, the norms and the check schedule the status kernel decides claims with
  // (copied from host vectors: the stream is synchronised before they change)
  auto upload_state = [&]() {
    KRR_CHECK_HIP(hipMemcpyAsync(active.p, act.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
    KRR_CHECK_HIP(hipMemcpyAsync(next_check_d, next_check.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
    acols.clear();
    ashift.clear();
    for (int c = 0; c < R; ++c)
      if (act[c]) {
        acols.push_back(c);
        ashift.push_back(betas[c]);
      }
    const bool sub = R > 1 && !acols.empty() && (int)acols.size() < R;
    if (sub) KRR_CHECK_HIP(hipMemcpyAsync(cols_d.p, acols.data(), sizeof(int) * acols.size(), hipMemcpyHostToDevice, s));
    if ((sub ? cols_d.p : nullptr) != colsp || (sub ? (int)acols.size() : R) != ncols) graphs_stale = true;
    colsp = sub ? cols_d.p : nullptr;
    ncols = sub ? (int)acols.size() : R;
    KRR_CHECK_HIP(hipStreamSynchronize(s));
  };
  // out = (K + diag(beta)) v with operator A over the active columns
  auto product = [&](Operator& A, const double* v, double* out, hipStream_t st, const hipEvent_t* kev) {
    A.apply(v, colsp ? ashift.data() : betas, out, st, kev, colsp, ncols);
  };
  KRR_CHECK_HIP(hipMemcpyAsync(ynorm_d, ynorm.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  upload_state();
  // zero-rhs columns: alpha = 0
  // initial residual r = y - (K + beta I) x0 (FP64), skipped for a zero initial guess
  KRR_CHECK_HIP(hipMemsetAsync(flags.p, 0, 2 * sizeof(int), s));
  hipLaunchKernelGGL(k_absmax_flag, dim3(std::min<unsigned>(nb(nR), 2048)), dim3(256), 0, s, x, nR, flags.p);
  int hflags[2];
  KRR_CHECK_HIP(hipMemcpyAsync(hflags, flags.p, sizeof(hflags), hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  if (hflags[0]) {
    tm.start(&res.st.t_mvm_fp64_ms);
    product(*Atrue, x, q.p, s, nullptr);
    tm.stop();
    res.st.n_mvm_fp64++;
    KRR_CHECK_HIP(hipMemcpyAsync(r.p, Y, sizeof(double) * nR, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_residual, dim3(nb(nR)), dim3(256), 0, s, r.p, Y, q.p, active.p, n, R, Gate());
  } else {
    KRR_CHECK_HIP(hipMemcpyAsync(r.p, Y, sizeof(double) * nR, hipMemcpyDeviceToDevice, s));
  }
  auto precondition = [&](const double* in, double* out, hipStream_t st) {
    if (P) {
      tm.start(&res.st.t_precond_ms);
      woodbury_apply(*P, in, ww, prec != KRR_FP64, out, st);
      tm.stop();
    } else {
      hipLaunchKernelGGL(k_copy, dim3(nb(nR)), dim3(256), 0, st, out, in, nR);
      KRR_LAUNCH_CHECK();
    }
  };
  precondition(r.p, z.p, s);
  KRR_CHECK_HIP(hipMemcpyAsync(pp, z.p, sizeof(double) * nR, hipMemcpyDeviceToDevice, s));
  red.dot(r.p, z.p, n, rho, s);

  // Lanczos coefficients of column 0, recorded until its recursive residual first claims convergence:
  // the true-residual check that follows replaces r by a vector of rounding-error size relative to the
  // recurrence, after which the coefficients no longer describe a Lanczos process of the operator.
  std::vector<double> lanczos_g, lanczos_b;
  bool lanczos_open = true, pending_b = false;
  // host-mapped status words: one status per iteration of a cycle, the true residuals of its check, and
  // the control words [first iteration, halt]
  const size_t SS = 4 * (size_t)R + 2;
  double* hs = status_buffer(B * SS + R + 2);
  double* hcheck = hs + B * SS;
  double* hctrl = hcheck + R;
  // the same statuses and check in device memory, for the captured cycles
  DevBuf<double> dstat(graph_on ? B * SS + R : 0, s);
  double* dhs = dstat.p;
  double* dcheck = graph_on ? dstat.p + B * SS : nullptr;
  // Safeguards: the best iterate by true residual is kept per column.  The residual 2-norm of CG is
  // not monotone (CG minimises the A-norm of the error), so a column is only stopped (KRR_ENOCONV, best
  // iterate returned) when its true residual is not finite or exceeds 1e6 times its best, or when its
  // recursive residual has claimed convergence 8 times without the true residual reaching tol (the
  // attainable accuracy of the recurrence is reached).  After a failed convergence check a column is
  // not checked again for max(replace_every, 5) iterations.
  DevBuf<double> xbest(nR, s);
  DevBuf<int> mask(R, s);
  std::vector<double> best_rel(R, HUGE_VAL);
  std::vector<int> stall(R, 0), gave_up(R, 0);
  std::vector<char> claim(R, 0);
  const int recheck = std::max(replace_every, 5);
  auto copy_columns = [&](double* dst, const double* src, const std::vector<int>& m) {
    KRR_CHECK_HIP(hipMemcpyAsync(mask.p, m.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_copy_active, dim3(nb(nR)), dim3(256), 0, s, dst, src, mask.p, n, R);
    KRR_LAUNCH_CHECK();
    KRR_CHECK_HIP(hipStreamSynchronize(s));
  };
  bool any_active = false;
  for (int c = 0; c < R; ++c) any_active |= act[c] != 0;
  int it = 0;
  bool breakdown = false;
  // KRR_PROGRESS=k prints the iteration count and the largest recursive relative residual every k iterations
  const char* prog_env = std::getenv("KRR_PROGRESS");
  const int progress = prog_env ? std::atoi(prog_env) : 0;
  // scalar steps carried by the final kernels of the dot products
  auto epi_gamma = [&](const double* rho_cur) {
    DotEpilogue e;
    e.mode = DotEpilogue::kGamma;
    e.rho = rho_cur;
    e.active = active.p;
    e.gamma = gamma;
    e.flags = flags.p + 1;
    return e;
  };
  auto epi_beta = [&](const double* rho_cur) {
    DotEpilogue e;
    e.mode = DotEpilogue::kBeta;
    e.rho = rho_cur;
    e.active = active.p;
    e.beta = beta;
    return e;
  };
  // the status of iteration *it_base + it_off into `slot`; halt: the cycle's gate (null in the host loop)
  auto epi_status = [&](double* slot, const int* it_base, int it_off, int* halt) {
    DotEpilogue e;
    e.mode = DotEpilogue::kStatus;
    e.active = active.p;
    e.gamma = gamma;
    e.beta = beta;
    e.flags = flags.p;
    e.hs = slot;
    e.next_check = next_check_d;
    e.ynorm = ynorm_d;
    e.tol = tol;
    e.it_base = it_base;
    e.it_off = it_off;
    e.halt = halt;
    return e;
  };
  // Reads the status of iteration `it`: Lanczos coefficients, iteration counts, the columns' claims.
  // Returns false on a breakdown.
  auto read_status = [&](const double* st, bool& candidate) -> bool {
    candidate = false;
    if (st[4 * R + 1] != 0.0) return false;
    if (pending_b) lanczos_b.push_back(st[2 * R]);   // beta of the previous iteration, column 0
    pending_b = false;
    if (act[0] && lanczos_open) lanczos_g.push_back(st[R]);
    for (int c = 0; c < R; ++c) {
      h[c] = st[c];
      claim[c] = st[3 * R + c] != 0.0;
      if (!act[c]) continue;
      res.iters[c] = it;
      if (claim[c]) {
        candidate = true;
        if (c == 0) lanczos_open = false;
      }
    }
    if (progress > 0 && it % progress == 0) {
      double worst = 0;
      for (int c = 0; c < R; ++c)
        if (act[c]) worst = std::max(worst, std::sqrt(h[c]) / ynorm[c]);
      std::fprintf(stderr, "krr pcg: iteration %d, max recursive relres %.3e, %.1f ms\n", it, worst,
                   std::chrono::duration<double, std::milli>(clk::now() - t_start).count());
      std::fflush(stderr);
    }
    return true;
  };
  bool fresh_true = false;  // the true residuals of the current x were computed by this iteration's check
  // The decisions on the squared true residual norms rrt of the current x (a check): converged columns stop,
  // the best iterate is kept, stalled or diverging columns stop.
  auto decide = [&](const double* rrt) {
    bool changed = false, improved = false;
    std::vector<int> imp(R, 0);
    for (int c = 0; c < R; ++c) {
      if (!act[c]) continue;
      const double rel = std::sqrt(rrt[c]) / ynorm[c];
      res.relres[c] = rel;
      if (rel <= tol) {
        act[c] = 0;
        changed = true;
        continue;
      }
      // only a column whose recursive residual claimed convergence and failed the check waits before
      // its next check; a scheduled replacement leaves the others free to claim at the next iteration
      if (claim[c]) {
        next_check[c] = it + recheck;
        ++stall[c];
        changed = true;
      }
      if (rel < best_rel[c]) {
        best_rel[c] = rel;
        imp[c] = 1;
        improved = true;
      }
      if (stall[c] >= 8 || rel > 1e6 * best_rel[c] || !std::isfinite(rel)) {
        act[c] = 0;
        gave_up[c] = 1;
        changed = true;
      }
    }
    if (improved) copy_columns(xbest.p, x, imp);
    if (changed) upload_state();
    fresh_true = true;
  };
  // true residual in FP64 (replaces the recursive one), then the decisions
  auto check = [&](bool scheduled) {
    tm.start(&res.st.t_mvm_fp64_ms);
    product(*Atrue, x, qq, s, nullptr);
    tm.stop();
    res.st.n_mvm_fp64++;
    if (scheduled) res.st.n_replace++;
    hipLaunchKernelGGL(k_residual, dim3(nb(nR)), dim3(256), 0, s, r.p, Y, qq, active.p, n, R, Gate());
    red.dot(r.p, nullptr, n, rr, s);
    KRR_CHECK_HIP(hipMemcpyAsync(h.data(), rr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    tm.collect();
    decide(h.data());
  };
  // Small problems run each reduction step as one workgroup (k_step_small, k_dir_small), larger ones as the
  // two-stage column reductions; both drivers take the same choice.
  const bool small = (int64_t)n * R <= kSmallElems;
  int CBs = 1;
  while (CBs * 2 <= R && CBs < 64) CBs *= 2;
  // one iteration's update after its product q = A p: gamma, x += gamma p, r -= gamma q, and its status
  auto step = [&](hipStream_t st, const DotEpilogue& es, Gate gate) {
    if (small) {
      hipLaunchKernelGGL(k_step_small, dim3(1), dim3(kSmallThreads), 0, st, x, r.p, (const double*)pp,
                         (const double*)qq, n, R, CBs, pq, rr, epi_gamma(rho), es, gate);
      KRR_LAUNCH_CHECK();
    } else {
      red.dot(pp, qq, n, pq, st, epi_gamma(rho), gate);
      red.axpy2_rr(x, r.p, pp, qq, gamma, n, rr, st, es, gate);
    }
  };
  // z = M^{-1} r, rho_new = r^T z, beta = rho_new / rho, pout = z + beta pin (pin for inactive columns)
  auto direction = [&](hipStream_t st, double* pin, double* pout, Gate gate) {
    precondition(r.p, z.p, st);
    if (small) {
      hipLaunchKernelGGL(k_dir_small, dim3(1), dim3(kSmallThreads), 0, st, (const double*)r.p, (const double*)z.p,
                         (const double*)pin, pout, (const int*)active.p, n, R, CBs, rho_new, epi_beta(rho), gate);
    } else {
      red.dot(r.p, z.p, n, rho_new, st, epi_beta(rho), gate);
      if (pout == pin)
        hipLaunchKernelGGL(k_update_p, dim3(nb(nR)), dim3(256), 0, st, pin, z.p, beta, active.p, n, R, gate);
      else
        hipLaunchKernelGGL(k_update_p_to, dim3(nb(nR)), dim3(256), 0, st, pout, (const double*)pin,
                           (const double*)z.p, (const double*)beta, (const int*)active.p, n, R);
    }
    KRR_LAUNCH_CHECK();
  };
  // the step (do_step, with its status es) and then the next direction pout = z + beta pin (do_dir)
  auto step_dir = [&](hipStream_t st, bool do_step, const DotEpilogue& es, Gate gstep, bool do_dir, double* pin,
                      double* pout, Gate gdir) {
    if (do_step) step(st, es, gstep);
    if (do_dir) direction(st, pin, pout, gdir);
  };
  // the next direction after a decision, in place
  auto enqueue_direction = [&](hipStream_t st, Gate gate) {
    step_dir(st, false, DotEpilogue(), Gate(), true, pp, pp, gate);
    std::swap(rho, rho_new);
  };
  hipEvent_t ev_status;
  KRR_CHECK_HIP(hipEventCreateWithFlags(&ev_status, hipEventDisableTiming));
  struct EventGuard {
    hipEvent_t e;
    ~EventGuard() { (void)hipEventDestroy(e); }
  } ev_guard{ev_status};

  // Graph-captured cycles.  A cycle starts after the host's decisions on the previous iteration and holds:
  // the next direction, `B` iterations (the MVM, p^T q, the x / r update with the status, and, except after
  // the last, the next direction), then, with scheduled replacements, the check of the last iteration (FP64
  // product, r = y - (K + beta I) x, its norms).  The status kernels decide the claims on the device; a claim or a breakdown
  // closes the halt gate, after which the remaining kernels that change the solver's state do nothing, so x,
  // r, p and the scalars are those of the iteration that asked, exactly as the host loop leaves them.  The
  // host then reads the statuses and continues as the host loop does.  The products of the iterations after
  // a halt still run (on scratch buffers; their results are not used).  One graph is captured per set of
  // buffer pointers it reads (the direction / product buffers and the parity of the two rho buffers).
  struct CycleGraph {
    const double *pp, *qq, *rho;
    hipGraphExec_t exec;
  };
  std::vector<CycleGraph> graphs;
  hipStream_t cs = nullptr;   // capture stream (a graph is captured on it and launched on s)
  struct GraphGuard {
    std::vector<CycleGraph>& g;
    hipStream_t& cs;
    ~GraphGuard() {
      for (auto& c : g) (void)hipGraphExecDestroy(c.exec);
      if (cs) (void)hipStreamDestroy(cs);
    }
  } graph_guard{graphs, cs};
  auto cycle_graph = [&]() -> hipGraphExec_t {
    if (graphs_stale) {
      for (auto& c : graphs) (void)hipGraphExecDestroy(c.exec);
      graphs.clear();
      graphs_stale = false;
    }
    for (auto& c : graphs)
      if (c.pp == pp && c.qq == qq && c.rho == rho) return c.exec;
    if (!cs) KRR_CHECK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    KRR_CHECK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipGraph_t graph = nullptr;
    double* rho0 = rho;
    double* rho_new0 = rho_new;
    try {
      hipLaunchKernelGGL(k_cycle_begin, dim3(1), dim3(64), 0, cs, halt_d, it_base_d, (const double*)hctrl);
      enqueue_direction(cs, Gate());
      for (int u = 0; u < B; ++u) {
        product(Aw, pp, qq, cs, nullptr);
        step_dir(cs, true, epi_status(dhs + u * SS, it_base_d, u + 1, halt_d), Gate{halt_d, u + 1}, u + 1 < B, pp,
                 pp, Gate{halt_d, u + 2});
        if (u + 1 < B) std::swap(rho, rho_new);
      }
      if (cycle_check) {
        product(*Atrue, x, qq, cs, nullptr);
        hipLaunchKernelGGL(k_residual, dim3(nb(nR)), dim3(256), 0, cs, r.p, Y, qq, active.p, n, R,
                           Gate{halt_d, B});
        DotEpilogue ec;
        ec.mode = DotEpilogue::kCheck;
        ec.hs = dcheck;
        red.dot(r.p, nullptr, n, rr, cs, ec, Gate{halt_d, B});
      }
      hipLaunchKernelGGL(k_cycle_end, dim3(1), dim3(256), 0, cs, (const int*)halt_d, hctrl, (const double*)dhs, hs,
                         (int)(B * SS + R));
      KRR_LAUNCH_CHECK();
    } catch (...) {
      (void)hipStreamEndCapture(cs, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      rho = rho0;
      rho_new = rho_new0;
      throw;
    }
    rho = rho0;   // the capture only recorded the launches; the host's pointers advance when a cycle runs
    rho_new = rho_new0;
    KRR_CHECK_HIP(hipStreamEndCapture(cs, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    KRR_CHECK_HIP(ie);
    graphs.push_back(CycleGraph{pp, qq, rho, exec});
    return exec;
  };

  // Host loop.  Look-ahead: after iteration i's status kernel the host also enqueues iteration i+1's
  // preconditioner apply, p update and product (into the second p / q buffers), and then waits for the status
  // only, so the GPU is not idle while the host reads it and launches the next kernels.  The look-ahead is
  // kept when the status asks for nothing (the common case): its kernels are the ones the iteration would
  // have launched, on the same data, so the iterates are unchanged.  It is not started before a scheduled
  // residual replacement, and it is discarded (rho left as it was, its product's time not counted) when the
  // status reports a claim or a breakdown.  With graphs on, every B iterations (at the scheduled replacements,
  // else every kGraphCycle iterations; no look-ahead there) the loop hands over to a captured cycle when a
  // whole cycle fits before maxit, and takes over again after a cycle that halted, until the next such point.
  double discarded_ms = 0.0;
  bool have_next = false;   // this iteration's product was enqueued by the previous look-ahead
  bool need_dir = false;    // the next direction after a decision has not been enqueued yet
  while (any_active && it < maxit) {
    if (graph_on && need_dir && it % B == 0 && it + B <= maxit) {
      hipGraphExec_t exec = cycle_graph();
      hctrl[0] = (double)it;
      hctrl[1] = 0.0;
      KRR_CHECK_HIP(hipGraphLaunch(exec, s));
      KRR_CHECK_HIP(hipEventRecord(ev_status, s));
      KRR_CHECK_HIP(hipEventSynchronize(ev_status));
      res.st.n_graph_cycles++;
      need_dir = false;
      fresh_true = false;
      std::swap(rho, rho_new);   // the cycle's first direction
      pending_b = act[0] && lanczos_open;
      const int halt = (int)hctrl[1];
      KRR_REQUIRE(halt >= 0 && halt <= B, "internal: cycle halt word out of range");
      const int nu = halt ? halt : B;   // iterations whose status is valid
      bool candidate = false;
      for (int u = 0; u < nu; ++u) {
        ++it;
        res.st.n_mvm++;
        res.st.n_graph_iters++;
        if (!read_status(hs + u * SS, candidate)) {
          breakdown = true;
          break;
        }
        KRR_REQUIRE(!candidate || u + 1 == nu, "internal: a claim did not halt the cycle");
        if (u + 1 < nu) {   // this iteration's next direction ran
          std::swap(rho, rho_new);
          pending_b = act[0] && lanczos_open;
        }
      }
      if (breakdown) break;
      if (cycle_check && (halt == 0 || halt == B)) {   // the check of the last (scheduled) iteration ran
        res.st.n_mvm_fp64++;
        res.st.n_replace++;
        decide(hcheck);
      } else if (candidate) {
        check(false);   // a claim that the cycle's own check does not cover
      }
      any_active = false;
      for (int c = 0; c < R; ++c) any_active |= act[c] != 0;
      if (!any_active || it >= maxit) break;
      need_dir = true;
      continue;
    }
    if (need_dir) {
      enqueue_direction(s, Gate());
      pending_b = act[0] && lanczos_open;   // read with the next iteration's status
      need_dir = false;
    }
    ++it;
    fresh_true = false;
    // q = (K + beta I) p in the working precision
    if (!have_next) {
      tm.start(&res.st.t_mvm_ms);
      product(Aw, pp, qq, s, tm.external(&res.st.t_mvm_kernel_ms));
      tm.stop();
    }
    have_next = false;
    res.st.n_mvm++;
    const bool scheduled = replace_every > 0 && it % replace_every == 0;
    const bool handover = graph_on && it % B == 0;   // a cycle may start after this iteration
    const bool ahead = !scheduled && !handover && it < maxit;
    step(s, epi_status(hs, nullptr, it, nullptr), Gate());
    KRR_CHECK_HIP(hipEventRecord(ev_status, s));
    const size_t tmark = tm.marks();
    if (ahead) {
      direction(s, pp, pa, Gate());
      tm.start(&res.st.t_mvm_ms);
      product(Aw, pa, qa, s, tm.external(&res.st.t_mvm_kernel_ms));
      tm.stop();
    }
    KRR_CHECK_HIP(hipEventSynchronize(ev_status));
    tm.collect(tmark);
    bool candidate = false;
    if (!read_status(hs, candidate)) {
      tm.retarget(&discarded_ms);
      breakdown = true;
      break;
    }
    if (ahead && !candidate) {   // keep the look-ahead: it is the next iteration's direction and product
      std::swap(pp, pa);
      std::swap(qq, qa);
      std::swap(rho, rho_new);
      have_next = true;
      pending_b = act[0] && lanczos_open;   // read with the next iteration's status
      continue;
    }
    if (ahead) tm.retarget(&discarded_ms);   // discard it: the true-residual check below replaces r first
    if (candidate || scheduled) check(scheduled);
    any_active = false;
    for (int c = 0; c < R; ++c) any_active |= act[c] != 0;
    if (!any_active || it >= maxit) break;   // no next direction is needed after the last iteration
    need_dir = true;
  }
  // final true residuals for columns still active (maxit or breakdown); stopped columns return their
  // best iterate
  bool unfinished = false;
  for (int c = 0; c < R; ++c) unfinished |= act[c] != 0;
  if (unfinished && !fresh_true) {   // (after a check in the last iteration its residuals are current)
    product(*Atrue, x, qq, s, nullptr);
    res.st.n_mvm_fp64++;
    hipLaunchKernelGGL(k_residual, dim3(nb(nR)), dim3(256), 0, s, r.p, Y, qq, active.p, n, R, Gate());
    red.dot(r.p, nullptr, n, rr, s);
    KRR_CHECK_HIP(hipMemcpyAsync(h.data(), rr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < R; ++c)
      if (act[c]) {
        res.relres[c] = std::sqrt(h[c]) / ynorm[c];
        if (!(res.relres[c] <= best_rel[c])) gave_up[c] = 1;
      }
  }
  bool restore = false;
  std::vector<int> rest(R, 0);
  for (int c = 0; c < R; ++c)
    if (gave_up[c] && best_rel[c] < HUGE_VAL) {
      rest[c] = 1;
      res.relres[c] = best_rel[c];
      restore = true;
    }
  if (restore) copy_columns(x, xbest.p, rest);
  bool any_gave_up = false;
  for (int c = 0; c < R; ++c) any_gave_up |= gave_up[c] != 0;
  if (breakdown) {
    res.status = KRR_EBREAKDOWN;
    set_error("PCG breakdown at iteration " + std::to_string(it) + ": p^T A p <= 0 or not finite");
  } else if (unfinished || any_gave_up) {
    res.status = KRR_ENOCONV;
    set_error(any_gave_up ? "PCG stopped: true residual stagnated or diverged; best iterate returned"
                          : "PCG reached maxit; last iterate returned");
  }
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  tm.collect();
  // Lanczos tridiagonal of column 0 (rebuilt from the CG step lengths and ratios) -> its smallest and
  // largest eigenvalues by Sturm-sequence bisection inside the Gershgorin interval.
  {
    const int m = (int)std::min(lanczos_g.size(), lanczos_b.size() + 1);
    if (m >= 2) {
      std::vector<double> dg(m), od(m > 1 ? m - 1 : 0);
      for (int j = 0; j < m; ++j) {
        dg[j] = 1.0 / lanczos_g[j] + (j > 0 ? lanczos_b[j - 1] / lanczos_g[j - 1] : 0.0);
        if (j + 1 < m) od[j] = std::sqrt(std::max(lanczos_b[j], 0.0)) / lanczos_g[j];
      }
      auto count_below = [&](double x) {   // Sturm count of eigenvalues < x
        int cnt = 0;
        double dd = dg[0] - x;
        if (dd < 0) ++cnt;
        for (int j = 1; j < m; ++j) {
          const double den = dd == 0.0 ? 1e-300 : dd;
          dd = dg[j] - x - od[j - 1] * od[j - 1] / den;
          if (dd < 0) ++cnt;
        }
        return cnt;
      };
      double lo = 1e300, hi = -1e300;
      for (int j = 0; j < m; ++j) {
        const double rad = (j > 0 ? std::fabs(od[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(od[j]) : 0.0);
        lo = std::min(lo, dg[j] - rad);
        hi = std::max(hi, dg[j] + rad);
      }
      auto kth = [&](int k) {   // k-th smallest eigenvalue (0-based)
        double a = lo, b = hi;
        for (int t = 0; t < 200; ++t) {
          const double mid = 0.5 * (a + b);
          if (count_below(mid) > k) b = mid;
          else a = mid;
        }
        return 0.5 * (a + b);
      };
      const double emin = kth(0), emax = kth(m - 1);
      res.st.kappa_est = emin > 0 ? emax / emin : 0.0;
      res.st.lam_min_est = emin;
      res.st.lam_max_est = emax;
    }
  }
  int mx = 0;
  for (int c = 0; c < R; ++c) mx = std::max(mx, res.iters[c]);
  res.st.iters_max = mx;
  res.st.t_total_ms = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
  return res;
}

}  // namespace krr

extern "C" int krr_set_pcg_mode(int32_t mode) {
  return krr::guarded([&] {
    KRR_REQUIRE(mode >= -1 && mode <= 1, "mode must be -1 (automatic), 0 (host loop) or 1 (graph cycles)");
    krr::set_pcg_mode(mode);
    return (int)KRR_OK;
  });
}

extern "C" int krr_pcg_solve(const double* X, int64_t n, int32_t d, double eps, const double* Yrhs, int32_t R,
                             const double* betas, const krr_precond* P, double tol, int32_t maxit,
                             int32_t replace_every, int32_t prec, double* alpha, int32_t* iters, double* relres,
                             krr_solve_stats* stats, int32_t timing, void* stream) {
  return krr::guarded([&] {
    krr::validate_common(n, n, d, eps);
    krr::validate_prec(prec);
    KRR_REQUIRE(X && Yrhs && betas && alpha && iters && relres, "null pointer argument");
    KRR_REQUIRE(R >= 1 && R <= 256, "R must be in [1, 256]");
    KRR_REQUIRE(tol > 0 && std::isfinite(tol), "tol must be positive");
    KRR_REQUIRE(maxit >= 0, "maxit must be >= 0");
    KRR_REQUIRE(replace_every >= 0, "replace_every must be >= 0");
    for (int c = 0; c < R; ++c) KRR_REQUIRE(betas[c] > 0 && std::isfinite(betas[c]), "beta must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(X, n * (int64_t)d, "X", s);
    krr::check_finite_device(Yrhs, n * (int64_t)R, "y", s);
    krr::check_finite_device(alpha, n * (int64_t)R, "initial alpha", s);
    krr::PcgResult res =
        krr::pcg_solve(X, n, d, eps, Yrhs, R, betas, P, tol, maxit, replace_every, prec, alpha, timing != 0, s);
    for (int c = 0; c < R; ++c) {
      iters[c] = res.iters[c];
      relres[c] = res.relres[c];
    }
    if (stats) *stats = res.st;
    return res.status;
  });
}
