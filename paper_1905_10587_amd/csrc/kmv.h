// Kernel matrix-vector products U = K(Xt, Xs) V on gfx950 (the operation the paper delegates
// to FIG(targets, sources, h, V), Sec. 2.4; computed here by exact direct summation, never
// storing K).
#pragma once

#include "krr_internal.h"

#include <string>

namespace krr {

// Derived device copies of a point set used by the MVM kernels (stage inputs).
//   x64: npad x dpad FP64 (zero padded rows/columns)
//   x32: npad x dpad FP32, (x - center) * sqrt(log2(e)/eps)
//   sa / sb: npad x ka bf16 split vectors of (x - center) for the MFMA cross term
//            (target side / source side), ka = 32 * nchunk
struct Staged {
  int64_t n = 0, npad = 0;
  int d = 0, dpad = 0, ka = 0;
  int prec = KRR_FP64;
  double eps = 0;
  DevBuf<double> x64;
  // FP64 staging: every pair's base-2 exponent -log2(e) |x_i - x_j|^2 / eps is provably >= -1020 (the box
  // of the points gives log2(e) diag^2 / eps <= 1000 and log2(e) max|x|^2 / eps <= 1e10, so the rounding of
  // the matrix-core form's norms cannot take it past that), and the FP64 exp2 runs without its clamp
  bool q_floor = false;
  DevBuf<float> x32;
  DevBuf<uint16_t> sa, sb;
  DevBuf<double> center;   // dpad
  // Spatial order for exact far-tile culling (symmetric mixed form): the staged copies hold the points in
  // Morton order of their grid cells, perm[i] = original index of staged point i; box16 holds, for every
  // group of 16 staged points, the bounding box of z' = (x - center) sqrt(log2(e) / eps): lo[dpad] then
  // hi[dpad].  Empty: the caller's order, no culling.
  DevBuf<int64_t> perm;
  DevBuf<double> box16;
  // skip masks of the symmetric kernel for target groups of 16 NF points (built on first use)
  mutable DevBuf<uint16_t> cull_mask;
  mutable int cull_nf = 0;
};

constexpr int kRowPad = 1024;   // targets/sources are padded to multiples of this
constexpr int kPrefetchRows = 32;   // extra allocated rows after the padded sources (prefetch reads)

// Pads d up to the instantiated widths of the direct (FP64/FP32) kernels.
int padded_dim(int d);
// Number of 32-wide K chunks of the split-BF16 cross term for dimension d.
int mixed_chunks(int d);

// Stage a point set.  center: dpad FP64 on device (translation applied to FP32 and split copies;
// the kernel is translation invariant).  Pass the same center for targets and sources.
// sort: stage a square operator's points in spatial order with culling boxes (MIXED only; see Staged).
void stage_points(Staged& st, const double* X, int64_t n, int d, double eps, int prec,
                  const double* center, bool as_target, bool as_source, hipStream_t s, bool sort = false);

// Exact far-tile culling of the symmetric mixed form.  A 16-source step of a wave's 16 NF targets is skipped
// when every kernel value in it is exactly zero in FP32: the boxes' minimum scaled squared distance exceeds
// 161 (exp2 of anything below -150 is 0) plus a bound on the split cross term's rounding error.
//   cull_mode: -1 automatic (square mixed one-column products whose bounding-box diagonal reaches past the
//   threshold), 0 off, 1 on, 2 spatial order without skipping (for comparisons).
int cull_mode();
void set_cull_mode(int mode);
// Whether a square mixed product of these points should be staged in spatial order under the current mode.
bool cull_wanted(const double* X, int64_t n, int d, double eps, hipStream_t s);
// Skip masks for target groups of 16 NF points against 256-source groups (cached in S).
const uint16_t* cull_masks(const Staged& S, int NF, hipStream_t s);
// Device counters of skipped 16-source steps (diagonal and off-diagonal super-tiles) of culled launches.
unsigned long long* cull_counters();
void cull_reset_counters(hipStream_t s);
// Mean of the points (FP64), written to center[dpad].
void point_mean(const double* X, int64_t n, int d, int dpad, double* center, hipStream_t s);

// V (n x R FP64, row-major) -> padded column-block layout used by the kernels.
struct StagedVec {
  int64_t npad = 0;
  int R = 0;            // columns padded to a multiple of 8
  int Rreal = 0;
  // column c of the staged vectors is column cols[c] of the caller's V (row stride ldv), and the products
  // go to the same columns of U; nullptr: columns 0 .. Rreal - 1 of a V with Rreal columns
  const int* cols = nullptr;
  int ldv = 0;
  DevBuf<double> v64;   // npad x R
  DevBuf<float> v32;    // npad x R
  // block-MVM operands: BF16 parts in groups of four sources, V4[((j/4) * Rb + r) * 4 + j%4]
  int Rb = 0;
  DevBuf<uint16_t> vh, vm, vl;
  // staged-V block form: the parts in the MFMA B-operand lane layout, per 32-source step and 16-column tile
  DevBuf<uint16_t> vt;
};
// Block path: stage V into the BF16 parts (Rb = R padded to rpad).
// Staged-V block form: stage V into the B-operand lane layout (Rb = R padded to 16).
void stage_vectors_vt(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int nsplit, hipStream_t s);
void stage_vectors_block(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int rpad, int nsplit,
                         hipStream_t s);
// Whether kmv_launch takes the block (multi right-hand side) path for these parameters.
bool kmv_uses_block(int prec, int d, int R, int deriv);
// perm: the operator's staged order (Staged::perm), nullptr for the caller's order.  cols (device, R entries)
// and ldv: stage columns cols[0 .. R) of a V whose rows hold ldv values (a subset of its columns); the kernel
// MVM then writes its products to those columns of U (one product without the derivative kernel).
void stage_vectors(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int prec,
                   hipStream_t s, const int64_t* perm = nullptr, const int* cols = nullptr, int ldv = 0);

// Core launcher: U[i, col0 + c] (row stride ldu) for the staged operands.
//   deriv: 0 K, 1 K', 2 both (K columns first, then K' columns).
//   shift: per-column ridge term added as shift[c] * V[i, c] (targets == sources) or nullptr.
//   Vraw: the original FP64 V (n x R) for the shift term.
//   variant >= 0 forces a variant (else the launch table, else the default); split_req > 0 forces the sources
//   per block of the direct forms (rounded up to 256; at most nsrc / 256 splits) or the super-tile edge of the
//   symmetric forms (else the table's, else the launcher's own choice).
void kmv_launch(const Staged& T, const Staged& S, StagedVec& V, int deriv,
                const double* shift_host, const double* Vraw, int prec, double* U, int64_t ldu,
                hipStream_t s, int variant = -1, DevBuf<double>* ws = nullptr,
                const hipEvent_t* kev = nullptr,   // kev: two events recorded around the main kernel
                int split_req = 0);

// Launch table entry and the record of the last launch on this thread.
struct KmvChoice {
  int variant = -1;   // -1: none
  int split = 0;      // sources per block (direct forms) or super-tile edge (symmetric forms); 0: launcher's choice
};
struct KmvLaunchInfo {
  int variant = -1, split = 0, symmetric = 0;
  int culled = 0;          // the symmetric form ran with far-tile culling (counters valid)
  int64_t npad = 0;        // padded point count of the launch
  int nf = 0;              // target fragments per wave (16 NF targets per wave)
};
KmvLaunchInfo kmv_last_launch();
KmvChoice kmv_lookup(int prec, int d, int R, int64_t n, bool square);
void kmv_set_tuned(int prec, int d, int R, int64_t n, bool square, KmvChoice c);
std::string device_arch();

// W = K(Xt, Xs) T on the FP64 matrix cores without forming K(Xt, Xs) (Algorithm 3: C U^{1/2} with the
// kernel block applied on the fly): Xt m x d, Xs k x d (FP64, row-major, device), T k x ncol (row stride
// ldt), W m x ncol (row stride ldw).  Needs padded_dim(d) <= 16 (returns false otherwise, nothing launched).
bool kernel_times_matrix_f64(const double* Xt, int64_t m, const double* Xs, int64_t k, int d, double eps,
                             const double* T, int64_t ldt, int ncol, double* W, int64_t ldw, hipStream_t s);

// Variant bookkeeping for the autotuner.
int kmv_num_variants(int prec, int R);
int kmv_default_variant(int prec, int d, int R, int64_t m, int64_t n, bool square = false);
// FP64 with several columns, variant 3: the FP64 matrix-core kernel (needs the column count padded to 16)
bool kmv_f64_uses_mfma(int prec, int d, int R, int deriv, int variant);
// Whether variant v runs the symmetric square-product form for these parameters.
bool kmv_is_symmetric(int prec, int d, int R, int deriv, bool square, int v);
void kmv_set_override(int d, int R, int prec, int variant);
int kmv_get_override(int d, int R, int prec);
std::string kmv_table_json();
void kmv_table_from_json(const std::string& s);

}  // namespace krr
