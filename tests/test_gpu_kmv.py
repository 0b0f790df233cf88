"""GPU parity of the kernel MVM (krr_kernel_mv) against the oracle, element by element.

Sizes span several 1024-row tiles with ragged tails, single points, cross-set products,
several right-hand sides, the derivative kernel and the ridge shift.  Errors are measured
per entry relative to sum_j K_ij |V_jc| (the scale of the sum, which avoids dividing by
cancelled sums).  Bars:
  FP64  <= 1e-14   (direct differences, FP64 exp from its series; measured <= 3e-16); the symmetric form
                   with the cross term on the FP64 matrix cores: the cancellation bar of
                   _f64_cross_term_bar (at least 1e-14)
  FP32  <= 1e-6    (FP32 differences/exp/partial sums; measured <= 1.4e-7)
  MIXED <= 1e-6    (split-BF16 MFMA cross term with FP32 accumulation; measured <= 1e-7)
"""
import numpy as np
import pytest
import torch

from oracle import kernel as ok

TOL = {"fp64": 1e-14, "fp32": 1e-6, "mixed": 1e-6}
BLOCK_TOL = {"fp32": 1e-6, "mixed": 5e-6}

CASES = [
    # (m, n, d, same, R)
    (1, 1, 3, True, 1),
    (37, 53, 3, False, 1),
    (1000, 1500, 4, False, 1),
    (2000, 2000, 3, True, 1),
    (3000, 2100, 8, False, 1),
    (1100, 900, 16, False, 1),
    (700, 800, 6, False, 3),
    (1030, 1030, 4, True, 9),
    (257, 300, 1, False, 1),
    (400, 350, 40, False, 2),
]


def _data(m, n, d, same, R, seed):
    rng = np.random.default_rng(seed)
    Xs = rng.random((n, d))
    Xt = Xs if same else rng.random((m, d))
    V = rng.standard_normal((n, R))
    eps = 0.05 * d
    return Xt, Xs, V, eps


def _scaled_err(U, ref, Kabs_V):
    return float(np.max(np.abs(U - ref) / np.maximum(Kabs_V, 1e-300)))


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[f"m{c[0]}_n{c[1]}_d{c[2]}_R{c[4]}" for c in CASES])
def test_kernel_mv_parity(gpu_lib, prec, case):
    m, n, d, same, R = case
    Xt, Xs, V, eps = _data(m, n, d, same, R, seed=m + n + d)
    print(f"case m={m} n={n} d={d} R={R} prec={prec}", flush=True)
    K = ok.kernel_matrix(Xt, Xs, eps)
    ref = K @ V
    scale = K @ np.abs(V)
    U = gpu_lib.kernel_mv(torch.from_numpy(Xt), None if same else torch.from_numpy(Xs), eps,
                          torch.from_numpy(V), prec=prec).cpu().numpy()
    err = _scaled_err(U, ref, scale)
    print(f"  max scaled error {err:.3e}", flush=True)
    # several mixed-precision columns take the block path (two BF16 parts of K and V: ~2^-17 each)
    tol = BLOCK_TOL["mixed"] if (prec == "mixed" and R > 1) else TOL[prec]
    assert err <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_kernel_mv_deriv_and_shift(gpu_lib, prec):
    rng = np.random.default_rng(11)
    X = rng.random((1500, 4))
    V = rng.standard_normal((1500, 2))
    eps = 0.2
    K = ok.kernel_matrix(X, X, eps)
    Kp = ok.kernel_deriv_matrix(X, X, eps)
    Xg, Vg = torch.from_numpy(X), torch.from_numpy(V)
    both = gpu_lib.kernel_mv(Xg, None, eps, Vg, deriv=2, prec=prec).cpu().numpy()
    tol = TOL[prec]
    assert _scaled_err(both[:, :2], K @ V, K @ np.abs(V)) <= tol
    assert _scaled_err(both[:, 2:], Kp @ V, Kp @ np.abs(V) + 1e-3 * (K @ np.abs(V))) <= 10 * tol
    only = gpu_lib.kernel_mv(Xg, None, eps, Vg, deriv=1, prec=prec).cpu().numpy()
    np.testing.assert_allclose(only, both[:, 2:], rtol=0, atol=1e-12 * np.abs(both).max())
    sh = gpu_lib.kernel_mv(Xg, None, eps, Vg, shift=[1e-3, 0.5], prec=prec).cpu().numpy()
    ref = K @ V + V * np.array([1e-3, 0.5])
    assert _scaled_err(sh, ref, K @ np.abs(V) + np.abs(V) * 0.5) <= BLOCK_TOL.get(prec, tol)


@pytest.mark.gpu
def test_kernel_mv_rejects_bad_arguments(gpu_lib):
    X = torch.rand(10, 3, dtype=torch.float64)
    v = torch.rand(10, dtype=torch.float64)
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.kernel_mv(X, None, -1.0, v)
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.kernel_mv(X, None, float("inf"), v)


BLOCK_CASES = [
    # (m, n, d, R) for the block (many right-hand sides) MFMA path
    (1500, 1700, 6, 16),
    (2100, 1100, 4, 40),
    (1030, 2000, 6, 128),
    (900, 700, 16, 33),
    (1200, 1500, 16, 96),    # shared-tile form (variant 12): three of its four waves hold columns, four K chunks
    (800, 1300, 6, 200),     # shared-tile form over two 128-column groups (224 padded columns: 3 live waves in the second)
    (1, 1, 3, 64),           # one target, one source
    (5, 3001, 8, 130),       # few targets, ragged sources, 130 columns (one live wave in the second group)
    (1100, 1000, 3, 128),    # staged-V form with every block full (static tile loop), one K chunk
    (700, 900, 16, 256),     # the same over two full column groups, four K chunks (one tile read ahead)
    (600, 1400, 8, 112),     # staged-V form, one block of seven column tiles (static tile loop)
    (400, 900, 4, 70),       # one block of five column tiles, 70 real columns
]


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("mixed", 5e-6), ("fp32", 1e-6)])
@pytest.mark.parametrize("case", BLOCK_CASES, ids=[f"m{c[0]}_n{c[1]}_d{c[2]}_R{c[3]}" for c in BLOCK_CASES])
def test_block_mv_parity(gpu_lib, prec, tol, case):
    """K V for many columns: exp'd tiles feed a second MFMA (split-BF16 parts of K and V).

    MIXED uses two BF16 parts (three products; measured <= 1e-6); FP32 three parts (six products;
    measured <= 8e-8)."""
    m, n, d, R = case
    if n == 1 and prec == "mixed":
        # one source: nothing averages, so the bar is the per-element worst case of the two-part split,
        # |K - (Kh + Km)| <= 2^-18 |K| and the same for V, plus the dropped Km Vm <= 2^-18 |K V|: 3 x 2^-18
        # = 1.14e-5, with the exp and cross-term rounding below 1e-6
        tol = 1.25e-5
    rng = np.random.default_rng(m + R)
    Xs = rng.random((n, d))
    Xt = rng.random((m, d))
    V = rng.standard_normal((n, R))
    eps = 0.1 * d
    K = ok.kernel_matrix(Xt, Xs, eps)
    ref, scale = K @ V, K @ np.abs(V)
    for variant in range(gpu_lib.num_variants(prec, R)):
        gpu_lib.set_variant(d, R, prec, variant)
        U = gpu_lib.kernel_mv(torch.from_numpy(Xt), torch.from_numpy(Xs), eps, torch.from_numpy(V),
                              prec=prec).cpu().numpy()
        err = _scaled_err(U, ref, scale)
        print(f"block {prec} m={m} n={n} d={d} R={R} variant={variant}: max scaled error {err:.2e}", flush=True)
        assert err <= tol
    gpu_lib.set_variant(d, R, prec, -1)


F64_MANY_CASES = [
    # (m, n, d, R): FP64 products with several columns; variant 3 runs the FP64 matrix-core kernel
    # (16 * NRG columns per block, NRG = 1, 2, 4, 6, 8, the last block possibly partly filled; more than 8
    # columns are padded to a multiple of 16)
    (1500, 1700, 6, 16),
    (2100, 1100, 4, 48),     # 48 columns: one block of 64, three live groups of 16
    (1030, 2000, 6, 128),    # NRG 8, ragged targets
    (900, 700, 16, 64),      # NRG 4, widest instantiated dimension
    (800, 1300, 3, 32),      # odd padded dimension, NRG 2
    (700, 900, 2, 200),      # 200 columns padded to 208: 128 + 80 (five live groups in the second block)
    (600, 700, 3, 170),      # the dense-sketch width of the small workload: 176 = 128 + 48
    (600, 1100, 40, 24),     # d = 40: no matrix-core form (variant 3 runs variant 1)
    (500, 800, 5, 9),        # 9 columns padded to 16
    (1000, 1000, 8, 256),    # two 128-column blocks
    (1, 1, 2, 16),           # one target, one source
    (3, 4099, 16, 128),      # three targets, a ragged source tail
    (800, 900, 5, 90),       # 90 columns padded to 96: NRG 6, one block
    (500, 700, 4, 80),       # 80 columns: NRG 6 with one dead column group
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", F64_MANY_CASES, ids=[f"m{c[0]}_n{c[1]}_d{c[2]}_R{c[3]}" for c in F64_MANY_CASES])
def test_fp64_many_columns_variants(gpu_lib, case):
    """FP64 K V with several columns, every variant (direct TM 1, 2, 4 and the matrix-core form) against
    the oracle at the FP64 bar."""
    m, n, d, R = case
    rng = np.random.default_rng(m + 3 * R)
    Xs = rng.random((n, d))
    Xt = rng.random((m, d))
    V = rng.standard_normal((n, R))
    eps = 0.1 * d
    K = ok.kernel_matrix(Xt, Xs, eps)
    ref, scale = K @ V, K @ np.abs(V)
    for variant in range(gpu_lib.num_variants("fp64", R)):
        gpu_lib.set_variant(d, R, "fp64", variant)
        U = gpu_lib.kernel_mv(torch.from_numpy(Xt), torch.from_numpy(Xs), eps, torch.from_numpy(V),
                              prec="fp64").cpu().numpy()
        err = _scaled_err(U, ref, scale)
        print(f"fp64 m={m} n={n} d={d} R={R} variant={variant}: max scaled error {err:.2e}", flush=True)
        assert err <= TOL["fp64"]
    gpu_lib.set_variant(d, R, "fp64", -1)


MIXED_VARIANT_CASES = [
    # (m, n, d, deriv): d = 3, 8, 13, 20 give 1, 2, 3, 4 K chunks of the split cross term; d = 30 has none
    # of the pipelined forms (it falls back to the plain kernel)
    (1100, 2500, 3, 0),
    (2100, 1300, 8, 0),
    (1030, 1700, 13, 0),
    (1500, 1100, 20, 0),
    (600, 1500, 30, 0),
    (1100, 1900, 8, 1),
    (900, 1200, 3, 2),
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", MIXED_VARIANT_CASES, ids=[f"m{c[0]}_n{c[1]}_d{c[2]}_deriv{c[3]}"
                                                           for c in MIXED_VARIANT_CASES])
def test_mixed_single_column_variants(gpu_lib, case):
    """Every single-column MFMA variant (plain NF 1, 2, 4, 8; pipelined NF 2, 4, 8; pipelined with LDS-staged
    source tiles NF 2, 4, 8), incl. K' and (K, K')."""
    m, n, d, deriv = case
    rng = np.random.default_rng(m * 7 + d)
    Xs = rng.random((n, d))
    Xt = rng.random((m, d))
    v = rng.standard_normal(n)
    eps = 0.05 * d
    refs = ok.kernel_mv(Xt, Xs, eps, v, deriv=deriv)
    scales = ok.kernel_mv(Xt, Xs, eps, np.abs(v), deriv=deriv)
    if deriv != 2:
        refs, scales = [refs], [scales]
    outs = {}
    for variant in range(gpu_lib.num_variants("mixed", 1)):
        gpu_lib.set_variant(d, 1, "mixed", variant)
        U = gpu_lib.kernel_mv(torch.from_numpy(Xt), torch.from_numpy(Xs), eps, torch.from_numpy(v), deriv=deriv,
                              prec="mixed").cpu().numpy()
        cols = [U[:, c] for c in range(2)] if deriv == 2 else [U.reshape(-1)]
        for c, (ref, scale) in enumerate(zip(refs, scales)):
            err = _scaled_err(cols[c], ref, scale)
            print(f"mixed m={m} n={n} d={d} deriv={deriv} variant={variant} part={c}: max scaled error {err:.2e}",
                  flush=True)
            assert err <= TOL["mixed"]
        outs[variant] = U
    gpu_lib.set_variant(d, 1, "mixed", -1)
    # the pipelined kernels keep the plain kernels' per-lane summation order, and at these sizes every
    # variant runs in one round of resident blocks with the same source split: identical results
    for plain, piped, staged in ((1, 4, 7), (2, 5, 8), (3, 6, 9)):
        assert np.array_equal(outs[plain], outs[piped]), (plain, piped)
        assert np.array_equal(outs[plain], outs[staged]), (plain, staged)


SYM_CASES = [
    # (n, d): square products K(X, X) v; n spans several 1024-point super-tiles with a ragged tail
    (2500, 3),
    (3100, 8),
    (2049, 13),
    (4100, 20),
    (700, 4),
    (3000, 6),
    (2600, 16),
]


SYM_VARIANTS = {"mixed": (10, 11), "fp64": (3, 4, 5, 6)}


def _f64_cross_term_bar(X, eps):
    """Bar of the FP64 symmetric forms whose exponent is contracted on the matrix cores (variants 5, 6): q =
    c'(|x_i|^2 + |x_j|^2 - 2 x_i.x_j), c' = log2(e) / eps, on centred coordinates, carries a rounding error of at
    most about k u max|x - mean|^2 |c'|: the norms 2(d + 1), the scaled source coordinates 2, and either
    (padded width 4 mod 4: row norms as the contraction's accumulator input) d accumulation steps on partial
    sums up to 3 |c'| max|x|^2 and a final addition of the source norm, 4, so k = 5d + 8, or (padded width
    2 mod 4: both norms inside the contraction) d + 2 steps on partial sums up to 4 |c'| max|x|^2, so
    k = 6d + 12; a relative error ln2 times that in each kernel value.  The bar is twice that bound, and never
    below the direct form's."""
    d = X.shape[1]
    width = next((w for w in (2, 3, 4, 6, 8, 16) if d <= w), d)   # the kernel's padded width (no such form above 16)
    k = 6 * d + 12 if width % 4 == 2 else 5 * d + 8
    M = float(np.max(np.sum((X - X.mean(axis=0)) ** 2, axis=1)))
    return max(TOL["fp64"], 2.0 * np.log(2.0) * (np.log2(np.e) / eps) * k * 2.0 ** -53 * M)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("case", SYM_CASES, ids=[f"n{c[0]}_d{c[1]}" for c in SYM_CASES])
def test_symmetric_square_product(gpu_lib, case, prec):
    """The symmetric form (each off-diagonal super-tile evaluated once, feeding row and column sums) against
    the oracle, with and without the ridge shift, for both of its variants (shapes without a symmetric
    form run the direct kernel: FP64 at odd padded widths, mixed above 20 dimensions)."""
    n, d = case
    rng = np.random.default_rng(n + 31 * d)
    X = rng.random((n, d))
    v = rng.standard_normal(n)
    eps = 0.05 * d
    beta = 1e-3
    K = ok.kernel_matrix(X, X, eps)
    ref, scale = K @ v, K @ np.abs(v)
    for variant in SYM_VARIANTS[prec]:
        gpu_lib.set_variant(d, 1, prec, variant)
        U = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(v), prec=prec).cpu().numpy()
        err = _scaled_err(U, ref, scale)
        Us = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(v), shift=beta,
                               prec=prec).cpu().numpy()
        err_s = _scaled_err(Us, ref + beta * v, scale + beta * np.abs(v))
        form = gpu_lib.kmv_variant(d, 1, prec, square=True)
        bar = _f64_cross_term_bar(X, eps) if prec == "fp64" and variant >= 5 else TOL[prec]
        print(f"symmetric {prec} n={n} d={d} variant={variant} {form}: max scaled error {err:.2e} "
              f"(with shift {err_s:.2e}; bar {bar:.1e})", flush=True)
        assert err <= bar and err_s <= bar
    gpu_lib.set_variant(d, 1, prec, -1)


@pytest.mark.gpu
@pytest.mark.parametrize("case", [(3000, 4, 0.01, "uniform"), (2600, 16, 4.0, "normal")],
                         ids=["d4_eps0.01_uniform", "d16_eps4_normal"])
def test_fp64_cross_term_form_at_workload_arithmetic(gpu_lib, case):
    """Variants 5 and 6 at the mixed workload's arithmetic (uniform points in the unit 4-cube, eps = 0.01: the
    largest |c'| max|x|^2 of the workloads) and the adjoint workload's (d = 16, x ~ N(0, I/4), eps = 4), with
    and without the shift, against the oracle within the cancellation bar; the direct symmetric form (variant
    4) on the same data stays within the FP64 bar."""
    n, d, eps, kind = case
    rng = np.random.default_rng(n + d)
    X = rng.random((n, d)) if kind == "uniform" else 0.5 * rng.standard_normal((n, d))
    v = rng.standard_normal(n)
    K = ok.kernel_matrix(X, X, eps)
    ref, scale = K @ v, K @ np.abs(v)
    bar = _f64_cross_term_bar(X, eps)
    errs = {}
    try:
        for variant in (4, 5, 6):
            gpu_lib.set_variant(d, 1, "fp64", variant)
            U = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(v), prec="fp64").cpu().numpy()
            Us = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(v), shift=1e-3,
                                   prec="fp64").cpu().numpy()
            errs[variant] = (_scaled_err(U, ref, scale),
                             _scaled_err(Us, ref + 1e-3 * v, scale + 1e-3 * np.abs(v)))
    finally:
        gpu_lib.set_variant(d, 1, "fp64", -1)
    print(f"fp64 d={d} eps={eps}: direct symmetric {errs[4][0]:.2e}, cross term on matrix cores {errs[5][0]:.2e} / "
          f"{errs[6][0]:.2e} (bar {bar:.1e})", flush=True)
    assert max(errs[4]) <= TOL["fp64"]
    assert max(errs[5]) <= bar and max(errs[6]) <= bar


@pytest.mark.gpu
@pytest.mark.parametrize("R", [16, 40, 128])
@pytest.mark.parametrize("d", [3, 8])
def test_fp64_many_columns(gpu_lib, R, d):
    """FP64 products with many right-hand sides (wide column chunks of 16 or 32: one exp per pair shared by
    the chunk), a ragged last chunk at R = 40, square and cross-set."""
    rng = np.random.default_rng(R + d)
    Xs = rng.random((1300, d))
    Xt = rng.random((700, d))
    V = rng.standard_normal((1300, R))
    eps = 0.05 * d
    for targets, same in ((Xs, True), (Xt, False)):
        K = ok.kernel_matrix(targets, Xs, eps)
        ref, scale = K @ V, K @ np.abs(V)
        U = gpu_lib.kernel_mv(torch.from_numpy(targets), None if same else torch.from_numpy(Xs), eps,
                              torch.from_numpy(V), prec="fp64").cpu().numpy()
        err = _scaled_err(U, ref, scale)
        print(f"fp64 R={R} d={d} square={same}: max scaled error {err:.2e}", flush=True)
        assert err <= TOL["fp64"]


@pytest.mark.gpu
@pytest.mark.parametrize("eps", [0.05, 1e-3, 1e-5], ids=["exponent_bounded", "exponent_unbounded", "isolated"])
def test_fp64_cross_term_form_exp_clamp(gpu_lib, eps):
    """The FP64 matrix-core symmetric form runs its exp2 without the clamp at -1020 only when the points' box
    bounds every exponent log2(e) |x_i - x_j|^2 / eps by 1000 (eps = 0.05 in the unit 4-cube: at most 115);
    with eps = 1e-3 (exponents down to -5771: far pairs underflow, the oracle's values are exactly zero) and
    1e-5 (most points isolated: their products are v_i itself) the clamped exp2 runs.  All against the oracle
    within the cancellation bar, finite everywhere."""
    n, d = 2500, 4
    rng = np.random.default_rng(97)
    X = rng.random((n, d))
    v = rng.standard_normal(n)
    K = ok.kernel_matrix(X, X, eps)
    ref, scale = K @ v, K @ np.abs(v)
    bar = _f64_cross_term_bar(X, eps)
    try:
        gpu_lib.set_variant(d, 1, "fp64", 5)
        U = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(v), prec="fp64").cpu().numpy()
    finally:
        gpu_lib.set_variant(d, 1, "fp64", -1)
    err = _scaled_err(U, ref, scale)
    print(f"fp64 variant 5 eps={eps}: max scaled error {err:.2e} (bar {bar:.1e})", flush=True)
    assert np.all(np.isfinite(U))
    assert err <= bar
