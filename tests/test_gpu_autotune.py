"""The kernel MVM's launch table: after krr_autotune the tuned entry (variant and, when the search chose one,
split) is what a product of that size class launches, and that launch passes parity against the oracle."""
import json

import numpy as np
import pytest
import torch

from oracle import kernel as ok
from test_gpu_kmv import _f64_cross_term_bar


@pytest.mark.gpu
@pytest.mark.parametrize("prec,d,R,n_tune,n_run,bar", [("mixed", 4, 1, 32768, 40000, 2e-6),
                                                      ("fp64", 4, 1, 16384, 20000, 1e-14),
                                                      ("mixed", 6, 32, 16384, 17000, 5e-6)])
def test_tuned_entry_is_launched_and_passes_parity(gpu_lib, tmp_path, prec, d, R, n_tune, n_run, bar):
    gpu_lib.set_variant(d, R, prec, -1)
    best = gpu_lib.autotune(d, R, prec, n=n_tune)
    assert 0 <= best < gpu_lib.num_variants(prec, R)
    f = tmp_path / "table.json"
    gpu_lib.autotune_save(str(f))
    tab = json.loads(f.read_text())
    assert tab["arch"].startswith("gfx9")
    rclass = 1 if R == 1 else 3 if prec == "mixed" else 2
    key = f"{ {'fp64': 0, 'fp32': 1, 'mixed': 2}[prec] }:{d}:{rclass}:{n_tune.bit_length() - 1}:1"
    variant, split = tab["entries"][key]
    assert variant == best
    rng = np.random.default_rng(7)
    X = rng.random((n_run, d))
    V = rng.standard_normal((n_run, R)) if R > 1 else rng.standard_normal(n_run)
    eps = 0.05 * d
    U = gpu_lib.kernel_mv(torch.from_numpy(X), None, eps, torch.from_numpy(V), prec=prec).cpu().numpy()
    lv, lsplit, _ = gpu_lib.kmv_last_launch()
    print(f"{prec} d={d} R={R}: tuned variant {variant} split {split}; launched {lv} split {lsplit}")
    assert lv == variant
    if split > 0:
        assert lsplit == split
    # parity on sampled rows, each scaled by sum_j K_ij |v_j| (the conditioning of the row's sum)
    rows = rng.choice(n_run, 64, replace=False)
    ref = ok.kernel_mv(X[rows], X, eps, V)
    scale = ok.kernel_mv(X[rows], X, eps, np.abs(V))
    err = np.abs((U[rows] - ref) / scale).max()
    if prec == "fp64" and variant >= 5:   # the cross term on the FP64 matrix cores: its cancellation bar
        bar = max(bar, _f64_cross_term_bar(X, eps))
    assert err <= bar, err
    gpu_lib.set_variant(d, R, prec, -1)
