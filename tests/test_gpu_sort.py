"""The device radix sort (krr_radix_sort_pairs) against NumPy's stable sort, pair for pair.

The sort orders the pivoted QR's candidate columns and the Morton staging of culled operators; both need
the stable order (equal keys keep their input order).  Cases: sizes below one sub-tile, ragged multiples of
the 256-pair sub-tile and the 2048-pair chunk, more blocks than the sort launches (chunks of several
sub-tiles), keys with many duplicates, all-equal keys, keys already sorted or reversed, full 64-bit keys
(the QR's, with the top bit set) and partial bit ranges (the Morton codes'), where the bits above end_bit
take no part in the order.
"""
import numpy as np
import pytest
import torch


def _reference(keys_u64, vals, end_bit):
    mask = np.uint64((1 << end_bit) - 1) if end_bit < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(keys_u64 & mask, kind="stable")
    return keys_u64[order], vals[order]


def _run(gpu_lib, keys_u64, vals, end_bit):
    k = torch.from_numpy(keys_u64.view(np.int64).copy())
    v = torch.from_numpy(vals.copy())
    ko, vo = gpu_lib.radix_sort_pairs(k, v, end_bit)
    return ko.cpu().numpy().view(np.uint64), vo.cpu().numpy()


def _keys(kind, n, rng):
    if kind == "random64":
        return rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    if kind == "dups":
        return rng.integers(0, 37, n, dtype=np.uint64) << np.uint64(rng.integers(0, 56))
    if kind == "equal":
        return np.full(n, 0xDEADBEEF12345678, dtype=np.uint64)
    if kind == "sorted":
        return np.sort(rng.integers(0, 2**40, n, dtype=np.uint64))
    if kind == "reversed":
        return np.sort(rng.integers(0, 2**40, n, dtype=np.uint64))[::-1].copy()
    if kind == "norms":   # the QR's keys: order-reversed bit patterns of non-negative doubles, ~0 for taken
        v = np.abs(rng.standard_normal(n)) * 10.0 ** rng.integers(-5, 5, n)
        v[rng.random(n) < 0.05] = -1.0
        v[rng.random(n) < 0.05] = 1.0   # ties
        bits = v.view(np.uint64)
        return np.where(v < 0, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0x7FFFFFFFFFFFFFFF) - bits)
    raise ValueError(kind)


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 7, 255, 256, 2049, 70_001, 1_500_007])
@pytest.mark.parametrize("kind", ["random64", "dups", "equal", "sorted", "reversed", "norms"])
def test_radix_sort_matches_stable_sort(gpu_lib, n, kind):
    rng = np.random.default_rng(n * 7 + len(kind))
    keys = _keys(kind, n, rng)
    vals = rng.permutation(n).astype(np.int64) + 3 * n   # a permutation: the output must be one too
    ko, vo = _run(gpu_lib, keys, vals, 64)
    rk, rv = _reference(keys, vals, 64)
    assert np.array_equal(ko, rk) and np.array_equal(vo, rv)


@pytest.mark.gpu
@pytest.mark.parametrize("end_bit", [1, 8, 13, 48, 63])
def test_radix_sort_bit_range(gpu_lib, end_bit):
    """Only bits [0, end_bit) order the pairs (stable among equal low bits); keys come back whole."""
    n = 100_003
    rng = np.random.default_rng(end_bit)
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    vals = np.arange(n, dtype=np.int64)
    ko, vo = _run(gpu_lib, keys, vals, end_bit)
    rk, rv = _reference(keys, vals, end_bit)
    assert np.array_equal(ko, rk) and np.array_equal(vo, rv)


@pytest.mark.gpu
def test_radix_sort_empty_and_inputs_untouched(gpu_lib):
    ko, vo = gpu_lib.radix_sort_pairs(torch.empty(0, dtype=torch.int64), torch.empty(0, dtype=torch.int64))
    assert ko.numel() == 0 and vo.numel() == 0
    k = torch.arange(5000, 0, -1, dtype=torch.int64, device="cuda")
    v = torch.arange(5000, dtype=torch.int64, device="cuda")
    k0, v0 = k.clone(), v.clone()
    ko, vo = gpu_lib.radix_sort_pairs(k, v)
    assert torch.equal(k, k0) and torch.equal(v, v0)
    assert torch.equal(ko, torch.arange(1, 5001, dtype=torch.int64, device="cuda"))
    assert torch.equal(vo, torch.arange(4999, -1, -1, dtype=torch.int64, device="cuda"))
