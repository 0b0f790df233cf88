"""krr_precond_apply_noalloc (the Woodbury apply for callers that cannot allocate device memory) against
krr_precond_apply, called through the C ABI: two calls in a row, the second on a smaller problem, so stale
scratch from the first call cannot leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

import datagen


def _precond(gpu_lib, n, d, k, eps, betas, prec, seed):
    X = np.random.default_rng(seed).random((n, d))
    idx, sign = datagen.sketch_sparse_draws(n, k + 20, 16, seed + 1)
    return gpu_lib.Preconditioner(torch.from_numpy(X), eps, betas, k, k + 20, idx=torch.from_numpy(idx),
                                  sign=torch.from_numpy(sign), prec=prec)


def _raw_apply(lib, P, x, betas, prec, noalloc, out=None):
    """The C ABI call itself (ctypes), on torch device buffers and torch's current stream."""
    R = 1 if x.dim() == 1 else x.shape[1]
    out = torch.empty_like(x) if out is None else out
    bh = (ctypes.c_double * R)(*[float(b) for b in betas])
    fn = lib.krr_precond_apply_noalloc if noalloc else lib.krr_precond_apply
    st = fn(P.handle, ctypes.c_void_p(x.data_ptr()), R, bh, {"fp64": 0, "mixed": 2}[prec],
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.krr_last_error()
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_apply_matches_apply_twice(gpu_lib, prec):
    lib = gpu_lib.load()
    rng = np.random.default_rng(3)
    cases = [(30000, 3, 400, 0.02, [1e-3, 1e-2], 3), (2500, 2, 120, 0.05, [1e-2], 1)]   # second: smaller
    for n, d, k, eps, betas, R in cases:
        P = _precond(gpu_lib, n, d, k, eps, betas, prec, 10 + n % 7)
        x = torch.from_numpy(rng.standard_normal((n, R)) if R > 1 else rng.standard_normal(n)).cuda()
        cols = [betas[c % len(betas)] for c in range(R)]
        ref = _raw_apply(lib, P, x, cols, prec, noalloc=False)
        got = torch.empty_like(x)
        torch.cuda.synchronize()
        alloc_before = torch.cuda.memory_allocated()
        _raw_apply(lib, P, x, cols, prec, noalloc=True, out=got)
        torch.cuda.synchronize()
        # nothing was allocated through the library's allocator (torch's caching allocator) for the call
        assert torch.cuda.memory_allocated() == alloc_before
        err = (torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item()
        print(f"n={n} k={k} R={R} {prec}: no-alloc vs apply rel diff {err:.2e}")
        if R == 1:
            # one column: the same kernels in the same order
            assert torch.equal(got, ref)
        else:
            assert err <= 1e-12
        # the binding's wrapper gives the same
        out = torch.empty_like(x)
        P.apply_noalloc(x, out, betas=cols, prec=prec)
        assert torch.equal(out, got)


@pytest.mark.gpu
def test_noalloc_rejects_too_large(gpu_lib):
    """ceil(n / 256) * kept + 2 kept doubles above the 64 MiB scratch (n = 4e6, kept = 600: 75 MB): KRR_EINVAL
    before any GPU work, and the handle still works with the allocating entry point."""
    n, d, k, eps = 4_000_000, 2, 600, 1e-3
    X = np.random.default_rng(21).random((n, d))
    S = np.random.default_rng(22).choice(n, size=k, replace=False).astype(np.int64)
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [1e-2], k, anchors=torch.from_numpy(S), prec="fp64")
    kept = P.info()["kept"]
    need = -(-n // 256) * kept + 2 * kept
    assert need * 8 > 64 << 20, f"kept {kept}: the case no longer exceeds the scratch"
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(gpu_lib.KRRError, match="scratch") as e:
        P.apply_noalloc(x, out, prec="fp64")
    assert e.value.status == -1
    y = P.apply(x, prec="fp64")
    assert torch.isfinite(y).all()
