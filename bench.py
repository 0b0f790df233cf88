"""Benchmark: Gaussian KRR hot path on one MI355X (one JSON line on stdout).

Default workload "mixed": n = 1,000,000 points uniform in [0,1]^4, y = sum_m sin(2 pi m x_m)/m + 0.1 N(0,1),
eps = 0.01, beta = 1e-3, k = 2000 anchors from an Algorithm 2 sketch (l = 2020, r = 32), mixed precision
(split-BF16 MFMA cross term, FP32 exp/accumulate, FP64 scalars and residual replacement every 10
iterations), tol 1e-6.  Its full solve takes minutes, so a step is one replacement cycle of the PCG
(Algorithm 5): 10 mixed iterations and the FP64 residual replacement, cold-started on the resident
inputs; the preconditioner build (Algorithms 2-3) is timed once beside the steps.  After the timed
region: the same cycle with the FP64 and the FP32 kernels, the CPU oracle, and the full solve to 1e-6
(its iteration cap set by --budget-s so the run stays within its wall-clock budget).

value = kernel pairs evaluated by the step's MVMs (mixed and FP64) / step wall time, in Gpairs/s.
roofline: the mixed MVM kernel (HIP events around its launches inside the library), against the VALU
bound of the form that ran.  Other workloads (--workload fp32|small|block|adjoint): a step is the whole
build + solve (or build + gradient).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PCG solve s to rel-res 1e-6 + kernel-MVM Gpairs/s; mixed vs FP64, same GPU"
# VALU-only bound of the kernel MVM on MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 lane-slots/s.
# Direct form: one pair needs one v_exp_f32 (half rate: 2 slots) and one FMA (1 slot) -> 13.1e12 pairs/s.
# Symmetric form (square products): one exp and two FMAs (row and column sums) serve two pairs of the
# product -> 2 slots per pair -> 19.7e12 pairs/s.  Pairs are the product's n^2 (the algorithmic units).
SLOTS = 256 * 4 * 16 * 2.4e9
PEAK_PAIRS = SLOTS / 3.0
PEAK_PAIRS_SYM = SLOTS / 2.0
# The mixed forms also issue NCH MFMAs (v_mfma_f32_16x16x32_bf16, 16 cycles each at full rate) per 256
# evaluated pairs, and on this part MFMA and VALU work barely overlap (about 6%, measured with a register-only probe
# and with the kernel's own counters), so the bound is VALU cycles + MFMA cycles per 256 evaluated pairs:
# direct 48 + 16 NCH, symmetric 64 + 16 NCH (symmetric: two product pairs per evaluated pair).
SIMD_CYCLES = 256 * 4 * 2.4e9


def mixed_chunks(d):
    need = -(-(6 * d + 6) // 32)
    return next(c for c in (1, 2, 3, 4, 6, 8, 13, 25) if c >= need)


def peak_mixed(d, sym):
    nch = mixed_chunks(d)
    return (2.0 if sym else 1.0) * 256 * SIMD_CYCLES / ((64 if sym else 48) + 16 * nch)


def f64_symm_slots(d):
    """VALU instructions per evaluated pair of the FP64 symmetric matrix-core form (see peak_direct)."""
    width = next((w for w in (2, 3, 4, 6, 8, 16) if d <= w), d)   # the kernel's padded width (no such form above 16)
    return 17 if width % 4 == 2 else 18


def peak_direct(d, prec, sym, variant=None):
    """VALU bound of the FP32 / FP64 forms (one lane-slot per VALU instruction, exp2 in FP32 counted as two):
    FP32 per pair d subtractions + d FMAs + exp + one FMA; FP64 per pair d subtractions + d FMAs + a
    16-instruction exp2 (scaling by -log2(e)/eps, reduction, degree-10 polynomial, 2^n) + one FMA, + one more
    FMA in the symmetric form, whose evaluated pair serves two pairs of the product.  The FP64 symmetric forms
    with the exponent's cross term on the matrix cores (variants 5, 6) issue 18 VALU instructions per evaluated
    pair whatever d (q from the contraction, which starts from the row norm, and the source norm: 1; exp2 without
    the scaling: 15; row and column FMAs: 2), 17 where both norms are contracted with it (padded widths 2, 6);
    their MFMAs run on the matrix cores."""
    if prec == "fp32":
        return SLOTS / (2 * d + 3)
    if sym and variant is not None and variant >= 5:
        return 2.0 * SLOTS / f64_symm_slots(d)
    return (2.0 * SLOTS / (2 * d + 18)) if sym else SLOTS / (2 * d + 17)
# Files whose contents define the mixed MVM kernels and their launch: a stored counter summary is used
# for roofline.traffic only while these hash to the value recorded with it.
KERNEL_SOURCES = ("paper_1905_10587_amd/csrc/kmv_kernels.h", "paper_1905_10587_amd/csrc/kmv_mixed.hip",
                  "paper_1905_10587_amd/csrc/kmv.hip", "paper_1905_10587_amd/csrc/kmv.h",
                  "paper_1905_10587_amd/csrc/kmv_dispatch.h")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload):
    """HBM bytes per launch of the mixed MVM kernel from the committed counter summary, or None when the
    summary is missing, is for another workload, or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    return rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(X, eps, seconds=15.0, threads=None):
    """CPU oracle (FP64 NumPy, as written) timed on a bounded row sample of one kernel MVM, on the host's
    cores: each worker thread runs the oracle's row-sampled product on its own rows (NumPy's array loops
    release the GIL; BLAS kept to one thread per worker).  Returns (pairs/s over wall time, rows, seconds,
    threads)."""
    import concurrent.futures as cf
    import threading

    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import kernel as ok

    threads = threads or max(1, min(16, os.cpu_count() or 1))
    v = np.random.default_rng(0).standard_normal(X.shape[0])
    stop = threading.Event()
    counts = [0] * threads

    def worker(w):
        rng = np.random.default_rng(100 + w)
        while not stop.is_set():
            ok.kernel_mv_rows(X, eps, v, rng.integers(0, X.shape[0], 8))
            counts[w] += 8

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            futs = [ex.submit(worker, w) for w in range(threads)]
            time.sleep(seconds)
            stop.set()
            for f in futs:
                f.result()
        secs = time.perf_counter() - t0
    rows = sum(counts)
    return rows * float(X.shape[0]) / secs, rows, secs, threads


def kernels_only(a, wl, Xg, krr, torch):
    """Plain copy of known size, then the workload's kernel MVMs (for rocprofv3 traces and counters)."""
    dev = Xg.device
    # calibration: a 1 GiB copy whose source has been pushed out of the last-level cache by a second 1 GiB fill
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    src.fill_(1.0)
    flush = torch.empty_like(src)
    flush.fill_(2.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, flush, dst
    out = {"copy_bytes": nbytes}
    R = wl.y.shape[1] if wl.y.ndim == 2 else 1   # the workload's right-hand sides (the block MVM for R > 1)
    v = torch.randn(wl.n, R, dtype=torch.float64, device=dev) if R > 1 else torch.randn(wl.n, dtype=torch.float64,
                                                                                            device=dev)
    out["columns"] = R
    for prec, reps in (("mixed", a.reps), ("fp64", 1)):
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            krr.kernel_mv(Xg, None, wl.eps, v, shift=wl.betas[0], prec=prec)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        out[f"{prec}_ms"] = times
        out[f"{prec}_gpairs_s"] = round(float(wl.n) * wl.n / min(times) / 1e6, 1)
        log(f"bench: {prec} MVM n={wl.n}: {min(times):.2f} ms")
    print(json.dumps(out), flush=True)
    return 0


def traffic_record(a):
    """CPU only: summarise the FETCH_SIZE and WRITE_SIZE counter passes (rocprofv3 --pmc ... --output-format
    csv -- python3 bench.py --kernels-only) into profiles/traffic_<workload>.json, the HBM bytes per launch of
    the workload's mixed MVM kernel that the benchmark reports as roofline.traffic.  Each counter is scaled by
    what it reads for the 1 GiB copy that --kernels-only runs first (bytes copied / counter)."""
    import csv

    def per_dispatch(path):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                d = acc.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])
                d[1] += float(r["Counter_Value"])
        return [acc[k] for k in sorted(acc)]

    fetch, write = (per_dispatch(p) for p in a.traffic_record)
    copy_bytes = 1 << 30

    def copy_kib(rows):
        c = [v for n, v in rows if "copy" in n.lower()]
        if not c:
            raise SystemExit("no copy kernel in the counter file")
        return max(c)

    def kernel_kib(rows):
        v = [x for n, x in rows if a.kernel_name in n]
        if not v:
            raise SystemExit(f"no dispatch of a kernel named like {a.kernel_name!r}")
        return v, [n for n, _ in rows if a.kernel_name in n][0]

    cf, cw = copy_kib(fetch), copy_kib(write)
    (kf, name), (kw, _) = kernel_kib(fetch), kernel_kib(write)
    fs, ws = copy_bytes / 1024 / cf, copy_bytes / 1024 / cw
    mf, mw = sum(kf) / len(kf), sum(kw) / len(kw)
    rec = {"workload": a.workload, "kernel": name[:80], "sources_sha256": kernel_sources_sha256(),
           "files": list(KERNEL_SOURCES), "fetch_kib_per_launch_raw": round(mf, 1),
           "write_kib_per_launch_raw": round(mw, 1), "launches": len(kf), "copy_bytes": copy_bytes,
           "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw, "fetch_scale": round(fs, 4),
           "write_scale": round(ws, 4), "hbm_bytes_per_launch": int(mf * 1024 * fs + mw * 1024 * ws)}
    path = os.path.join(ROOT, "profiles", f"traffic_{a.workload}.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))
    return 0


def study_anchors(a, wl, Xg, Yg, krr, torch, datagen, prec, replace_every):
    """Anchor-selection variants on one workload (remark in Sec. 3; the l-versus-iterations tradeoff):
    Algorithm 1 (dense sketch), Algorithm 2 over r, random sampling, farthest point sampling and no
    preconditioner.  Build time, iterations and solve time for each."""
    import numpy as np
    dev = Xg.device
    n, k, l = wl.n, wl.k, wl.l
    beta = float(wl.betas[0])
    seed = datagen.sketch_seed(wl.name)
    rows = []
    # warm-up: first use of the build's kernels and BLAS handles, not timed
    krr.Preconditioner(Xg, wl.eps, [beta], 64, 84, omega=torch.from_numpy(datagen.sketch_dense_omega(n, 84, 1)).to(dev),
                       prec=prec)
    torch.cuda.synchronize()
    cases = [("alg1_dense", {}), *[(f"alg2_sparse_r{r}", {"r": r}) for r in (8, 32, 128)],
             ("random", {}), ("fps", {}), ("none", {})]
    for name, opt in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "alg1_dense":
            om = torch.from_numpy(datagen.sketch_dense_omega(n, l, seed)).to(dev)
            P = krr.Preconditioner(Xg, wl.eps, [beta], k, l, omega=om, prec=prec)
        elif name.startswith("alg2"):
            idx, sign = datagen.sketch_sparse_draws(n, l, opt["r"], seed)
            P = krr.Preconditioner(Xg, wl.eps, [beta], k, l, idx=torch.from_numpy(idx).to(dev),
                                   sign=torch.from_numpy(sign).to(dev), prec=prec)
        elif name == "random":
            S = torch.from_numpy(datagen.random_anchors(n, k, seed)).to(dev)
            P = krr.Preconditioner(Xg, wl.eps, [beta], k, anchors=S, prec=prec)
        elif name == "fps":
            P = krr.Preconditioner(Xg, wl.eps, [beta], k, anchors="fps", fps_start=0, prec=prec)
        else:
            P = None
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        alpha, its, rel, st, status = krr.pcg_solve(Xg, Yg, wl.eps, [beta], P, tol=wl.tol, maxit=a.maxit,
                                                    replace_every=replace_every, prec=prec)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0 - tb
        row = {"anchors": name, "build_s": round(tb, 3), "solve_s": round(ts, 3), "iterations": max(its),
               "relres_true": max(rel), "status": status, "kappa_est": round(st["kappa_est"], 1)}
        if P is not None:
            row["build_phases_ms"] = {kk: round(v, 1) for kk, v in P.timings().items()}
            row["kept"] = P.info()["kept"]
        log(f"bench: anchors {name}: build {tb:.3f} s, {max(its)} iterations, solve {ts:.3f} s")
        rows.append(row)
        del P
    print(json.dumps({"study": "anchors", "workload": f"{wl.name}: n={n} d={wl.d} eps={wl.eps} beta={beta} "
                                                      f"k={k} l={l} tol={wl.tol}",
                      "precision": prec, "replace_every": replace_every, "data": "synthetic", "rows": rows}))
    return 0


def study_cond(a, krr, torch, datagen):
    """Condition numbers with and without the preconditioner on 10,000-point draws of each workload's
    distribution (the setting of Sec. 5.1: k = 100, 500, 1000, Algorithm 2 anchors with l = k + 5), measured
    as the extreme Ritz
    values of FP64 CG/PCG on a Gaussian right-hand side run to 1e-10; beside them the rank that
    Corollary tradeoff asks for."""
    import numpy as np
    dev = torch.device("cuda:0")
    out = []
    for name in ("fp32", "mixed", "adjoint", "block"):
        wl = datagen.make_workload(name, **({"n": 10_000, "m": 1000} if name == "adjoint" else {"n": 10_000}))
        X = torch.from_numpy(wl.X).to(dev)
        # a Gaussian right-hand side excites every eigenvector, so the Ritz values reach both ends of
        # the spectrum (a label vector may have almost nothing at the bottom)
        yg = torch.from_numpy(np.random.default_rng(7).standard_normal(wl.n)).to(dev)
        beta = float(wl.betas[0])
        seed = datagen.sketch_seed(name)
        entry = {"workload": name, "n": wl.n, "d": wl.d, "eps": wl.eps, "beta": beta, "rows": []}
        for k in (0, 100, 500, 1000):
            P = None
            t0 = time.perf_counter()
            if k:
                idx, sign = datagen.sketch_sparse_draws(wl.n, k + 5, min(32, wl.n), seed)
                P = krr.Preconditioner(X, wl.eps, [beta], k, k + 5, idx=torch.from_numpy(idx).to(dev),
                                       sign=torch.from_numpy(sign).to(dev), prec="fp64")
            _, its, rel, st, status = krr.pcg_solve(X, yg, wl.eps, [beta], P, tol=1e-10, maxit=20_000,
                                                    prec="fp64")
            torch.cuda.synchronize()
            entry["rows"].append({"k": k, "cond": st["kappa_est"], "lam_min": st["lam_min_est"],
                                  "lam_max": st["lam_max_est"], "iterations": max(its), "relres_true": max(rel),
                                  "s": round(time.perf_counter() - t0, 3)})
            log(f"bench: cond {name} k={k}: {st['kappa_est']:.4g} ({max(its)} iterations)")
        g, kb, q = krr.rank_for_cond(X, wl.eps, beta, 2.0)
        entry["corollary_tradeoff_xi2"] = {"gamma": g, "k_bound": kb, "q": q}
        out.append(entry)
    print(json.dumps({"study": "cond", "data": "synthetic", "subsets": out}))
    return 0


def mvm_roofline(prec, d, R, n, avg_ms, launches, variant, sym, traffic):
    """Roofline record of the dominant kernel (the working-precision MVM).  frac is against the VALU-only
    hardware bound of the form that ran (the exp and FMAs it must issue); for the mixed forms the bound that
    also charges the MFMA cross term, which on this part does not overlap the VALU work, is given beside it
    as an implementation figure."""
    achieved = float(n) * n / (avg_ms * 1e-3)
    if prec == "mixed":
        peak = PEAK_PAIRS_SYM if sym else PEAK_PAIRS
        ser = peak_mixed(d, sym)
        form = "symmetric form (exp + 2 FMA per evaluated pair, two pairs each)" if sym else \
            "direct form (exp + FMA per pair)"
    else:
        peak = ser = peak_direct(d, prec, sym, variant)
        form = f"{'symmetric' if sym else 'direct'} form, {prec} VALU ops per pair"
        if prec == "fp64" and sym and variant is not None and variant >= 5:
            form = (f"symmetric form, exponent's cross term on the FP64 matrix cores, {f64_symm_slots(d)} "
                    f"VALU ops per evaluated pair")
    rec = {"bound": "alu", "kernel": f"{prec} MVM, variant {variant}, {form}, d={d}",
           "achieved": round(achieved / 1e12, 3), "peak": round(peak / 1e12, 2), "unit": "Tpairs/s",
           "frac": round(achieved / peak, 3), "traffic": traffic,
           "avg_kernel_ms": round(avg_ms, 4), "launches": launches,
           "pairs_per_launch": float(n) * n}
    if prec == "mixed":
        rec["peak_valu_plus_mfma_serialized"] = round(ser / 1e12, 2)
        rec["frac_of_serialized_bound"] = round(achieved / ser, 3)
    return rec


def load_launch_table(krr, torch):
    """The kernel MVM launch table tuned for this GPU (paper_1905_10587_amd/tuned/<arch>.json, written by
    python -m paper_1905_10587_amd.tune), if present; its path, else None (the launcher's defaults)."""
    from paper_1905_10587_amd import tune
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tune.table_path(arch)
    if not os.path.exists(path):
        return None
    krr.autotune_load(path)
    return os.path.relpath(path, ROOT)


def cycle_bench(a, wl, Xg, Yg, sk, krr, torch, t_proc0):
    """Default benchmark: the n = 1,000,000, d = 4 mixed-precision solve.  A step is one replacement cycle of
    its PCG (Algorithm 5): replace_every mixed iterations (split-BF16 MFMA cross term, FP32 exp, Woodbury
    apply with the FP32 factor, FP64 scalars) and the FP64 residual replacement, from a cold start on the
    resident inputs; the preconditioner is built once, timed beside the steps.  After the timed region:
    one cycle each with the FP64 and FP32 kernels (same preconditioner, same GPU), the CPU oracle, and the
    full solve to rel-res tol under the run's wall-clock budget."""
    prec, rep = "mixed", 10
    beta = float(wl.betas[0])
    n = wl.n
    table = load_launch_table(krr, torch)
    # one product first: the launch the solve's MVMs take (variant, split) is read back from the library
    krr.kernel_mv(Xg, None, wl.eps, Yg, shift=beta, prec=prec)
    launched = dict(zip(("variant", "split", "symmetric"), krr.kmv_last_launch()))
    c_tot, c_skip = krr.cull_stats()
    # warm-up build on a slice (first use of the build's kernels), not timed
    m0 = min(n, 16384)
    import datagen
    idx0, sign0 = datagen.sketch_sparse_draws(m0, 84, 8, 1)
    krr.Preconditioner(Xg[:m0], wl.eps, [beta], 64, 84, idx=torch.from_numpy(idx0).to(Xg.device),
                       sign=torch.from_numpy(sign0).to(Xg.device), prec=prec)
    torch.cuda.synchronize()
    log(f"bench: building the preconditioner (k={wl.k}, l={wl.l}, r={wl.r})")
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    P = krr.Preconditioner(Xg, wl.eps, [beta], wl.k, wl.l, prec=prec, **sk)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    # device memory the build held at its peak beyond the resident inputs (all of it comes through torch's
    # caching allocator)
    build_peak_gb = round((torch.cuda.max_memory_allocated() - base) / 1e9, 2)
    phases = {k: round(v, 1) for k, v in P.timings().items()}
    log(f"bench: build {build_s:.3f} s {phases}")

    def cycle(p=prec, r=rep):
        return krr.pcg_solve(Xg, Yg, wl.eps, [beta], P, tol=wl.tol, maxit=10, replace_every=r, prec=p,
                             timing=True)

    for w in range(a.warmup):
        log(f"bench: warmup step {w + 1}/{a.warmup}")
        cycle()
    torch.cuda.synchronize()
    log(f"bench: timing {a.steps} step(s)")
    tot = {"n_mvm": 0, "n_mvm_fp64": 0, "t_mvm_kernel_ms": 0.0, "t_mvm_ms": 0.0, "t_mvm_fp64_ms": 0.0,
           "t_precond_ms": 0.0}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(a.steps):
        _, its, rel, st, status = cycle()
        for k in tot:
            tot[k] += st[k]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    step_s = t_total / a.steps
    n_mvm, n_fp64 = tot["n_mvm"] // a.steps, tot["n_mvm_fp64"] // a.steps
    pairs_step = (n_mvm + n_fp64) * float(n) * n
    variant, sym = krr.kmv_variant(wl.d, 1, prec, square=True)
    avg_ms = tot["t_mvm_kernel_ms"] / max(tot["n_mvm"], 1)
    traffic = stored_traffic(wl.name)
    out = {
        "metric": METRIC,
        "value": round(pairs_step / step_s / 1e9, 2),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * step_s, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-split/f32/f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: n={n} d={wl.d} eps={wl.eps} beta={beta} k={wl.k} l={wl.l} "
                               f"r={wl.r} tol={wl.tol}; uniform points in [0,1]^4, "
                               f"y = sum_m sin(2 pi m x_m)/m + 0.1 N(0,1)",
                   "step": f"one replacement cycle of the PCG solve: {rep} mixed iterations + FP64 residual "
                           f"replacement, cold start", "precision": prec, "replace_every": rep},
        "step_mvms": {"mixed": n_mvm, "fp64": n_fp64},
        "step_split_ms": {"mixed_mvm": round(tot["t_mvm_ms"] / a.steps, 2),
                          "fp64_mvm": round(tot["t_mvm_fp64_ms"] / a.steps, 2),
                          "woodbury": round(tot["t_precond_ms"] / a.steps, 2)},
        "build_s": round(build_s, 3),
        "build_phases_ms": phases,
        "build_peak_gb": build_peak_gb,
        "launch_table": table,
        "mixed_mvm_launch": launched,
        "mvm_gpairs_s": round(float(n) * n / avg_ms / 1e6, 1),
        "roofline": mvm_roofline(prec, wl.d, 1, n, avg_ms, tot["n_mvm"], variant, sym,
                                 None if traffic is None else traffic["hbm_bytes_per_launch"]),
    }
    # the same cycle with the FP64 and the FP32 kernels (library kernel events, as for the mixed kernel)
    for p2, r2 in (("fp64", 0), ("fp32", 10)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its2, _, st2, _ = krr.pcg_solve(Xg, Yg, wl.eps, [beta], P, tol=wl.tol, maxit=10, replace_every=r2,
                                           prec=p2, timing=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        k_ms = st2["t_mvm_kernel_ms"] / max(st2["n_mvm"], 1)
        v2, s2 = krr.kmv_variant(wl.d, 1, p2, square=True) if p2 == "fp64" else (None, False)
        out[f"{p2}_cycle"] = {"s": round(dt, 3), "iterations": max(its2), "n_mvm": st2["n_mvm"],
                              "n_mvm_fp64": st2["n_mvm_fp64"], "mvm_kernel_ms": round(k_ms, 3),
                              "mvm_gpairs_s": round(float(n) * n / k_ms / 1e6, 1)}
        if p2 == "fp64":   # the FP64 form's VALU bound (its operation count is fixed by its arithmetic)
            out[f"{p2}_cycle"]["roofline"] = mvm_roofline(p2, wl.d, 1, n, k_ms, st2["n_mvm"], v2, s2, None)
        out[f"mvm_gpairs_s_{p2}"] = out[f"{p2}_cycle"]["mvm_gpairs_s"]
        log(f"bench: {p2} cycle {dt:.3f} s, MVM kernel {k_ms:.2f} ms")
    out["mvm_speedup_vs_fp64"] = round(out["mvm_gpairs_s"] / out["mvm_gpairs_s_fp64"], 2)
    out["cycle_speedup_vs_fp64"] = round(out["fp64_cycle"]["s"] / step_s, 2)
    # exact far-tile culling: pairs of the product whose evaluation was skipped, and the same cycle without it
    off, skipped = {}, {}
    try:
        for mode in (1, 2, 0):   # culling forced on; spatial order without skipping; the caller's order
            krr.set_cull(mode)
            krr.kernel_mv(Xg, None, wl.eps, Yg, shift=beta, prec=prec)
            skipped[mode] = krr.cull_stats()[1]
            _, _, _, st0, _ = krr.pcg_solve(Xg, Yg, wl.eps, [beta], P, tol=wl.tol, maxit=10, replace_every=rep,
                                            prec=prec, timing=True)
            off[mode] = st0["t_mvm_kernel_ms"] / max(st0["n_mvm"], 1)
    finally:
        krr.set_cull(-1)
    out["culling"] = {"pairs_per_product": c_tot, "pairs_skipped_default": c_skip,
                      "pairs_skippable": skipped[1],
                      "evaluated_fraction_forced": round(1.0 - skipped[1] / max(c_tot, 1), 4),
                      "mvm_kernel_ms_default": round(avg_ms, 3), "mvm_kernel_ms_culling_forced": round(off[1], 3),
                      "mvm_kernel_ms_spatial_order_only": round(off[2], 3),
                      "mvm_kernel_ms_caller_order": round(off[0], 3),
                      "note": "pairs counted over the points padded to a multiple of 1024; skipped pairs are "
                              "those whose kernel value is exactly zero in FP32; the default (automatic) mode "
                              "skips only when at least 10% of the steps can be skipped"}
    log(f"bench: culling could skip {skipped[1] / max(c_tot, 1):.4f} of the pairs (default skipped "
        f"{c_skip / max(c_tot, 1):.4f}); mixed MVM {avg_ms:.2f} ms default, {off[1]:.2f} forced, "
        f"{off[2]:.2f} spatial order only, {off[0]:.2f} caller's order")
    if not a.no_cpu:
        log("bench: CPU oracle baseline")
        rate, rows, secs, thr = oracle_baseline(wl.X, wl.eps)
        out["cpu_baseline"] = {"value": round(rate / 1e9, 4), "unit": "Gpairs/s", "cores": thr, "kind": "oracle",
                               "cpu": cpu_model(),
                               "sample": f"oracle kernel_mv_rows (FP64 NumPy) on {rows} random rows x {n} sources "
                                         f"({rows * float(n):.3g} pairs, {secs:.1f} s wall, {thr} threads); the "
                                         f"oracle's solve runs the same product once per iteration"}
        log(f"bench: CPU oracle {rate / 1e9:.4f} Gpairs/s on {thr} threads")
    if not a.no_full_solve:
        # the full solve to tol, capped so that the whole run stays inside its wall-clock budget
        per_it = step_s / 10.0
        left = a.budget_s - (time.perf_counter() - t_proc0) - 15.0
        maxit = int(min(a.maxit, max(0.0, left) / (per_it * 1.05)))
        log(f"bench: full solve to {wl.tol} (maxit {maxit} from the {a.budget_s:.0f} s budget)")
        if maxit >= 10:
            os.environ.setdefault("KRR_PROGRESS", "200")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            alpha, its, rel, st, status = krr.pcg_solve(Xg, Yg, wl.eps, [beta], P, tol=wl.tol, maxit=maxit,
                                                        replace_every=rep, prec=prec, timing=True)
            torch.cuda.synchronize()
            solve_s = time.perf_counter() - t0
            fp64_per_it = out["fp64_cycle"]["s"] / max(out["fp64_cycle"]["iterations"], 1)
            out["solve"] = {"solve_s": round(solve_s, 2), "build_plus_solve_s": round(build_s + solve_s, 2),
                            "iterations": max(its), "relres_true": max(rel), "status": status,
                            "converged": bool(status == 0 and max(rel) <= wl.tol), "maxit": maxit,
                            "n_mvm": st["n_mvm"], "n_mvm_fp64": st["n_mvm_fp64"],
                            "t_mvm_s": round(st["t_mvm_ms"] / 1e3, 2),
                            "t_mvm_fp64_s": round(st["t_mvm_fp64_ms"] / 1e3, 2),
                            "t_woodbury_s": round(st["t_precond_ms"] / 1e3, 2),
                            "fp64_replacement_share": round(st["t_mvm_fp64_ms"] / 1e3 / solve_s, 3),
                            "kappa_est": round(st["kappa_est"], 1),
                            "fp64_solve_s_projected": round(fp64_per_it * max(its), 1),
                            "solve_speedup_vs_fp64_projected": round(fp64_per_it * max(its) / solve_s, 2),
                            "projection": "FP64 cycle time per iteration (same GPU, same preconditioner) x "
                                          "the mixed solve's iteration count"}
            log(f"bench: solve {solve_s:.1f} s, {max(its)} iterations, relres {max(rel):.3e}, status {status}")
    return out


def main(argv=None):
    t_proc0 = time.perf_counter()
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed", choices=["mixed", "fp32", "small", "block", "adjoint"])
    ap.add_argument("--prec", default=None, help="working precision (default: the workload's)")
    ap.add_argument("--fp64-solve", action="store_true", help="also run the full FP64 solve (minutes)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-full-solve", action="store_true", help="mixed workload: skip the full solve after "
                                                                 "the timed cycles")
    ap.add_argument("--budget-s", type=float, default=525.0,
                    help="wall-clock budget of the whole run; caps the full solve's iterations")
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--beta-columns", type=float, nargs="*", default=None,
                    help="block workload: solve only the columns of these betas")
    ap.add_argument("--column-slice", type=int, nargs=2, default=None, metavar=("START", "STOP"),
                    help="with --beta-columns: the selected columns [START, STOP) only")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling mode: a 1 GiB device copy (counter calibration), then the workload's "
                         "mixed and FP64 kernel MVMs; prints their HIP-event times")
    ap.add_argument("--reps", type=int, default=3, help="MVM launches per precision in --kernels-only")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="CPU only: write profiles/traffic_<workload>.json from the two counter passes")
    ap.add_argument("--kernel-name", default="k_kmv_mixed_sym",
                    help="kernel whose traffic --traffic-record summarises (a substring of its name)")
    ap.add_argument("--save-alpha", default=None, help="write the timed solve's alpha (.npy) after the run")
    ap.add_argument("--study", default=None, choices=["anchors", "cond"],
                    help="instead of the benchmark step: anchor-selection variants on the workload, or "
                         "condition numbers with/without the preconditioner on 10,000-point subsets")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: the solver has no multi-GPU path "
                                   "(row sharding of the targets is designed, not implemented)",
                          "n_gpus": a.gpus}))
        return 2
    if a.traffic_record:
        return traffic_record(a)

    import numpy as np
    import torch

    import datagen
    import paper_1905_10587_amd as krr

    krr.load()
    assert torch.cuda.is_available(), "bench needs a GPU"
    load_launch_table(krr, torch)   # every mode launches the tuned kernels (the default step records the path)
    if a.study == "cond":
        return study_cond(a, krr, torch, datagen)
    wl = datagen.make_workload(a.workload)
    prec = a.prec or {"mixed": "mixed", "fp32": "mixed", "small": "fp64", "block": "mixed", "adjoint": "mixed"}[a.workload]
    replace_every = 0 if prec == "fp64" else 10
    log(f"bench: workload {wl.name} n={wl.n} d={wl.d} eps={wl.eps} betas={wl.betas} k={wl.k} l={wl.l} "
        f"r={wl.r} tol={wl.tol} prec={prec}")
    dev = torch.device("cuda:0")
    Xg = torch.from_numpy(wl.X).to(dev)
    Y = wl.y if wl.y.ndim == 1 else wl.y
    Yg = torch.from_numpy(Y).to(dev)
    if wl.col_beta is not None:
        betas_col = [float(b) for b in wl.col_beta]
        if a.beta_columns:
            # the columns of the listed betas only (their recurrences are independent of the others; the
            # preconditioner is still built for every beta of the workload, as in the full run)
            keep = [c for c, b in enumerate(betas_col) if any(abs(b - x) <= 1e-12 * x for x in a.beta_columns)]
            if not keep:
                raise SystemExit("--beta-columns selects no column")
            if a.column_slice:
                keep = keep[a.column_slice[0]:a.column_slice[1]]
            Yg = Yg[:, keep].contiguous()
            betas_col = [betas_col[c] for c in keep]
            log(f"bench: {len(keep)} of {len(wl.col_beta)} columns (betas {sorted(set(betas_col))}, "
                f"columns {keep[0]}..{keep[-1]})")
    else:
        betas_col = [float(wl.betas[0])] * (1 if Y.ndim == 1 else Y.shape[1])
    if wl.r > 0:
        idx, sign = datagen.sketch_sparse_draws(wl.n, wl.l, wl.r, datagen.sketch_seed(wl.name))
        sk = dict(idx=torch.from_numpy(idx).to(dev), sign=torch.from_numpy(sign).to(dev))
    else:
        sk = dict(omega=torch.from_numpy(datagen.sketch_dense_omega(wl.n, wl.l, datagen.sketch_seed(wl.name))).to(dev))
    torch.cuda.synchronize()
    if a.kernels_only:
        return kernels_only(a, wl, Xg, krr, torch)
    if a.study == "anchors":
        return study_anchors(a, wl, Xg, Yg, krr, torch, datagen, prec, replace_every)
    if a.workload == "mixed" and prec == "mixed":
        out = cycle_bench(a, wl, Xg, Yg, sk, krr, torch, t_proc0)
        print(json.dumps(out), flush=True)
        return 0
    return solve_bench(a, wl, Xg, Yg, sk, betas_col, prec, replace_every, krr, torch)


def solve_bench(a, wl, Xg, Yg, sk, betas_col, prec, replace_every, krr, torch):
    """Other workloads: a step is the whole solve (preconditioner build + PCG to tol, or for the adjoint
    workload build + gradient)."""
    dev = Xg.device
    adjoint = wl.X_val is not None
    if adjoint:
        Xvg = torch.from_numpy(wl.X_val).to(dev)
        yvg = torch.from_numpy(wl.y_val).to(dev)
    grad_out = {}

    def step():
        t0 = time.perf_counter()
        P = krr.Preconditioner(Xg, wl.eps, list(wl.betas), wl.k, wl.l, prec=prec, **sk)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        if adjoint:
            # the step of this workload is the validation-loss gradient: forward solve, adjoint solve and the
            # FP64 products that assemble loss and gradient
            loss, ge, gb, alpha, lam, gstatus, sts = krr.grad(Xg, Yg, Xvg, yvg, wl.eps, wl.betas[0], P,
                                                              tol=wl.tol, maxit=a.maxit,
                                                              replace_every=replace_every, prec=prec,
                                                              return_stats=True)
            torch.cuda.synchronize()
            grad_out.update(loss=loss, dloss_dlog_eps=ge, dloss_dlog_beta=gb, stats=sts, status=gstatus)
            st = {k: sts[0][k] + sts[1][k] for k in sts[0] if k not in ("kappa_est", "iters_max")}
            st["kappa_est"] = sts[0]["kappa_est"]
            st["iters_max"] = max(sts[0]["iters_max"], sts[1]["iters_max"])
            its, rel = [sts[0]["iters_max"], sts[1]["iters_max"]], [0.0]
            return P, alpha, its, rel, st, gstatus, tb, time.perf_counter() - t0
        alpha, its, rel, st, status = krr.pcg_solve(Xg, Yg, wl.eps, betas_col, P, tol=wl.tol, maxit=a.maxit,
                                                    replace_every=replace_every, prec=prec, timing=True)
        torch.cuda.synchronize()
        return P, alpha, its, rel, st, status, tb, time.perf_counter() - t0

    os.environ.setdefault("KRR_PROGRESS", "100")
    for w in range(a.warmup):
        log(f"bench: warmup step {w + 1}/{a.warmup}")
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {a.steps} step(s)")
    t_start = time.perf_counter()
    results = []
    for s in range(a.steps):
        results.append(step())
        log(f"bench: step {s + 1}: build {results[-1][6]:.2f} s, total {results[-1][7]:.2f} s, "
            f"iterations {max(results[-1][2])}, relres {max(results[-1][3]):.2e}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    P, alpha, its, rel, st, status, t_build, t_step = results[-1]
    pcg_drivers = None
    if not adjoint and float(wl.n) * wl.n * len(betas_col) <= 2.0 ** 34:   # (automatic mode: 2^30)
        # after the timed region: the same solve under each PCG driver (phase timers off), the second of two
        # calls timed (the first captures the graphs), and whether the two return the same bits
        pcg_drivers = {}
        ref = None
        try:
            for mode, name in ((0, "host_loop"), (1, "graph_cycles")):
                krr.set_pcg_mode(mode)
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    al, its2, _, st2, _ = krr.pcg_solve(Xg, Yg, wl.eps, betas_col, P, tol=wl.tol, maxit=a.maxit,
                                                        replace_every=replace_every, prec=prec)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                pcg_drivers[name] = {"solve_ms": round(1e3 * dt, 2), "iterations": max(its2),
                                     "us_per_iteration": round(1e6 * dt / max(max(its2), 1), 1),
                                     "graph_cycles": st2["n_graph_cycles"]}
                if ref is None:
                    ref = al.clone()
                else:
                    pcg_drivers["bit_identical"] = bool(torch.equal(ref, al))
        finally:
            krr.set_pcg_mode(-1)
    if a.save_alpha:
        import numpy as np
        np.save(a.save_alpha, alpha.cpu().numpy())
    R = len(betas_col)
    n = wl.n
    pairs_step = (st["n_mvm"] + st["n_mvm_fp64"]) * float(n) * n
    if adjoint:   # + fused (K, K') on validation x training, K^T r_v, K' alpha (FP64)
        m = wl.X_val.shape[0]
        pairs_step += 2.0 * m * n + float(n) * n
    ms_per_step = 1e3 * t_total / a.steps
    value = pairs_step / (t_total / a.steps) / 1e9
    avg_mvm_ms = st["t_mvm_kernel_ms"] / max(st["n_mvm"], 1)
    achieved = float(n) * n / (avg_mvm_ms * 1e-3)
    variant, sym = krr.kmv_variant(wl.d, R, prec, square=True) if prec in ("mixed", "fp64") else (None, False)
    traffic = stored_traffic(wl.name) if prec == "mixed" and R == 1 else None
    block_mvm = prec == "mixed" and R > 1
    if block_mvm:
        # many right-hand sides: the exp'd tile is contracted with V on MFMA; the method's work per pair is one
        # exp and 2R flops (K V); the split products (three per column) and the cross term are the
        # implementation's cost.  Dense BF16 peak 2.5 PFLOP/s.
        nch = -(-(6 * wl.d + 6) // 32)
        flop_impl = 2.0 * 3 * R + 2.0 * 32 * nch
        roofline = {"bound": "mfma", "kernel": f"block MVM (variant {variant}), R={R}, d={wl.d}",
                    "achieved": round(achieved * flop_impl / 1e12, 1), "peak": 2500.0, "unit": "TFLOP/s",
                    "frac": round(achieved * flop_impl / 2.5e15, 3), "traffic": None,
                    "flop_per_pair_issued": flop_impl, "flop_per_pair_method": 2.0 * R,
                    "frac_method_flops": round(achieved * 2.0 * R / 2.5e15, 3),
                    "frac_of_split_bound": round(achieved / min(PEAK_PAIRS, 2.5e15 / (2.0 * R * 3)), 3),
                    "avg_kernel_ms": round(avg_mvm_ms, 4), "launches": st["n_mvm"]}
    else:
        roofline = mvm_roofline(prec, wl.d, R, n, avg_mvm_ms, st["n_mvm"], variant, sym,
                                None if traffic is None else traffic["hbm_bytes_per_launch"])
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16x3-split/f32/f64", "fp32": "f32/f64", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: n={n} d={wl.d} eps={wl.eps} beta={list(wl.betas)} k={wl.k} "
                               f"l={wl.l} r={wl.r} tol={wl.tol} rhs={R}",
                   "precision": prec, "replace_every": replace_every},
        "step_s": round(t_step, 3),
        "build_s": round(t_build, 3),
        "build_phases_ms": {k: round(v, 1) for k, v in P.timings().items()},
        "solve_s": round(t_step - t_build, 3),
        "iterations": max(its),
        "relres_true": None if adjoint else max(rel),
        "status": status,
        "n_mvm": st["n_mvm"],
        "n_mvm_fp64": st["n_mvm_fp64"],
        "t_mvm_s": round(st["t_mvm_ms"] / 1e3, 3),
        "t_mvm_fp64_s": round(st["t_mvm_fp64_ms"] / 1e3, 3),
        "t_precond_s": round(st["t_precond_ms"] / 1e3, 3),
        "kappa_est": round(st["kappa_est"], 1),
        "mvm_gpairs_s": round(achieved / 1e9, 1),
        "roofline": roofline,
    }
    if R > 1:   # per-beta summary of the block solve's columns
        by_beta = {}
        for c in range(R):
            e = by_beta.setdefault(str(betas_col[c]), {"columns": 0, "converged": 0, "iterations_max": 0,
                                                        "relres_max": 0.0})
            e["columns"] += 1
            e["converged"] += int(rel[c] <= wl.tol)
            e["iterations_max"] = max(e["iterations_max"], int(its[c]))
            e["relres_max"] = max(e["relres_max"], float(rel[c]))
        out["columns_by_beta"] = by_beta
        out["ms_per_iteration"] = round(1e3 * (t_step - t_build) / max(max(its), 1), 1)
    if pcg_drivers is not None:
        out["pcg_drivers"] = pcg_drivers
    if adjoint:
        sts = grad_out.pop("stats")
        out["gradient"] = {**{k: v for k, v in grad_out.items()},
                           "forward": {"iterations": sts[0]["iters_max"], "n_mvm": sts[0]["n_mvm"],
                                       "n_mvm_fp64": sts[0]["n_mvm_fp64"]},
                           "adjoint": {"iterations": sts[1]["iters_max"], "n_mvm": sts[1]["n_mvm"],
                                       "n_mvm_fp64": sts[1]["n_mvm_fp64"]},
                           "validation_points": int(wl.X_val.shape[0])}
    if R == 1 and not adjoint and prec != "fp64" and (a.fp64_solve or n <= 200_000):
        # the same system solved with the FP64 and the FP32 kernels (same preconditioner), after the timed region
        for p2, rep in (("fp64", 0), ("fp32", 10)):
            log(f"bench: {p2} solve on the same GPU for comparison")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a2, its2, rel2, st2, status2 = krr.pcg_solve(Xg, Yg, wl.eps, betas_col, P, tol=wl.tol,
                                                         maxit=a.maxit, replace_every=rep, prec=p2, timing=True)
            torch.cuda.synchronize()
            out[f"{p2}_solve_s"] = round(time.perf_counter() - t0, 3)
            out[f"{p2}_iterations"] = max(its2)
            out[f"{p2}_relres_true"] = max(rel2)
            k_ms = st2["t_mvm_kernel_ms"] / max(st2["n_mvm"], 1)
            out[f"mvm_gpairs_s_{p2}"] = round(float(n) * n / k_ms / 1e6, 1)
            if p2 == "fp64":
                out["alpha_rel_err_vs_fp64"] = float(torch.linalg.norm(alpha - a2) / torch.linalg.norm(a2))
        out["solve_speedup_vs_fp64"] = round(out["fp64_solve_s"] / (t_step - t_build), 2)
        out["mvm_speedup_vs_fp64"] = round(out["mvm_gpairs_s"] / out["mvm_gpairs_s_fp64"], 2)
    if not a.no_cpu:
        log("bench: CPU oracle baseline")
        rate, rows, secs, thr = oracle_baseline(wl.X, wl.eps)
        out["cpu_baseline"] = {"value": round(rate / 1e9, 4), "unit": "Gpairs/s", "cores": thr, "kind": "oracle",
                               "cpu": cpu_model(),
                               "sample": f"oracle kernel_mv_rows (FP64 NumPy) on {rows} random rows x {n} sources "
                                         f"({rows * float(n):.3g} pairs, {secs:.1f} s wall, {thr} threads)"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
