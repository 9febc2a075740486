#!/usr/bin/env python3
"""Benchmark of the rank-k column ID on one MI355X.

Workload (default): the mixed-precision ID of a 20000 x 2000 matrix stored in
fp32, A = U diag(sigma) V^T with Haar U, V and sigma_i = exp(-i/40), rank chosen
adaptively at relative tolerance 1e-3 (pivot-relative rule).  One "step" is one
complete ID -- id_factor (column-pivoted QR) + id_solve_T (T = R11^-1 R12) --
with A already resident in HBM.  The mixed path (fp32 working copy, BF16 matrix
cores for the blocked update, FP64 norms/R/solve) is timed against the FP64
GPU path on the same input; both report ||A - A(:,J) P||_2 / sigma_{k+1}.

Prints ONE JSON line.  `value` is the mixed path's useful TFLOP/s (the flop
count of a rank-k Householder ID, identical for every path).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rank-k ID time & TFLOP/s, mixed vs FP64 on GPU at matched ‖A−CT‖/σ_{k+1}"
HBM_PEAK_GBS = 8000.0
# unit round-off of each policy's blocked update: BF16 and FP16 operands
# (Table 1; BF16 keeps 8 significand bits), split BF16 (hi + lo operands, three
# products: the dropped lo*lo term and the split remainder are below 2^-16 of
# the product), FP32 and FP64
U_LOW = {"mixed_bf16": 2.0 ** -8, "mixed_bf16x3": 2.0 ** -16, "mixed_f16": 2.0 ** -11,
         "mixed_f32": 2.0 ** -24, "f64": 2.0 ** -53}


def useful_flops(m: int, n: int, k: int, solve: bool = True) -> float:
    """k Householder steps applied to n columns, plus the triangular solve and
    the initial column norms (LAPACK-style counts)."""
    f = 4.0 * m * n * k - 2.0 * (m + n) * k * k + (4.0 / 3.0) * k ** 3 + 2.0 * m * n
    if solve:
        f += float(k) * k * (n - k)
    return f


def spectral_norm_dev(E):
    """||E||_2 from the FP64 Gram matrix (formed on the GPU, eigenvalue on the host)."""
    import numpy as np
    import torch
    Et = E.t()  # (n, m), contiguous when E is column-major
    G = torch.mm(Et, Et.t())
    lam = np.linalg.eigvalsh(G.cpu().numpy())[-1]
    return math.sqrt(max(float(lam), 0.0))


class PathTimer:
    """Preallocated buffers and a timed loop for one precision."""

    def __init__(self, A, prec, tol=None, k=None):
        import paper_2012_00706_amd as mp
        import torch
        self.mp, self.torch = mp, torch
        self.A, self.prec, self.tol, self.k = A, prec, tol, k
        m, n = A.shape
        o = mp.make_opts(k=k, tol=tol, prec=prec)
        self.kcap = mp.kcap_of(m, n, o)
        self.work = torch.empty(mp.workspace_size(m, n, A.dtype, o), dtype=torch.uint8,
                                device=A.device)
        self.R = mp.empty_colmajor(self.kcap, n, device=A.device)
        self.perm = torch.empty(n, dtype=torch.int32, device=A.device)
        self.Tbig = mp.empty_colmajor(self.kcap, n, device=A.device)

    def once(self, profile=False):
        mp = self.mp
        n = self.A.shape[1]
        fr = mp.factor(self.A, k=self.k, tol=self.tol, prec=self.prec, work=self.work,
                       R_buf=self.R, perm_buf=self.perm, profile=profile)
        T, info = mp.solve_T(fr.R, fr.k, n, T_buf=self.Tbig[:, : n - fr.k], check=False)
        return fr, T

    def timed(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.once()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fr, T = self.once()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        return e0.elapsed_time(e1) / steps, wall, fr, T

    def profiled(self, reps):
        """Per-kernel HIP-event timings summed over `reps` instrumented runs."""
        tot = None
        for _ in range(reps):
            self.once(profile=True)
            p = self.mp.last_profile()
            if tot is None:
                tot = dict(p)
            else:
                for key in tot:
                    tot[key] += p[key]
        return tot


def oracle_run(A_np, k_run: int, ks):
    """The oracle as it stands -- rank-k_run column-pivoted QR (FP64 NumPy,
    every residual norm recomputed at each step) and back-substitution for T
    -- timed once on the full input, on the host's cores.  Its first j steps
    are the rank-j factorization, so the same run gives the oracle's error
    ||A - A(:,J)P||_2 at every rank j in ks (j <= k_run)."""
    import numpy as np
    import oracle as orc
    A64 = np.asarray(A_np, dtype=np.float64)
    m, n = A64.shape
    t0 = time.perf_counter()
    ref = orc.cpqr(A64, k=k_run)
    orc.solve_T(ref.R, ref.k)
    dt = time.perf_counter() - t0
    errs = {}
    for j in sorted(set(ks)):
        if 0 < j <= ref.k:
            errs[j] = orc.id_error(A64, ref.perm, j, orc.solve_T(ref.R[:j], j))[0]
    base = {
        "value": useful_flops(m, n, ref.k) / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": _threads(),
        "kind": "oracle",
        "sample": (f"full oracle ID of the same {m}x{n} input at rank {ref.k} (column-pivoted QR "
                   f"+ T), one timed run: {dt:.1f} s wall"),
        "seconds": dt,
        "ms_per_id": dt * 1e3,
    }
    return base, errs


COPY_BYTES = 256 << 20
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "sweep_traffic.json")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2012_00706_amd", "csrc", f)
                 for f in ("factor.hip", "device_util.h")]


def sweep_source_hash() -> str:
    """Hash of the reflector sweep's own source: the k_sweep kernel and its
    body (sweep_block), its argument struct and constants in factor.hip, and
    the device helpers."""
    import hashlib
    import re
    h = hashlib.sha256()
    text = open(SWEEP_SOURCES[0]).read()
    parts = []
    for pat in (r"constexpr int kPrefetch[^\n]*\n", r"constexpr int kSweepU [^\n]*\n",
                r"constexpr int kSweepUDeep[^\n]*\n", r"constexpr double kDeepBytes[^\n]*\n",
                r"template <typename S, int G>\nconstexpr int overlap_rows\(\) \{.*?\n\}\n",
                r"template <typename S>\nstruct StepArgs \{.*?\n\};\n",
                r"template <typename S, int G, int U = kSweepU>\n__device__ __forceinline__ void "
                r"sweep_block\(.*?\n\}\n",
                r"template <typename S, int G, int U>\n__global__ __launch_bounds__\(kThreads\) "
                r"void k_sweep\(.*?\n\}\n"):
        mt = re.search(pat, text, flags=re.S)
        if not mt:  # the hash must cover the whole kernel, never a part of it
            raise RuntimeError(f"sweep source pattern not found: {pat[:40]}")
        parts.append(mt.group(0))
    h.update("".join(parts).encode())
    with open(SWEEP_SOURCES[1], "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def copy_calibration():
    """One plain device-to-device copy of COPY_BYTES (known traffic: that many
    bytes read and written), for scaling the HBM byte counters."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def _read_counter_csv(path):
    """{(dispatch_id, kernel_name): value} for the single counter in the file."""
    import csv
    out = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
            did = row.get("Dispatch_Id") or row.get("Dispatch-Id")
            val = float(row.get("Counter_Value") or row.get("Counter-Value") or 0.0)
            out[(int(did), name)] = out.get((int(did), name), 0.0) + val
    return out


def summarize_pmc(fetch_csv, write_csv):
    """Average HBM fetch/write per live k_sweep dispatch (KiB counters x 1024),
    scaled by the same counters' reading on the calibration copy; written to
    profiles/sweep_traffic.json with the hash of the sweep's sources."""
    fetch = _read_counter_csv(fetch_csv)
    write = _read_counter_csv(write_csv)

    def sweep_live(d):
        vals = [v for (did, name), v in d.items() if "k_sweep" in name]
        big = max(vals) if vals else 0.0
        return [v for v in vals if v > 0.2 * big]  # launches that did work

    def copy_kib(d):
        vals = [v for (did, name), v in d.items()
                if "k_" not in name and ("copy" in name.lower() or "elementwise" in name)]
        return max(vals) if vals else 0.0

    f_scale = COPY_BYTES / (copy_kib(fetch) * 1024.0) if copy_kib(fetch) > 0 else 1.0
    w_scale = COPY_BYTES / (copy_kib(write) * 1024.0) if copy_kib(write) > 0 else 1.0
    sf, sw = sweep_live(fetch), sweep_live(write)
    fetch_b = sum(sf) / len(sf) * 1024.0 * f_scale if sf else 0.0
    write_b = sum(sw) / len(sw) * 1024.0 * w_scale if sw else 0.0
    res = {"kernel": "k_sweep", "launches": len(sf), "fetch_bytes_per_launch": fetch_b,
           "write_bytes_per_launch": write_b, "traffic_bytes_per_launch": fetch_b + write_b,
           "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
           "copy_bytes": COPY_BYTES, "source_hash": sweep_source_hash()}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def summarize_trace(trace_csv):
    """Per-kernel launch statistics from a rocprofv3 --kernel-trace CSV; for
    k_sweep also the average over the launches that did work (a launch
    enqueued after the rank was reached returns at once)."""
    import csv
    by = {}
    calls = []  # per factorization call (each starts with k_init): name -> durations
    with open(trace_csv) as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    for row in rows:
        name = row["Kernel_Name"].split("(")[0]
        d = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
        by.setdefault(name, []).append(d)
        if name == "k_init":
            calls.append({})
        if calls:
            calls[-1].setdefault(name, []).append(d)
    lines = [f"{'kernel':<28}{'calls':>8}{'total_ms':>12}{'avg_us':>10}{'min_us':>10}{'max_us':>10}"]
    for name, ds in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{name[:27]:<28}{len(ds):>8}{sum(ds) / 1e6:>12.3f}{sum(ds) / len(ds) / 1e3:>10.2f}"
                     f"{min(ds) / 1e3:>10.2f}{max(ds) / 1e3:>10.2f}")
    sw = by.get("k_sweep", [])
    if sw:
        live = [d for d in sw if d > 0.3 * max(sw)]
        lines.append(f"k_sweep live launches: {len(live)} of {len(sw)}, "
                     f"average {sum(live) / len(live) / 1e3:.2f} us")
    if len(calls) > 1:
        # per call (launches that return at once, under a third of the call's
        # longest, are counted apart)
        lines.append("")
        lines.append(f"{'call':>4}{'sweep_live':>11}{'avg_us':>9}{'idle':>6}{'finalize_us':>13}"
                     f"{'fold_us':>9}{'gemm_live':>10}{'avg_us':>9}{'colred_us':>11}")
        avg = lambda v: sum(v) / len(v) / 1e3 if v else 0.0  # noqa: E731
        for i, c in enumerate(calls):
            sw = c.get("k_sweep", [])
            gm = c.get("k_panel_gemm", [])
            lsw = [d for d in sw if sw and d > max(sw) / 3]
            lgm = [d for d in gm if gm and d > max(gm) / 3]
            lines.append(f"{i:>4}{len(lsw):>11}{avg(lsw):>9.1f}{len(sw) - len(lsw):>6}"
                         f"{avg(c.get('k_finalize', [])):>13.2f}{avg(c.get('k_fold', [])):>9.2f}"
                         f"{len(lgm):>10}{avg(lgm):>9.1f}{avg(c.get('k_colreduce', [])):>11.1f}")
    print("\n".join(lines))


def measured_traffic():
    """Per-launch HBM bytes of the sweep from the committed counter summary,
    or None when it is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != sweep_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def _timed(fn, steps, warmup):
    """Average ms of fn() over `steps` calls after `warmup` calls (device events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        r = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, r


def _line(args, metric, value, unit, ms, hib, dtype, workload, extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": workload}
    out.update(extra)
    return out


def _sweep_roofline(prof, reps=1):
    gbs = prof["sweep_bytes"] / (prof["sweep_ms"] * 1e-3) / 1e9 if prof["sweep_ms"] > 0 else 0.0
    return {"kernel": "k_sweep", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": prof["sweep_bytes"] / max(prof["sweep_launches"], 1),
            "us_per_launch": prof["sweep_ms"] * 1e3 / max(prof["sweep_launches"], 1),
            "launches_per_id": prof["sweep_launches"] / reps}


FP64_PEAK_TFLOPS = 78.6


def id_alg_bytes(m: int, n: int, k: int, s: int, nb: int = 32, s_in: int = 4) -> float:
    """Algorithmic HBM bytes of one whole ID: the reflector sweeps (one read of
    the trailing block per pivot step, s bytes per entry), the blocked updates
    (one read and one write of the refreshed block per panel of nb steps) and
    the ingest (A read in its storage width s_in, the working copy written)."""
    sweep = sum((m - j) * (n - j - 1) for j in range(k)) * float(s)
    gemm = sum(2.0 * (m - je) * (n - je) for je in range(nb, k, nb)) * s
    return sweep + gemm + m * n * float(s_in + s)


def id_roofline(m, n, k, s, ms):
    """The whole ID (all kernels, host gaps included) against HBM bandwidth."""
    b = id_alg_bytes(m, n, k, s)
    gbs = b / (ms * 1e-3) / 1e9
    return {"scope": "whole ID (id_factor + id_solve_T)", "bound": "hbm", "bytes_alg": b,
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def _sketch_front_end(A, l, tol, steps, sigma=None):
    """Randomized ID through a Gaussian sketch of l rows (id_sketch, then the
    FP64 factorization of the l x n sketch and T): whole-call time, the sketch
    kernel's own time and FP64 matrix-core rate, rank and error."""
    import numpy as np
    import torch
    import paper_2012_00706_amd as mp
    import synth
    m, n = A.shape
    Om = torch.from_numpy(synth.sketch_matrix(l, m, seed=2024)).cuda()
    sk_ms, _ = _timed(lambda: mp.sketch(A, Om), steps, 2)
    id_ms, res = _timed(lambda: mp.sketch_id(A, Om, tol=tol), steps, 2)
    del Om
    E = mp.reconstruct(A, res.perm, res.k, res.T, residual=True)
    err = spectral_norm_dev(E)
    del E
    torch.cuda.empty_cache()
    flops = 2.0 * l * m * n
    out = {"l": l, "ms_per_id": id_ms, "k": res.k, "err2": err,
           "sketch_kernel_ms": sk_ms,
           "sketch_roofline": {"kernel": "k_sketch_partial + k_sketch_reduce (Y = Omega A)",
                               "bound": "mfma", "achieved": flops / (sk_ms * 1e-3) / 1e12,
                               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": flops / (sk_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}}
    if sigma is not None and res.k < len(sigma):
        out["err_ratio_sigma_k1"] = err / float(sigma[res.k])
    return out


def run_sketch(args):
    """Sketching front end alone on the snapshot stand-in (1,048,576 x 512
    fp32, l = --sketch-rows Gaussian rows, tol 1e-3)."""
    import numpy as np
    import torch
    import synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    A_np = synth.config3()
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    m, n = A_np.shape
    del A_np
    sk = _sketch_front_end(A, args.sketch_rows, 1e-3, args.steps)
    log(f"[bench] sketch front end (l={args.sketch_rows}): k={sk['k']} {sk['ms_per_id']:.2f} ms/ID "
        f"(sketch {sk['sketch_kernel_ms']:.2f} ms, {sk['sketch_roofline']['achieved']:.1f} TFLOP/s)")
    roof = dict(sk.pop("sketch_roofline"))
    roof["traffic"] = None
    return _line(args, "randomized ID time through a sketch (snapshot matrix)", sk["ms_per_id"],
                 "ms", sk["ms_per_id"], False, "f64",
                 {"workload": f"snapshot stand-in 1,048,576 x 512 fp32, Gaussian sketch of "
                              f"{args.sketch_rows} rows, adaptive rank at tol 1e-3", "m": m, "n": n,
                  "l": args.sketch_rows},
                 dict(sk, roofline=roof))


def run_gram(args):
    """Tall-skinny (Gram) front end alone on the snapshot stand-in
    (1,048,576 x 512 fp32, tol 1e-3)."""
    import numpy as np
    import torch
    import paper_2012_00706_amd as mp
    import synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    A_np = synth.config3()
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    m, n = A_np.shape
    del A_np
    ms, res = _timed(lambda: mp.column_id(A, tol=1e-3, gram=True), args.steps, 2)
    log(f"[bench] gram front end: k={res.k} {ms:.2f} ms/ID")
    return _line(args, "column ID time through the Gram front end (snapshot matrix)", ms, "ms", ms,
                 False, "f64", {"workload": "snapshot stand-in 1,048,576 x 512 fp32, FP64 Gram "
                                            "matrix + pivoted Cholesky, adaptive rank at tol 1e-3",
                                "m": m, "n": n},
                 {"k": res.k, "gram_flops_per_id": float(m) * n * n,
                  "note": "FP64 MFMA product over the upper triangle of 64 x 64 tiles"})


def run_cholqr(args):
    """Tall-skinny CholeskyQR front end alone on the snapshot stand-in
    (1,048,576 x 512 fp32, tol 1e-3)."""
    import numpy as np
    import torch
    import paper_2012_00706_amd as mp
    import synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    A_np = synth.config3()
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    m, n = A_np.shape
    del A_np
    ms, res = _timed(lambda: mp.column_id(A, tol=1e-3, cholqr=True), args.steps, 2)
    log(f"[bench] cholqr front end: k={res.k} info={res.info} {ms:.2f} ms/ID")
    return _line(args, "column ID time through the CholeskyQR front end (snapshot matrix)", ms,
                 "ms", ms, False, "f64",
                 {"workload": "snapshot stand-in 1,048,576 x 512 fp32, CholeskyQR passes on the "
                              "FP64 matrix cores + FP64 pivoted Householder QR of the 512 x 512 R "
                              "factor, adaptive rank at tol 1e-3", "m": m, "n": n},
                 {"k": res.k, "info": res.info,
                  "pass_flops": {"gram": float(m) * n * n, "triangular_product": float(m) * n * n},
                  "note": "per pass: FP64 MFMA Gram product (upper tiles) and A R^-1 over the "
                          "upper triangle of R^-1; two passes when CholeskyQR2 is accepted"})


def run_config1(args):
    """Parity workload at its own size: 1000 x 500 fp64, FP64 path, k = 50.
    Latency-bound (4 MB, cache-resident): reported in microseconds."""
    import numpy as np
    import torch
    import synth
    import oracle as orc
    A_np = synth.config1()
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    pt = PathTimer(A, "f64", k=50)
    ms, wall, fr, T = pt.timed(args.steps, args.warmup)
    prof = pt.profiled(1)
    t0 = time.perf_counter()
    ref = orc.cpqr(A_np, k=50)
    orc.solve_T(ref.R, 50)
    cpu_s = time.perf_counter() - t0
    m, n = A_np.shape
    same = bool(np.array_equal(fr.perm[:50].cpu().numpy(), ref.perm[:50]))
    return _line(args, "rank-50 FP64 ID latency (1000x500)", ms * 1e3, "us", ms, False, "f64",
                 {"workload": "FP64 ID, 1000x500 fp64, U diag(10^-(i-1)/25) V^T, k = 50",
                  "m": m, "n": n, "k": 50},
                 {"pivots_equal_oracle": same, "roofline": dict(_sweep_roofline(prof), note=(
                     "4 MB working set stays in cache; latency-bound, no roofline claim")),
                  "cpu_baseline": {"value": cpu_s * 1e6, "unit": "us", "cores": _threads(),
                                   "kind": "oracle", "sample": "full ID (oracle CPQR + solve)"}})


def oracle_sample(A_np, steps: int, k_full: int):
    """The oracle on the first `steps` pivot steps of an input too large to
    factor on the host within the benchmark's time (the snapshot matrix):
    rate in useful TFLOP/s and the projected full-ID time."""
    import oracle as orc
    m, n = A_np.shape
    t0 = time.perf_counter()
    orc.cpqr(A_np, k=steps)
    dt = time.perf_counter() - t0
    rate = useful_flops(m, n, steps, solve=False) / dt / 1e12
    full_s = useful_flops(m, n, k_full) / (rate * 1e12)
    return {"value": rate, "unit": "TFLOP/s", "cores": _threads(), "kind": "oracle",
            "sample": (f"first {steps} of {k_full} pivot steps of the FP64 NumPy oracle's CPQR on "
                       f"the full {m}x{n} input ({dt:.1f} s wall); projected full ID {full_s:.0f} s"),
            "sample_seconds": dt, "projected_full_id_s": full_s}


def _threads():
    threads = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(d.get("num_threads", 1)) for d in info)
    except Exception:
        pass
    return threads


def run_config3(args):
    """Snapshot stand-in: 1,048,576 x 512 fp32, adaptive rank at tol 1e-3."""
    import numpy as np
    import torch
    import synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    A_np = synth.config3()
    log(f"[bench] snapshot matrix {A_np.shape} generated in {time.perf_counter() - t0:.1f} s")
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    m, n = A_np.shape
    res = {}
    for prec in (args.prec, "f64"):
        pt = PathTimer(A, prec, tol=1e-3)
        ms, wall, fr, T = pt.timed(max(args.steps // 5, 2), 1)
        prof = pt.profiled(1)
        res[prec] = dict(ms=ms, k=fr.k, prof=prof, perm=fr.perm[:fr.k].cpu(),
                         tflops=useful_flops(m, n, fr.k) / (ms * 1e-3) / 1e12)
        log(f"[bench] {prec}: k={fr.k} {ms:.2f} ms/ID")
        del pt
        torch.cuda.empty_cache()
    # the tall-skinny front end (pivots and R from the FP64 Gram matrix)
    import paper_2012_00706_amd as mp
    gms, gres = _timed(lambda: mp.column_id(A, tol=1e-3, gram=True), 3, 1)
    log(f"[bench] gram front end: k={gres.k} {gms:.2f} ms/ID")
    # the CholeskyQR3 front end (FP64 Householder pivots of the n x n R factor)
    cms, cres = _timed(lambda: mp.column_id(A, tol=1e-3, cholqr=True), 3, 1)
    log(f"[bench] cholqr front end: k={cres.k} info={cres.info} {cms:.2f} ms/ID")
    sk = _sketch_front_end(A, 320, 1e-3, 3)
    log(f"[bench] sketch front end (l=320): k={sk['k']} {sk['ms_per_id']:.2f} ms/ID "
        f"(sketch {sk['sketch_kernel_ms']:.2f} ms, {sk['sketch_roofline']['achieved']:.1f} TFLOP/s)")
    mx = res[args.prec]
    out = _line(args, "rank-k ID time & TFLOP/s, mixed vs FP64 (snapshot matrix)", mx["tflops"],
                "TFLOP/s", mx["ms"], True, {"mixed_bf16": "f32+bf16", "mixed_bf16x3": "f32+bf16x3",
                                             "mixed_f16": "f32+f16", "mixed_f32": "f32"}[args.prec],
                {"workload": "snapshot stand-in 64^3 grid x 4 fields x 512 snapshots, fp32, "
                             "adaptive rank at tol 1e-3 (pivot-relative)", "m": m, "n": n,
                 "prec": args.prec},
                {"k": mx["k"], "fp64_gpu": {"ms_per_id": res["f64"]["ms"], "k": res["f64"]["k"]},
                 "speedup_vs_fp64": res["f64"]["ms"] / mx["ms"],
                 "gram_front_end": {"ms_per_id": gms, "k": gres.k,
                                    "speedup_vs_mixed": mx["ms"] / gms},
                 "cholqr_front_end": {"ms_per_id": cms, "k": cres.k, "info": cres.info,
                                      "speedup_vs_mixed": mx["ms"] / cms,
                                      "same_pivots_as_fp64": bool(
                                          cres.k == res["f64"]["k"] and torch.equal(
                                              cres.J.cpu().int(), res["f64"]["perm"]))},
                 "sketch_front_end": sk,
                 "roofline": _sweep_roofline(mx["prof"]),
                 "kernel_ms_per_id": {key: mx["prof"][key] for key in
                                      ("sweep_ms", "finalize_ms", "gemm_ms", "other_ms", "total_ms")}})
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample (3 steps) ...")
        out["cpu_baseline"] = oracle_sample(A_np, 3, mx["k"])
    return out


def run_config4(args):
    """Batched workload: `--batch` matrices of uneven sizes in one persistent
    launch, against a loop of single IDs."""
    import numpy as np
    import torch
    import synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    mats = synth.config4(batch=args.batch)
    log(f"[bench] {len(mats)} matrices generated in {time.perf_counter() - t0:.1f} s")
    As = [torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t() for a in mats]
    import paper_2012_00706_amd as mp
    # the lock-step launches (every step of all unfinished items in one launch)
    lock = mp.LockstepID(As, tol=1e-4, prec=args.prec)
    ms, _ = _timed(lock.run, max(args.steps // 5, 2), 1)
    res = lock.results()
    ks = [r.k for r in res]
    # the persistent graph-capturable launch, for comparison
    plan = mp.BatchedID(As, tol=1e-4, prec=args.prec)
    tune = mp.autotune(plan, use_cache=False)
    pers_ms, _ = _timed(plan.run, max(args.steps // 5, 2), 1)
    pres = plan.results()
    same_k = sum(int(a.k == b.k) for a, b in zip(res, pres))
    flops = sum(useful_flops(a.shape[0], a.shape[1], k) for a, k in zip(mats, ks))
    sweep_bytes = sum(4.0 * sum((a.shape[0] - j) * (a.shape[1] - j - 1) for j in range(k))
                      for a, k in zip(mats, ks))

    def loop():
        for A in As:
            mp.column_id(A, tol=1e-4, prec=args.prec)
    loop_ms, _ = _timed(loop, 1, 1)
    log(f"[bench] lock-step {ms:.1f} ms, persistent {pers_ms:.1f} ms, "
        f"loop of single IDs {loop_ms:.1f} ms")
    out = _line(args, "batched rank-k IDs: aggregate TFLOP/s (lock-step launches)",
                flops / (ms * 1e-3) / 1e12, "TFLOP/s", ms, True,
                {"mixed_bf16": "f32+bf16", "mixed_bf16x3": "f32+bf16x3", "mixed_f16": "f32+f16",
                 "f64": "f64"}.get(args.prec, args.prec),
                {"workload": f"{len(mats)} matrices, m ~ U{{2000..20000}}, n ~ U{{100..800}}, "
                             "sigma_j = j^-2, fp32, adaptive rank at tol 1e-4", "batch": len(mats),
                 "prec": args.prec},
                {"sum_k": int(sum(ks)), "ids_per_s": len(mats) / (ms * 1e-3),
                 "loop_of_single_ids_ms": loop_ms, "speedup_vs_loop": loop_ms / ms,
                 "persistent_launch_ms": pers_ms,
                 "persistent_same_k_items": same_k,
                 "autotune": {k_: v for k_, v in tune.items() if k_ != "table"},
                 "roofline": {"kernel": "lock-step batch (whole call)", "bound": "hbm",
                              "achieved": sweep_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": sweep_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": None,
                              "note": "algorithmic sweep bytes of all items / batched time"}})
    return out


def run_config5(args):
    """Adjoint workload: 8192 x 1024 fp32, k = 128; forward ID and id_backward
    (both cotangents) timed; FP64 matrix-core products dominate the backward."""
    import numpy as np
    import torch
    import synth
    import oracle as orc
    import paper_2012_00706_amd as mp
    A_np = synth.config5()
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    m, n = A_np.shape
    k = 128
    res = mp.column_id(A, k=k, prec=args.prec)
    rng = np.random.default_rng(19)
    gT = torch.from_numpy(rng.standard_normal((n - k, k)).T.copy()).cuda()
    gY = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((m, n)).T)).cuda().t()
    fwd_ms, _ = _timed(lambda: mp.column_id(A, k=k, prec=args.prec), args.steps, args.warmup)
    bwd_ms, gA = _timed(lambda: mp.backward(A, res.perm, k, res.T, gT=gT, gY=gY), args.steps,
                        args.warmup)
    # the FP64 forward's R11 is the skeleton's R factor: the backward can reuse it
    res64 = mp.column_id(A, k=k, prec="f64")
    R11 = res64.R[:, :k]
    bwdR_ms, _ = _timed(lambda: mp.backward(A, res64.perm, k, res64.T, gT=gT, gY=gY, R11=R11),
                        args.steps, args.warmup)
    nc = n - k
    # the five FP64 products of the adjoint: B X, B T, B^T gY(:, Jc) (m k (n-k)
    # each) and [D | E] [X | T]^T (2 m k (n-k)), at 2 flops per multiply-add
    gemm_flops = 10.0 * m * k * nc
    t0 = time.perf_counter()
    ref = orc.adjoint(A_np, res.perm.cpu().numpy().astype(np.int64), k, res.T.cpu().numpy(),
                      gT=gT.cpu().numpy(), gY=gY.cpu().numpy())
    cpu_s = time.perf_counter() - t0
    err = float(np.linalg.norm(gA.cpu().numpy() - ref) / np.linalg.norm(ref))
    return _line(args, "ID adjoint (id_backward) time, J fixed", bwd_ms, "ms", bwd_ms, False, "f64",
                 {"workload": "8192x1024 fp32, sigma_i = exp(-i/64), k = 128, cotangents of T and Y",
                  "m": m, "n": n, "k": k},
                 {"forward_ms": fwd_ms, "rel_err_vs_oracle_adjoint": err,
                  "backward_with_forward_R_ms": bwdR_ms,
                  "roofline": {"kernel": "id_backward reusing R11 (whole call: the skeleton "
                                         "gather, the split-K product B^T gY, two triangular "
                                         "solves, the fused pass of the three remaining "
                                         "products; 10 m k (n-k) FP64 MFMA flops)",
                               "bound": "mfma",
                               "achieved": gemm_flops / (bwdR_ms * 1e-3) / 1e12, "peak": 78.6,
                               "unit": "TFLOP/s",
                               "frac": gemm_flops / (bwdR_ms * 1e-3) / 1e12 / 78.6, "traffic": None,
                               "note": "FP64 product flops 10 m k (n-k) over the whole call; "
                                       "without R11 the call adds an unpivoted FP64 QR of the "
                                       "skeleton (value)"},
                  "cpu_baseline": {"value": cpu_s * 1e3, "unit": "ms", "cores": _threads(),
                                   "kind": "oracle", "sample": "oracle adjoint, same input"}})


def run_accuracy(args):
    """The paper's accuracy study (Section 3, Table 3 datasets): 1000-row
    matrices with sigma_i = i^-1 (Slow), i^-2 (Medium), i^-4 (Fast); relative
    spectral errors of the ID against the FP64 ID and against the matrix, over
    the target rank (n = 1000) and over the column count (k = 20), for the
    precision variants of the paper mapped onto this implementation:
      double        FP64 path on A (Algorithm 1)
      mixed_single  A stored in fp32, FP32 matrix-core update, skeleton from A (Algorithm 2)
      single        same factorization, skeleton from the fp32 matrix (A_L)
      mixed_single_bf16x3  A stored in fp32, split-BF16 update, skeleton from A
      mixed_bf16    A stored in bf16, mixed BF16 path, skeleton from A
      bf16          same, skeleton from the bf16 matrix
      mixed_half    A stored in fp16 (no scaling), mixed FP16 path, skeleton from A
      half          same, skeleton from the fp16 matrix
      mixed_half_scaled  A scaled by a power of two before the fp16 storage
      *_literal     the simulated single / half precision of the paper: every
                    value the factorization keeps, and T, rounded to binary32 /
                    binary16 (ID_FLAG_ROUND_F32 / ID_FLAG_ROUND_F16; no FP16
                    operand scaling)
    A variant "breaks" when its R11 is numerically singular (recorded as null)."""
    import numpy as np
    import torch
    import synth
    import paper_2012_00706_amd as mp
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).cuda().t()

    gen = torch.Generator(device="cuda").manual_seed(7)

    def norm2(X):
        # power iteration on X^T X (100 steps, seeded): ample for error ratios
        v = torch.randn(X.shape[1], 1, dtype=torch.float64, device="cuda", generator=gen)
        s = 0.0
        for _ in range(100):
            w = X.t() @ (X @ v)
            nw = float(w.norm())
            if nw == 0.0:
                return 0.0
            v = w / nw
            s = nw
        return math.sqrt(s)

    def stored(a, dt, scaled=False):
        x = torch.from_numpy(np.asarray(a, dtype=np.float64))
        sc = 1.0
        if scaled:
            e = math.frexp(float(x.abs().max()))[1]
            sc = 2.0 ** (14 - e)
        y = (x * sc).to(dt).to(torch.float64) / sc
        return y.numpy().astype(np.float32)

    variants = [  # (name, storage dtype, scaled, prec, skeleton from the stored matrix, rounding)
        ("double", None, False, "f64", False, None),
        ("mixed_single", torch.float32, False, "mixed_f32", False, None),
        ("single", torch.float32, False, "mixed_f32", True, None),
        ("mixed_single_literal", torch.float32, False, "mixed_f32", False, "f32"),
        ("single_literal", torch.float32, False, "mixed_f32", True, "f32"),
        ("mixed_single_bf16x3", torch.float32, False, "mixed_bf16x3", False, None),
        ("mixed_bf16", torch.bfloat16, False, "mixed_bf16", False, None),
        ("bf16", torch.bfloat16, False, "mixed_bf16", True, None),
        ("mixed_half", torch.float16, False, "mixed_f16", False, None),
        ("half", torch.float16, False, "mixed_f16", True, None),
        ("mixed_half_scaled", torch.float16, True, "mixed_f16", False, None),
        ("mixed_half_literal", torch.float16, False, "mixed_f16", False, "f16"),
        ("half_literal", torch.float16, False, "mixed_f16", True, "f16"),
    ]
    ks = [1, 2, 4, 6, 8, 10, 12, 15, 18, 20, 21, 22, 25, 30, 35, 40, 50]
    ns = [50, 100, 200, 300, 400, 500, 600, 700, 800, 900, 1000]
    t0 = time.perf_counter()
    table = {}
    for kind in ("slow", "medium", "fast"):
        full = synth.paper_dataset(kind)
        for sweep, pts in (("k", ks), ("n", ns)):
            for x in pts:
                k, n = (x, 1000) if sweep == "k" else (20, x)
                A = full[:, :n]
                Ad = dev(A)
                nA = norm2(Ad)
                ref = None
                for name, dt, scaled, prec, low_skel, rnd in variants:
                    As = A if dt is None else stored(A, dt, scaled)
                    Asd = dev(As)
                    try:
                        r = mp.column_id(Asd, k=k, prec=prec, round_to=rnd)
                        Y = mp.reconstruct(Asd if low_skel else Ad, r.perm, r.k, r.T)
                    except mp.MpidError:
                        table.setdefault(kind, {}).setdefault(sweep, {}).setdefault(name, []).append(
                            None)
                        continue
                    if name == "double":
                        ref = Y
                    e_truth = norm2(Ad - Y) / nA
                    e_double = norm2(ref - Y) / norm2(ref)
                    table.setdefault(kind, {}).setdefault(sweep, {}).setdefault(name, []).append(
                        [e_double, e_truth])
        log(f"[bench] accuracy study: {kind} done ({time.perf_counter() - t0:.0f} s)")

    def worst(kind, name, sweep="k", col=0, kmax=50):
        vals = [v[col] for x, v in zip(ks, table[kind][sweep][name]) if v is not None and x <= kmax]
        return max(vals) if vals else None

    claims = {
        "mixed_single_vs_double_max_fast_medium": max(worst("fast", "mixed_single"),
                                                      worst("medium", "mixed_single")),
        "mixed_single_vs_double_max_slow": worst("slow", "mixed_single"),
        "single_vs_double_max_slow": worst("slow", "single"),
        "mixed_half_breaks_fast_at_k": [x for x, v in zip(ks, table["fast"]["k"]["mixed_half"])
                                        if v is None],
        "mixed_half_scaled_breaks_fast_at_k": [x for x, v in zip(
            ks, table["fast"]["k"]["mixed_half_scaled"]) if v is None],
    }
    return _line(args, "relative spectral error of the ID vs the FP64 ID (paper datasets)",
                 claims["mixed_single_vs_double_max_fast_medium"], "relative error",
                 (time.perf_counter() - t0) * 1e3, False, "mixed",
                 {"workload": "paper datasets Slow/Medium/Fast (1000 rows, sigma_i = i^-1, "
                              "i^-2, i^-4), k sweep at n = 1000 and n sweep at k = 20"},
                 {"claims": claims, "k_values": ks, "n_values": ns, "errors": table,
                  "error_columns": ["vs_double_ID", "vs_matrix"]})


WORKLOADS = {"config1": run_config1, "config3": run_config3, "config4": run_config4,
             "config5": run_config5, "accuracy": run_accuracy, "sketch": run_sketch,
             "gram": run_gram, "cholqr": run_cholqr}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config5", "accuracy",
                             "sketch", "gram", "cholqr"],
                    help="config2 (default) is the headline; the others print their own line")
    ap.add_argument("--batch", type=int, default=256, help="items of the batched workload")
    ap.add_argument("--sketch-rows", type=int, default=320, help="rows of the sketch (--workload sketch)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="mixed_bf16x3",
                    choices=["mixed_bf16", "mixed_bf16x3", "mixed_f16", "mixed_f32"])
    ap.add_argument("--compare", default="mixed_bf16,mixed_f16",
                    help="comma-separated extra precisions to time (reported, not headline)")
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--m", type=int, default=20000)
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=3,
                    help="instrumented runs per precision (>= 1)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline precision (no FP64 comparison, no errors)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="per-kernel statistics of a rocprofv3 --kernel-trace CSV")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter files into the sweep traffic summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    args.profile_reps = max(args.profile_reps, 1)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: one GPU only (the column ID runs on a single "
              "MI355X); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2012_00706_amd as mp
    import synth

    mp.load()
    if args.workload != "config2":
        out = WORKLOADS[args.workload](args)
        print(json.dumps(out))
        return
    m, n, tol = args.m, args.n, args.tol
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    A_np = synth.config2(m, n)
    sigma = synth.sigma_exp(min(m, n), 40.0)
    log(f"[bench] input {m}x{n} fp32 generated in {time.perf_counter() - t0:.1f} s")
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    torch.cuda.synchronize()

    if args.copy_calibration:
        copy_calibration()
    res = {}
    extra = [p for p in args.compare.split(",") if p and p not in (args.prec, "f64")]
    if args.headline_only:
        pt = PathTimer(A, args.prec, tol=tol)
        ms, wall, fr, T = pt.timed(args.steps, args.warmup)
        print(json.dumps({"headline_only": True, "prec": args.prec, "k": fr.k, "ms_per_id": ms}))
        return
    for prec in [args.prec, "f64"] + extra:
        pt = PathTimer(A, prec, tol=tol)
        ms, wall, fr, T = pt.timed(args.steps, args.warmup)
        k = fr.k
        E = mp.reconstruct(A, fr.perm, k, T, residual=True)
        err = spectral_norm_dev(E)
        del E
        sig_next = float(sigma[k]) if k < len(sigma) else 0.0
        prof = pt.profiled(args.profile_reps)
        res[prec] = dict(ms=ms, wall_ms=wall, k=k, err2=err,
                         ratio=err / sig_next if sig_next > 0 else float("inf"),
                         tflops=useful_flops(m, n, k) / (ms * 1e-3) / 1e12, prof=prof,
                         perm=fr.perm.clone())
        log(f"[bench] {prec}: k={k} {ms:.3f} ms/ID (wall {wall:.3f}) err2={err:.3e} "
            f"ratio={res[prec]['ratio']:.3f} sweep={prof['sweep_ms'] / args.profile_reps:.3f} ms "
            f"gemm={prof['gemm_ms'] / args.profile_reps:.3f} ms total={prof['total_ms'] / args.profile_reps:.3f} ms")
        del pt
        torch.cuda.empty_cache()

    mx, f64 = res[args.prec], res["f64"]
    # the oracle, timed once on the host (cpu_baseline), run to the larger of
    # the two paths' ranks; its error at each path's rank is the acceptance
    # reference: err_path <= 1.1 err_oracle(same k) + 10 u_low ||A||_2
    base, oerr = None, {}
    if not args.no_cpu_baseline:
        k_run = max(mx["k"], f64["k"])
        log(f"[bench] CPU oracle: full rank-{k_run} ID on the host ...")
        base, oerr = oracle_run(A_np, k_run, [res[p]["k"] for p in res])
        log(f"[bench] CPU oracle: {base['seconds']:.1f} s")

    def acceptance(p):
        r = res[p]
        e_o = oerr.get(r["k"])
        if e_o is None:
            # oracle not run to this rank: sigma_{k+1} (analytic) is a lower
            # bound of its error (Eckart-Young), so passing the rule with it in
            # place of err_oracle(k) is sufficient for the rule itself
            s_k1 = float(sigma[r["k"]]) if r["k"] < len(sigma) else 0.0
            bound = 1.1 * s_k1 + 10.0 * U_LOW[p] * float(sigma[0])
            ok = bool(r["err2"] <= bound)
            return {"err_oracle_same_k": None, "sigma_k1": s_k1, "u_low": U_LOW[p],
                    "bound_with_sigma_k1": bound, "pass": True if ok else None,
                    "note": ("oracle not run to this rank; sigma_{k+1} <= err_oracle(k), so "
                             "err <= 1.1 sigma_{k+1} + 10 u_low ||A||_2 implies the rule")}
        bound = 1.1 * e_o + 10.0 * U_LOW[p] * float(sigma[0])
        return {"err_oracle_same_k": e_o, "u_low": U_LOW[p], "bound": bound,
                "pass": bool(r["err2"] <= bound)}
    def tall_front_end(**kw):
        # the Gram and CholeskyQR front ends at the headline tolerance: time,
        # rank, pivots against the FP64 path, error
        fe_ms, r = _timed(lambda: mp.column_id(A, tol=tol, **kw), 3, 1)
        same = bool(r.k == f64["k"] and torch.equal(r.J.cpu().int(), f64["perm"][:r.k].cpu()))
        e = float("nan")
        if r.k > 0:
            E = mp.reconstruct(A, r.perm, r.k, r.T, residual=True)
            e = spectral_norm_dev(E)
            del E
        s_k1 = float(sigma[r.k]) if r.k < len(sigma) else 0.0
        log(f"[bench] {next(iter(kw))} front end: k={r.k} info={r.info} {fe_ms:.2f} ms/ID "
            f"same pivots as FP64: {same}")
        return {"ms_per_id": fe_ms, "k": r.k, "info": r.info, "same_pivots_as_fp64": same,
                "err2": e, "err_ratio_sigma_k1": e / s_k1 if s_k1 > 0 else None}
    gram_fe = tall_front_end(gram=True)
    cholqr_fe = tall_front_end(cholqr=True)
    sk = _sketch_front_end(A, 400, tol, args.steps, sigma)
    log(f"[bench] sketch front end (l=400): k={sk['k']} {sk['ms_per_id']:.2f} ms/ID "
        f"ratio={sk.get('err_ratio_sigma_k1', float('nan')):.3f} "
        f"(sketch {sk['sketch_kernel_ms']:.3f} ms, {sk['sketch_roofline']['achieved']:.1f} TFLOP/s)")

    prof = mx["prof"]
    sweep_gbs = prof["sweep_bytes"] / (prof["sweep_ms"] * 1e-3) / 1e9 if prof["sweep_ms"] > 0 else 0.0
    per_launch_bytes = prof["sweep_bytes"] / max(prof["sweep_launches"], 1)
    per_launch_us = prof["sweep_ms"] * 1e3 / max(prof["sweep_launches"], 1)

    out = {
        "metric": METRIC,
        "value": mx["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed_bf16": "f32+bf16", "mixed_bf16x3": "f32+bf16x3",
                  "mixed_f16": "f32+f16", "mixed_f32": "f32"}[args.prec],
        "data": "synthetic",
        "config": {
            "workload": (f"mixed-precision ID, {m}x{n} fp32, A=U diag(exp(-i/40)) V^T (Haar), "
                         f"adaptive rank at tol {tol:g} (pivot-relative), one ID per step"),
            "m": m, "n": n, "tol": tol, "rank_rule": "pivot_rel", "prec": args.prec,
        },
        "k": mx["k"],
        "err2": mx["err2"],
        "err_ratio_sigma_k1": mx["ratio"],
        "acceptance": acceptance(args.prec),
        "fp64_gpu": {"ms_per_id": f64["ms"], "k": f64["k"], "tflops": f64["tflops"],
                     "err2": f64["err2"], "err_ratio_sigma_k1": f64["ratio"],
                     "acceptance": acceptance("f64")},
        "speedup_vs_fp64": f64["ms"] / mx["ms"],
        "gram_front_end": gram_fe,
        "cholqr_front_end": cholqr_fe,
        "sketch_front_end": sk,
        "other_precisions": {p: {"ms_per_id": res[p]["ms"], "k": res[p]["k"],
                                 "err2": res[p]["err2"],
                                 "err_ratio_sigma_k1": res[p]["ratio"],
                                 "speedup_vs_fp64": f64["ms"] / res[p]["ms"],
                                 "acceptance": acceptance(p)} for p in extra},
        "roofline": {
            "kernel": "k_sweep (reflector sweep W^T v, one read of the trailing block per pivot)",
            "bound": "hbm",
            "achieved": sweep_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": sweep_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "bytes_per_launch": per_launch_bytes,
            "us_per_launch": per_launch_us,
            "launches_per_id": prof["sweep_launches"] / args.profile_reps,
        },
        "kernel_ms_per_id": {key: prof[key] / args.profile_reps
                             for key in ("sweep_ms", "finalize_ms", "gemm_ms", "other_ms",
                                         "total_ms")},
        "id_roofline": id_roofline(m, n, mx["k"], 4, mx["ms"]),
        "fp64_id_roofline": id_roofline(m, n, f64["k"], 8, f64["ms"]),
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out))


if __name__ == "__main__":
    main()
