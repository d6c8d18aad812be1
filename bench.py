"""Benchmark of the compressed-NMF hot path on one MI355X.

A step is one cnmf_factorize call on the FP32 20000 x 5000 workload
(A = W H + |N(0, 0.05)|, r = 50, k = 60, q = 4, two-sided structured
compression, 200 compressed-ADMM iterations, FP64 relative residual), with
A, the test matrices and the initial factors resident in HBM before the
clock starts.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-precision]

The line also carries a "precision" object: the two-sided sketch of the
100000 x 20000 FP32 workload (r = 100, k = 120, q = 4) with FP32, BF16 and
FP8 E4M3 (+ BF16 final pass) range-finder passes, each with its projection
residual ||A - L L^T A||_F / ||A||_F accumulated in FP64.  That input is
generated on the device (torch's seeded generator, same recipe).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1505_04650_amd import workloads as WL  # noqa: E402

METRIC = "sketch TFLOP/s + NMF solves/s at stated rel. residual; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_traffic(w):
    """HBM bytes per range-pass launch from the committed counter profile
    (FETCH_SIZE / WRITE_SIZE scaled by a copy of known size), or None when
    the profile is for another workload or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_range_passes_{w.name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    with open(os.path.join(ROOT, prof["kernel_source"]), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != prof["kernel_source_sha256"]:
        return None
    return prof["hbm_bytes_per_launch"]


def cpu_baseline(inp, w, lam, budget_s=15.0):
    """The FP64 oracle, as it stands, on the host: full solves of the same
    workload (sketch + 200 ADMM iterations + residual) until ~budget_s."""
    from oracle import cnmf_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    A64 = inp["A"].astype(np.float64)
    done, t0, res = 0, time.perf_counter(), None
    while True:
        sk = O.sketch(A64, inp["Omega_L"], inp["Omega_R"], w.q)
        adm = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, w.iters)
        res = O.rel_residual(A64, adm["U"], adm["V"])
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / done * (done + 1) > 2.5 * budget_s:
            break
    el = time.perf_counter() - t0
    hi = host_info()
    return {"value": done / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": hi["cpu_model"], "blas": hi["blas"], "logical_cpus": hi["logical_cpus"],
            "sample": f"{done} full solve(s) of the same 20000x5000 workload (FP64 NumPy, "
                      f"sketch q=4 + {w.iters} ADMM iterations + residual) in {el:.1f} s"}, res


def _proj_residual(A, L, norm_a, blk=8192):
    """||A - L (L^T A)||_F / ||A||_F formed directly (not through ||A||^2 -
    ||L^T A||^2, which assumes L^T L = I) in FP64 over row blocks, and the
    orthonormality error max|L^T L - I|, from plain PyTorch FP64 products."""
    import torch
    k, n = L.shape[1], A.shape[1]
    Ld = L.double()
    B = torch.zeros(k, n, dtype=torch.float64, device=A.device)
    for i in range(0, A.shape[0], blk):
        B += Ld[i:i + blk].T @ A[i:i + blk].double()
    ss = 0.0
    for i in range(0, A.shape[0], blk):
        R = A[i:i + blk].double() - Ld[i:i + blk] @ B
        ss += float((R * R).sum())
    orth = float((Ld.T @ Ld - torch.eye(k, dtype=torch.float64, device=A.device)).abs().max())
    return math.sqrt(ss) / norm_a, orth


def _fp64_reference_sketch(A, oml, omr, q, blk=8192):
    """An FP64 reference of the two-sided sketch with plain PyTorch on the
    device: A in FP64, Householder QR (torch.linalg.qr) after every product,
    signs fixed so that diag(R) >= 0.  Returns L (m x k), R (k x n), B, At."""
    import torch

    def orth(Y):
        Q, Rr = torch.linalg.qr(Y)
        sg = torch.sign(torch.diagonal(Rr))
        sg[sg == 0] = 1.0
        return Q * sg

    def av(X):   # A X, X n x k
        return torch.cat([A[i:i + blk].double() @ X for i in range(0, A.shape[0], blk)])

    def atv(Z):  # A^T Z, Z m x k
        out = torch.zeros(A.shape[1], Z.shape[1], dtype=torch.float64, device=A.device)
        for i in range(0, A.shape[0], blk):
            out += A[i:i + blk].double().T @ Z[i:i + blk]
        return out

    Lq = orth(av(oml))
    for _ in range(q):
        Lq = orth(av(orth(atv(Lq))))
    Rq = orth(atv(omr))
    for _ in range(q):
        Rq = orth(atv(orth(av(Rq))))
    B = atv(Lq).T.contiguous()          # k x n
    At = B @ Rq                          # k x k  (B R^T with R = Rq^T)
    return Lq, Rq.T.contiguous(), B, At


def _sin_max_angle(Q1, Q2):
    """sin of the largest principal angle between the column spans of the
    orthonormal Q1, Q2 (2-norm of Q1's part outside span(Q2))."""
    import torch
    D = Q1 - Q2 @ (Q2.T @ Q1)
    return float(torch.linalg.matrix_norm(D, ord=2))


def precision_section(h, steps, warmup, reference=True):
    """Sketch of the 100000 x 20000 precision workload in FP32, BF16 and FP8
    (reference=False skips the FP64 reference sketch and the errors against
    it, for kernel profiles under hardware counters)."""
    import torch
    from paper_1505_04650_amd import api
    w = WL.WORKLOADS["precision_100000x20000"]
    dev = torch.device("cuda", 0)
    g = torch.Generator(device=dev)
    g.manual_seed(100 * w.index)
    A = torch.rand(w.m, w.r, device=dev, generator=g) @ torch.rand(w.r, w.n, device=dev, generator=g)
    for i in range(0, w.m, 8192):
        A[i:i + 8192] += (w.sigma * torch.randn(A[i:i + 8192].shape, device=dev, generator=g)).abs_()
    oml = torch.randn(w.n, w.k, device=dev, dtype=torch.float64, generator=g)
    omr = torch.randn(w.m, w.k, device=dev, dtype=torch.float64, generator=g)
    norm_a = math.sqrt(sum(float((A[i:i + 8192].double() ** 2).sum()) for i in range(0, w.m, 8192)))
    refL = refR = refB = refAt = None
    if reference:
        t_ref = time.perf_counter()
        refL, refR, refB, refAt = _fp64_reference_sketch(A, oml, omr, w.q)
        ref_res, ref_orth = _proj_residual(A, refL, norm_a)
        torch.cuda.synchronize()
        log(f"precision: FP64 reference sketch (PyTorch FP64, Householder QR) in {time.perf_counter() - t_ref:.1f} "
            f"s, projection residual {ref_res:.6e}")
    flops = 2.0 * w.m * w.n * w.k * (2 * (1 + 2 * w.q) + 1)  # two chains of 2q + 1 products, and B
    out = {"workload": w.name, "m": w.m, "n": w.n, "r": w.r, "k": w.k, "q": w.q, "sides": "both",
           "data": "synthetic, generated on the device"}
    st = h.stream
    for pd, fd in (("f32", "f32"), ("bf16", "bf16"), ("fp8", "bf16")):
        for _ in range(warmup):
            api.sketch(A, w.r, w.k, w.q, oml, omr, pass_dtype=pd, final_dtype=fd, handle=h)
        torch.cuda.synchronize()
        h.set_timing(True)
        agg = {}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sk = None
        for _ in range(steps):
            sk = api.sketch(A, w.r, w.k, w.q, oml, omr, pass_dtype=pd, final_dtype=fd, handle=h)
            for name, (ms, fl, nl) in h.stages().items():
                a = agg.setdefault(name, [0.0, 0.0, 0])
                if not math.isnan(ms):
                    a[0] += ms
                a[1] += fl
                a[2] += nl
        e1.record(st)
        torch.cuda.synchronize()
        h.set_timing(False)
        ms = e0.elapsed_time(e1) / steps
        pn, pt = agg.get("pass_AX", [0, 0, 0]), agg.get("pass_ATZ", [0, 0, 0])
        pass_ms = (pn[0] + pt[0]) / steps
        pres, porth = _proj_residual(A, sk.L, norm_a)
        r_ = w.r
        vs_ref = None
        if reference:
            vs_ref = {"proj_residual_gap": abs(pres - ref_res),
                      "orth_err_L": porth,
                      "sin_angle_L_leading_r": _sin_max_angle(sk.L.double()[:, :r_], refL[:, :r_]),
                      "sin_angle_R_leading_r": _sin_max_angle(sk.R.double().T[:, :r_].contiguous(), refR.T[:, :r_]),
                      "rel_err_B": float(torch.linalg.norm(sk.B.double() - refB) / torch.linalg.norm(refB)),
                      "rel_err_At": float(torch.linalg.norm(sk.At.double() - refAt) / torch.linalg.norm(refAt))}
        out[pd] = {"final_dtype": fd, "sketch_ms": ms, "sketch_tflops": flops / (ms * 1e-3) / 1e12,
                   "pass_ms": pass_ms, "pass_tflops": flops / (pass_ms * 1e-3) / 1e12,
                   "stages_ms": {k: v[0] / steps for k, v in agg.items() if v[2]},
                   "proj_residual": pres, "vs_fp64_reference": vs_ref}
        log(f"precision {pd}/{fd}: {ms:.3f} ms per sketch, projection residual {out[pd]['proj_residual']:.6e}")
    ref = out["f32"]["proj_residual"]
    for pd in ("bf16", "fp8"):
        out[pd]["proj_residual_gap_vs_f32"] = abs(out[pd]["proj_residual"] - ref)
        out[pd]["speedup_vs_f32"] = out["f32"]["sketch_ms"] / out[pd]["sketch_ms"]
    if reference:
        out["fp64_reference"] = {"kind": "PyTorch FP64 on the device (A cast to FP64 per row block, Householder "
                                         "QR after every product, diag(R) >= 0), the same test matrices",
                                 "proj_residual": ref_res, "orth_err_L": ref_orth}
    del A, refL, refR, refB, refAt
    torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model, logical cores and the BLAS NumPy uses (for cpu_baseline)."""
    info = {"cpu_model": None, "logical_cpus": os.cpu_count(), "blas": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{d.get('internal_api')} {d.get('version')} ({d.get('num_threads')} threads)"
                for d in threadpool_info() if d.get("user_api") == "blas"]
        info["blas"] = ", ".join(libs) or None
    except Exception:  # pragma: no cover
        pass
    return info


def attainable_peaks():
    """Measured attainable peaks on this GPU: HBM (a 4 GiB device copy,
    bytes read + written per second) and the dense matrix engines through
    the vendor GEMM (hipBLASLt via torch.matmul, 8192^3) in FP32, BF16, FP64."""
    import torch
    dev = torch.device("cuda", 0)
    out = {}
    src = torch.empty(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["hbm_copy_GBps"] = 2 * src.numel() * 4 / (ms * 1e-3) / 1e9
    del src, dst
    nn = 8192
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16), ("fp64", torch.float64)):
        a = torch.randn(nn, nn, device=dev, dtype=torch.float32).to(dt)
        b = torch.randn(nn, nn, device=dev, dtype=torch.float32).to(dt)
        for _ in range(2):
            c = a @ b
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"gemm_{name}_TFLOPs"] = 2.0 * nn ** 3 / (ms * 1e-3) / 1e12
        del a, b, c
    torch.cuda.empty_cache()
    out["note"] = ("vendor GEMM through torch.matmul (8192^3, square) and a device copy; fractions in the "
                   "roofline objects are against the published peaks")
    return out


def extra_workloads_section(h, lam_c2, inp_c2, w_c2):
    """The other workloads, measured beside the headline:
    * 1000 x 500 FP64 (q 4, 100 ADMM iterations): device time per stage and
      the factors' gap to the oracle (the parity workload);
    * 20000 x 5000 FP32: compressed MU and alternating NNLS, and
      uncompressed ADMM / MU / alternating NNLS (L = I, R = I), 200
      iterations each, time and FP64 residual beside compressed ADMM;
    * 10000 x 100000 separable FP32 (two-sided, q 2): sketch time and GB/s of
      A read, SPA time, and whether SPA returns exactly the planted columns."""
    import torch
    from oracle import cnmf_oracle as O
    from paper_1505_04650_amd import api
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev)
    out = {}
    # 1000 x 500 FP64
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w)
    sk = O.sketch(inp["A"], inp["Omega_L"], inp["Omega_R"], w.q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[w.r - 1])
    ref = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, w.iters)
    args = (t(inp["A"]), w.r, w.k, w.q, t(inp["U1"]), t(inp["V1"]), t(inp["Omega_L"]), t(inp["Omega_R"]))
    for _ in range(2):
        api.factorize(*args, iters=w.iters, lam=lam, phi=lam, handle=h)
    torch.cuda.synchronize()
    h.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    f = api.factorize(*args, iters=w.iters, lam=lam, phi=lam, handle=h)
    e1.record(h.stream)
    torch.cuda.synchronize()
    st = {k: (v[0] * 1e3 if not math.isnan(v[0]) else None) for k, v in h.stages().items() if v[2]}
    h.set_timing(False)
    U = f.U.cpu().numpy()
    # the same solve captured once as a graph and replayed (launch latency
    # dominates at this size)
    gph = api.FactorizeGraph(*args, iters=w.iters, lam=lam, phi=lam)
    for _ in range(3):
        gph.replay()
    gph.synchronize()
    ge0, ge1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ge0.record(gph.stream)
    for _ in range(10):
        gph.replay()
    ge1.record(gph.stream)
    gph.synchronize()
    us_graph = ge0.elapsed_time(ge1) * 1e3 / 10
    same_graph = bool(torch.equal(gph.U, f.U) and torch.equal(gph.V, f.V))
    gph.close()
    out["plain_fp64_1000x500"] = {
        "us_per_solve": e0.elapsed_time(e1) * 1e3, "us_per_solve_graph_replay": us_graph,
        "graph_replay_identical": same_graph, "us_per_stage": st,
        "rel_diff_U_vs_oracle": float(np.linalg.norm(U - ref["U"]) / np.linalg.norm(ref["U"])),
        "rel_residual": float(f.rel_residual.item()),
        "rel_residual_oracle": O.rel_residual(inp["A"], ref["U"], ref["V"])}
    log(f"1000x500 FP64: {out['plain_fp64_1000x500']['us_per_solve']:.0f} us per solve, "
        f"{us_graph:.0f} us as a graph replay")
    # 20000 x 5000: compressed MU and the uncompressed comparators
    A = torch.as_tensor(inp_c2["A"], device=dev)
    c2 = {}
    for method in ("mu", "anls", "admm_full", "mu_full", "anls_full"):
        fa = (A, w_c2.r, w_c2.k, w_c2.q, t(inp_c2["U1"]), t(inp_c2["V1"]), t(inp_c2["Omega_L"]),
              t(inp_c2["Omega_R"]))
        api.factorize(*fa, method=method, iters=w_c2.iters, lam=lam_c2, phi=lam_c2, mu_eps=1e-16, handle=h)
        torch.cuda.synchronize()
        e0.record(h.stream)
        f = api.factorize(*fa, method=method, iters=w_c2.iters, lam=lam_c2, phi=lam_c2, mu_eps=1e-16, handle=h)
        e1.record(h.stream)
        torch.cuda.synchronize()
        c2[method] = {"ms_per_solve": e0.elapsed_time(e1), "rel_residual": float(f.rel_residual.item())}
        log(f"20000x5000 {method}: {c2[method]['ms_per_solve']:.2f} ms, residual {c2[method]['rel_residual']:.6e}")
    out["nmf_fp32_20000x5000_methods"] = dict(c2, iters=w_c2.iters, lam=lam_c2)
    del A
    # 10000 x 100000 separable, two-sided
    ws = WL.WORKLOADS["separable_fp32_10000x100000"]
    As, planted = WL.separable_on_device(ws.m, ws.n, ws.r, ws.sep_noise, 100 * ws.index, dev)
    planted = planted.tolist()
    for _ in range(2):
        K, _, _ = api.select(As, ws.r, ws.k, ws.q, sides="both", seed=300, handle=h)
    torch.cuda.synchronize()
    h.set_timing(True)
    e0.record(h.stream)
    K, score, Bsk = api.select(As, ws.r, ws.k, ws.q, sides="both", seed=300, want_scores=True, want_B=True, handle=h)
    e1.record(h.stream)
    torch.cuda.synchronize()
    stg = {k: v for k, v in h.stages().items() if v[2]}
    h.set_timing(False)
    total = e0.elapsed_time(e1)
    spa_ms = stg.get("spa", (float("nan"),))[0]
    sketch_ms = total - spa_ms
    npass = 2 * ws.q + 2
    # the right factor H (r x n) by per-column NNLS on B
    api.snmf_nnls(Bsk, K, handle=h)
    torch.cuda.synchronize()
    e0.record(h.stream)
    Hn, ninfo = api.snmf_nnls(Bsk, K, want_info=True, handle=h)
    e1.record(h.stream)
    torch.cuda.synchronize()
    nnls_ms = e0.elapsed_time(e1)
    ninfo = ninfo.cpu().tolist()
    out["separable_fp32_10000x100000"] = {
        "ms_total": total, "ms_sketch": sketch_ms, "ms_spa": spa_ms, "passes": npass,
        "ms_right_factor_nnls": nnls_ms, "nnls_columns_not_converged": ninfo[0], "nnls_max_steps": ninfo[1],
        "sketch_GBps_of_A": npass * ws.m * ws.n * 4 / (sketch_ms * 1e-3) / 1e9,
        "K_equals_planted_set": sorted(K.cpu().tolist()) == planted,
        "K": K.cpu().tolist()}
    log(f"10000x100000 separable: sketch {sketch_ms:.2f} ms, SPA {spa_ms:.3f} ms, planted recovered "
        f"{out['separable_fp32_10000x100000']['K_equals_planted_set']}")
    del As, Bsk, Hn
    torch.cuda.empty_cache()
    out.update(input_formats_section(h, inp_c2, w_c2))
    return out


def _timed(h, fn, reps=3):
    """Median wall time (ms) of fn() with the device synchronised around it."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), fn


def input_formats_section(h, inp_c2, w_c2):
    """The other input forms and test matrices, measured beside the dense
    device-resident path:
    * 20000 x 5000 FP32 in pinned host memory, streamed through the device
      (two-sided sketch, q 4: 10 passes over A);
    * SRHT instead of Gaussian test matrices on the same sketch;
    * a sparse A from the paper's sparse recipe (W, H with density 0.01, N
      with density 1e-4; n = 0.75 m), 40000 x 30000, r 50, as CSR: sketch
      and 100 compressed ADMM iterations."""
    import torch
    from paper_1505_04650_amd import api
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev)
    out = {}
    w = w_c2
    A = torch.as_tensor(inp_c2["A"])
    Ah = A.pin_memory()
    Ad = A.to(dev)
    oml, omr = t(inp_c2["Omega_L"]), t(inp_c2["Omega_R"])
    npass = 2 * w.q + 2
    ms_dev, _ = _timed(h, lambda: api.sketch(Ad, w.r, w.k, w.q, oml, omr, handle=h))
    ms_host, _ = _timed(h, lambda: api.sketch(Ah, w.r, w.k, w.q, oml, omr, handle=h))
    Lh = api.sketch(Ah, w.r, w.k, w.q, oml, omr, handle=h).L
    Ld = api.sketch(Ad, w.r, w.k, w.q, oml, omr, handle=h).L
    A64 = Ad.double()
    nA = float(torch.linalg.norm(A64))
    pr = lambda L_: float(torch.linalg.norm(A64 - L_.double() @ (L_.double().T @ A64))) / nA
    out["host_streamed_fp32_20000x5000"] = {
        "sketch_ms": ms_host, "device_resident_sketch_ms": ms_dev, "passes": npass,
        "block_rows": int(max(64, (64 << 20) // (w.n * 4) // 64 * 64)),
        "host_to_device_GBps": npass * w.m * w.n * 4 / (ms_host * 1e-3) / 1e9,
        "proj_residual": pr(Lh), "proj_residual_device_path": pr(Ld)}
    log(f"host-streamed 20000x5000 sketch: {ms_host:.1f} ms ({out['host_streamed_fp32_20000x5000']['host_to_device_GBps']:.1f}"
        f" GB/s of A), device-resident {ms_dev:.2f} ms")
    ms_srht, _ = _timed(h, lambda: api.sketch(Ad, w.r, w.k, w.q, seed=5, test_matrix="srht", handle=h))
    ms_gauss, _ = _timed(h, lambda: api.sketch(Ad, w.r, w.k, w.q, seed=5, handle=h))
    Ls = api.sketch(Ad, w.r, w.k, w.q, seed=5, test_matrix="srht", handle=h).L
    Lg = api.sketch(Ad, w.r, w.k, w.q, seed=5, handle=h).L
    out["srht_vs_gaussian_fp32_20000x5000"] = {
        "sketch_ms_srht": ms_srht, "sketch_ms_gaussian": ms_gauss,
        "proj_residual_srht": pr(Ls), "proj_residual_gaussian": pr(Lg)}
    del Ah, Ad, A64, Lh, Ld, Ls, Lg
    torch.cuda.empty_cache()
    # sparse recipe on the device
    m, n, r, k, delta = 40000, 30000, 50, 60, 0.01
    g = torch.Generator(device=dev)
    g.manual_seed(7000)
    W = torch.rand(m, r, device=dev, generator=g) * (torch.rand(m, r, device=dev, generator=g) < delta)
    H = torch.rand(r, n, device=dev, generator=g) * (torch.rand(r, n, device=dev, generator=g) < delta)
    Ad = W @ H
    Ad += torch.randn(m, n, device=dev, generator=g) * (torch.rand(m, n, device=dev, generator=g) < delta * delta)
    As = Ad.to_sparse_csr()
    nnz = int(As.values().numel())
    # the initialisation and penalties of the dense workloads: c U[0,1)
    # factors with E[U V] = mean(A), lambda = phi = sigma_r(At)
    c = math.sqrt(4.0 * max(float(Ad.mean()), 1e-12) / r)
    U0 = c * torch.rand(m, r, device=dev, dtype=torch.float64, generator=g)
    V0 = c * torch.rand(r, n, device=dev, dtype=torch.float64, generator=g)
    ms_sk, _ = _timed(h, lambda: api.sketch(As, r, k, 4, seed=9, handle=h))
    lam = float(torch.linalg.svdvals(api.sketch(As, r, k, 4, seed=9, handle=h).At.double())[r - 1])
    f = None

    def fz():
        nonlocal f
        f = api.factorize(As, r, k, 4, U0, V0, None, None, iters=100, lam=lam, phi=lam, seed=9, handle=h)
    ms_f, _ = _timed(h, fz)
    res_sparse = float(f.rel_residual.item())
    # the same factors against the dense copy (FP64 on the device): the
    # sparse residual formula must agree
    Ud, Vd = f.U.double(), f.V.double()
    A64 = Ad.double()
    res_dense = float(torch.linalg.norm(A64 - Ud @ Vd) / torch.linalg.norm(A64))
    out["sparse_fp32_40000x30000"] = {
        "recipe": "W, H density 0.01, N density 1e-4 (the paper's sparse synthetic case), n = 0.75 m",
        "nnz": nnz, "density": nnz / (m * n), "r": r, "k": k, "q": 4,
        "sketch_ms": ms_sk, "factorize_ms_100_admm_iterations": ms_f, "lambda": lam,
        "rel_residual": res_sparse, "rel_residual_dense_check": res_dense}
    log(f"sparse 40000x30000 ({nnz} nonzeros): sketch {ms_sk:.2f} ms, factorize {ms_f:.2f} ms, residual "
        f"{res_sparse:.6f} (dense check {res_dense:.6f})")
    del W, H, Ad, As, A64, f
    torch.cuda.empty_cache()
    return out


def serving_section(n_req, qps=None, max_batch=128, workers=3, budget_bytes=16 << 30, baseline_n=40):
    """The serving workload: n_req uneven compressed-ADMM requests (FP32,
    k = r + 10, q = 2, 100 iterations), all generated on the device before
    the clock starts (the device-resident path), through the continuous-
    batching server under an HBM budget.  Protocol: the saturation
    throughput X_sat with every request arriving at t = 0, then Poisson
    arrivals at 0.5, 0.8 and 0.95 X_sat; the 0.8 run is the headline (a
    given `qps` runs that rate alone).  Beside it: the first `baseline_n`
    requests run one at a time through cnmf_factorize (the plain FP32
    path), whose factors every served copy equals bit for bit."""
    import torch
    from paper_1505_04650_amd import api
    S = WL.SERVING
    m, n, r, k, _ = WL.serving_requests(n_req, 0.0)
    dev = torch.device("cuda", 0)
    noise_mean = S["sigma"] * math.sqrt(2.0 / math.pi)

    def gen(i):
        g = torch.Generator(device=dev)
        g.manual_seed(10_000 + i)
        mi, ni, ri, ki = int(m[i]), int(n[i]), int(r[i]), int(k[i])
        A = torch.rand(mi, ri, device=dev, generator=g) @ torch.rand(ri, ni, device=dev, generator=g)
        A += (S["sigma"] * torch.randn(mi, ni, device=dev, generator=g)).abs_()
        oml = torch.randn(ni, ki, device=dev, dtype=torch.float64, generator=g)
        omr = torch.randn(mi, ki, device=dev, dtype=torch.float64, generator=g)
        c = math.sqrt(4.0 * (ri / 4.0 + noise_mean) / ri)
        U0 = c * torch.rand(mi, ri, device=dev, dtype=torch.float64, generator=g)
        V0 = c * torch.rand(ri, ni, device=dev, dtype=torch.float64, generator=g)
        lam = WL.expected_rms(ri, S["sigma"]) * math.sqrt(min(mi, ni))
        return dict(A=A, r=ri, k=ki, q=S["q"], U0=U0, V0=V0, omega_left=oml, omega_right=omr, lam=lam)

    t_gen = time.perf_counter()
    reqs = [gen(i) for i in range(n_req)]
    torch.cuda.synchronize()
    log(f"serving: {n_req} requests generated on the device in {time.perf_counter() - t_gen:.1f} s "
        f"({sum(q['A'].numel() for q in reqs) * 4 / 1e9:.1f} GB of A)")

    # the plain path: one request at a time through cnmf_factorize
    h = api.default_handle()
    base = []
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for i in range(baseline_n):
        q = reqs[i]
        t1 = time.perf_counter()
        f = api.factorize(q["A"], q["r"], q["k"], q["q"], q["U0"], q["V0"], q["omega_left"], q["omega_right"],
                          iters=S["iters"], lam=q["lam"], phi=q["lam"], handle=h)
        torch.cuda.synchronize()
        base.append(((time.perf_counter() - t1) * 1e3, f.U, f.V, float(f.rel_residual.item())))
    base_wall = time.perf_counter() - tb0
    base_ms = np.array([b[0] for b in base])

    def run(rate, budget=budget_bytes, graphs=False):
        t_arr = WL.serving_requests(n_req, rate)[4]
        lat, queue, res, same = [], [], [], []
        with api.Server(budget, max_batch=max_batch, workers=workers, graphs=graphs) as srv:
            outstanding = {}

            def drain(block=False):
                while outstanding:
                    done_any = False
                    for i in list(outstanding):
                        t = outstanding[i]
                        info = srv.poll(t)
                        if info["done"]:
                            if info["status"] != 0:
                                raise RuntimeError(f"request {i} failed: {info['message']}")
                            lat.append(info["total_ms"])
                            queue.append(info["queue_ms"])
                            res.append(float(t.rel_residual.item()))
                            if i < baseline_n:
                                same.append(bool(torch.equal(t.U, base[i][1]) and torch.equal(t.V, base[i][2])))
                            srv.release(t)
                            del outstanding[i]
                            done_any = True
                    if not block or not outstanding:
                        return
                    if not done_any:
                        time.sleep(2e-4)

            t0 = time.perf_counter()
            for i in range(n_req):
                while time.perf_counter() - t0 < t_arr[i]:
                    drain()
                    time.sleep(1e-4)
                q = reqs[i]
                outstanding[i] = srv.submit(q["A"], q["r"], q["k"], q["q"], q["U0"], q["V0"], q["omega_left"],
                                            q["omega_right"], iters=S["iters"], lam=q["lam"], phi=q["lam"])
                if i % 64 == 63:
                    drain()
            t_sub = time.perf_counter() - t0
            drain(block=True)
            wall = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array(lat)
        o = {"qps_offered": rate or None, "qps_submitted": n_req / t_sub if t_sub > 0 else None,
             "solves_per_s": n_req / wall, "wall_s": wall,
             "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                            "mean": float(lat.mean()), "max": float(lat.max())},
             "queue_ms_p50": float(np.percentile(queue, 50)),
             "rel_residual_mean": float(np.mean(res)), "rel_residual_max": float(np.max(res)),
             "results_identical_to_plain_path": bool(all(same)) if same else None,
             "hbm_budget_bytes": budget, "graph_replays": graphs,
             "server": {k2: st[k2] for k2 in ("batch_steps", "graph_replays", "graphs_built", "batched_iterations",
                                              "max_batch_seen", "peak_arena_bytes")}}
        log(f"serving at {rate or 0:.0f} QPS (budget {budget / 2**30:.1f} GiB, graphs {graphs}): "
            f"{o['solves_per_s']:.1f} solves/s, p50 {o['latency_ms']['p50']:.1f} ms, "
            f"p99 {o['latency_ms']['p99']:.1f} ms, max batch {o['server']['max_batch_seen']}, "
            f"peak arena {o['server']['peak_arena_bytes'] / 2**30:.2f} GiB")
        return o

    if qps:
        runs = [run(qps)]
        head = runs[0]
        x_sat = None
    else:
        sat = run(0.0)
        x_sat = sat["solves_per_s"]
        runs = [sat] + [run(f * x_sat) for f in (0.5, 0.8, 0.95)]
        head = runs[2]
        # the same saturation run with graph replays of the fixed-grid step
        # instead of direct launches, and the headline rate under a budget
        # that binds (below the arena's peak at that rate, so admission has
        # to hold requests)
        runs.append(run(0.0, graphs=True))
        runs.append(run(0.8 * x_sat, budget=max(1 << 30, int(0.6 * head["server"]["peak_arena_bytes"]))))
    out = {"workload": f"serving_{n_req}", "requests": n_req,
           "m": list(S["m"]), "n": list(S["n"]), "r": list(S["r"]), "q": S["q"], "iters": S["iters"],
           "data": "synthetic, every request generated on the device before the clock starts",
           "max_batch": max_batch, "workers": workers, "hbm_budget_bytes": budget_bytes,
           "x_sat_solves_per_s": x_sat, "headline": "0.8 x X_sat" if x_sat else "offered QPS",
           "runs_order": "X_sat, 0.5, 0.8, 0.95 X_sat; X_sat with graph replays; 0.8 X_sat under a binding budget"
           if x_sat else "offered QPS",
           "solves_per_s": head["solves_per_s"], "latency_ms": head["latency_ms"],
           "results_identical_to_plain_path": all(o["results_identical_to_plain_path"] is not False for o in runs),
           "runs": runs,
           "plain_path": {"requests": baseline_n, "solves_per_s": baseline_n / base_wall,
                          "latency_ms_p50": float(np.percentile(base_ms, 50)),
                          "latency_ms_p99": float(np.percentile(base_ms, 99))}}
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--precision-only", action="store_true",
                    help="only the precision sketches (for kernel profiles); prints that object")
    ap.add_argument("--no-reference", action="store_true",
                    help="with --precision-only: skip the FP64 reference sketch (for hardware-counter runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, the attainable peaks and the host information")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB FP32 tensor three times (a plain copy kernel of known size, so that "
                         "hardware byte counters can be scaled)")
    ap.add_argument("--serving-only", action="store_true", help="only the serving run; prints that object")
    ap.add_argument("--serving-requests", type=int, default=WL.SERVING["count"])
    ap.add_argument("--serving-qps", type=float, default=None,
                    help="one Poisson arrival rate instead of the X_sat / 0.5 / 0.8 / 0.95 X_sat protocol")
    ap.add_argument("--workload", default="nmf_fp32_20000x5000")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see the design notes on "
              "sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1505_04650_amd import api

    w = WL.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB (read 1 GiB, write 1 GiB each)")
        del src, dst
    if args.precision_only:
        print(json.dumps({"precision": precision_section(api.default_handle(), max(1, args.steps), args.warmup,
                                                         reference=not args.no_reference)}),
              flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_section(args.serving_requests, args.serving_qps)}), flush=True)
        return
    log(f"workload {w.name}: generating inputs")
    inp = WL.make_inputs(w)
    A = torch.as_tensor(inp["A"], device=dev)
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev)
    oml, omr, U1, V1 = t(inp["Omega_L"]), t(inp["Omega_R"]), t(inp["U1"]), t(inp["V1"])
    h = api.default_handle()

    # penalty: sigma_r of the compressed core (fixed before timing)
    sk = api.sketch(A, w.r, w.k, w.q, oml, omr)
    torch.cuda.synchronize()
    lam = float(np.linalg.svd(sk.At.double().cpu().numpy(), compute_uv=False)[w.r - 1])
    log(f"lambda = phi = sigma_r(At) = {lam:.6g}")

    def step():
        return api.factorize(A, w.r, w.k, w.q, U1, V1, oml, omr, method="admm", iters=w.iters, lam=lam, phi=lam,
                             handle=h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    h.set_timing(True)
    st = h.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    agg = {}
    torch.cuda.synchronize()
    ev0.record(st)
    t0 = time.perf_counter()
    f = None
    for _ in range(args.steps):
        f = step()
        for name, (ms, fl, n) in h.stages().items():  # waits on the step's own events
            a = agg.setdefault(name, [0.0, 0.0, 0])
            if not math.isnan(ms):
                a[0] += ms
            a[1] += fl
            a[2] += n
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    h.set_timing(False)
    ms_per_step = gpu_ms / args.steps
    res_gpu = float(f.rel_residual.item())
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step)")

    # sketch alone (TFLOP/s on the algorithmic 2 m n k x 19 flops)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        api.sketch(A, w.r, w.k, w.q, oml, omr, handle=h)
    e1.record(st)
    torch.cuda.synchronize()
    sketch_ms = e0.elapsed_time(e1) / args.steps
    sketch_flops = 2.0 * w.m * w.n * w.k * (2 * (1 + 2 * w.q) + 1)
    sketch_tflops = sketch_flops / (sketch_ms * 1e-3) / 1e12

    # the same solve captured as a graph and replayed (a context figure; the
    # headline is the call above)
    gph = api.FactorizeGraph(A, w.r, w.k, w.q, U1, V1, oml, omr, method="admm", iters=w.iters, lam=lam, phi=lam)
    gph.replay()
    gph.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(gph.stream)
    for _ in range(args.steps):
        gph.replay()
    g1.record(gph.stream)
    gph.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    graph_same = bool(torch.equal(gph.U, f.U) and torch.equal(gph.V, f.V))
    gph.close()
    log(f"graph replay: {graph_ms:.3f} ms/step (identical factors: {graph_same})")

    stages = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[2] / args.steps,
                  "gflop_per_step": v[1] / args.steps / 1e9} for k, v in agg.items() if v[2]}
    # dominant kernel: the range-finder pass kernels (A X and A^T Z launches)
    pn, pt = agg.get("pass_AX", [0, 0, 0]), agg.get("pass_ATZ", [0, 0, 0])
    pass_ms = pn[0] + pt[0]
    pass_fl = pn[1] + pt[1]
    pass_n = pn[2] + pt[2]
    achieved = pass_fl / (pass_ms * 1e-3) / 1e12 if pass_ms > 0 else None
    roofline = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": (achieved / FP32_PEAK_TFLOPS) if achieved else None, "traffic": pass_traffic(w),
                "kernel": "gemm_n_dma_kernel + gemm_t_dma_kernel (range-finder passes, FP32 16x16x4 MFMA)",
                "avg_launch_ms": pass_ms / pass_n if pass_n else None,
                "gflop_per_launch": pass_fl / pass_n / 1e9 if pass_n else None}

    out = {"metric": METRIC, "value": 1000.0 / ms_per_step, "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "m": w.m, "n": w.n, "r": w.r, "k": w.k, "q": w.q, "iters": w.iters,
                      "method": "compressed ADMM (two-sided)", "lambda": lam, "rel_residual": res_gpu},
           "sketch_tflops": sketch_tflops, "sketch_ms": sketch_ms, "stages": stages, "roofline": roofline,
           "graph_replay": {"ms_per_step": graph_ms, "identical_factors": graph_same}}

    if not args.no_extras:
        out["workloads"] = extra_workloads_section(h, lam, inp, w)
        out["attainable_peaks"] = attainable_peaks()
        out["host"] = host_info()
    if not args.no_precision:
        out["precision"] = precision_section(h, max(2, min(args.steps, 5)), 1)
    if not args.no_serving:
        out["serving"] = serving_section(args.serving_requests, args.serving_qps)

    if not args.no_cpu_baseline:
        log("cpu baseline: running the FP64 oracle on the host")
        cb, res_o = cpu_baseline(inp, w, lam)
        out["cpu_baseline"] = cb
        out["config"]["rel_residual_oracle"] = res_o
        out["config"]["rel_residual_gap"] = abs(res_gpu - res_o)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
