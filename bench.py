#!/usr/bin/env python3
"""Benchmark of the two-stage Householder orthogonalization on one MI355X.

Default workload (graded): one step = one call of tho_two_stage (Algorithm 1
with the second choice of P, every row-streaming step in libtho's HIP
kernels) on real FP64, n = 2^22, k0 = 128, k = 64, V the Q factor of a
Gaussian matrix, A = X diag(s) Y^T with s log-spaced from 1 to 1e-8
(cond(A) = 1e8).  Inputs are generated on the GPU from a fixed seed and are
resident in HBM before the timed region.

Other workloads (--workload):
  graded-f32x2, graded-bf16  the same problem with FP32 hi+lo / BF16 panels
  grad      forward + adjoint (tho_two_stage_backward), n = 2^20, k0 = 64,
            k = 32, Gaussian loss weights G_Q, G_R
  batched   4096 problems (n ~ U[2048, 65536], k0 in {8,16,32,64},
            k in {4,8,16}) in one graph-captured persistent launch
  complex   complex128, n = 2^20, k0 = 64, k = 32, A = V C + 1e-10 G
            (cond([V, A]) ~ 1e10), with BCGS and full Householder QR beside it

value   = algorithmic bytes / time.  Two-stage: B_alg = 8 n (3 k0 + 4 k) (V
          and A streamed once in each of the three phases their dependences
          force, Q written once).  Adjoint: + 8 n (2 k0 + 4 k) (V, A, Q and
          the Q adjoint read once, dV and dA written once).  Batched: the sum
          of B_alg over the problems.
roofline: the dominant kernel (largest share of the timed region, from HIP
          events the library records around each launch on the call's
          stream), its algorithmic work per launch over its average duration,
          against the FP64 peak (two-stage leaf/formation) or the HBM peak
          (batched, streaming kernels).
cpu_baseline: the CPU oracle (NumPy FP64, test infrastructure) timed on this
          host on a sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
HERE = os.path.dirname(os.path.abspath(__file__))
WORKLOADS = ["graded", "graded-f32x2", "graded-bf16", "grad", "batched", "complex"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="graded", choices=WORKLOADS)
    p.add_argument("--n", type=int, default=None)
    p.add_argument("--k0", type=int, default=None)
    p.add_argument("--k", type=int, default=None)
    p.add_argument("--cpu-rows", type=int, default=1 << 22)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-check", action="store_true")
    p.add_argument("--no-compare", action="store_true", help="skip the comparison methods (graded only)")
    p.add_argument("--copy-calib", action="store_true",
                   help="launch one plain 1 GiB device copy first (HBM counter calibration)")
    return p.parse_args()


def make_inputs(n, k0, k, seed=3, device="cuda"):
    """Graded workload on the GPU (input generation only)."""
    import torch
    g = torch.Generator(device=device).manual_seed(260214449 + seed)
    V, _ = torch.linalg.qr(torch.randn(n, k0, dtype=torch.float64, device=device, generator=g))
    X, _ = torch.linalg.qr(torch.randn(n, k, dtype=torch.float64, device=device, generator=g))
    Y, _ = torch.linalg.qr(torch.randn(k, k, dtype=torch.float64, device=device, generator=g))
    s = 10.0 ** (-8.0 * torch.arange(k, dtype=torch.float64, device=device) / max(k - 1, 1))
    A = (X * s[None, :]) @ Y.T.contiguous()
    del X
    return V.contiguous(), A.contiguous()


def kernel_model(name, n, k0, k):
    """Algorithmic (bytes, flops) per launch of the main kernels."""
    m = n - k0
    if name == "xty_partial":      # C = V^T A over all rows
        return 8.0 * n * (k0 + k), 2.0 * n * k0 * k
    if name == "leaf_l0":          # A + V Z, Householder QR, V^T Q chain
        return 8.0 * m * (k0 + 2 * k), m * (4.0 * k0 * k + 2.0 * k * k)
    if name == "form_l0":          # Q_ = Q_loc G, + V N
        return 8.0 * m * (k0 + 2 * k), m * (2.0 * k0 * k + 2.0 * k * k)
    return None


def gram_loss(V, Q):
    """||[V,Q]^T [V,Q] - I||_2 on the GPU (FP64, 2^18-row chunks)."""
    import numpy as np
    import torch
    n = Q.shape[0]
    G = None
    for i in range(0, n, 1 << 18):
        blk = torch.cat([V[i:i + (1 << 18)], Q[i:i + (1 << 18)]], 1)
        gg = blk.mH.contiguous() @ blk
        G = gg if G is None else G + gg
    Gm = G.cpu().numpy() - np.eye(G.shape[0])
    return float(np.max(np.abs(np.linalg.eigvalsh(0.5 * (Gm + Gm.conj().T)))))


def rel_res(V, A, Q, R, S):
    import numpy as np
    n = A.shape[0]
    ge = ga = None
    for i in range(0, n, 1 << 18):
        sl = slice(i, i + (1 << 18))
        eb = A[sl] - V[sl] @ S - Q[sl] @ R
        ab = A[sl]
        x = eb.mH.contiguous() @ eb
        y = ab.mH.contiguous() @ ab
        ge = x if ge is None else ge + x
        ga = y if ga is None else ga + y
    return float(np.sqrt(np.max(np.linalg.eigvalsh(ge.cpu().numpy())) /
                         np.max(np.linalg.eigvalsh(ga.cpu().numpy()))))


def threads_used():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def time_steps(fn, steps, warmup, stream):
    """Headline time: `steps` calls bracketed by events on `stream`, with the
    library's per-kernel event recording off.  The per-kernel breakdown then
    comes from a separate run of the same number of steps with recording on
    (its totals are per-kernel sums; they are divided by `steps` below)."""
    import torch
    from paper_2602_14449_amd import _lib
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    _lib.tho_profile_reset()
    _lib.tho_profile_enable(1)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    _lib.tho_profile_enable(0)
    return ms, _lib.profile_read()


def roofline(prof, model_fn, bound, traffic_tag=None):
    """`traffic_tag` names the workload the committed HBM counters were taken
    on; the traffic field stays null for any other workload."""
    dname, (dms, dcnt) = max(prof.items(), key=lambda kv: kv[1][0])
    davg = dms / max(dcnt, 1)
    model = model_fn(dname)
    if model is None:
        return None
    bts, fl = model
    if bound == "mfma":
        ach = fl / (davg * 1e-3) / 1e12
        peak, unit = FP64_PEAK_TFS, "TFLOP/s"
    else:
        ach = bts / (davg * 1e-3) / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    roof = {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": None, "kernel": dname, "avg_ms": round(davg, 4),
            "alg_bytes_per_launch": bts, "alg_flops_per_launch": fl}
    tf = os.path.join(HERE, "profiles", "traffic.json")
    if traffic_tag is not None and os.path.exists(tf):
        try:
            tj = json.load(open(tf))
            ent = tj.get(dname) if tj.get("_calibration", {}).get("workload") == traffic_tag else None
            if ent and ent.get("valid", False):
                roof["traffic"] = ent["bytes_per_launch"]
        except Exception:
            pass
    return roof


def cpu_baseline_two_stage(n_s, k0, k, full_n):
    from oracle import two_stage as oracle_two_stage
    V, A = make_inputs(n_s, k0, k, seed=33)
    Vh, Ah = V.cpu().numpy(), A.cpu().numpy()
    del V, A
    t0 = time.perf_counter()
    oracle_two_stage(Vh, Ah)
    t = time.perf_counter() - t0
    gbs = 8.0 * n_s * (3 * k0 + 4 * k) / t / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": int(threads_used()), "kind": "oracle",
            "sample": "graded workload at n=%d (1/%d of the rows), k0=%d, k=%d; one oracle run, %.1f s"
                      % (n_s, max(1, full_n // n_s), k0, k, t)}


def base_line(a, metric, value, ms, dtype, workload, extra_cfg):
    cfg = {"workload": workload}
    cfg.update(extra_cfg)
    return {"metric": metric, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}


def run_graded(a, panel):
    import torch
    import paper_2602_14449_amd as tho
    n = a.n or (1 << 22)
    k0 = a.k0 if a.k0 is not None else 128
    k = a.k or 64
    dev = torch.device("cuda:0")
    V, A = make_inputs(n, k0, k)
    Q = torch.empty(n, k, dtype=torch.float64, device=dev)
    R = torch.empty(k, k, dtype=torch.float64, device=dev)
    S = torch.empty(max(k0, 0), k, dtype=torch.float64, device=dev)
    ws = torch.empty(tho.workspace_bytes(n, k0, k, panel=panel), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    if a.copy_calib:
        # known traffic: 2^30 bytes read + 2^30 bytes written
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)              # runtime copy (hipMemcpy device to device)
        torch.neg(src, out=dst)     # elementwise kernel, same traffic
        torch.cuda.synchronize()
        del src, dst
    ms, prof = time_steps(lambda: tho.two_stage(V, A, panel=panel, out=(Q, R, S), workspace=ws),
                          a.steps, a.warmup, stream)
    B_alg = 8.0 * n * (3 * k0 + 4 * k)
    F_alg = float(n) * (8 * k0 * k + 4 * k * k)
    gbs = B_alg / (ms * 1e-3) / 1e9
    full = (n, k0, k) == (1 << 22, 128, 64)
    wl = ("graded: real two-stage, n=2^22, k0=128, k=64, cond(A)=1e8, %s panels" % panel.upper()) if full \
        else "graded: n=%d, k0=%d, k=%d, %s panels" % (n, k0, k, panel)
    out = base_line(a, "two-stage orth GB/s (% HBM peak) vs full HHQR of [V,A]; orth loss vs FP64", gbs, ms,
                    "f64" if panel == "fp64" else panel + "+f64", wl, {"n": n, "k0": k0, "k": k, "panel": panel})
    out["pct_hbm_peak"] = round(100.0 * gbs / HBM_PEAK_GBS, 2)
    out["pct_fp64_peak"] = round(100.0 * F_alg / (ms * 1e-3) / 1e12 / FP64_PEAK_TFS, 2)
    out["roofline"] = roofline(prof, lambda nm: kernel_model(nm, n, k0, k), "mfma",
                               traffic_tag="graded n=%d k0=%d k=%d panel=%s" % (n, k0, k, panel))
    out["kernels_ms_per_step"] = {kn: round(v[0] / a.steps, 4) for kn, v in
                                  sorted(prof.items(), key=lambda kv: -kv[1][0])}
    if not a.no_check:
        out["accuracy"] = {"orth_loss": gram_loss(V, Q), "rel_residual": rel_res(V, A, Q, R, S)}
    if panel == "fp64" and not a.no_compare:
        out["comparisons"] = compare(a, V, A, Q, R, S, stream)
        # the paper's comparison (two-stage vs Householder QR of [V, A]) on
        # floors: algorithmic bytes at the HBM peak vs flops at the FP64 peak
        b_hh = 8.0 * n * (2 * k0 + 3 * k)
        f_hh = float(n) * (2 * k0 * k0 + 6 * k0 * k + 4 * k * k)
        fl_ts = max(B_alg / (HBM_PEAK_GBS * 1e9), F_alg / (FP64_PEAK_TFS * 1e12)) * 1e3
        fl_hh = max(b_hh / (HBM_PEAK_GBS * 1e9), f_hh / (FP64_PEAK_TFS * 1e12)) * 1e3
        hh_ms = out["comparisons"]["hhqr_full"]["ms"]
        out["hhqr_vs_two_stage"] = {
            "two_stage_floor_ms": round(fl_ts, 3), "hhqr_floor_ms": round(fl_hh, 3),
            "floor_ratio": round(fl_hh / fl_ts, 3), "measured_ratio": round(hh_ms / ms, 3),
            "note": "hhqr_full is Algorithm 4 over 64-column panels (three chained two-stage steps); "
                    "the floor ratio is what an ideal Householder QR of [V, A] would allow"}
    if not a.no_cpu_baseline:
        del Q, ws
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline_two_stage(min(a.cpu_rows, n), k0, k, n)
    else:
        out["cpu_baseline"] = None
    return out


def compare(a, V, A, Q, R, S, stream):
    """The comparison methods on the same inputs (3 timed calls each)."""
    import torch
    import paper_2602_14449_amd as tho
    res = {}
    cands = [("hhqr_full", lambda: tho.hhqr_full(V, A, out=(Q, R, S))),
             ("bcgs_1_1", lambda: tho.bcgs(V, A, 1, 1, out=(Q, R, S))),
             ("bcgs_1_2", lambda: tho.bcgs(V, A, 1, 2, out=(Q, R, S))),
             ("two_stage_p_mlu", lambda: tho.two_stage(V, A, p_choice="mlu", out=(Q, R, S))),
             ("two_stage_p_polar", lambda: tho.two_stage(V, A, p_choice="polar", out=(Q, R, S))),
             ("two_stage_f32x2", lambda: tho.two_stage(V, A, panel="f32x2", out=(Q, R, S))),
             ("two_stage_bf16", lambda: tho.two_stage(V, A, panel="bf16", out=(Q, R, S)))]
    for name, fn in cands:
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ent = {"ms": round(e0.elapsed_time(e1) / 3, 3)}
        if not a.no_check:
            ent["orth_loss"] = gram_loss(V, Q)
            ent["rel_residual"] = rel_res(V, A, Q, R, S)
        res[name] = ent
    # vendor Householder QR of [V, A] (rocSOLVER geqrf + orgqr through torch), one call
    B = torch.cat([V, A], 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    torch.linalg.qr(B)
    torch.cuda.synchronize()
    res["torch_linalg_qr_of_VA"] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "calls": 1}
    del B
    return res


def run_grad(a):
    import numpy as np
    import torch
    import paper_2602_14449_amd as tho
    n = a.n or (1 << 20)
    k0 = a.k0 if a.k0 is not None else 64
    k = a.k or 32
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(260214449 + 5)
    V, _ = torch.linalg.qr(torch.randn(n, k0, dtype=torch.float64, device=dev, generator=g))
    V = V.contiguous()
    A = torch.randn(n, k, dtype=torch.float64, device=dev, generator=g)
    GQ = torch.randn(n, k, dtype=torch.float64, device=dev, generator=g)
    GR = torch.randn(k, k, dtype=torch.float64, device=dev, generator=g)
    stream = torch.cuda.current_stream(dev)

    def step():
        Q, R, S = tho.two_stage(V, A)
        return tho.two_stage_backward(V, A, Q, R, GQ, GR)

    ms, prof = time_steps(step, a.steps, a.warmup, stream)
    B = 8.0 * n * (3 * k0 + 4 * k) + 8.0 * n * (2 * k0 + 4 * k)
    gbs = B / (ms * 1e-3) / 1e9
    out = base_line(a, "two-stage forward + adjoint GB/s (algorithmic bytes)", gbs, ms, "f64",
                    "grad: real FP64 forward + adjoint, n=%d, k0=%d, k=%d, Gaussian G_Q, G_R" % (n, k0, k),
                    {"n": n, "k0": k0, "k": k})
    out["pct_hbm_peak"] = round(100.0 * gbs / HBM_PEAK_GBS, 2)

    m = n - k0
    # rows_gemm launches of one adjoint: Q_ and its adjoint (V_low with Q_low,
    # G_Q low), the A1 adjoint (2 inputs, 1 output), dV over all rows (3
    # inputs), the two bottom-row corrections of dV and dA: per row
    # 8 (6 k0 + 13 k) bytes over 6 launches.
    rg_launches = prof.get("rows_gemm", (0.0, 1))[1] / max(a.steps, 1)

    def model(nm):
        if nm == "xty_partial":
            return 8.0 * n * (k0 + k), 2.0 * n * k0 * k
        if nm == "rows_gemm":
            return (8.0 * (m * (6 * k0 + 13 * k) + k0 * (k0 + 3 * k)) / max(rg_launches, 1),
                    2.0 * n * (4 * k0 * k + 2 * k * k) / max(rg_launches, 1))
        return kernel_model(nm, n, k0, k)
    dname = max(prof.items(), key=lambda kv: kv[1][0])[0]
    out["roofline"] = roofline(prof, model, "hbm" if dname in ("xty_partial", "rows_gemm") else "mfma")
    out["kernels_ms_per_step"] = {kn: round(v[0] / a.steps, 4) for kn, v in
                                  sorted(prof.items(), key=lambda kv: -kv[1][0])}
    if not a.no_cpu_baseline:
        from oracle.adjoint import two_stage_vjp
        ns = min(a.cpu_rows, n) // 4
        Vh, Ah = V[:ns].cpu().numpy(), A[:ns].cpu().numpy()
        Vh, _ = np.linalg.qr(Vh)
        GQh, GRh = GQ[:ns].cpu().numpy(), GR.cpu().numpy()
        t0 = time.perf_counter()
        two_stage_vjp(Vh, Ah, GQh, GRh)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(8.0 * ns * (3 * k0 + 4 * k + 2 * k0 + 4 * k) / t / 1e9, 4),
                               "unit": "GB/s", "cores": int(threads_used()), "kind": "oracle",
                               "sample": "grad workload at n=%d, k0=%d, k=%d: oracle reverse-mode gradient "
                                         "(forward intermediates included), %.1f s" % (ns, k0, k, t)}
    else:
        out["cpu_baseline"] = None
    return out


def run_batched(a):
    import torch
    import paper_2602_14449_amd as tho
    import tho_workloads as W
    dev = torch.device("cuda:0")
    count = 4096
    pairs = W.batched_gpu(count)
    plan = tho.BatchedPlan(pairs)
    stream = torch.cuda.current_stream(dev)
    ms, prof = time_steps(plan.run, a.steps, a.warmup, stream)
    B = sum(8.0 * V.shape[0] * (3 * V.shape[1] + 4 * A_.shape[1]) for V, A_ in pairs)
    F = sum(float(V.shape[0]) * (8 * V.shape[1] * A_.shape[1] + 4 * A_.shape[1] ** 2) for V, A_ in pairs)
    gbs = B / (ms * 1e-3) / 1e9
    out = base_line(a, "batched two-stage GB/s (algorithmic bytes, % HBM peak)", gbs, ms, "f64",
                    "batched: 4096 real FP64 problems, n~U[2048,65536], k0 in {8,16,32,64}, k in {4,8,16}, "
                    "one graph-captured persistent launch", {"problems": count, "tuning": plan.info()})
    out["pct_hbm_peak"] = round(100.0 * gbs / HBM_PEAK_GBS, 2)
    out["roofline"] = roofline(prof, lambda nm: (B, F) if nm == "batched" else None, "hbm")
    if not a.no_check:
        outs = plan.outputs
        losses = []
        for j in range(0, count, count // 16):
            V, A_ = pairs[j]
            losses.append(gram_loss(V, outs[j][0]))
        out["accuracy"] = {"max_orth_loss_16_sampled": max(losses)}
    if not a.no_cpu_baseline:
        from oracle import two_stage as oracle_two_stage
        t0 = time.perf_counter()
        done = 0.0
        j = 0
        while time.perf_counter() - t0 < 10.0 and j < count:
            V, A_ = pairs[j]
            oracle_two_stage(V.cpu().numpy(), A_.cpu().numpy())
            done += 8.0 * V.shape[0] * (3 * V.shape[1] + 4 * A_.shape[1])
            j += 1
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(done / t / 1e9, 4), "unit": "GB/s", "cores": int(threads_used()),
                               "kind": "oracle",
                               "sample": "first %d of the 4096 problems through the oracle, %.1f s" % (j, t)}
    else:
        out["cpu_baseline"] = None
    plan.close()
    return out


def run_complex(a):
    import torch
    import paper_2602_14449_amd as tho
    n = a.n or (1 << 20)
    k0 = a.k0 if a.k0 is not None else 64
    k = a.k or 32
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(260214449 + 2)
    c128 = torch.complex128

    def cn(*shape):
        return torch.randn(*shape, dtype=c128, device=dev, generator=g)
    V, _ = torch.linalg.qr(cn(n, k0))
    V = V.contiguous()
    A = (V @ cn(k0, k) + 1e-10 * cn(n, k)).contiguous()
    Q = torch.empty(n, k, dtype=c128, device=dev)
    R = torch.empty(k, k, dtype=c128, device=dev)
    S = torch.empty(k0, k, dtype=c128, device=dev)
    stream = torch.cuda.current_stream(dev)
    ms, prof = time_steps(lambda: tho.two_stage(V, A, out=(Q, R, S)), a.steps, a.warmup, stream)
    B_alg = 16.0 * n * (3 * k0 + 4 * k)
    gbs = B_alg / (ms * 1e-3) / 1e9
    out = base_line(a, "two-stage orth GB/s (% HBM peak) vs full HHQR of [V,A]; orth loss vs FP64", gbs, ms,
                    "c128", "complex: complex128 two-stage, n=%d, k0=%d, k=%d, A = V C + 1e-10 G" % (n, k0, k),
                    {"n": n, "k0": k0, "k": k})
    out["pct_hbm_peak"] = round(100.0 * gbs / HBM_PEAK_GBS, 2)

    def model(nm):
        m = n - k0
        if nm == "zleaf_l0":   # complex Householder of the m x k block: read, write vectors
            return 16.0 * m * 2 * k, 8.0 * m * k * k
        if nm == "zform_l0":
            return 16.0 * m * 2 * k, 8.0 * m * k * k
        if nm == "rows_gemm":  # A + V Z and Q_ + V N (average of the two)
            return 16.0 * m * (k0 + 2 * k), 8.0 * m * k0 * k
        if nm == "xty_partial":
            return 16.0 * n * (k0 + k), 8.0 * n * k0 * k
        return None
    dname = max(prof.items(), key=lambda kv: kv[1][0])[0]
    out["roofline"] = roofline(prof, model, "hbm" if dname in ("rows_gemm", "xty_partial") else "mfma")
    out["kernels_ms_per_step"] = {kn: round(v[0] / a.steps, 4) for kn, v in
                                  sorted(prof.items(), key=lambda kv: -kv[1][0])}
    if not a.no_check:
        out["accuracy"] = {"orth_loss": gram_loss(V, Q), "rel_residual": rel_res(V, A, Q, R, S)}
        comp = {}
        for name, fn in [("hhqr_full", lambda: tho.hhqr_full(V, A, out=(Q, R, S))),
                         ("bcgs_1_1", lambda: tho.bcgs(V, A, 1, 1, out=(Q, R, S))),
                         ("bcgs_1_2", lambda: tho.bcgs(V, A, 1, 2, out=(Q, R, S)))]:
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            comp[name] = {"ms": round((time.perf_counter() - t0) / 3 * 1e3, 3), "orth_loss": gram_loss(V, Q),
                          "rel_residual": rel_res(V, A, Q, R, S)}
        out["comparisons"] = comp
    if not a.no_cpu_baseline:
        from oracle import two_stage as oracle_two_stage
        ns = min(a.cpu_rows, n) // 4
        Vh, Ah = V[:ns].cpu().numpy(), A[:ns].cpu().numpy()
        t0 = time.perf_counter()
        oracle_two_stage(Vh, Ah)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(16.0 * ns * (3 * k0 + 4 * k) / t / 1e9, 4), "unit": "GB/s",
                               "cores": int(threads_used()), "kind": "oracle",
                               "sample": "complex workload rows 0..%d (first rows of the same V, A), k0=%d, k=%d; "
                                         "one oracle run, %.1f s" % (ns, k0, k, t)}
    else:
        out["cpu_baseline"] = None
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    sys.path.insert(0, HERE)
    torch.cuda.set_device(0)
    if a.workload == "graded":
        out = run_graded(a, "fp64")
    elif a.workload == "graded-f32x2":
        out = run_graded(a, "f32x2")
    elif a.workload == "graded-bf16":
        out = run_graded(a, "bf16")
    elif a.workload == "grad":
        out = run_grad(a)
    elif a.workload == "complex":
        out = run_complex(a)
    else:
        out = run_batched(a)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
