"""Benchmark: generalized Hermitian-definite eigensolve on one MI355X.

Workload (default): n = 10000 complex128 pencil with a constructed spectrum
(A = L Q diag(D) Q^H L^H, B = L L^H, |D| log-uniform over [1e-3, 1e1] with random
sign), all eigenpairs, FP64.  One step = one call of hgv_zhegvx (Cholesky, reduction to
standard form, dense->band, bulge chasing, divide and conquer, the two back-transforms
and the back-substitution).  Inputs are resident in HBM; each step starts from a
device copy of the pencil (the solve destroys A and overwrites B).

Prints ONE JSON line (rank 0).  Extra fields: per-stage milliseconds, the accuracy of
the last step (residual, B-orthogonality, eigenvalue error against the constructed
spectrum), the lower-fraction solves (10 % / 25 % of the eigenpairs) in FP64 and in
mixed precision (complex64 reduction + FP64 refinement) side by side with their
residuals, the GEMM roofline from HIP events recorded around every MFMA GEMM launch,
and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix (and vector) peak
PEAK_HBM_GBS = 8000.0


def solve_flops(n, m):
    """Algorithmic flops (LAPACK complex leading terms): potrf 4/3 n^3, hegst 4 n^3,
    he2hb 16/3 n^3, Q2 8 n^2 m, Q1 8 n^2 m, back-substitution 4 n^2 m."""
    return (4.0 / 3.0 + 4.0 + 16.0 / 3.0) * n ** 3 + 20.0 * n * n * m


def gemm_traffic():
    """HBM bytes per launch of the complex-double GEMM tile kernel, from the committed counter
    summary, or None when the kernel's device code has changed since the counters were taken."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", "gemm_tz_hbm_traffic_fp64_n10000.md")).read()
        src = open(os.path.join(root, "paper_1207_1773_amd", "csrc", "gemm.hip"), "rb").read()
    except OSError:
        return None
    import hashlib
    import re
    mb = re.search(r"^hbm_bytes_per_launch: (\d+)$", text, re.M)
    mh = re.search(r"^gemm\.hip tile kernel sha256: ([0-9a-f]{64})$", text, re.M)
    s = src.decode()
    b0, b1 = s.find("// ---- device code of the tile kernel (begin) ----"), s.find("// ---- device code of the tile kernel (end) ----")
    if not mb or not mh or b0 < 0 or b1 < 0 or hashlib.sha256(s[b0:b1].encode()).hexdigest() != mh.group(1):
        return None
    return int(mb.group(1))


def run_config1(ctx, dev, reps=3):
    """n = 4096 GUE-like pencil (cond(B) = 1e3), all pairs, band width 64: seconds (median
    of `reps` after a warm-up), algorithmic TFLOP/s and the accuracy on 2000 columns."""
    import numpy as np
    import torch
    import paper_1207_1773_amd as hgv
    from inputs import gue_pair
    n = 4096
    A, B = gue_pair(n, 1, cond_b=1e3, device=dev)
    Ac0, Bc0 = hgv.colmajor(A), hgv.colmajor(B)
    Ac, Bc = torch.empty_like(Ac0), torch.empty_like(Bc0)
    times, r = [], None
    for it in range(reps + 1):
        Ac.copy_(Ac0)
        Bc.copy_(Bc0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = ctx.zhegvx(Ac, Bc, 1, n, "fp64", 64, stats=True, inplace=True)
        e1.record()
        torch.cuda.synchronize()
        if it > 0:
            times.append(e0.elapsed_time(e1))
    W, X, info, st = r
    ms = float(np.median(times))
    n1 = lambda M: float(M.abs().sum(0).max())
    idx = torch.cat([torch.arange(1000), torch.arange(n - 1000, n)]).to(dev)
    Xs, Ws = X[:, idx], W[idx].to(torch.complex128)
    BX = B @ Xs
    res = n1(A @ Xs - BX * Ws[None, :]) / (n * n1(A) * n1(Xs))
    G = Xs.conj().T @ BX
    orth = n1(G - torch.eye(G.shape[0], dtype=G.dtype, device=dev))
    print("[bench] GUE n=4096 all pairs: %.1f ms" % ms, file=sys.stderr, flush=True)
    return {"workload": "GUE-like pencil A=(G+G^H)/2, B=U diag(logspace(0,3,n)) U^H, n=4096, all pairs, FP64, nb=64",
            "s": ms / 1e3, "tflops": solve_flops(n, n) / (ms * 1e-3) / 1e12, "info": info,
            "stage_ms": {k: v for k, v in st["ms"].items() if v > 0},
            "gemm_stage_ms": sum(st["ms"][k] for k in ("potrf", "hegst", "he2hb", "q2", "q1", "trsm")),
            "residual": res, "orthogonality": orth, "orth_over_n": orth / n, "checked_columns": 2000,
            "times_ms": times}


def run_config3(ctx, dev, reps=3):
    """Batched workload: 64 pencils, n uniform in [500, 3000], lowest 20 % of each, the whole
    batch captured in one HIP graph (FP64 and mixed precision), against the same problems
    solved one after another."""
    import numpy as np
    import torch
    import paper_1207_1773_amd as hgv
    from inputs import batch_problem, batch_sizes
    sizes = batch_sizes()
    il = [1] * len(sizes)
    iu = [int(math.ceil(0.2 * n)) for n in sizes]
    flops = sum(solve_flops(n, m) for n, m in zip(sizes, iu))
    As, Bs = [], []
    for i, n in enumerate(sizes):
        A, B = batch_problem(i, n, device=dev)
        As.append(A)
        Bs.append(B)
    nb = [hgv.hgv_default_nb(n) for n in sizes]
    out = {"workload": "64 GUE-like pencils (cond(B)=1e2), n uniform in [500,3000], lowest 20%% of each; "
                       "sum n^3 = %.3e" % sum(float(n) ** 3 for n in sizes),
           "algorithmic_flops": flops}
    for precision in ("fp64", "mixed"):
        bs = hgv.tensors.BatchedSolve(ctx, As, Bs, il, iu, nb, precision=precision,
                                      max_refine_iters=2 if precision == "mixed" else 0)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                bs.run()
        torch.cuda.current_stream().wait_stream(side)
        ctx._sync_stream()
        times = []
        for it in range(reps + 1):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            if it > 0:
                times.append(e0.elapsed_time(e1))
        # the same batch launched eagerly (no graph), for comparison
        eager = []
        for it in range(2):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            bs.run()
            e1.record()
            torch.cuda.synchronize()
            eager.append(e0.elapsed_time(e1))
        Ws, Xs, infos = bs.results()
        worst_res = worst_orth = 0.0
        n1 = lambda M: float(M.abs().sum(0).max())
        for i, n in enumerate(sizes):
            BX = Bs[i] @ Xs[i]
            res = n1(As[i] @ Xs[i] - BX * Ws[i].to(torch.complex128)[None, :]) / (n * n1(As[i]) * n1(Xs[i]))
            G = Xs[i].conj().T @ BX
            orth = n1(G - torch.eye(G.shape[0], dtype=G.dtype, device=dev)) / n
            worst_res, worst_orth = max(worst_res, res), max(worst_orth, orth)
        ms = float(np.median(times))
        out[precision] = {"s": ms / 1e3, "tflops": flops / (ms * 1e-3) / 1e12, "times_ms": times,
                          "eager_s": min(eager) / 1e3,
                          "infos_nonzero": int(sum(1 for x in infos if x != 0)),
                          "max_residual": worst_res, "max_orth_over_n": worst_orth}
        print("[bench] batched 64 pencils %s (one graph): %.1f ms" % (precision, ms), file=sys.stderr, flush=True)
        del g, bs
    # the same problems solved one after another (one call each, FP64)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i, n in enumerate(sizes):
        ctx.zhegvx(As[i], Bs[i], il[i], iu[i], "fp64", nb[i])
    e1.record()
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    out["one_by_one_fp64"] = {"s": ms1 / 1e3, "tflops": flops / (ms1 * 1e-3) / 1e12,
                              "note": "each call synchronises to read back d_info"}
    out["batched_speedup_vs_one_by_one"] = ms1 / (out["fp64"]["s"] * 1e3)
    print("[bench] 64 pencils one by one: %.1f ms" % ms1, file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--frac", type=float, default=1.0, help="fraction of eigenpairs (lowest) in the timed step")
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--fractions", type=str, default="0.1,0.25", help="extra untimed-by-contract fractions")
    ap.add_argument("--mixed-fractions", type=str, default="0.1,0.25,1.0",
                    help="fractions also solved in mixed precision (side by side with FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured FP64 MFMA / copy peaks")
    ap.add_argument("--cpu-n", type=int, default=2560)
    ap.add_argument("--no-values-only", action="store_true", help="skip the eigenvalues-only solve")
    ap.add_argument("--no-one-stage", action="store_true", help="skip the one-stage solve")
    ap.add_argument("--no-config1", action="store_true", help="skip the n=4096 GUE-pencil solve")
    ap.add_argument("--no-config3", action="store_true", help="skip the batched 64-pencil solve")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only copy a device buffer of this size 5 times and exit (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the solver runs on one device)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1207_1773_amd as hgv
    from inputs import constructed

    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}), flush=True)
        return
    ctx = hgv.Context.get(dev)
    n = args.n
    m = max(1, int(math.ceil(args.frac * n)))

    t0 = time.time()
    A, B, parts = constructed(n, 2, "loguniform", device=dev, return_parts=True)
    D_sorted = np.sort(parts["D"])
    del parts
    Ac0 = hgv.colmajor(A)
    Bc0 = hgv.colmajor(B)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    print("[bench] pencil n=%d generated in %.1f s" % (n, t_gen), file=sys.stderr, flush=True)

    Ac = torch.empty_like(Ac0)
    Bc = torch.empty_like(Bc0)

    def step(mm, stats, precision="fp64"):
        Ac.copy_(Ac0)
        Bc.copy_(Bc0)
        return ctx.zhegvx(Ac, Bc, 1, mm, precision, args.nb, stats=stats, inplace=True)

    n1 = lambda M: float(M.abs().sum(0).max())

    def accuracy(W, X, mm, cols=2000):
        """residual ||AX - BX W||_1 / (n ||A||_1 ||X||_1), ||X^H B X - I||_1 and the eigenvalue error
        against the constructed spectrum (all eigenvalues), on `cols` pairs: all of them, or the
        first and the last cols/2 when there are more."""
        Wn = W.cpu().numpy()
        lerr = float(np.abs(Wn - D_sorted[:mm]).max() / np.abs(D_sorted).max())
        if mm <= cols:
            idx = torch.arange(mm, device=X.device)
        else:
            idx = torch.cat([torch.arange(cols // 2), torch.arange(mm - cols // 2, mm)]).to(X.device)
        Xs = X[:, idx]
        Ws = W[idx].to(torch.complex128)
        BX = B @ Xs
        R = A @ Xs - BX * Ws[None, :]
        res = n1(R) / (n * n1(A) * n1(Xs))
        G = Xs.conj().T @ BX
        orth = n1(G - torch.eye(G.shape[0], dtype=G.dtype, device=dev))
        return {"residual": res, "orthogonality": orth, "orth_over_n": orth / n,
                "max_rel_eig_err_vs_constructed": lerr, "checked_columns": int(Xs.shape[1])}

    for i in range(args.warmup):
        step(m, False)
        torch.cuda.synchronize()
        print("[bench] warmup %d done" % i, file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    stage_ms = {}
    gemm_ms = gemm_flops = 0.0
    gemm_launches = 0
    t_start = time.time()
    ev0.record()
    last = None
    for i in range(args.steps):
        last = step(m, True)
        st = last[3]
        for k, v in st["ms"].items():
            stage_ms[k] = stage_ms.get(k, 0.0) + v
        gemm_ms += st["gemm_ms"]
        gemm_flops += st["gemm_flops"]
        gemm_launches += st["gemm_launches"]
        print("[bench] step %d: %.1f ms" % (i, sum(st["ms"].values())), file=sys.stderr, flush=True)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.time() - t_start
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    W, X, info, st = last
    flops = solve_flops(n, m)
    tflops = flops / (ms_per_step * 1e-3) / 1e12

    # accuracy of the last timed step (verification on the device with torch products)
    acc_main = accuracy(W, X, m)
    acc_main["info"] = info

    def timed_fraction(f, precision):
        mf = max(1, int(math.ceil(f * n)))
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = step(mf, True, precision)
        e1.record()
        torch.cuda.synchronize()
        msf = e0.elapsed_time(e1)
        st_f = r[3]
        rec = {"m": mf, "s": msf / 1e3, "tflops": solve_flops(n, mf) / (msf * 1e-3) / 1e12,
               "stage_ms": {k: v for k, v in st_f["ms"].items() if v > 0}, "info": r[2]}
        if precision == "mixed":
            rec.update({"refine_iters": st_f["refine_iters"], "refine_resid": st_f["refine_resid"],
                        "fallback": st_f["fallback"]})
        rec["accuracy"] = accuracy(r[0], r[1], mf)
        print("[bench] %s fraction %.2f: %.1f ms" % (precision, f, msf), file=sys.stderr, flush=True)
        return rec

    extra = {}
    for f in [float(x) for x in args.fractions.split(",") if x]:
        extra["%d%%" % round(100 * f)] = timed_fraction(f, "fp64")
    mixed = {}
    for f in [float(x) for x in args.mixed_fractions.split(",") if x]:
        key = "%d%%" % round(100 * f)
        rec = timed_fraction(f, "mixed")
        base = extra.get(key)
        if base is None and abs(f * n - m) < 1:
            base = {"s": ms_per_step / 1e3}
        if base is not None:
            rec["speedup_vs_fp64"] = base["s"] / rec["s"]
        mixed[key] = rec

    # eigenvalues only (no second-stage reflectors, Sturm-count multisection, no back-transforms)
    values_only = None
    if not args.no_values_only:
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        Ac.copy_(Ac0)
        Bc.copy_(Bc0)
        e0.record()
        rv = ctx.zhegvx(Ac, Bc, 1, n, "fp64", args.nb, stats=True, inplace=True, values_only=True)
        e1.record()
        torch.cuda.synchronize()
        msv = e0.elapsed_time(e1)
        Wv = rv[0].cpu().numpy()
        values_only = {"m": n, "s": msv / 1e3, "info": rv[2],
                       "stage_ms": {k: v for k, v in rv[3]["ms"].items() if v > 0},
                       "max_rel_eig_err_vs_constructed": float(np.abs(Wv - D_sorted).max() / np.abs(D_sorted).max()),
                       "speedup_vs_all_vectors": ms_per_step / msv}
        print("[bench] eigenvalues only: %.1f ms" % msv, file=sys.stderr, flush=True)

    # the one-stage tridiagonalisation (Sec. 4.1) as the comparison path, all pairs
    one_stage = None
    if not args.no_one_stage:
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        Ac.copy_(Ac0)
        Bc.copy_(Bc0)
        e0.record()
        r1 = ctx.zhegvx(Ac, Bc, 1, n, "fp64", args.nb, stats=True, inplace=True, one_stage=True)
        e1.record()
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1)
        one_stage = {"m": n, "s": ms1 / 1e3, "tflops": solve_flops(n, n) / (ms1 * 1e-3) / 1e12, "info": r1[2],
                     "stage_ms": {k: v for k, v in r1[3]["ms"].items() if v > 0},
                     "note": "he2hb = one-stage tridiagonalisation (hemv-based), q1 = its back-transformation",
                     "accuracy": accuracy(r1[0], r1[1], n),
                     "two_stage_speedup": ms1 / ms_per_step}
        print("[bench] one-stage, all pairs: %.1f ms" % ms1, file=sys.stderr, flush=True)

    del Ac, Bc, Ac0, Bc0, A, B, X
    torch.cuda.empty_cache()
    config1 = run_config1(ctx, dev) if not args.no_config1 else None
    config3 = run_config3(ctx, dev) if not args.no_config3 else None

    # roofline denominators measured on this device (after the timed steps)
    peaks = None
    if not args.no_peaks:
        wb = 2 << 30
        w = torch.empty(wb, dtype=torch.uint8, device=dev)
        ptf, pgbs = hgv.hgv_device_peaks(ctx.handle, w.data_ptr(), wb)
        del w
        peaks = {"fp64_mfma_tflops": ptf, "copy_gbs": pgbs, "published_fp64_mfma_tflops": PEAK_FP64_TFLOPS,
                 "published_hbm_gbs": 8000.0,
                 "method": "hgv_device_peaks: v_mfma_f64_16x16x4f64 chains with no memory traffic (16 waves/CU); "
                           "16-byte copy of 1 GiB to 1 GiB, bytes read + written"}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        An, Bn = constructed(args.cpu_n, 2, "loguniform")
        An, Bn = An.numpy(), Bn.numpy()
        tc = time.time()
        _, _, cinfo = oracle.zhegv(An, Bn)
        tcpu = time.time() - tc
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cores = min(cores, os.cpu_count() or cores)
        model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = {"value": solve_flops(args.cpu_n, args.cpu_n) / tcpu / 1e12, "unit": "TFLOP/s", "cores": cores,
               "kind": "oracle",
               "cpu_model": model,
               "sample": "oracle full solve (all pairs) of the same pencil recipe at n=%d: %.2f s (info %d), "
                         "TFLOP/s with the n=%d flop count; an n^3-scaled ESTIMATE (not measured) for n=%d: %.0f s"
                         % (args.cpu_n, tcpu, cinfo, args.cpu_n, n, tcpu * (n / args.cpu_n) ** 3)}

    stage_avg = {k: v / args.steps for k, v in stage_ms.items() if v > 0}
    stage_tflops = {k: st["flops"][k] / (v * 1e-3) / 1e12 for k, v in stage_avg.items() if st["flops"].get(k)}
    nbw = st["nb"] if st else max(args.nb, 1)
    hb2st_gbs = (24.0 * n * n * nbw / (stage_avg["hb2st"] * 1e-3) / 1e9) if stage_avg.get("hb2st") else None
    gemm_avg_ms = gemm_ms / max(gemm_launches, 1)
    achieved = (gemm_flops / (gemm_ms * 1e-3) / 1e12) if gemm_ms > 0 else None
    out = {
        "metric": "generalized eigensolve s & TFLOP/s, n=10k c128; FP64 vs mixed at equal residual",
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "constructed-spectrum pencil, |D| log-uniform [1e-3,1e1], n=%d, lowest %d "
                               "eigenpairs (%.0f%%), FP64, nb=%s" % (n, m, 100.0 * m / n,
                                                                   st["nb"] if st else args.nb),
                   "n": n, "m": m, "precision": "fp64"},
        "seconds_per_solve": ms_per_step / 1e3,
        "stage_ms": stage_avg,
        "stage_tflops": stage_tflops,
        "hb2st_algorithmic_gbs": hb2st_gbs,
        "accuracy": acc_main,
        "fractions": extra,
        "mixed": mixed,
        "eigenvalues_only": values_only,
        "one_stage_all_pairs": one_stage,
        "config_gue_n4096": config1,
        "config_batched_64": config3,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP64_TFLOPS) if achieved else None, "traffic": gemm_traffic(),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE / WRITE_SIZE counters, copy-calibrated)",
                     "kernel": "hgv::gemm_kernel<hgv::TZ, 64, 64, 4> (complex-double MFMA GEMM tiles, every launch "
                               "of a step; split-K reductions excluded)",
                     "launches_per_step": gemm_launches / args.steps,
                     "avg_launch_ms": gemm_avg_ms,
                     "gemm_share_of_step": (gemm_ms / args.steps) / ms_per_step,
                     "peak_measured": peaks["fp64_mfma_tflops"] if peaks else None,
                     "frac_of_measured": (achieved / peaks["fp64_mfma_tflops"]) if (peaks and achieved) else None},
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
        "input_generation_s": t_gen,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
