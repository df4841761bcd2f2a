#!/usr/bin/env python
"""Benchmark of the parareal / L1 / sine-Galerkin solver on one MI355X.

Workload (1D, config 2 of the method's benchmark set): D = 1 + 1/(1+u^2), f = 0.1 u (1-u),
M = 256 sine modes, Q = 384 Gauss points, N = 4096 fine L1 steps, P = 64 parareal slices,
three batched runs (alpha = 0.3, 0.7, 1.0) of 32 instances each with u0 coefficients
c_k ~ N(0, k^-3) (seeds 0..31).  Synthetic, seeded inputs.

One step = the three batched parareal solves (plain coarse L1 propagator G) run to the
iteration count k*(alpha) at which every instance's slice ends are within 1e-8 (relative
L2 over all P+1 slice ends) of the serial solution.  k* is found before the timed region
from the GPU serial solution (itself parity-checked against the CPU oracle by the tests)
and the parareal iterates.  Metric: useful mode-steps/s = sum_b M N / time-to-1e-8.

The JSON line also carries:
  roofline      the dominant kernel: the fine-sweep step kernel (2048 units per launch;
                evaluation, cosine-moment stiffness, register-resident Cholesky, solves).
                Algorithmic flops per unit = M^3/3 + M^2/2 + M/6 (Cholesky) + 2 M^2
                (two triangular solves) + 4 M Q (u_q and the load vector) + 2 (2M+1) Q
                (cosine moments); divided by the average launch time measured with HIP
                events on the launch stream over the timed region; peak = 78.6 TFLOP/s
                (MI355X dense FP64 matrix).
  gemm_assembly the same step with the stiffness formed as the quadrature GEMM
                dphi^T diag(w D) dphi on FP64 MFMA (assembly = 1), timed for one step; its
                assembly kernel's roofline counts Q M (M+1) flops per unit (the M(M+1)/2
                distinct entries of the symmetric stiffness, 2Q flops each).
  cpu_baseline  the CPU oracle (plain serial C) timed on this host's cores on a bounded
                sample: the first slice (64 fine steps) of 16 instances of the alpha = 0.3
                batch, one instance per thread.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8-rel solution: learned-G vs plain-G parareal; mode-steps/s"
PEAK_FP64_MFMA_TFLOPS = 78.6
TARGET = 1e-8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_err_max(its_k, Us):
    # max over instances of ||U^k_b - U_b|| / ||U_b||
    d = (its_k - Us).flatten(1).norm(dim=1)
    n = Us.flatten(1).norm(dim=1)
    return float((d / n).max())


def cpu_baseline(kw, u0_np, n_inst):
    import concurrent.futures as cf

    import oracle

    oracle.lib()
    po = oracle.problem(**kw)
    S = kw["steps"] // kw["slices"]
    threads = max(1, min(16, os.cpu_count() or 1, n_inst))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda b: oracle.fine_F(po, 0, u0_np[b:b + 1]), range(n_inst)))
    dt = time.perf_counter() - t0
    mode_steps = n_inst * S * kw["modes"]
    return {"value": mode_steps / dt, "unit": "mode-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle serial fine propagator, first slice ({S} steps) of {n_inst} "
                      f"alpha={kw['alpha']} instances, one instance per thread, {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["full", "kernels"], default="full",
                    help="kernels: one parareal sweep of the alpha=0.3 batch and a 1 GiB plain "
                         "device copy (for hardware-counter runs); prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_11023_amd as l1
    from paper_2510_11023_amd import _lib
    from paper_2510_11023_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = dict(W.C2)
    M, N, P, Q = base["modes"], base["steps"], base["slices"], base["quad"]
    B, alphas = W.C2_BATCH, W.C2_ALPHAS
    u0_np = W.u0_batch_1d(M, range(B))
    u0 = torch.tensor(u0_np, dtype=torch.float64, device=dev)
    probs = {a: l1.make_problem(**W.with_(base, alpha=a)) for a in alphas}
    probs_gemm = {a: l1.make_problem(assembly=1, **W.with_(base, alpha=a)) for a in alphas}
    p0 = probs[alphas[0]]
    ws_par = torch.empty(l1.workspace_bytes(p0, B, 1), dtype=torch.uint8, device=dev)
    ws_ser = torch.empty(l1.workspace_bytes(p0, B, 0), dtype=torch.uint8, device=dev)
    log(f"workspace: parareal {ws_par.numel() / 2**30:.2f} GiB, serial {ws_ser.numel() / 2**20:.0f} MiB")

    if args.mode == "kernels":
        # one coarse sweep + one fine sweep + one correction sweep, then a plain copy of
        # 2^27 doubles (1 GiB read + 1 GiB written) that calibrates the byte counters
        l1.solve_parareal(probs[alphas[0]], u0, 1, tol=0.0, workspace=ws_par)
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("kernels mode done")
        return

    # serial reference and its time
    Us, t_serial = {}, {}
    for a in alphas:
        l1.solve_serial(probs[a], u0, workspace=ws_ser)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, _ = l1.solve_serial(probs[a], u0, workspace=ws_ser)
        torch.cuda.synchronize()
        t_serial[a] = time.perf_counter() - t0
        Us[a] = U
        log(f"serial alpha={a}: {t_serial[a] * 1e3:.1f} ms")

    # k*(alpha): first sweep count whose iterate is within 1e-8 of the serial solution
    kstar, errs = {}, {}
    for a in alphas:
        res = l1.solve_parareal(probs[a], u0, P, tol=1e-11, want_iterates=True, workspace=ws_par)
        torch.cuda.synchronize()
        e = [rel_err_max(res.iterates[k], Us[a]) for k in range(res.iters + 1)]
        ks = next((k for k, v in enumerate(e) if v <= TARGET), None)
        if ks is None:
            ks = P  # exact after P sweeps
        kstar[a] = max(ks, 1)
        errs[a] = e
        log(f"parareal alpha={a}: k*={kstar[a]} errors " + " ".join(f"{v:.1e}" for v in e[: kstar[a] + 1]))

    def step(pr=probs):
        out = {}
        for a in alphas:
            out[a] = l1.solve_parareal(pr[a], u0, kstar[a], tol=0.0, want_incr=False,
                                       workspace=ws_par).U
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = _lib.profile_stop()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    achieved_err = {a: rel_err_max(out[a], Us[a]) for a in alphas}
    log(f"timed: {ms_per_step:.1f} ms/step; error vs serial " + str(achieved_err))
    for k in sorted(stats):
        n, tot = stats[k]
        log(f"  {k:32s} launches {n:7d}  avg {tot / n * 1e3:9.1f} us  total {tot:9.1f} ms")

    useful = len(alphas) * B * M * N
    value = useful / (ms_per_step / 1e3)
    executed = sum(kstar[a] for a in alphas) * B * M * N
    serial_total = sum(t_serial.values())

    # dominant kernel: the fine-sweep step kernel
    units = B * P
    key = f"step/fine/{units}"
    n_l, tot_l = stats.get(key, (0, 0.0))
    roofline = None
    if n_l:
        avg_s = tot_l / n_l / 1e3
        per_unit = M ** 3 / 3 + M ** 2 / 2 + M / 6 + 2 * M ** 2 + 4 * M * Q + 2 * (2 * M + 1) * Q
        flops = units * per_unit
        achieved = flops / avg_s / 1e12
        roofline = {"bound": "mfma", "kernel": "k_step1d_reg<moments> (fine sweep, 2048 units)",
                    "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4),
                    "avg_launch_ms": round(avg_s * 1e3, 4), "flops_per_launch": int(flops),
                    "traffic": None}
    share = {k: round(v[1] / sum(x[1] for x in stats.values()), 4) for k, v in stats.items()}

    # the same step with the quadrature-GEMM stiffness (assembly = 1)
    step(probs_gemm)
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    out_g = step(probs_gemm)
    torch.cuda.synchronize()
    t_gemm = time.perf_counter() - t0
    stats_g = _lib.profile_stop()
    n_a, tot_a = stats_g.get(f"assemble/fine/{units}", (0, 0.0))
    gemm = {"ms_per_step": t_gemm * 1e3,
            "achieved_rel_err": {str(a): rel_err_max(out_g[a], Us[a]) for a in alphas}}
    if n_a:
        avg_a = tot_a / n_a / 1e3
        fl = units * Q * M * (M + 1)
        gemm["assemble_roofline"] = {
            "bound": "mfma", "kernel": "k_assemble1d<64> (fine sweep, 2048 units)",
            "achieved": round(fl / avg_a / 1e12, 3), "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s", "frac": round(fl / avg_a / 1e12 / PEAK_FP64_MFMA_TFLOPS, 4),
            "avg_launch_ms": round(avg_a * 1e3, 4), "flops_per_launch": fl}
    for k in sorted(stats_g):
        n, tot = stats_g[k]
        log(f"  gemm {k:27s} launches {n:7d}  avg {tot / n * 1e3:9.1f} us  total {tot:9.1f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(W.with_(base, alpha=alphas[0]), u0_np, 16)
        log(f"cpu baseline: {cpu['value']:.3g} mode-steps/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "mode-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "config2: 1D, M=256, Q=384, N=4096, P=64, D=1+1/(1+u^2), f=0.1u(1-u), "
                        "alpha in {0.3,0.7,1.0} x 32 instances (seeds 0..31); plain-G parareal "
                        "run to 1e-8 relative of the serial solution",
            "coarse": "plain L1 (learned G not in this line)",
            "kstar": {str(a): kstar[a] for a in alphas},
            "achieved_rel_err": {str(a): achieved_err[a] for a in alphas},
        },
        "time_to_1e8_ms": ms_per_step,
        "serial_ms": serial_total * 1e3,
        "serial_mode_steps_per_s": useful / serial_total,
        "executed_mode_steps_per_s": executed / (ms_per_step / 1e3),
        "kernel_time_share": share,
        "roofline": roofline,
        "gemm_assembly": gemm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
