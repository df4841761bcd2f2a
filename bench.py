#!/usr/bin/env python
"""Benchmark of the parareal / L1 / sine-Galerkin solver on one MI355X.

Main workload (1D): D = 1 + 1/(1+u^2), f = 0.1 u (1-u), M = 256 sine modes, Q = 384 Gauss
points, N = 4096 fine L1 steps, P = 64 parareal slices, three batched runs (alpha = 0.3,
0.7, 1.0) of 32 instances each, u0 coefficients c_k ~ N(0, k^-3) (seeds 0..31).  Synthetic,
seeded inputs.

One step = the three batched parareal solves (plain coarse L1 propagator G) run to the
iteration count k*(alpha) at which every instance's slice ends are within 1e-8 (relative
L2 over all P+1 slice ends) of the serial solution.  k* is found before the timed region
from the GPU serial solution (itself parity-checked against the CPU oracle by the tests)
and the parareal iterates.  Metric value: useful mode-steps/s = sum_b M N / time-to-1e-8.

The JSON line also carries:
  roofline        the dominant kernel, the register-resident factor-and-solve kernel of the
                  fine sweep (2048 units per launch).  Algorithmic flops per unit =
                  M^3/3 + M^2/2 + M/6 (Cholesky) + 2 M^2 (two triangular solves), divided by
                  the average launch time measured with HIP events on the launch stream over
                  the timed region; peak = 78.6 TFLOP/s (MI355X dense FP64).  traffic = HBM
                  bytes per launch from the FETCH_SIZE and WRITE_SIZE counters, scaled by
                  what the counters read for a plain device copy, recorded for the kernel
                  source with the hash below (null once the source differs).
  history_hbm     the L1 history-sum kernel of the fine sweep: algorithmic bytes per sweep
                  (every unit's trajectory rows 0..r-1, each instance's slice ends once, the
                  output rows) over its summed launch time, against 8 TB/s.
  gemm_assembly   the same step with the stiffness formed as the quadrature GEMM
                  dphi^T diag(w D) dphi on FP64 MFMA (assembly = 1); its assembly kernel's
                  roofline counts Q M (M+1) flops per unit (the M(M+1)/2 distinct entries of
                  the symmetric stiffness, 2Q flops each).
  uneven_batch    256 instances with their own modes, steps per slice and order, grouped by
                  padded mode count, all groups' parareal runs in one HIP graph (one branch per
                  group, tiles autotuned per group); useful mode-steps/s and per-instance
                  latency percentiles from device stamps at each instance's convergence sweep.
  learned_vs_plain  the learned-coarse workload: 1D, M = 128, Q = 192, N = 2048, P = 64,
                  alpha ~ U(0.2, 1), D and f as above; the residual network is trained on
                  4096 seeded serial trajectories (one-off, untimed but reported), then plain
                  and learned parareal are each run to 1e-8 of the serial solution on 64
                  held-out instances and timed.
  config3_2d      the 2D workload: 64 x 64 tensor sine modes (4096 coefficients), 96 x 96 Gauss
                  points, N = 2048, P = 128, alpha = 0.6, D = 1 + exp(-u^2)/2, f = sin u: one
                  fine sweep over all 128 slices (16 steps of 128 systems of size 4096 through
                  the blocked device-memory factorisation), with its FP64 rate against the
                  78.6 TFLOP/s peak (M^3/3 + M^2/2 + M/6 + 2 M^2 flops per system); the serial
                  solve; plain parareal run to 1e-8 of the serial solution.
  cpu_baseline    the CPU oracle (plain serial C) timed on this host's cores on a bounded
                  sample: the first slice (64 fine steps) of 16 instances of the alpha = 0.3
                  batch, one instance per thread.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8-rel solution: learned-G vs plain-G parareal; mode-steps/s"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
TARGET = 1e-8

# HBM traffic of the fine-sweep factor-and-solve kernel, per full launch (2048 units), from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE on `python bench.py --mode kernels`, divided by
# the counters' reading for a plain copy of known size (fetch and write factors below).
# Valid only for the kernel sources and build flags with this hash.
TRAFFIC_SOURCES = ("paper_2510_11023_amd/csrc/step1d_reg.hip", "paper_2510_11023_amd/csrc/l1pr_internal.h",
                   "paper_2510_11023_amd/build.py")
TRAFFIC_RECORD = {"sha256": "b2229fb70e4db912dd049b76d91d20f06c8d8463067e94761883de4c68135b6e",
                  "fetch_kib": 8721.5, "write_kib": 4096, "fetch_factor": 2.0, "write_factor": 1.0,
                  "bytes_per_launch": int((2 * 8721.5 + 4096) * 1024)}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_hash():
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def rel_err_max(its_k, Us):
    # max over instances of ||U^k_b - U_b|| / ||U_b||
    d = (its_k - Us).flatten(1).norm(dim=1)
    n = Us.flatten(1).norm(dim=1)
    return float((d / n).max())


def cpu_baseline(kw, u0_np, n_inst, min_seconds=10.0):
    """The oracle's fine propagator on the first slice of n_inst instances, one instance per
    thread, repeated until about min_seconds of wall time have passed."""
    import concurrent.futures as cf

    import oracle

    oracle.lib()
    po = oracle.problem(**kw)
    S = kw["steps"] // kw["slices"]
    threads = max(1, min(16, os.cpu_count() or 1, n_inst))
    rounds = 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        while True:
            list(ex.map(lambda b: oracle.fine_F(po, 0, u0_np[b:b + 1]), range(n_inst)))
            rounds += 1
            if time.perf_counter() - t0 >= min_seconds or rounds >= 64:
                break
    dt = time.perf_counter() - t0
    mode_steps = rounds * n_inst * S * kw["modes"]
    return {"value": mode_steps / dt, "unit": "mode-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle serial fine propagator, first slice ({S} steps, M={kw['modes']}) of "
                      f"{n_inst} alpha={kw['alpha']} instances, one instance per thread, "
                      f"{rounds} rounds, {dt:.1f} s wall"}


def find_kstar(l1, p, u0, Us, ws, max_iter, **kw):
    res = l1.solve_parareal(p, u0, max_iter, tol=0.0, want_iterates=True, workspace=ws, **kw)
    e = [rel_err_max(res.iterates[k], Us) for k in range(res.iters + 1)]
    ks = next((k for k, v in enumerate(e) if v <= TARGET), None)
    return ks, e


def learned_vs_plain(l1, torch, W, dev):
    from paper_2510_11023_amd.learned import LearnedCoarse, training_data

    kw = dict(W.C4)
    M, N, P = kw["modes"], kw["steps"], kw["slices"]
    p = l1.make_problem(**kw)
    ntrain, epochs = len(W.C4_TRAIN_SEEDS), 10
    t0 = time.perf_counter()
    model = LearnedCoarse(M, seed=0)
    ta = W.alphas_uniform(ntrain, W.C4_TRAIN_ALPHA_SEED)
    u0t = torch.tensor(W.u0_batch_1d(M, W.C4_TRAIN_SEEDS), device=dev)
    x, t = training_data(p, u0t, ta, model, sweeps=W.C4_TRAIN_SWEEPS)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    nsamples = x.shape[0]
    model.set_stats(x, t)
    t0 = time.perf_counter()
    losses = model.train(x, t, epochs=epochs, batch=1024, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, t, u0t
    log(f"learned G: data {t_data:.1f} s, training {t_train:.1f} s, loss {losses[0]:.3g} -> {losses[-1]:.3g}")
    # training work on BF16 MFMA: forward 2 (in_p H + 2 H^2 + H out_p) per sample at the padded
    # widths the kernels multiply, backward twice that (input and weight gradients)
    i = model.info
    fwd = 2 * (i.in_padded * i.hidden + 2 * i.hidden * i.hidden + i.hidden * i.out_padded)
    train_flops = 3 * fwd * (nsamples // 1024) * 1024 * epochs
    bf16 = {"bound": "mfma", "achieved": round(train_flops / t_train / 1e12, 3), "peak": PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s", "frac": round(train_flops / t_train / 1e12 / PEAK_BF16_TFLOPS, 5),
            "flops": train_flops, "note": "whole training loop over its wall time (BF16 MFMA "
            "16x16x16, FP32 accumulation; launch-bound at batch 1024)"}

    ea = [float(a) for a in W.alphas_uniform(len(W.C4_EVAL_SEEDS), W.C4_EVAL_ALPHA_SEED)]
    u0 = torch.tensor(W.u0_batch_1d(M, W.C4_EVAL_SEEDS), device=dev)
    B = u0.shape[0]
    Us, _ = l1.solve_serial(p, u0, alpha=ea)
    ws = l1.parareal_workspace(p, B, dev, learned=True)
    out = {"workload": f"1D, M={M}, Q={kw['quad']}, N={N}, P={P}, D=1+1/(1+u^2), f=0.1u(1-u), "
                       f"{B} held-out instances with alpha~U(0.2,1); network 3x512 SiLU, "
                       f"trained on {ntrain} seeded serial trajectories and their first "
                       f"{W.C4_TRAIN_SWEEPS} plain parareal iterates ({nsamples} samples)",
           "train": {"data_s": round(t_data, 2), "train_s": round(t_train, 2), "epochs": epochs,
                     "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1]),
                     "bf16_roofline": bf16}}
    for name, extra in (("plain", {}), ("learned", {"coarse": l1.COARSE_LEARNED, "mlp_params": model.params})):
        ks, e = find_kstar(l1, p, u0, Us, ws, 30, alpha=ea, **extra)
        log(f"{name} G: k*={ks} errors " + " ".join(f"{v:.1e}" for v in e[: (ks or 30) + 1]))
        rec = {"kstar": ks, "rel_err_by_sweep": [float(f"{v:.3e}") for v in e[: (ks or 30) + 1]]}
        if ks is not None:
            run = lambda: l1.solve_parareal(p, u0, ks, alpha=ea, tol=0.0, want_incr=False,
                                            workspace=ws, **extra)
            run()
            torch.cuda.synchronize()
            times = []
            for _ in range(3):
                t0 = time.perf_counter()
                U = run().U
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            tm = sorted(times)[1]
            rec.update({"ms": round(tm * 1e3, 2), "mode_steps_per_s": B * M * N / tm,
                        "achieved_rel_err": rel_err_max(U, Us)})
        out[name] = rec
    if out["plain"].get("ms") and out["learned"].get("ms"):
        out["speedup_learned_over_plain"] = round(out["plain"]["ms"] / out["learned"]["ms"], 3)
    return out


def c5_network(l1, torch, W, dev, log_prefix="uneven learned G"):
    """One residual network of 256 modes for the whole uneven workload: trained on plain-G
    pairs of config-5-type problems (u0 = sin(pi x), D = 1 + sin^2(u)/2, manufactured f) at
    M in {64, 128, 192, 256}, Q = 2M, S in {8, 24, 40, 64} (64 seeded orders each; serial
    trajectories and the first three plain parareal iterates), the coefficients a problem
    does not carry padded with zeros."""
    import numpy as np

    from paper_2510_11023_amd.learned import LearnedCoarse, training_data_padded

    t0 = time.perf_counter()
    model = LearnedCoarse(256, seed=0)
    xs, ts = [], []
    k = 0
    for M in (64, 128, 192, 256):
        for S in (8, 24, 40, 64):
            p = l1.make_problem(**W.with_(W.C5, modes=M, quad=2 * M, steps=W.C5["slices"] * S))
            u0 = torch.zeros((64, M), dtype=torch.float64, device=dev)
            u0[:, 0] = 2.0 ** -0.5
            al = W.alphas_uniform(64, seed=7000 + k)
            x, t = training_data_padded(p, u0, al, model, sweeps=3)
            xs.append(x)
            ts.append(t)
            k += 1
    x, t = torch.cat(xs), torch.cat(ts)
    del xs, ts
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    model.set_stats(x, t)
    t0 = time.perf_counter()
    losses = model.train(x, t, epochs=10, batch=1024, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n = x.shape[0]
    del x, t
    log(f"{log_prefix}: data {t_data:.1f} s, training {t_train:.1f} s ({n} samples), "
        f"loss {losses[0]:.3g} -> {losses[-1]:.3g}")
    return model, {"data_s": round(t_data, 2), "train_s": round(t_train, 2), "samples": int(n),
                   "epochs": 10, "loss_first_epoch": float(losses[0]),
                   "loss_last_epoch": float(losses[-1])}


def uneven_batch(l1, torch, W, dev, learned_model=None):
    """Config 5: 256 instances with their own modes, steps per slice and order, grouped by
    padded mode count; every group's parareal run is one branch of a single HIP graph; each
    instance stops at its first sweep whose increment is <= 1e-8 (its units then return at
    entry).  Plain coarse step, then (with a network) the learned one with the plain step as
    fallback."""
    import numpy as np

    from paper_2510_11023_amd import solver

    modes, spp, alpha = W.c5_instances()
    P = W.C5["slices"]
    mp = (modes + 15) // 16 * 16
    groups = []
    t_ser = 0.0
    for Mp in sorted(set(mp.tolist())):
        idx = np.nonzero(mp == Mp)[0]
        B = len(idx)
        kw = W.with_(W.C5, modes=int(Mp), quad=2 * int(Mp), steps=P * int(spp[idx].max()))
        p = l1.make_problem(**kw)
        ws = solver.uneven_workspace(p, B, dev, learned=learned_model is not None)
        p.tune = l1.autotune(p, B, workspace=ws)
        u0 = torch.zeros((B, int(Mp)), dtype=torch.float64, device=dev)
        u0[:, 0] = 2.0 ** -0.5
        g = dict(idx=idx, p=p, ws=ws, u0=u0, B=B, Mp=int(Mp),
                 modes=torch.tensor(modes[idx], dtype=torch.int32, device=dev),
                 spp=torch.tensor(spp[idx], dtype=torch.int32, device=dev),
                 alpha=torch.tensor(alpha[idx], dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g["Us"] = l1.solve_serial_uneven(p, u0, g["modes"], g["spp"], g["alpha"])
        torch.cuda.synchronize()
        t_ser += time.perf_counter() - t0
        groups.append(g)
    useful = float((modes.astype(np.int64) * P * spp).sum())
    cap, tol = 24, 1e-8

    def graph_run(extra):
        # sweeps per group: until every instance's increment is <= 1e-8 (capped), found untimed
        for g in groups:
            U, conv, _ = l1.solve_parareal_uneven(g["p"], g["u0"], cap, g["modes"], g["spp"],
                                                  g["alpha"], conv_tol=tol, workspace=g["ws"], **extra)
            c = conv.cpu().numpy()
            g["sweeps"] = int(cap if (c < 0).any() else c.max())
            g["out"] = torch.empty_like(U)
            g["conv"] = torch.empty(g["B"], dtype=torch.int32, device=dev)
            g["stamps"] = torch.zeros(g["sweeps"] + 1, dtype=torch.int64, device=dev)
            g["stream"] = torch.cuda.Stream()
        t_start = torch.zeros(1, dtype=torch.int64, device=dev)

        def run_all():
            solver.device_stamp(t_start)
            main = torch.cuda.current_stream()
            for g in groups:
                g["stream"].wait_stream(main)
                with torch.cuda.stream(g["stream"]):
                    l1.solve_parareal_uneven(g["p"], g["u0"], g["sweeps"], g["modes"], g["spp"],
                                             g["alpha"], conv_tol=tol, workspace=g["ws"],
                                             out=g["out"], conv=g["conv"], stamps=g["stamps"],
                                             **extra)
            for g in groups:
                main.wait_stream(g["stream"])

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run_all()  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            run_all()
        graph.replay()
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            graph.replay()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t_graph = sorted(times)[1]
        khz = solver.wall_clock_khz()
        lat, err, sweeps_inst = [], 0.0, []
        t0d = int(t_start.item())
        for g in groups:
            conv = g["conv"].cpu().numpy()
            st = g["stamps"].cpu().numpy()
            for b in range(g["B"]):
                k = conv[b] if conv[b] > 0 else g["sweeps"]
                sweeps_inst.append(int(k))
                lat.append((st[k] - t0d) / khz)  # ms
            d = (g["out"] - g["Us"]).flatten(1).norm(dim=1) / g["Us"].flatten(1).norm(dim=1)
            err = max(err, float(d.max()))
        lat = np.array(lat)
        del graph
        return {"graph_ms": round(t_graph * 1e3, 2), "useful_mode_steps_per_s": useful / t_graph,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                               "p99": float(np.percentile(lat, 99))},
                "mean_sweeps_per_instance": float(np.mean(sweeps_inst)),
                "groups": [{"Mp": g["Mp"], "instances": g["B"], "sweeps": g["sweeps"], "tune": g["p"].tune}
                           for g in groups],
                "max_rel_err_vs_serial": err}

    plain = graph_run({})
    log(f"uneven batch, plain G: {len(groups)} groups, graph {plain['graph_ms']:.1f} ms, serial "
        f"{t_ser * 1e3:.1f} ms, error vs serial {plain['max_rel_err_vs_serial']:.2e}, mean sweeps "
        f"{plain['mean_sweeps_per_instance']:.2f}")
    out = {"workload": "256 instances, P=64, M~U{64..256}, S~U{8..64} (N=64 S), alpha~U(0.2,1), "
                       "D=1+sin^2(u)/2, manufactured f, u0=sin(pi x); grouped by roundup16(M) "
                       "(Q = 2 roundup16(M)); one HIP graph with one branch per group; each "
                       "instance stops at its first sweep with increment <= 1e-8",
           "serial_ms": round(t_ser * 1e3, 2), "plain": plain,
           # the headline fields keep their former names (plain coarse step)
           "graph_ms": plain["graph_ms"], "useful_mode_steps_per_s": plain["useful_mode_steps_per_s"],
           "latency_ms": plain["latency_ms"], "max_rel_err_vs_serial": plain["max_rel_err_vs_serial"]}
    if learned_model is not None:
        model, train = learned_model
        lr = graph_run({"coarse": l1.COARSE_LEARNED, "mlp_params": model.params, "mlp_modes": 256})
        lr["train"] = train
        out["learned"] = lr
        out["speedup_learned_over_plain"] = round(plain["graph_ms"] / lr["graph_ms"], 3)
        log(f"uneven batch, learned G: graph {lr['graph_ms']:.1f} ms, error vs serial "
            f"{lr['max_rel_err_vs_serial']:.2e}, mean sweeps {lr['mean_sweeps_per_instance']:.2f}")
    return out


def config3_2d(l1, torch, W, dev, with_parareal=True):
    """Config 3 (2D): fine-sweep throughput of the blocked device-memory factorisation, the
    serial solve, and plain parareal to 1e-8 of the serial solution."""
    from paper_2510_11023_amd import _lib

    kw = dict(W.C3)
    M1, N, P = kw["modes"], kw["steps"], kw["slices"]
    Md, S = M1 * M1, N // P
    p = l1.make_problem(**kw)
    u0 = torch.tensor(W.u0_random_2d(M1, 0)[None], device=dev)
    ws = l1.parareal_workspace(p, 1, dev)
    log(f"config 3: workspace {ws.numel() / 2**30:.1f} GiB")
    # one fine sweep over all P slices from the coarse initial guess (P units per step)
    Z = l1.solve_parareal(p, u0, 0, tol=0.0, want_iterates=True, workspace=ws).iterates[0]
    Z = Z.contiguous()
    l1.fine_apply(p, Z, workspace=ws)
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    l1.fine_apply(p, Z, workspace=ws)
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t0
    st = _lib.profile_stop()
    n_s, tot_s = st.get(f"blk_solve/fine/{P}", (0, 0.0))
    per_unit = Md ** 3 / 3 + Md ** 2 / 2 + Md / 6 + 2 * Md ** 2  # Cholesky + two triangular solves
    out = {"workload": f"2D, {M1}x{M1} modes (Md={Md}), {kw['quad']}x{kw['quad']} Gauss points, N={N}, "
                       f"P={P} (S={S}), alpha={kw['alpha']}, D=1+exp(-u^2)/2, f=sin(u), "
                       f"u0 c_k1k2 ~ N(0,(k1^2+k2^2)^-1.5) seed 0",
           "fine_sweep_ms": round(t_sweep * 1e3, 1),
           "fine_sweep_mode_steps_per_s": P * S * Md / t_sweep,
           "fine_sweep_tflops": round(P * S * per_unit / t_sweep / 1e12, 2)}
    if n_s:
        avg = tot_s / n_s / 1e3
        ach = P * per_unit / avg / 1e12
        out["solve_roofline"] = {"bound": "mfma", "kernel": f"blocked factorisation and solve "
                                 f"(k_blk_diag, k_blk_panel, k_blk_trail, k_blk_bs_*), {P} units per step",
                                 "achieved": round(ach, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(ach / PEAK_FP64_TFLOPS, 4), "avg_step_ms": round(avg * 1e3, 2),
                                 "flops_per_step": int(P * per_unit)}
    share = {k: round(v[1] / sum(x[1] for x in st.values()), 4) for k, v in st.items()}
    out["fine_sweep_share"] = share
    log(f"config 3: fine sweep {t_sweep * 1e3:.0f} ms ({out['fine_sweep_tflops']} TFLOP/s)")
    ws_s = torch.empty(l1.workspace_bytes(p, 1, 0), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Us, _ = l1.solve_serial(p, u0, workspace=ws_s)
    torch.cuda.synchronize()
    t_ser = time.perf_counter() - t0
    out["serial_ms"] = round(t_ser * 1e3, 1)
    out["serial_mode_steps_per_s"] = N * Md / t_ser
    log(f"config 3: serial {t_ser * 1e3:.0f} ms")
    del ws_s
    if with_parareal:
        ks, e = find_kstar(l1, p, u0, Us, ws, 14)
        rec = {"kstar": ks, "rel_err_by_sweep": [float(f"{v:.3e}") for v in e]}
        if ks is not None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U = l1.solve_parareal(p, u0, ks, tol=0.0, want_incr=False, workspace=ws).U
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            rec.update({"ms": round(tp * 1e3, 1), "mode_steps_per_s": N * Md / tp,
                        "achieved_rel_err": rel_err_max(U, Us)})
        out["parareal_plain"] = rec
        log(f"config 3: parareal k*={ks} " + (f"{rec.get('ms')} ms" if ks is not None else ""))
    out["conjugate_gradients"] = config3_cg(l1, torch, W, dev, Us)
    return out


def config3_cg(l1, torch, W, dev, Us_direct=None):
    """Config 3 with the step systems solved by preconditioned conjugate gradients
    (solver = 1): fine sweep, serial solve and plain parareal to 1e-8 of that serial
    solution; the stiffness products' MFMA rate; agreement with the Cholesky path."""
    from paper_2510_11023_amd import _lib

    kw = dict(W.C3)
    M1, N, P = kw["modes"], kw["steps"], kw["slices"]
    Md, S, Q = M1 * M1, N // P, kw["quad"]
    p = l1.make_problem(solver=1, **kw)
    u0 = torch.tensor(W.u0_random_2d(M1, 0)[None], device=dev)
    ws = l1.parareal_workspace(p, 1, dev)
    Z = l1.solve_parareal(p, u0, 0, tol=0.0, want_iterates=True, workspace=ws).iterates[0]
    Z = Z.contiguous()
    l1.fine_apply(p, Z, workspace=ws)
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    l1.fine_apply(p, Z, workspace=ws)
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t0
    st = _lib.profile_stop()
    out = {"workload": "config 3 with solver = 1 (conjugate gradients)",
           "workspace_gib": round(ws.numel() / 2 ** 30, 3),
           "fine_sweep_ms": round(t_sweep * 1e3, 1),
           "fine_sweep_mode_steps_per_s": P * S * Md / t_sweep}
    n_a, tot_a = st.get(f"cg_grid/fine/{P}", (0, 0.0))
    n_u, tot_u = st.get(f"cg_step/fine/{P}", (0, 0.0))
    if n_a and n_u:
        avg = (tot_a / n_a + tot_u / n_u) / 1e3
        fl = P * 2 * (4 * Q * M1 * M1 + 4 * Q * Q * M1)
        out["apply_roofline"] = {"bound": "mfma", "kernel": f"separable stiffness product and CG "
                                 f"update (k_stiff2d_grid, k_cg_part, k_cg_step; {P} units)",
                                 "achieved": round(fl / avg / 1e12, 2), "peak": PEAK_FP64_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(fl / avg / 1e12 / PEAK_FP64_TFLOPS, 4),
                                 "avg_apply_us": round(avg * 1e6, 1), "flops_per_apply": fl}
        out["cg_iterations_per_step"] = round((n_u - S) / S, 2)
    tot = sum(v[1] for v in st.values())
    out["fine_sweep_share"] = {k: round(v[1] / tot, 4) for k, v in st.items()}
    ws_s = torch.empty(l1.workspace_bytes(p, 1, 0), dtype=torch.uint8, device=dev)
    l1.solve_serial(p, u0, workspace=ws_s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Us, _ = l1.solve_serial(p, u0, workspace=ws_s)
    torch.cuda.synchronize()
    t_ser = time.perf_counter() - t0
    out["serial_ms"] = round(t_ser * 1e3, 1)
    out["serial_mode_steps_per_s"] = N * Md / t_ser
    if Us_direct is not None:
        out["rel_diff_vs_cholesky_serial"] = rel_err_max(Us, Us_direct)
    ks, e = find_kstar(l1, p, u0, Us, ws, 14)
    rec = {"kstar": ks, "rel_err_by_sweep": [float(f"{v:.3e}") for v in e]}
    if ks is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U = l1.solve_parareal(p, u0, ks, tol=0.0, want_incr=False, workspace=ws).U
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        rec.update({"ms": round(tp * 1e3, 1), "mode_steps_per_s": N * Md / tp,
                    "achieved_rel_err": rel_err_max(U, Us), "speedup_over_serial": round(t_ser / tp, 2)})
    out["parareal_plain"] = rec
    log(f"config 3 (CG): fine sweep {t_sweep * 1e3:.0f} ms, serial {t_ser * 1e3:.0f} ms, "
        f"parareal k*={ks} {rec.get('ms')} ms")
    return out


def median_time(torch, fn, reps=5):
    fn()
    torch.cuda.synchronize()
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], out


def config1_latency(l1, torch, W, dev):
    """Config 1 (one instance, M = 32, N = 256, P = 8): serial and parareal latency; parareal
    stops at its first sweep whose increment is <= 1e-8 (the flowchart's test)."""
    kw = dict(W.C1)
    M, N, P = kw["modes"], kw["steps"], kw["slices"]
    p = l1.make_problem(**kw)
    u0 = torch.tensor(W.u0_sine_mode(M)[None, :], device=dev)
    t_ser, (Us, _) = median_time(torch, lambda: l1.solve_serial(p, u0))
    t_par, r = median_time(torch, lambda: l1.solve_parareal(p, u0, P, tol=1e-8))
    err = rel_err_max(r.U, Us)
    log(f"config 1: serial {t_ser * 1e3:.2f} ms, parareal {t_par * 1e3:.2f} ms ({r.iters} sweeps, "
        f"error vs serial {err:.1e})")
    return {"workload": f"1D, M={M}, Q={kw['quad']}, N={N}, P={P}, alpha={kw['alpha']}, "
                        "D=1+sin^2(u)/2, manufactured f, u0=sin(pi x), one instance",
            "serial_ms": round(t_ser * 1e3, 3), "parareal_ms": round(t_par * 1e3, 3),
            "parareal_sweeps": r.iters, "parareal_rel_err_vs_serial": err,
            "serial_mode_steps_per_s": M * N / t_ser, "parareal_mode_steps_per_s": M * N / t_par,
            "stop": "per-instance increment <= 1e-8"}


def soe_history(l1, torch, W, dev, alpha=0.3):
    """The sum-of-exponentials far history (history = 2) against the exact full history
    (history = 1) on the config-2 batch, serial solves at N = 4096 and 16384: wall time, the
    history kernel's time per step, and the gap between the two solutions."""
    from paper_2510_11023_amd import _lib

    B, M = W.C2_BATCH, 256
    u0 = torch.tensor(W.u0_batch_1d(M, range(B)), dtype=torch.float64, device=dev)
    out = {"workload": f"1D, M={M}, Q=384, P=64, alpha={alpha}, {B} instances, config-2 D and f, "
                       "serial solve with the full uniform L1 history: exact (history 1, prefix "
                       "blocks of 64 steps) against the sum-of-exponentials far history (history 2)",
           "runs": []}
    for N in (4096, 16384):
        rec = {"steps": N}
        res = {}
        for h in (1, 2):
            p = l1.make_problem(**W.with_(W.C2, alpha=alpha, steps=N, history=h))
            ws = torch.empty(l1.workspace_bytes(p, B, 0), dtype=torch.uint8, device=dev)
            l1.solve_serial(p, u0, workspace=ws)
            torch.cuda.synchronize()
            _lib.profile_start(only=("history", "prefix"))
            t0 = time.perf_counter()
            U, _ = l1.solve_serial(p, u0, workspace=ws)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st = _lib.profile_stop()
            hist_ms = sum(v[1] for k, v in st.items())
            res[h] = U
            key = "exact" if h == 1 else "soe"
            rec[key] = {"ms": round(t * 1e3, 1), "mode_steps_per_s": B * M * N / t,
                        "history_us_per_step": round(hist_ms * 1e3 / N, 2),
                        "workspace_mib": round(ws.numel() / 2**20, 1)}
            del ws
        if 2 in res:
            rec["rel_gap_soe_vs_exact"] = rel_err_max(res[2], res[1])
        out["runs"].append(rec)
        log(f"soe history N={N}: exact {rec['exact']['ms']} ms ({rec['exact']['history_us_per_step']} us/step), "
            f"soe {rec['soe']['ms']} ms ({rec['soe']['history_us_per_step']} us/step), gap {rec['rel_gap_soe_vs_exact']:.1e}")
    return out


def full_history(l1, torch, W, dev, alpha=0.3):
    """Full-history parareal on the config-2 batch (one alpha): its fixed point is the uniform
    L1 solution with full history (the full-history serial solve); sweeps to 1e-8 of it, wall
    time of both, and the per-sweep prefix kernel against the FP64 vector peak."""
    from paper_2510_11023_amd import _lib

    kw = W.with_(W.C2, alpha=alpha, history=1)
    M, N, P = kw["modes"], kw["steps"], kw["slices"]
    S, B = N // P, W.C2_BATCH
    p = l1.make_problem(**kw)
    u0 = torch.tensor(W.u0_batch_1d(M, range(B)), dtype=torch.float64, device=dev)
    ws = torch.empty(l1.workspace_bytes(p, B, 1), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(l1.workspace_bytes(p, B, 0), dtype=torch.uint8, device=dev)
    l1.solve_serial(p, u0, workspace=ws_s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Us, _ = l1.solve_serial(p, u0, workspace=ws_s)
    torch.cuda.synchronize()
    t_ser = time.perf_counter() - t0
    del ws_s
    ks, e = find_kstar(l1, p, u0, Us, ws, 24)
    out = {"workload": f"1D, M={M}, Q={kw['quad']}, N={N}, P={P}, alpha={alpha}, {B} instances "
                       f"(seeds 0..{B - 1}), config-2 D and f, full-history fine propagator",
           "serial_ms": round(t_ser * 1e3, 1), "serial_mode_steps_per_s": B * M * N / t_ser,
           "kstar": ks, "rel_err_by_sweep": [float(f"{v:.3e}") for v in e]}
    k = ks if ks is not None else P
    l1.solve_parareal(p, u0, k, tol=0.0, want_incr=False, workspace=ws)
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    U = l1.solve_parareal(p, u0, k, tol=0.0, want_incr=False, workspace=ws).U
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    st = _lib.profile_stop()
    out.update({"parareal_ms": round(tp * 1e3, 1), "mode_steps_per_s": B * M * N / tp,
                "achieved_rel_err": rel_err_max(U, Us), "speedup_over_serial": round(t_ser / tp, 2)})
    n_p, tot_p = st.get(f"prefix/fine/{B * P}", (0, 0.0))
    if n_p:
        avg = tot_p / n_p / 1e3
        fmas = B * M * S * sum(n * S - 1 for n in range(1, P))
        ach = 2 * fmas / avg / 1e12
        out["prefix_roofline"] = {
            "bound": "alu", "kernel": f"k_hist_prefix (one launch per sweep, {B * P} units)",
            "achieved": round(ach, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP64_TFLOPS, 4), "avg_launch_ms": round(avg * 1e3, 3),
            "flops_per_launch": 2 * fmas, "launches": n_p,
            "hbm_bytes_unique": B * P * (2 * S + 1) * M * 8}
    n_h, tot_h = st.get(f"history/fine/{B * P}", (0, 0.0))
    if n_h:
        out["history_step_avg_us"] = round(tot_h / n_h * 1e3, 2)
    tot = sum(v[1] for v in st.values())
    out["kernel_time_share"] = {kk: round(v[1] / tot, 4) for kk, v in st.items()}
    log(f"full history: serial {t_ser * 1e3:.0f} ms, k*={ks}, parareal {tp * 1e3:.0f} ms, "
        f"prefix {out.get('prefix_roofline', {}).get('avg_launch_ms')} ms/launch")
    return out


def constant_d(l1, torch, W, dev, alpha=0.3):
    """Constant D on the config-2 batch (D = 1, the other settings as config 2): the diagonal
    step solve (solver = 2) against the Cholesky path on the quadrature stiffness, serial and
    parareal wall time, the diagonal kernel against the HBM peak; and one 2D fine sweep at the
    config-3 shape with constant D by both solvers."""
    from paper_2510_11023_amd import _lib

    kw = W.with_(W.C2, alpha=alpha, d_sel=0, d_param=1.0)
    M, N, P = kw["modes"], kw["steps"], kw["slices"]
    S, B = N // P, W.C2_BATCH
    u0 = torch.tensor(W.u0_batch_1d(M, range(B)), dtype=torch.float64, device=dev)
    out = {"workload": f"1D, M={M}, Q={kw['quad']}, N={N}, P={P}, alpha={alpha}, {B} instances "
                       f"(seeds 0..{B - 1}), D = 1, config-2 f"}
    res = {}
    for solver in (2, 0):
        p = l1.make_problem(solver=solver, **kw)
        ws = torch.empty(l1.workspace_bytes(p, B, 1), dtype=torch.uint8, device=dev)
        # GEMM tile variants for the fine steps (the serial solve uses the same ones)
        p.tune = l1.autotune(p, B, workspace=ws)
        ws_s = torch.empty(l1.workspace_bytes(p, B, 0), dtype=torch.uint8, device=dev)
        l1.solve_serial(p, u0, workspace=ws_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Us, _ = l1.solve_serial(p, u0, workspace=ws_s)
        torch.cuda.synchronize()
        t_ser = time.perf_counter() - t0
        del ws_s
        ks, e = find_kstar(l1, p, u0, Us, ws, 24)
        k = ks if ks is not None else P
        l1.solve_parareal(p, u0, k, tol=0.0, want_incr=False, workspace=ws)
        torch.cuda.synchronize()
        _lib.profile_start(only=("diag", "chol"))
        t0 = time.perf_counter()
        U = l1.solve_parareal(p, u0, k, tol=0.0, want_incr=False, workspace=ws).U
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        st = _lib.profile_stop()
        r = {"tune": int(p.tune), "serial_ms": round(t_ser * 1e3, 1), "serial_mode_steps_per_s": B * M * N / t_ser,
             "kstar": ks, "parareal_ms": round(tp * 1e3, 1), "mode_steps_per_s": B * M * N / tp,
             "achieved_rel_err": rel_err_max(U, Us), "speedup_over_serial": round(t_ser / tp, 2)}
        n_d, tot_d = st.get(f"diag/fine/{B * P}", (0, 0.0))
        if n_d:
            avg = tot_d / n_d / 1e3
            nbytes = B * P * M * 24  # rhs and F read, the new state written
            ach = nbytes / avg / 1e9
            r["diag_roofline"] = {
                "bound": "hbm", "kernel": f"k_diag_solve ({B * P} units, fine steps)",
                "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "avg_launch_us": round(avg * 1e6, 2),
                "bytes_per_launch": nbytes, "launches": n_d,
                "note": "a launch of a few microseconds: the two event records around it add "
                        "their own gap, so the kernel trace's duration is shorter"}
        res[solver] = (r, Us)
        del ws
    out["solver2_diagonal"] = res[2][0]
    out["solver0_cholesky"] = res[0][0]
    out["serial_speedup_diag_over_cholesky"] = round(res[0][0]["serial_ms"] / res[2][0]["serial_ms"], 2)
    # the two discretise the stiffness differently (exact integral against Q = 1.5 M Gauss points)
    out["rel_diff_vs_quadrature_stiffness"] = rel_err_max(res[2][1], res[0][1])
    kw2 = W.with_(W.C3, d_sel=0, d_param=1.0)
    u2 = torch.tensor(W.u0_random_2d(kw2["modes"], 0)[None], device=dev)
    two = {}
    for solver in (2, 0):
        p2 = l1.make_problem(solver=solver, **kw2)
        ws2 = l1.parareal_workspace(p2, 1, dev)
        Z2 = l1.solve_parareal(p2, u2, 0, tol=0.0, want_iterates=True, workspace=ws2).iterates[0]
        Z2 = Z2.contiguous()
        l1.fine_apply(p2, Z2, workspace=ws2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        l1.fine_apply(p2, Z2, workspace=ws2)
        torch.cuda.synchronize()
        two[solver] = (time.perf_counter() - t0) * 1e3
        del ws2
    out["2d_fine_sweep_ms"] = {"workload": f"2D, M={kw2['modes']}x{kw2['modes']}, Q={kw2['quad']}, "
                                           f"{kw2['slices']} slices of {kw2['steps'] // kw2['slices']} "
                                           f"steps, D = 1, config-3 f",
                               "solver2_diagonal": round(two[2], 2), "solver0_cholesky": round(two[0], 2)}
    # 1D, 2048 modes (Q = 3072) on the config-2 batch: beyond the factorisation paths
    kw1 = W.with_(kw, modes=2048, quad=3072)
    M1 = kw1["modes"]
    p1 = l1.make_problem(solver=2, **kw1)
    u1 = torch.tensor(W.u0_batch_1d(M1, range(B)), dtype=torch.float64, device=dev)
    ws1 = torch.empty(l1.workspace_bytes(p1, B, 1), dtype=torch.uint8, device=dev)
    p1.tune = l1.autotune(p1, B, workspace=ws1)
    Z1 = l1.solve_parareal(p1, u1, 0, tol=0.0, want_iterates=True, workspace=ws1).iterates[0].contiguous()
    l1.fine_apply(p1, Z1, workspace=ws1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l1.fine_apply(p1, Z1, workspace=ws1)
    torch.cuda.synchronize()
    t_f1 = time.perf_counter() - t0
    del Z1
    ws1s = torch.empty(l1.workspace_bytes(p1, B, 0), dtype=torch.uint8, device=dev)
    l1.solve_serial(p1, u1, workspace=ws1s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Us1, _ = l1.solve_serial(p1, u1, workspace=ws1s)
    torch.cuda.synchronize()
    t_s1 = time.perf_counter() - t0
    del ws1s
    ks1, _ = find_kstar(l1, p1, u1, Us1, ws1, 16)
    k1 = ks1 if ks1 is not None else 16
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U1 = l1.solve_parareal(p1, u1, k1, tol=0.0, want_incr=False, workspace=ws1).U
    torch.cuda.synchronize()
    t_p1 = time.perf_counter() - t0
    del ws1
    out["1d_2048_modes"] = {
        "workload": f"1D, M={M1}, Q={kw1['quad']}, N={N}, P={P}, alpha={alpha}, {B} instances, D = 1, "
                    f"config-2 f, diagonal solve (tune = {int(p1.tune)})",
        "fine_sweep_ms": round(t_f1 * 1e3, 2), "fine_sweep_mode_steps_per_s": B * M1 * N / t_f1,
        # lagged-state product and projection, 2 M Q flops each per unit step
        "gemm_tflops_over_sweep": round(4 * M1 * kw1["quad"] * B * N / t_f1 / 1e12, 2),
        "serial_ms": round(t_s1 * 1e3, 1), "serial_mode_steps_per_s": B * M1 * N / t_s1,
        "parareal_kstar": ks1, "parareal_ms": round(t_p1 * 1e3, 1),
        "parareal_mode_steps_per_s": B * M1 * N / t_p1, "parareal_rel_err": rel_err_max(U1, Us1),
        "parareal_speedup_over_serial": round(t_s1 / t_p1, 2)}
    # 256 x 256 modes (65536 coefficients): beyond the factorisation paths
    kw3 = W.with_(W.C3, modes=256, quad=384, d_sel=0, d_param=1.0)
    M3 = kw3["modes"] ** 2
    p3 = l1.make_problem(solver=2, **kw3)
    u3 = torch.tensor(W.u0_random_2d(kw3["modes"], 0)[None], device=dev)
    ws3 = l1.parareal_workspace(p3, 1, dev)
    Z3 = l1.solve_parareal(p3, u3, 0, tol=0.0, want_iterates=True, workspace=ws3).iterates[0].contiguous()
    l1.fine_apply(p3, Z3, workspace=ws3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l1.fine_apply(p3, Z3, workspace=ws3)
    torch.cuda.synchronize()
    t_fs = time.perf_counter() - t0
    del ws3
    ws3s = torch.empty(l1.workspace_bytes(p3, 1, 0), dtype=torch.uint8, device=dev)
    l1.solve_serial(p3, u3, workspace=ws3s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l1.solve_serial(p3, u3, workspace=ws3s)
    torch.cuda.synchronize()
    t_s3 = time.perf_counter() - t0
    del ws3s
    N3 = kw3["steps"]
    out["2d_256_modes"] = {
        "workload": f"2D, M=256x256 ({M3} coefficients), Q=384, N={N3}, P={kw3['slices']}, D = 1, "
                    f"config-3 f and alpha, one instance, diagonal solve",
        "fine_sweep_ms": round(t_fs * 1e3, 2), "fine_sweep_mode_steps_per_s": M3 * N3 / t_fs,
        # the four separable products per unit step (lagged state on the grid and back to the
        # load vector): 2 (2 M^2 Q + 2 Q^2 M) flops, over the sweep's wall time
        "products_tflops_over_sweep": round(
            2 * (2 * kw3["modes"] ** 2 * kw3["quad"] + 2 * kw3["quad"] ** 2 * kw3["modes"])
            * kw3["slices"] * (N3 // kw3["slices"]) / t_fs / 1e12, 2),
        "serial_ms": round(t_s3 * 1e3, 1), "serial_mode_steps_per_s": M3 * N3 / t_s3}
    log(f"constant D: serial {res[2][0]['serial_ms']:.0f} ms (diag) vs {res[0][0]['serial_ms']:.0f} ms "
        f"(Cholesky); parareal {res[2][0]['parareal_ms']:.0f} vs {res[0][0]['parareal_ms']:.0f} ms; "
        f"2D fine sweep {two[2]:.1f} vs {two[0]:.1f} ms; 1D 2048 modes: fine sweep {t_f1 * 1e3:.1f} ms, "
        f"serial {t_s1 * 1e3:.0f} ms, parareal k*={ks1} {t_p1 * 1e3:.0f} ms; 256x256 modes: fine sweep {t_fs * 1e3:.1f} ms, "
        f"serial {t_s3 * 1e3:.0f} ms")
    return out


def paper_model(l1, torch, W, dev, sizes=((8, 8), (16, 16), (32, 32), (64, 64), (128, 128),
                                               (128, 256))):
    """The paper's model problem on the sine path (qualitative re-runs of its two figures):
    - the error at t = T of parareal iterate k against the serial fine solution, with
      2^8 coarse intervals of 2^5 fine steps, against the hybrid serial solution (parareal's
      fixed point) and against the full-history serial solution (a different discrete
      solution: the error then levels off at the gap between the two);
    - serial and parareal (stop at increment <= 1e-10) wall time over the number of fine
      steps N_t x M, with N_t coarse intervals of M fine steps."""
    kw = dict(W.PAPER)
    M = kw["modes"]
    u0 = torch.tensor(W.u0_paper_1d(M)[None], dtype=torch.float64, device=dev)
    p = l1.make_problem(**kw)
    Us, _ = l1.solve_serial(p, u0)
    Uf, _ = l1.solve_serial(l1.make_problem(**W.with_(kw, history=1)), u0)
    res = l1.solve_parareal(p, u0, 12, tol=0.0, want_iterates=True)
    its = res.iterates[:, 0, -1]
    e_h = [float(f"{float((its[k] - Us[0, -1]).norm()):.3e}") for k in range(res.iters + 1)]
    e_f = [float(f"{float((its[k] - Uf[0, -1]).norm()):.3e}") for k in range(res.iters + 1)]
    out = {"workload": f"paper model: D=1+u, f=sin(pi x)e^-t, u0=x^4(1-x)^4, alpha=0.5, T=1, "
                       f"{M} sine modes, Q={kw['quad']}",
           "error_vs_iteration": {"N_t": kw["slices"], "M": kw["steps"] // kw["slices"],
                                  "vs_hybrid_serial": e_h, "vs_full_history_serial": e_f,
                                  "gap_hybrid_full_at_T": float(f"{float((Us[0, -1] - Uf[0, -1]).norm()):.3e}")}}
    runs = []
    for Nt, Ms in sizes:
        q = l1.make_problem(**W.with_(kw, slices=Nt, steps=Nt * Ms))
        l1.solve_serial(q, u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Uq, _ = l1.solve_serial(q, u0)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        l1.solve_parareal(q, u0, Nt, tol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = l1.solve_parareal(q, u0, Nt, tol=1e-10)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        runs.append({"N_t": Nt, "M": Ms, "fine_steps": Nt * Ms, "serial_ms": round(ts * 1e3, 2),
                     "parareal_ms": round(tp * 1e3, 2), "sweeps": r.iters,
                     "speedup": round(ts / tp, 2), "rel_err": rel_err_max(r.U, Uq)})
        log(f"paper model N_t={Nt} M={Ms}: serial {ts * 1e3:.1f} ms, parareal {tp * 1e3:.1f} ms "
            f"({r.iters} sweeps)")
    out["runtime_vs_fine_steps"] = runs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--no-full-history", action="store_true")
    ap.add_argument("--no-paper-model", action="store_true")
    ap.add_argument("--no-constant-d", action="store_true")
    ap.add_argument("--mode", choices=["full", "kernels", "kernels2d", "kernelsfh", "fullhistory",
                                       "cg2d", "constd", "uneven", "soe", "learned"],
                    default="full",
                    help="kernels: one parareal sweep of the alpha=0.3 batch and a 1 GiB plain "
                         "device copy (for hardware-counter runs); kernels2d: one fine sweep of "
                         "the 2D workload (128 slices) and the same copy; kernelsfh: one "
                         "full-history parareal sweep of the alpha=0.3 batch and the same copy; "
                         "none of these prints a JSON line; fullhistory: only the full-history "
                         "parareal section (its JSON); cg2d: only the config-3 conjugate-gradient "
                         "section (its JSON); constd: only the constant-D diagonal-solve "
                         "section (its JSON); uneven: only the uneven-batch section with its "
                         "learned coarse step (its JSON); soe: only the sum-of-exponentials "
                         "history section (its JSON); learned: only the config-4 learned "
                         "coarse step section (its JSON)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU; a run on several GPUs is not supported "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_11023_amd as l1
    from paper_2510_11023_amd import _lib
    from paper_2510_11023_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = dict(W.C2)
    M, N, P, Q = base["modes"], base["steps"], base["slices"], base["quad"]
    S = N // P
    Mp = M  # 256 is a multiple of 16
    B, alphas = W.C2_BATCH, W.C2_ALPHAS
    u0_np = W.u0_batch_1d(M, range(B))
    u0 = torch.tensor(u0_np, dtype=torch.float64, device=dev)
    probs = {a: l1.make_problem(**W.with_(base, alpha=a)) for a in alphas}
    probs_gemm = {a: l1.make_problem(assembly=1, **W.with_(base, alpha=a)) for a in alphas}
    p0 = probs[alphas[0]]
    ws_par = torch.empty(l1.workspace_bytes(p0, B, 1), dtype=torch.uint8, device=dev)
    ws_ser = torch.empty(l1.workspace_bytes(p0, B, 0), dtype=torch.uint8, device=dev)
    log(f"workspace: parareal {ws_par.numel() / 2**30:.2f} GiB, serial {ws_ser.numel() / 2**20:.0f} MiB")

    if args.mode == "kernels2d":
        kw2 = dict(W.C3)
        p2 = l1.make_problem(**kw2)
        u2 = torch.tensor(W.u0_random_2d(kw2["modes"], 0)[None], device=dev)
        ws2 = l1.parareal_workspace(p2, 1, dev)
        Z2 = l1.solve_parareal(p2, u2, 0, tol=0.0, want_iterates=True, workspace=ws2).iterates[0]
        l1.fine_apply(p2, Z2.contiguous(), workspace=ws2)
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("kernels2d mode done")
        return

    if args.mode == "kernelsfh":
        pf = l1.make_problem(**W.with_(base, alpha=alphas[0], history=1))
        wsf = torch.empty(l1.workspace_bytes(pf, B, 1), dtype=torch.uint8, device=dev)
        l1.solve_parareal(pf, u0, 1, tol=0.0, workspace=wsf)
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("kernelsfh mode done")
        return

    if args.mode == "cg2d":
        print(json.dumps(config3_cg(l1, torch, W, dev)), flush=True)
        return

    if args.mode == "constd":
        print(json.dumps(constant_d(l1, torch, W, dev)), flush=True)
        return

    if args.mode == "fullhistory":
        print(json.dumps(full_history(l1, torch, W, dev)), flush=True)
        return

    if args.mode == "uneven":
        print(json.dumps(uneven_batch(l1, torch, W, dev, learned_model=c5_network(l1, torch, W, dev))),
              flush=True)
        return

    if args.mode == "soe":
        print(json.dumps(soe_history(l1, torch, W, dev)), flush=True)
        return

    if args.mode == "learned":
        print(json.dumps(learned_vs_plain(l1, torch, W, dev)), flush=True)
        return

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

    # serial reference and its time: one call over all 3 x 32 instances, each with its own
    # alpha (the fair comparison: every instance's steps share the launches); the three groups
    # one after another for context.  An instance's result does not depend on its batch, so
    # both give the same solutions bit for bit.
    u96 = torch.cat([u0] * len(alphas)).contiguous()
    al96 = [a for a in alphas for _ in range(B)]
    ws_ser96 = torch.empty(l1.workspace_bytes(p0, len(alphas) * B, 0), dtype=torch.uint8, device=dev)
    l1.solve_serial(p0, u96, alpha=al96, workspace=ws_ser96)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U96, _ = l1.solve_serial(p0, u96, alpha=al96, workspace=ws_ser96)
    torch.cuda.synchronize()
    t_serial_all = time.perf_counter() - t0
    del ws_ser96
    log(f"serial, 96 instances in one call: {t_serial_all * 1e3:.1f} ms")
    Us, t_serial = {}, {}
    for gi, a in enumerate(alphas):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, _ = l1.solve_serial(probs[a], u0, workspace=ws_ser)
        torch.cuda.synchronize()
        t_serial[a] = time.perf_counter() - t0
        Us[a] = U
        assert torch.equal(U, U96[gi * B:(gi + 1) * B]), "batch independence"
        log(f"serial alpha={a}: {t_serial[a] * 1e3:.1f} ms")

    # k*(alpha): first sweep count whose iterate is within 1e-8 of the serial solution
    kstar = {}
    for a in alphas:
        ks, e = find_kstar(l1, probs[a], u0, Us[a], ws_par, 24)
        kstar[a] = max(ks if ks is not None else P, 1)   # exact after P sweeps
        log(f"parareal alpha={a}: k*={kstar[a]} errors " + " ".join(f"{v:.1e}" for v in e[: kstar[a] + 1]))

    # the three alpha groups are independent: each runs on a stream and a workspace of its own,
    # so that one group's fine launches take the CUs another group's coarse sweeps leave idle
    streams = [torch.cuda.Stream() for _ in alphas]
    ws_groups = [ws_par] + [torch.empty_like(ws_par) for _ in alphas[1:]]

    def step(pr=probs, wsg=None):
        out = {}
        cur = torch.cuda.current_stream()
        for a, s_, w in zip(alphas, streams, wsg or ws_groups):
            s_.wait_stream(cur)
            with torch.cuda.stream(s_):
                out[a] = l1.solve_parareal(pr[a], u0, kstar[a], tol=0.0, want_incr=False,
                                           workspace=w).U
        for s_ in streams:
            cur.wait_stream(s_)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_start(only=("chol", "history"))  # the roofline kernels only
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

    # the same 96 instances in one parareal call with the flowchart's stop rule applied per
    # instance (increment <= 1e-8, one host synchronisation per sweep): no offline k*
    ws96 = torch.empty(l1.workspace_bytes(p0, len(alphas) * B, 1), dtype=torch.uint8, device=dev)
    run96 = lambda: l1.solve_parareal(p0, u96, P, tol=TARGET, alpha=al96, want_incr=False,
                                      workspace=ws96)
    t96, r96 = median_time(torch, run96, reps=3)
    inst96 = r96.inst.cpu().numpy()
    tol_stop = {"ms": round(t96 * 1e3, 1), "mode_steps_per_s": useful / t96,
                "sweeps": r96.iters, "max_rel_err_vs_serial": rel_err_max(r96.U, U96),
                "sweeps_per_alpha": {str(a): int(inst96[g * B:(g + 1) * B].max()) for g, a in enumerate(alphas)},
                "note": "one call, 96 instances with their own alpha; each instance stops at its "
                        "first sweep whose relative increment is <= 1e-8"}
    del ws96
    log(f"parareal, one call with per-instance stop: {t96 * 1e3:.1f} ms, {r96.iters} sweeps, "
        f"error vs serial {tol_stop['max_rel_err_vs_serial']:.1e}")
    # sweep k launches only the slices n >= k (the earlier ones are converged)
    fine_units = [B * (P - min(k, P - 1)) for a in alphas for k in range(kstar[a])]
    executed = sum(u * S * M for u in fine_units)
    serial_total = sum(t_serial.values())
    # share of the step's wall time in the profiled kernels (summed over the three streams)
    share = {k: round(v[1] / (ms_per_step * args.steps), 4) for k, v in stats.items()}

    def fine_launches(kernel):
        # (units, launches, total ms) of every fine-sweep launch of `kernel`
        out = []
        for key, (n, tot) in stats.items():
            parts = key.split("/")
            if len(parts) == 3 and parts[0] == kernel and parts[1] == "fine":
                out.append((int(parts[2]), n, tot))
        return out

    # dominant kernel: the fine-sweep factor-and-solve kernel, over all its launches
    roofline = None
    chol = fine_launches("chol")
    if chol:
        per_unit = M ** 3 / 3 + M ** 2 / 2 + M / 6 + 2 * M ** 2
        flops = sum(u * per_unit * n for u, n, _ in chol)
        tot_s = sum(t for _, _, t in chol) / 1e3
        n_c = sum(n for _, n, _ in chol)
        achieved = flops / tot_s / 1e12
        traffic = None
        if TRAFFIC_RECORD and TRAFFIC_RECORD.get("sha256") == sources_hash():
            traffic = TRAFFIC_RECORD["bytes_per_launch"]
        units = B * P
        full = [x for x in chol if x[0] == units]
        roofline = {"bound": "mfma", "kernel": f"k_chol_reg<moments> (fine sweeps, {B * P} units "
                    f"per full launch; sweep k launches B (P - k))",
                    "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                    "traffic": traffic,
                    "avg_launch_ms": round(tot_s * 1e3 / n_c, 4),
                    "avg_full_launch_ms": round(full[0][2] / full[0][1], 4) if full else None,
                    "flops_per_full_launch": int(units * per_unit), "launches": n_c}

    # the same kernel with the GPU to itself: one alpha group alone, on one stream
    if roofline is not None:
        a_iso = alphas[0]
        l1.solve_parareal(probs[a_iso], u0, kstar[a_iso], tol=0.0, want_incr=False, workspace=ws_par)
        torch.cuda.synchronize()
        _lib.profile_start(only=("chol", "history"))
        l1.solve_parareal(probs[a_iso], u0, kstar[a_iso], tol=0.0, want_incr=False, workspace=ws_par)
        torch.cuda.synchronize()
        st_iso = _lib.profile_stop()
        iso = [(int(k.split("/")[2]), n, t) for k, (n, t) in st_iso.items() if k.startswith("chol/fine/")]
        fl_iso = sum(u * per_unit * n for u, n, _ in iso)
        t_iso = sum(t for _, _, t in iso) / 1e3
        full_iso = [x for x in iso if x[0] == B * P]
        roofline["isolated"] = {
            "note": f"one alpha group ({a_iso}) alone on one stream after the timed region; in the "
                    "timed region the three groups share the CUs, which lengthens each launch",
            "achieved": round(fl_iso / t_iso / 1e12, 3),
            "frac": round(fl_iso / t_iso / 1e12 / PEAK_FP64_TFLOPS, 4),
            "avg_full_launch_ms": round(full_iso[0][2] / full_iso[0][1], 4) if full_iso else None}

    # history sum: algorithmic bytes of the timed fine sweeps (launch with U units at step r:
    # rows 0..r-1 of every slot, the instance's slice ends once, the output rows)
    history = None
    hist = fine_launches("history")
    if hist:
        row = Mp * 8
        sweep_bytes = [(u * sum(range(1, S + 1)) + S * B * (P + 1) + S * u) * row for u in fine_units]
        tot_bytes = sum(sweep_bytes) * args.steps
        tot_h = sum(t for _, _, t in hist)
        n_h = sum(n for _, n, _ in hist)
        gbs = tot_bytes / (tot_h / 1e3) / 1e9
        history = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_full_sweep": sweep_bytes[0],
                   "avg_launch_us": round(tot_h / n_h * 1e3, 2)}
        if roofline is not None:  # the isolated pass above (one alpha group alone)
            hist_iso = [(n, t) for k, (n, t) in st_iso.items() if k.startswith("history/fine/")]
            if hist_iso:
                a_iso = alphas[0]
                units_iso = [B * (P - min(k, P - 1)) for k in range(kstar[a_iso])]
                b_iso = sum((u * sum(range(1, S + 1)) + S * B * (P + 1) + S * u) * row for u in units_iso)
                t_h = sum(t for _, t in hist_iso) / 1e3
                history["isolated"] = {"achieved": round(b_iso / t_h / 1e9, 1),
                                       "frac": round(b_iso / t_h / 1e9 / PEAK_HBM_GBS, 4),
                                       "avg_launch_us": round(t_h * 1e6 / sum(n for n, _ in hist_iso), 2)}

    # whole-step roofline: each phase at its own bound, summed (step solves at the FP64 MFMA
    # peak, history sums at the HBM bandwidth), over the measured step time.  Work per
    # unit-step: lagged state 2QM, moments 2Q(2M+1), load 2QM, factor and solves.
    unit_step = 2 * Q * M + 2 * Q * (2 * M + 1) + 2 * Q * M + (M ** 3 / 3 + M ** 2 / 2 + M / 6 + 2 * M ** 2)
    fine_unit_steps = sum(u * S for u in fine_units)
    coarse_unit_steps = sum((kstar[a] + 1) * P * B for a in alphas)
    solve_ms = (fine_unit_steps + coarse_unit_steps) * unit_step / (PEAK_FP64_TFLOPS * 1e12) * 1e3
    row = Mp * 8
    hist_bytes = sum((u * sum(range(1, S + 1)) + S * B * (P + 1) + S * u) * row for u in fine_units)
    hist_bytes += sum((kstar[a] + 1) * B * sum(range(1, P + 1)) * row for a in alphas)  # coarse
    hist_ms = hist_bytes / (PEAK_HBM_GBS * 1e9) * 1e3
    whole = {"solves_ms": round(solve_ms, 2), "history_ms": round(hist_ms, 2),
             "roofline_ms": round(solve_ms + hist_ms, 2), "measured_ms": round(ms_per_step, 1),
             "frac": round((solve_ms + hist_ms) / ms_per_step, 4),
             "flops_per_unit_step": int(unit_step),
             "unit_steps": {"fine": fine_unit_steps, "coarse": coarse_unit_steps}}

    # the same step with the quadrature-GEMM stiffness (assembly = 1), whose systems go through
    # device memory: workspaces of their own
    ws_gemm = [torch.empty(l1.workspace_bytes(probs_gemm[a], B, 1), dtype=torch.uint8, device=dev)
               for a in alphas]
    step(probs_gemm, ws_gemm)
    torch.cuda.synchronize()
    _lib.profile_start()
    t0 = time.perf_counter()
    out_g = step(probs_gemm, ws_gemm)
    torch.cuda.synchronize()
    t_gemm = time.perf_counter() - t0
    stats_g = _lib.profile_stop()
    units = B * P
    n_a, tot_a = stats_g.get(f"assemble/fine/{units}", (0, 0.0))
    gemm = {"ms_per_step": round(t_gemm * 1e3, 1),
            "achieved_rel_err": {str(a): rel_err_max(out_g[a], Us[a]) for a in alphas}}
    if n_a:
        avg_a = tot_a / n_a / 1e3
        fl = units * Q * M * (M + 1)
        gemm["assemble_roofline"] = {
            "bound": "mfma", "kernel": f"k_assemble1d<64> (fine sweep, {units} units)",
            "achieved": round(fl / avg_a / 1e12, 3), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(fl / avg_a / 1e12 / PEAK_FP64_TFLOPS, 4),
            "avg_launch_ms": round(avg_a * 1e3, 4), "flops_per_launch": fl}
    log(f"assembly=1 step: {t_gemm * 1e3:.1f} ms")
    del ws_gemm

    learned = None
    if not args.no_learned:
        learned = learned_vs_plain(l1, torch, W, dev)

    c1 = config1_latency(l1, torch, W, dev)

    soe = None
    if not args.no_full_history:
        soe = soe_history(l1, torch, W, dev)

    uneven = None
    if not args.no_uneven:
        net5 = None if args.no_learned else c5_network(l1, torch, W, dev)
        uneven = uneven_batch(l1, torch, W, dev, learned_model=net5)
        del net5

    paper = None
    if not args.no_paper_model:
        paper = paper_model(l1, torch, W, dev)

    constd = None
    if not args.no_constant_d:
        constd = constant_d(l1, torch, W, dev)

    fullh = None
    if not args.no_full_history:
        fullh = full_history(l1, torch, W, dev)

    two_d = None
    if not args.no_2d:
        two_d = config3_2d(l1, torch, W, dev)

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
            "workload": "1D, M=256, Q=384, N=4096, P=64, D=1+1/(1+u^2), f=0.1u(1-u), "
                        "alpha in {0.3,0.7,1.0} x 32 instances (seeds 0..31); plain-G parareal "
                        "run to 1e-8 relative of the serial solution",
            "coarse": "plain L1 (learned G: see learned_vs_plain)",
            "kstar": {str(a): kstar[a] for a in alphas},
            "achieved_rel_err": {str(a): achieved_err[a] for a in alphas},
        },
        "time_to_1e8_ms": ms_per_step,
        "serial_ms": t_serial_all * 1e3,
        "serial_mode_steps_per_s": useful / t_serial_all,
        "serial_note": "one l1pr_solve_serial call over all 96 instances (per-instance alpha); "
                       "the three alpha groups one after another take serial_ms_per_group_total",
        "serial_ms_per_group_total": serial_total * 1e3,
        "parareal_over_serial_time": round(ms_per_step / (t_serial_all * 1e3), 3),
        "parareal_tol_stop": tol_stop,
        "config1": c1,
        "soe_history": soe,
        "executed_mode_steps_per_s": executed / (ms_per_step / 1e3),
        "profiled_kernel_time_per_wall_time": share,
        "schedule": "the three alpha groups on three streams, one workspace each",
        "roofline": roofline,
        "history_hbm": history,
        "whole_step_roofline": whole,
        "gemm_assembly": gemm,
        "learned_vs_plain": learned,
        "uneven_batch": uneven,
        "config3_2d": two_d,
        "full_history": fullh,
        "constant_d": constd,
        "paper_model": paper,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
