#!/usr/bin/env python3
"""Benchmark of the far-field Stokeslet sum on one MI355X.

One step = one full pass of the hot path over the workload: the per-vesicle
preprocessing kernel and the pair-sum kernel (FP32-compensated), on inputs
already resident in HBM.  Workload: the dense suspension of 2,000 vesicles x
128 points (256,000 targets) at 30% area fraction, seeded and synthetic.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 19          # sub x2, q: mul+fma, log, rcp, r.F: mul+fma, scale, 2 x (2 fma)
ADJOINT_FLOPS_PER_PAIR = 68  # per ordered pair: r, q, rcp, log shared (7), v (12), position gradient (49)
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64
PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
METRIC = "Stokeslet pair-interactions/s (FP32-comp vs FP64) at ≤1e-5 rel err; % VALU peak"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_counters(tile, symmetric, name=None):
    """Figures of the committed rocprofv3 counter summary of the pair kernel (HBM bytes per launch,
    achieved shader clock, issue slots per pair), or {} when the kernel source (its file followed by the
    shared device header vesnet_internal.h) or the launch shape differs from the one measured."""
    import hashlib
    if name is None:
        name = "k_sym_main_fp32c_2000x128_counters.txt" if symmetric else "k_forward_fp32c_2000x128_counters.txt"
    src = "vesnet_symmetric.hip" if symmetric else "vesnet_kernels.hip"
    try:
        fields = {}
        for line in open(os.path.join(ROOT, "profiles", name)):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        csrc = os.path.join(ROOT, "paper_2606_25569_amd", "csrc")
        h = hashlib.sha1(open(os.path.join(csrc, src), "rb").read())
        h.update(open(os.path.join(csrc, "vesnet_internal.h"), "rb").read())
        sha = h.hexdigest()
        if fields.get("kernel_source_sha1") != sha or fields.get("tile") != tile:
            return {}
        out = {"profile": "profiles/" + name}
        for key in ("traffic_bytes_per_launch", "sclk_ghz", "slots_per_pair"):
            if key in fields:
                out[key] = float(fields[key])
        return out
    except (OSError, KeyError, ValueError):
        return {}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_one_core(frac, seed):
    """The oracle on one thread, in a child process (OMP_NUM_THREADS=1) that never touches the
    GPU, on a seeded target sample of the 2000 x 128 workload: (pairs/s, targets, seconds)."""
    import subprocess
    code = ("import json, sys, time; sys.path.insert(0, %r)\n"
            "from oracle import oracle as O\nfrom synth import suspension as S\n"
            "s = S.load_config(1); sel = S.sample_targets(s.n_points, %r, %r)\n"
            "t = time.perf_counter(); O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)\n"
            "dt = time.perf_counter() - t\n"
            "n = int(sum(s.n_points - (s.offsets[v + 1] - s.offsets[v]) for v in O.vesicle_ids(s.offsets)[sel]))\n"
            "print(json.dumps({'pairs': n, 'targets': int(sel.size), 's': dt, 'threads': O.num_threads()}))\n"
            % (ROOT, frac, seed))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        log(f"[bench] one-core oracle failed: {r.stderr[-500:]}")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true", help="autotune the launch shape instead of the library default")
    ap.add_argument("--tile", default=None,
                    help="T,B,splits[,staging]: fixed launch shape instead of the tuned one (staging 1 = SGPR, 2 = LDS)")
    ap.add_argument("--form", default="symmetric", choices=["symmetric", "direct"],
                    help="pair form of the FP32-compensated sum: symmetric (one evaluation per unordered pair, the "
                         "default) or direct (one gather per target)")
    ap.add_argument("--cpu-sample", type=float, default=0.03, help="fraction of targets the oracle evaluates")
    ap.add_argument("--workload", default="dense",
                    choices=["dense", "batched", "adjoint", "nearfield", "treecode", "force"],
                    help="dense: the benchmark line; batched / adjoint / nearfield / treecode / force: the other "
                         "forms, reported separately")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sum would shard by targets with one all-gather of source records).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration_mb} MiB three times")
        return

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "nearfield":
        return bench_nearfield(args)
    if args.workload == "treecode":
        return bench_treecode(args)
    if args.workload == "force":
        return bench_force(args)

    import paper_2606_25569_amd as V
    from synth import suspension as S

    t0 = time.time()
    s = S.load_config(1)
    P, M = s.n_points, s.n_vesicles
    pairs = s.cross_pairs()
    log(f"[bench] workload 2000x128: P={P} M={M} pairs={pairs:.4e} (generated in {time.time() - t0:.1f}s)")

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    X = torch.tensor(s.X, device=dev)
    f = torch.tensor(s.f, device=dev)
    w = torch.tensor(s.w, device=dev)
    part = V.Partition(s.offsets, dev)
    out = torch.empty((2, P), dtype=torch.float64, device=dev)
    lib = V._lib.lib()
    stream = torch.cuda.current_stream()
    sp = V.farfield._ptr

    cfg = None
    if args.tile:
        vals = [int(x) for x in args.tile.split(",")]
        cfg = V.TileConfig(vals[0], vals[1], vals[2], 1, vals[3] if len(vals) > 3 else 2, 1)
    elif args.tune:
        t1 = time.time()
        cfg, tms = V.autotune(X, X, f, w, part, s.mu, "fp32c", repeats=2)
        log(f"[bench] autotuned {cfg.as_dict()} ({tms:.3f} ms) in {time.time() - t1:.1f}s")
    if cfg is None:
        cfg = V.default_config(P, M, "fp32c")
    symmetric = args.form == "symmetric"
    cfg.pair_form = 2 if symmetric else 1
    if symmetric and not args.tile:
        cfg.targets_per_thread = 0  # the symmetric form's own default
    log(f"[bench] launch shape {cfg.as_dict()}")
    import ctypes
    cfg_ref = ctypes.byref(cfg)
    prec = V.FP32_COMPENSATED
    ws_n = lib.vesnet_farfield_workspace_bytes(P, M, prec, cfg_ref)
    ws = torch.empty(ws_n, dtype=torch.uint8, device=dev)
    sh = ctypes.c_void_p(stream.cuda_stream)

    def prepare(prec_code, c_ref, wsp):
        V._lib.check(lib.vesnet_farfield_prepare(sp(X), sp(f), sp(w), sp(part.device), M, P, prec_code, sp(wsp),
                                                 wsp.numel(), sh))

    def evaluate(prec_code, c_ref, wsp):
        V._lib.check(lib.vesnet_farfield_evaluate(sp(X), sp(part.device), M, P, float(s.mu), sp(out), prec_code,
                                                  c_ref, sp(wsp), wsp.numel(), sh))

    for _ in range(args.warmup):
        prepare(prec, cfg_ref, ws)
        evaluate(prec, cfg_ref, ws)
    torch.cuda.synchronize()
    log(f"[bench] warmup done; timing {args.steps} steps")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        prepare(prec, cfg_ref, ws)
        ev[k][1].record(stream)
        evaluate(prec, cfg_ref, ws)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prep_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
    eval_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
    ms_step = wall * 1e3 / args.steps
    value = pairs / (wall / args.steps)
    u32 = out.cpu().numpy()
    log(f"[bench] fp32c: {ms_step:.3f} ms/step, pair kernel {eval_ms.mean():.3f} ms (min {eval_ms.min():.3f}), "
        f"prepare {prep_ms.mean() * 1e3:.1f} us -> {value:.4e} pairs/s")

    # FP64 GPU kernels on the same inputs: the plain direct gather (the baseline), then the symmetric form
    prec64 = V.FP64

    def time64(pair_form):
        cfg64 = V.default_config(P, M, "fp64")
        cfg64.pair_form = pair_form
        if pair_form == 2:
            cfg64.targets_per_thread = 0  # the symmetric form's own default
        ws64 = torch.empty(lib.vesnet_farfield_workspace_bytes(P, M, prec64, ctypes.byref(cfg64)), dtype=torch.uint8,
                           device=dev)
        prepare(prec64, ctypes.byref(cfg64), ws64)
        evaluate(prec64, ctypes.byref(cfg64), ws64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.fp64_steps):
            prepare(prec64, ctypes.byref(cfg64), ws64)
            evaluate(prec64, ctypes.byref(cfg64), ws64)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.fp64_steps, out.cpu().numpy()

    ms64, u64 = time64(1)
    log(f"[bench] fp64 (direct): {ms64:.3f} ms/step -> {pairs / (ms64 * 1e-3):.4e} pairs/s")
    ms64s, u64s = time64(2)
    log(f"[bench] fp64 (symmetric): {ms64s:.3f} ms/step -> {pairs / (ms64s * 1e-3):.4e} pairs/s")

    # accuracy on a seeded target sample, and the CPU baseline on the same sample
    sel = S.sample_targets(P, args.cpu_sample, 101)
    errs = {}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log(f"[bench] oracle on {sel.size} targets x {P} sources ({O.num_threads()} threads)")
        tc = time.perf_counter()
        ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)
        tcpu = time.perf_counter() - tc
        sample_pairs = int(sum(P - (s.offsets[v + 1] - s.offsets[v]) for v in O.vesicle_ids(s.offsets)[sel]))
        scale = np.abs(ref).max()
        for name, u in (("fp32c", u32), ("fp64", u64), ("fp64_symmetric", u64s)):
            d = u[:, sel] - ref
            errs[name] = {"max_rel": float(np.abs(d).max() / scale),
                          "rms_rel": float(np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(ref * ref)))}
        rate = sample_pairs / tcpu
        cpu = {"value": rate, "unit": "pairs/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"seeded {100 * args.cpu_sample:g}% target sample: {sel.size} targets x all {P} sources of the "
                         f"same workload ({sample_pairs:.3e} pairs, {tcpu:.2f} s wall)",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "extrapolated_full_config_s": pairs / rate,
               "extrapolated_note": "the full 2000 x 128 sum at the sampled rate (extrapolated, not run)"}
        log(f"[bench] errors {errs}; oracle {rate:.3e} pairs/s on {cpu['cores']} threads")
        one = oracle_one_core(args.cpu_sample / 8, 103)
        if one:
            r1 = one["pairs"] / one["s"]
            cpu["one_core"] = {"value": r1, "unit": "pairs/s", "threads": one["threads"],
                               "sample": f"seeded {100 * args.cpu_sample / 8:g}% target sample: {one['targets']} targets "
                                         f"({one['pairs']:.3e} pairs, {one['s']:.2f} s wall)",
                               "extrapolated_full_config_s": pairs / r1}
            log(f"[bench] oracle on one thread: {r1:.3e} pairs/s")

    t_kernel = float(eval_ms.mean()) * 1e-3
    achieved = FLOPS_PER_PAIR * pairs / t_kernel / 1e12
    d = cfg.as_dict()
    tile_key = ",".join(str(d[k]) for k in ("targets_per_thread", "block_threads", "source_splits", "source_staging",
                                            "accumulate", "pair_form"))
    prof = measured_counters(tile_key, symmetric)
    prof64 = measured_counters("0,256,16,2,1,2", True, "k_sym64_main_fp64_2000x128_counters.txt")
    traffic = prof.get("traffic_bytes_per_launch")
    mix = None
    if "slots_per_pair" in prof:
        # the instruction-mix ceiling: every SIMD issues 32 FP32 lanes per cycle at the measured shader
        # clock, a transcendental takes four issue slots (counter basis in the profile summary)
        sclk = prof.get("sclk_ghz", 2.4)
        ceiling = 256 * 4 * 32 * sclk * 1e9 / prof["slots_per_pair"]
        mix = {"ceiling_pairs_per_s": ceiling, "frac": (pairs / t_kernel) / ceiling,
               "slots_per_pair": prof["slots_per_pair"], "sclk_ghz": sclk, "profile": prof["profile"]}
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense suspension: 2000 vesicles x 128 points (256000 targets), 30% area fraction "
                               "by RSA, gap 0.1, ellipses of perimeter 2pi and reduced area 0.65, force-free "
                               "Fourier forces k<=4, mu=1",
                   "n_points": P, "n_vesicles": M, "cross_vesicle_pairs": pairs,
                   "precision": "fp32-compensated (float32 pairs, float64 per-vesicle flush)",
                   "pair_form": args.form,
                   "tile": cfg.as_dict()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "kernel": "k_sym_main (symmetric pair sum)" if symmetric else "k_forward (pair sum)",
                     "kernel_ms": float(eval_ms.mean()), "kernel_ms_median": float(np.median(eval_ms)),
                     "kernel_ms_min": float(eval_ms.min()), "flops_per_pair": FLOPS_PER_PAIR,
                     "mix_ceiling_frac": mix["frac"] if mix else None, "mix_ceiling": mix,
                     "sclk_ghz": prof.get("sclk_ghz")},
        "cpu_baseline": cpu,
        "fp64": {"kernel": "k_forward<FP64> (plain direct gather, the baseline)",
                 "pairs_per_s": pairs / (ms64 * 1e-3), "ms_per_step": ms64,
                 "tflops": FLOPS_PER_PAIR * pairs / (ms64 * 1e-3) / 1e12,
                 "frac_fp64_peak": FLOPS_PER_PAIR * pairs / (ms64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                 "speedup_fp32c_over_fp64": ms64 / ms_step},
        "fp64_symmetric": {"kernel": "k_sym64_main (each unordered pair once, two-word fixed-point sums)",
                           "traffic": prof64.get("traffic_bytes_per_launch"), "sclk_ghz": prof64.get("sclk_ghz"),
                           "profile": prof64.get("profile"),
                           "pairs_per_s": pairs / (ms64s * 1e-3), "ms_per_step": ms64s,
                           "tflops": FLOPS_PER_PAIR * pairs / (ms64s * 1e-3) / 1e12,
                           "frac_fp64_peak": FLOPS_PER_PAIR * pairs / (ms64s * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                           "speedup_fp32c_over_fp64_symmetric": ms64s / ms_step},
        "max_rel_err": errs or None,
        "prepare_us": float(prep_ms.mean() * 1e3),
    }
    print(json.dumps(rec), flush=True)


def _time(fn, reps, stream):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(args):
    """64 independent suspensions: one persistent launch (eager and as a HIP graph)
    against one launch pair per suspension (eager and captured in a graph)."""
    import numpy as np
    import torch

    import paper_2606_25569_amd as V
    from synth import suspension as S

    t0 = time.time()
    b = S.load_config(3)
    pairs = b.cross_pairs()
    log(f"[bench] batched: S={b.n_suspensions} P={b.n_points} pairs={pairs:.4e} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    X = torch.tensor(b.X, device=dev)
    f = torch.tensor(b.f, device=dev)
    w = torch.tensor(b.w, device=dev)
    # the library's default shape (the batched symmetric form), the direct persistent form, and the
    # autotuner's choice, each eager and as a HIP graph
    forms = {}
    for name, cfg in (("symmetric_default", None), ("direct_default", {"pair_form": 1}), ("tuned", "tune")):
        bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c",
                              config=None if cfg == "tune" else cfg)
        if cfg == "tune":
            best, tms = V.autotune(None, None, None, None, None, batched=bp, repeats=2)
            log(f"[bench] batched autotune: {best.as_dict()} {tms:.3f} ms")
            bp.config = best
        te = _time(bp.run, args.steps, stream)
        bp.capture()
        tg = _time(bp.replay, args.steps, stream)
        bp.close()
        forms[name] = {"eager_ms": te, "graph_ms": tg, "pairs_per_s_graph": pairs / (tg * 1e-3),
                       "tflops_graph": FLOPS_PER_PAIR * pairs / (tg * 1e-3) / 1e12,
                       "frac_fp32_peak_graph": FLOPS_PER_PAIR * pairs / (tg * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                       "tile": (bp.config.as_dict() if bp.config is not None else "library default")}
        log(f"[bench] batched {name}: eager {te:.3f} ms, graph {tg:.3f} ms -> {pairs / (tg * 1e-3):.4e} pairs/s")
    t_eager, t_graph = forms["tuned"]["eager_ms"], forms["tuned"]["graph_ms"]
    # one prepare+evaluate per suspension, each with its own tuned-by-default shape
    parts, slices, wss, outs = [], [], [], []
    base = 0
    for k, m in enumerate(b.members):
        sl = slice(base, base + m.n_points)
        base += m.n_points
        parts.append(V.Partition(m.offsets, dev))
        slices.append((X[:, sl].contiguous(), f[:, sl].contiguous(), w[sl].contiguous()))
        wss.append(torch.empty(V.workspace_bytes(m.n_points, m.n_vesicles, "fp32c"), dtype=torch.uint8, device=dev))
        outs.append(torch.empty((2, m.n_points), dtype=torch.float64, device=dev))

    def loop():
        for k in range(len(b.members)):
            Xs, fs, ws_ = slices[k]
            V.farfield_forward(Xs, Xs, fs, ws_, parts[k], float(b.mu[k]), "fp32c", out=outs[k], workspace=wss[k])

    t_loop = _time(loop, args.steps, stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        loop()
    t_loop_graph = _time(g.replay, args.steps, stream)
    rec = {"workload": "batched: 64 independent suspensions, M log-uniform in [10,1500], N in {32,64,128}, "
                       "area fraction U[0.20,0.35], FP32-compensated",
           "n_points": b.n_points, "cross_vesicle_pairs": pairs, "tile": best.as_dict(), "forms": forms,
           "ms": {"persistent_eager": t_eager, "persistent_graph": t_graph, "loop_eager": t_loop,
                  "loop_graph": t_loop_graph},
           "pairs_per_s": {"persistent_graph": pairs / (t_graph * 1e-3), "loop_graph": pairs / (t_loop_graph * 1e-3)},
           "tflops_persistent_graph": FLOPS_PER_PAIR * pairs / (t_graph * 1e-3) / 1e12}
    print(json.dumps(rec), flush=True)


def bench_adjoint(args):
    """512 x 64 suspension: forward and the hand-written backward, FP32-compensated and FP64."""
    import numpy as np
    import torch

    import paper_2606_25569_amd as V
    from synth import suspension as S

    s = S.load_config(4)
    pairs = s.cross_pairs()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    X = torch.tensor(s.X, device=dev)
    f = torch.tensor(s.f, device=dev)
    w = torch.tensor(s.w, device=dev)
    g = torch.tensor(S.target_field(4, s.n_points), device=dev)
    part = V.Partition(s.offsets, dev)
    rec = {"workload": "adjoint: 512 vesicles x 64 points at 30% area fraction, dL/du = u - u*",
           "n_points": s.n_points, "cross_vesicle_pairs": pairs}
    rec["flops_per_pair"] = ADJOINT_FLOPS_PER_PAIR
    for prec in ("fp32c", "fp64"):
        tf = _time(lambda: V.farfield_forward(X, X, f, w, part, s.mu, prec), args.steps, stream)
        # the points form (one pass over unordered pairs under fp32c) and the two gathers
        tb = _time(lambda: V.farfield_backward_points(X, f, w, part, s.mu, g, prec), args.steps, stream)
        t2 = _time(lambda: V.farfield_backward(X, X, f, w, part, s.mu, g, prec), args.steps, stream)
        tfl = ADJOINT_FLOPS_PER_PAIR * pairs / (tb * 1e-3) / 1e12
        peak = PEAK_FP32_TFLOPS if prec == "fp32c" else PEAK_FP64_TFLOPS
        rec[prec] = {"forward_ms": tf, "backward_ms": tb, "backward_two_gathers_ms": t2,
                     "forward_pairs_per_s": pairs / (tf * 1e-3), "backward_pairs_per_s": pairs / (tb * 1e-3),
                     "backward_tflops": tfl, "backward_frac_peak": tfl / peak}
        log(f"[bench] adjoint {prec}: forward {tf:.3f} ms, backward {tb:.3f} ms (two gathers {t2:.3f} ms), "
            f"{tfl:.1f} TFLOP/s at {ADJOINT_FLOPS_PER_PAIR} flops per pair")
    print(json.dumps(rec), flush=True)


def bench_force(args):
    """The step before the sum: membrane force f = -kappa_b X_ssss + (sigma X_s)_s and trapezoid weights by
    spectral derivatives (five circulant N x N derivative products of two components per vesicle:
    20 N^2 flops per vesicle; 48 B of HBM traffic per point), 2000 vesicles of 128 and of 32 points, with
    a seeded smooth tension."""
    import numpy as np
    import torch

    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    from paper_2606_25569_amd.farfield import _ptr
    from synth import suspension as S

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    lib = L.lib()
    rec = {"workload": "membrane force and trapezoid weights (spectral derivatives, FP64), kappa_b = 1, "
                       "seeded tension 1 + 0.1 N(0, 1)", "cases": []}
    for name, s in (("2000 x 128", S.load_config(1)), ("2000 x 32", S.rsa_suspension(S.config_seed(5), 2000, 32, 0.30))):
        P, M = s.n_points, s.n_vesicles
        N = P // M
        X = torch.tensor(s.X, device=dev)
        sig_h = 1.0 + 0.1 * np.random.default_rng(S.config_seed(6)).normal(size=P)
        sig = torch.tensor(sig_h, device=dev)
        part = V.Partition(s.offsets, dev)
        f = torch.empty((2, P), dtype=torch.float64, device=dev)
        w = torch.empty((P,), dtype=torch.float64, device=dev)

        def step():
            L.check(lib.vesnet_elastic_force(_ptr(X), _ptr(sig), 1.0, _ptr(part.device), M, P, _ptr(f), _ptr(w),
                                             stream.cuda_stream))

        for _ in range(args.warmup):
            step()
        ms = _time(step, args.steps, stream)
        flops = 20.0 * N * N * M
        nbytes = 48.0 * P
        # the oracle (numpy FFT) on a bounded sample of vesicles, for context
        from oracle import spectral as SP
        sample = 200
        j1 = int(s.offsets[sample])
        t0 = time.time()
        SP.elastic_force(s.X[:, :j1], sig_h[:j1], 1.0, s.offsets[:sample + 1])
        cpu_vps = sample / (time.time() - t0)
        case = {"case": name, "n_points": P, "ms": ms, "points_per_s": P / (ms * 1e-3),
                "fp64": {"achieved_tflops": flops / (ms * 1e-3) / 1e12,
                         "frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
                "hbm": {"achieved_gbps": nbytes / (ms * 1e-3) / 1e9, "frac": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS},
                "cpu_baseline": {"value": cpu_vps, "unit": "vesicles/s", "kind": "oracle",
                                 "sample": f"{sample} vesicles, numpy FFT, one process"}}
        rec["cases"].append(case)
        log(f"[bench] force {name}: {ms * 1e3:.1f} us, {P / (ms * 1e-3):.3e} points/s, "
            f"{case['fp64']['achieved_tflops']:.2f} TFLOP/s FP64, {case['hbm']['achieved_gbps']:.0f} GB/s; "
            f"oracle {cpu_vps:.0f} vesicles/s")
    print(json.dumps(rec), flush=True)


def bench_nearfield(args):
    """Algorithm 4 with the layer velocities given (the paper predicts them with networks):
    masked far field with near-pair detection, five layers, Gaussian RBF fit by batched
    Cholesky, interpolation at the near pairs; 2000 vesicles x 32 points at 30% area fraction."""
    import numpy as np
    import torch

    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    from paper_2606_25569_amd.farfield import _ptr
    from synth import suspension as S

    t0 = time.time()
    s = S.rsa_suspension(S.config_seed(5), 2000, 32, 0.30)
    P, M, N = s.n_points, s.n_vesicles, 32
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    X = torch.tensor(s.X, device=dev)
    f = torch.tensor(s.f, device=dev)
    w = torch.tensor(s.w, device=dev)
    part = V.Partition(s.offsets, dev)
    lib = L.lib()
    prec = L.precision_code("fp32c")
    ws = torch.empty(V.workspace_bytes(P, M, "fp32c"), dtype=torch.uint8, device=dev)
    out = torch.empty((2, P), dtype=torch.float64, device=dev)
    cap = 8 * P
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    layers = torch.empty((2, 5 * P), dtype=torch.float64, device=dev)
    coeffs = torch.empty_like(layers)
    rws = torch.empty(lib.vesnet_rbf_workspace_bytes(N, M), dtype=torch.uint8, device=dev)
    width = 1.0

    def far():
        L.check(lib.vesnet_farfield_stokeslet_nearmasked(_ptr(X), _ptr(X), _ptr(f), _ptr(w), _ptr(part.device), M, P,
                                                         s.mu, _ptr(out), _ptr(pairs), cap, _ptr(count), prec, None,
                                                         _ptr(ws), ws.numel(), sp))

    def lay():
        L.check(lib.vesnet_near_layers(_ptr(X), _ptr(w), _ptr(part.device), M, P, _ptr(layers), sp))

    far()
    lay()
    torch.cuda.synchronize()
    n_near = int(count.item())
    assert n_near <= cap
    vel = torch.tensor(S.smooth_field(S.config_seed(5, 1), layers.cpu().numpy()), device=dev)

    def fit():
        L.check(lib.vesnet_rbf_fit(_ptr(layers), _ptr(vel), _ptr(w), _ptr(part.device), M, P, N, width, _ptr(coeffs),
                                   _ptr(rws), rws.numel(), sp))

    def ev():
        L.check(lib.vesnet_rbf_eval_near(_ptr(layers), _ptr(coeffs), _ptr(w), _ptr(part.device), M, P, width, _ptr(X),
                                         P, _ptr(pairs), _ptr(count), cap, _ptr(out), sp))

    def step():
        far()
        lay()
        fit()
        ev()

    # the same step with the masked far field by the fast multipole method (FP64, order 30)
    order = 30
    depth = lib.vesnet_fmm_default_depth(P, order)
    fws = torch.empty(lib.vesnet_fmm_nearmasked_workspace_bytes(P, M, depth, order), dtype=torch.uint8, device=dev)
    out_f = torch.empty_like(out)
    pairs_f = torch.empty_like(pairs)
    count_f = torch.zeros_like(count)

    def far_fmm():
        L.check(lib.vesnet_farfield_fmm_nearmasked(_ptr(X), _ptr(f), _ptr(w), _ptr(part.device), M, P, s.mu, order,
                                                   depth, _ptr(out_f), _ptr(pairs_f), cap, _ptr(count_f), _ptr(fws),
                                                   fws.numel(), sp))

    def ev_fmm():
        L.check(lib.vesnet_rbf_eval_near(_ptr(layers), _ptr(coeffs), _ptr(w), _ptr(part.device), M, P, width, _ptr(X),
                                         P, _ptr(pairs_f), _ptr(count_f), cap, _ptr(out_f), sp))

    def step_fmm():
        far_fmm()
        lay()
        fit()
        ev_fmm()

    far_fmm()
    torch.cuda.synchronize()
    assert int(count_f.item()) == n_near, (int(count_f.item()), n_near)
    fmm_diff = float((out_f - out).abs().max() / out.abs().max())  # both masked, before interpolation
    log(f"[bench] nearfield 2000x32: P={P}, {n_near} near pairs ({time.time() - t0:.1f}s)")
    times = {k: _time(fn, args.steps, stream) for k, fn in
             (("far_masked", far), ("layers", lay), ("rbf_fit", fit), ("rbf_eval", ev), ("step", step),
              ("far_masked_fmm", far_fmm), ("step_fmm", step_fmm))}
    n = 5 * N
    fit_flops = M * (n ** 3 / 3 + 4 * n * n)  # Cholesky and two triangular solves of two right-hand sides
    pairs_far = s.cross_pairs()
    # the oracle's fit (numpy Cholesky) of a sample of vesicles, for context
    from oracle import nearfield_rbf as NR
    lay_h = layers.cpu().numpy()
    vel_h = vel.cpu().numpy()
    sample = 100
    tc = time.time()
    for v in range(sample):
        a, b = 5 * s.offsets[v], 5 * s.offsets[v + 1]
        NR.vesicle_fit(lay_h[:, a:b], vel_h[:, a:b], width * s.w[s.offsets[v]:s.offsets[v + 1]].mean())
    cpu_fit_vps = sample / (time.time() - tc)
    rec = {"workload": "near field: 2000 vesicles x 32 points at 30% area fraction (gap >= 0.1 < h), "
                       "FP32-compensated masked far field + FP64 layers, RBF fit (width h) and interpolation; "
                       f"step_fmm: the masked far field by the fast multipole method (FP64, order {order}, depth {depth})",
           "n_points": P, "near_pairs": n_near, "ms": times,
           "far_masked_pairs_per_s": pairs_far / (times["far_masked"] * 1e-3),
           "rbf_fit": {"vesicles_per_s": M / (times["rbf_fit"] * 1e-3), "algorithmic_tflops_fp64": fit_flops / (times["rbf_fit"] * 1e-3) / 1e12,
                       "frac_of_fp64_peak": fit_flops / (times["rbf_fit"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                       "oracle_numpy_vesicles_per_s": cpu_fit_vps},
           "rbf_eval_pairs_per_s": n_near / (times["rbf_eval"] * 1e-3),
           "far_masked_fmm_vs_direct_rel_diff": fmm_diff}
    log(f"[bench] nearfield: " + ", ".join(f"{k} {v:.3f} ms" for k, v in times.items()))
    print(json.dumps(rec), flush=True)


def _treecode_work(X, sizes, depth):
    """Work of one treecode evaluation from its tree: (target, non-empty far box) evaluations,
    direct pairs with other vesicles' points in the 3 x 3 leaves (own vesicle assumed inside them),
    and the fast multipole method's (non-empty target box, non-empty source box) translations."""
    import numpy as np
    x, y = X
    side = max(x.max() - x.min(), y.max() - y.min())
    x0 = 0.5 * (x.min() + x.max()) - 0.5 * side
    y0 = 0.5 * (y.min() + y.max()) - 0.5 * side
    n = 1 << depth
    ix = np.clip(np.floor((x - x0) / (side / n)), 0, n - 1).astype(np.int64)
    iy = np.clip(np.floor((y - y0) / (side / n)), 0, n - 1).astype(np.int64)
    n_box = n_m2l = 0
    for l in range(2, depth + 1):
        nl = 1 << l
        bx, by = ix >> (depth - l), iy >> (depth - l)
        occ = np.bincount(bx * nl + by, minlength=nl * nl) > 0
        tb = np.flatnonzero(occ)
        tx, ty = tb // nl, tb % nl
        for a in range(-2, 4):
            for b in range(-2, 4):
                sx, sy = 2 * (bx >> 1) + a, 2 * (by >> 1) + b
                ok = (sx >= 0) & (sx < nl) & (sy >= 0) & (sy < nl) & ((np.abs(sx - bx) > 1) | (np.abs(sy - by) > 1))
                n_box += int(occ[np.where(ok, sx * nl + sy, 0)][ok].sum())
                sx, sy = 2 * (tx >> 1) + a, 2 * (ty >> 1) + b
                ok = (sx >= 0) & (sx < nl) & (sy >= 0) & (sy < nl) & ((np.abs(sx - tx) > 1) | (np.abs(sy - ty) > 1))
                n_m2l += int(occ[np.where(ok, sx * nl + sy, 0)][ok].sum())
    cnt = np.bincount(ix * n + iy, minlength=n * n).reshape(n, n)
    pad = np.pad(cnt, 1)
    near = sum(pad[1 + a:1 + a + n, 1 + b:1 + b + n] for a in (-1, 0, 1) for b in (-1, 0, 1))
    n_direct = int(near[ix, iy].sum() - np.repeat(sizes, sizes).sum())
    return n_box, n_direct, n_m2l


def _nonempty_leaves(X, depth):
    import numpy as np
    x, y = X
    side = max(x.max() - x.min(), y.max() - y.min())
    x0 = 0.5 * (x.min() + x.max()) - 0.5 * side
    y0 = 0.5 * (y.min() + y.max()) - 0.5 * side
    n = 1 << depth
    ix = np.clip(np.floor((x - x0) / (side / n)), 0, n - 1).astype(np.int64)
    iy = np.clip(np.floor((y - y0) / (side / n)), 0, n - 1).astype(np.int64)
    return int(np.unique(ix * n + iy).size)


def bench_treecode(args):
    """The 2000 x 128 workload by the FP64 treecode (default depth), at several orders, against the
    exact sum on a seeded target sample; the direct FP32-compensated sum timed alongside."""
    import numpy as np
    import torch

    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    from synth import suspension as S

    s = S.load_config(1)
    P, M = s.n_points, s.n_vesicles
    pairs = s.cross_pairs()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    X = torch.tensor(s.X, device=dev)
    f = torch.tensor(s.f, device=dev)
    w = torch.tensor(s.w, device=dev)
    part = V.Partition(s.offsets, dev)
    lib = L.lib()
    depth = int(lib.vesnet_treecode_default_depth(P))
    out = torch.empty((2, P), dtype=torch.float64, device=dev)
    sel = np.sort(np.random.default_rng(S.config_seed(1, 7)).choice(P, 2000, replace=False))
    from oracle import oracle as O
    t0 = time.time()
    exact = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)
    t_oracle = time.time() - t0
    scale = float(np.abs(exact).max())
    n_box, n_direct, n_m2l = _treecode_work(s.X, s.sizes(), depth)
    n_l2l = _nonempty_leaves(s.X, depth) * max(depth - 2, 0)  # (leaf, ancestor) shifts
    rec = {"workload": "treecode and fast multipole far field of the dense suspension: 2000 vesicles x 128 "
                       f"points (256000), uniform quadtree depth {depth}, FP64",
           "far_box_evaluations": n_box, "direct_pairs": n_direct, "m2l_translations": n_m2l, "l2l_shifts": n_l2l,
           "n_points": P, "cross_vesicle_pairs": pairs, "depth": depth, "orders": {}, "fmm_orders": {}}
    for order in (20, 30, 40):
        ws = torch.empty(lib.vesnet_treecode_workspace_bytes(P, depth, order), dtype=torch.uint8, device=dev)
        fn = lambda: V.farfield_treecode(X, f, w, part, s.mu, order, depth, out=out, workspace=ws)
        ms = _time(fn, args.steps, stream)
        fn()
        torch.cuda.synchronize()
        err = float(np.abs(out.cpu().numpy()[:, sel] - exact).max() / scale)
        flops = (24 * order + 60) * n_box + FLOPS_PER_PAIR * n_direct  # three complex Horner chains per box
        rec["orders"][order] = {"ms": ms, "max_rel_err_vs_exact": err,
                                "equivalent_pairs_per_s": pairs / (ms * 1e-3),
                                "algorithmic_tflops_fp64": flops / (ms * 1e-3) / 1e12,
                                "frac_of_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        log(f"[bench] treecode order {order}: {ms:.3f} ms, err {err:.2e} of max|u| on {sel.size} targets")
        ws = torch.empty(lib.vesnet_fmm_workspace_bytes(P, depth, order), dtype=torch.uint8, device=dev)
        fn = lambda: V.farfield_fmm(X, f, w, part, s.mu, order, depth, out=out, workspace=ws)
        ms = _time(fn, args.steps, stream)
        fn()
        torch.cuda.synchronize()
        err = float(np.abs(out.cpu().numpy()[:, sel] - exact).max() / scale)
        # M2L 3 series x (p+1)^2 complex-by-real MACs (4 flops) per translation; L2L 3 series x (p+1)(p+2)/2
        # complex FMAs (8 flops) per (leaf, ancestor); L2P three complex Horner chains (12p flops) per target
        fflops = (12 * (order + 1) ** 2 * n_m2l + 12 * (order + 1) * (order + 2) * n_l2l + 12 * order * P
                  + FLOPS_PER_PAIR * n_direct)
        rec["fmm_orders"][order] = {"ms": ms, "max_rel_err_vs_exact": err, "equivalent_pairs_per_s": pairs / (ms * 1e-3),
                                    "algorithmic_tflops_fp64": fflops / (ms * 1e-3) / 1e12,
                                    "frac_of_fp64_peak": fflops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        log(f"[bench] fmm order {order}: {ms:.3f} ms, err {err:.2e} of max|u| on {sel.size} targets")
    wsd = torch.empty(V.workspace_bytes(P, M, "fp32c"), dtype=torch.uint8, device=dev)
    ms_direct = _time(lambda: V.farfield_forward(X, X, f, w, part, s.mu, "fp32c", out=out, workspace=wsd), 5, stream)
    rec["direct_fp32c_ms"] = ms_direct
    # scaling in P: the fast multipole method, order 30 at the default depth, on twice the points
    s2 = S.load_config(2)
    P2 = s2.n_points
    X2, f2, w2 = (torch.tensor(a, device=dev) for a in (s2.X, s2.f, s2.w))
    part2 = V.Partition(s2.offsets, dev)
    depth2 = int(lib.vesnet_fmm_default_depth(P2, 30))
    out2 = torch.empty((2, P2), dtype=torch.float64, device=dev)
    ws2 = torch.empty(lib.vesnet_fmm_workspace_bytes(P2, depth2, 30), dtype=torch.uint8, device=dev)
    fn2 = lambda: V.farfield_fmm(X2, f2, w2, part2, s2.mu, 30, depth2, out=out2, workspace=ws2)
    ms2 = _time(fn2, args.steps, stream)
    fn2()
    torch.cuda.synchronize()
    sel2 = np.sort(np.random.default_rng(S.config_seed(2, 7)).choice(P2, 1000, replace=False))
    exact2 = O.farfield_suspension(s2.X, s2.f, s2.w, s2.offsets, s2.mu, select=sel2)
    err2 = float(np.abs(out2.cpu().numpy()[:, sel2] - exact2).max() / np.abs(exact2).max())
    rec["fmm_scaling"] = {"workload": "8000 vesicles x 64 points (512000), force-free", "depth": depth2, "order": 30,
                          "ms": ms2, "max_rel_err_vs_exact": err2, "cross_vesicle_pairs": s2.cross_pairs(),
                          "equivalent_pairs_per_s": s2.cross_pairs() / (ms2 * 1e-3)}
    log(f"[bench] fmm 8000 x 64, depth {depth2}, order 30: {ms2:.3f} ms, err {err2:.2e} of max|u| on {sel2.size} targets")
    rec["oracle_sample"] = {"targets": int(sel.size), "seconds": t_oracle}
    log(f"[bench] direct FP32-compensated sum: {ms_direct:.3f} ms")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
