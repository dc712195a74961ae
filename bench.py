"""Throughput of the fused D2Q37 time step on one MI355X.

Workload (one line of JSON on stdout): a 2048 x 2048 periodic lattice, shear
wave u_x = 0.05 sin(2 pi y / LY) plus 1e-4 seeded noise, tau = 0.8, FP64
populations in the CAoSoA layout (the layout the paper's Table 1 uses),
propagate and collide fused in one kernel with ping-pong buffers. `value` is million lattice updates per second (MLUPS)
over K timed steps with the state resident in HBM.

The same line carries the other forms of the step measured on the same GPU
(FP32-shifted and FP16-shifted storage with their per-field error against
the FP64 run on the shear wave and on a thermal Rayleigh-Taylor-like state,
the AoS/SoA/CSoA layouts, the split propagate + collide path, the learned
collide trained on the GPU from 10M pairs, and the 8192 x 8192
Rayleigh-Taylor-like lattice in FP64, FP32-shifted and learned form), a
roofline object for the dominant kernel and the CPU oracle timed on the host
cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS fused step, FP64 vs FP32-shifted/surrogate at stated err; % HBM roof"
LX = LY = 2048
TAU = 0.8
# Learned collide: training set and schedule, fallback threshold.
NPAIRS = 10_000_000
PAIR_SEED, INIT_SEED, ORDER_SEED = 11, 5, 17
EPOCHS, BATCH, LR = 32, 8192, 3e-3
THRESHOLD = 5e-5
# Step counts of the accuracy runs, fixed by the workloads themselves (not by
# --steps): 1000 steps on the 2048 x 2048 lattices, 500 on 8192 x 8192.
ERR_STEPS_2048 = 1000
ERR_STEPS_8192 = 500
HEADLINE_REPEATS = 5
# MFMA work of one site (37-128-128-37, multiply-adds counted as 2 flops).
MLP_FLOP_PER_SITE = 2 * (37 * 128 + 128 * 128 + 128 * 37)
BF16_PEAK_TFLOPS = 2500.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def timed_steps(lat, torch, nsteps: int, split: bool = False) -> float:
    """Seconds for nsteps, HIP events on the lattice's stream."""
    stream = lat.stream
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    if split:
        for _ in range(nsteps):
            lat.propagate()
            lat.collide()
    else:
        lat.step(nsteps)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def field_errors(ref, got):
    """Per-field max and rms absolute error against the FP64 run."""
    names = ("rho", "ux", "uy", "T")
    out = {}
    for n, a, b in zip(names, ref, got):
        d = (b - a)
        out[n] = {"max_abs": float(d.abs().max()), "rms": float(d.pow(2).mean().sqrt())}
    return out


def copy_bandwidth(torch, lb, nbytes: int, reps: int = 20) -> float:
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    lb.device_copy(dst, src)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        lb.device_copy(dst, src)
    stop.record(stream)
    stop.synchronize()
    dt = start.elapsed_time(stop) / 1e3 / reps
    return 2 * nbytes / dt / 1e9


def traffic_entry(kernel: str, per_launch_sites: int, field: str = "hbm_bytes_per_launch"):
    """A figure (HBM bytes per launch by default) from the committed
    rocprofv3 counter summary, if it was taken on the current kernel
    sources; else None."""
    from paper_1804_01918_amd.profsummary import source_digest
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    with open(PROFILE_TRAFFIC) as fh:
        rec = json.load(fh)
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("sites") != per_launch_sites or "source_files" not in k:
        return None
    if k.get("source_digest") != source_digest(k["source_files"]):
        return None
    return k.get(field)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS", "")
    visible = len(os.sched_getaffinity(0))
    return max(1, min(int(env), visible) if env.isdigit() and int(env) > 0 else visible)


def _oracle_mlups(lbm, inputs, n: int, seconds_target: float, min_steps: int = 1):
    f = lbm.init(*inputs.shear_wave(n, n, seed=0))
    t0 = time.perf_counter()
    f = lbm.run(f, TAU, 1)
    one = time.perf_counter() - t0
    steps = max(min_steps, int(seconds_target / max(one, 1e-3)))
    t0 = time.perf_counter()
    lbm.run(f, TAU, steps)
    dt = time.perf_counter() - t0
    return n * n * steps / dt / 1e6, steps, dt


def _oracle_config1(lbm, inputs):
    """The 128 x 64 correctness workload in full: 100 steps from the random
    equilibrium (seed 0)."""
    f = lbm.init(*inputs.random_equilibrium(128, 64, seed=0))
    t0 = time.perf_counter()
    lbm.run(f, TAU, 100)
    dt = time.perf_counter() - t0
    return 128 * 64 * 100 / dt / 1e6, dt


def cpu_baseline(seconds_target: float = 10.0):
    """The FP64 oracle (plain C, the same source built once) on the host's
    cores: all the threads the process may use (OpenMP over lattice columns)
    on the 2048 x 2048 shear-wave workload for at least 10 steps (a
    shortened run: the cost per step is constant), one thread on a 512 x 512
    lattice of the same state, and the 128 x 64 workload in full on both."""
    from oracle import lbm
    from paper_1804_01918_amd import inputs
    nthreads = _host_threads()
    try:
        lbm.set_threads(1)
        m1, s1, t1 = _oracle_mlups(lbm, inputs, 512, seconds_target)
        c1, ct1 = _oracle_config1(lbm, inputs)
        lbm.set_threads(nthreads)
        mn, sn, tn = _oracle_mlups(lbm, inputs, LX, seconds_target, min_steps=10)
        cn, ctn = _oracle_config1(lbm, inputs)
    finally:
        lbm.set_threads(1)
    return {"value": mn, "unit": "MLUPS", "cores": nthreads, "kind": "oracle",
            "sample": f"FP64 oracle, {LX}x{LY} shear-wave lattice (the benchmark workload), {sn} of its 1000 "
                      f"steps, {nthreads} threads (OpenMP over columns), {tn:.1f} s",
            "single_thread": {"value": m1, "unit": "MLUPS", "cores": 1,
                              "sample": f"FP64 oracle, 512x512 shear-wave lattice, {s1} steps, 1 thread, {t1:.1f} s"},
            "config_128x64_100_steps": {"single_thread_mlups": c1, "single_thread_s": ct1,
                                        "all_threads_mlups": cn, "all_threads_s": ctn},
            "cpu_model": _cpu_model(), "host_cpus_visible": len(os.sched_getaffinity(0))}


def train_network(torch, lb, train: bool = True):
    """Pairs from the plain FP32 collide, standardisation, Philox init and
    Adam, all on the GPU; returns the network and the training record. With
    train=False the network keeps its initial weights."""
    t0 = time.perf_counter()
    pre, post = lb.pairgen(NPAIRS, PAIR_SEED, TAU)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = lb.Mlp(BATCH)
    net.fit_normalization(pre, post, TAU)
    net.init(INIT_SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(pre, post, TAU, BATCH, EPOCHS, LR, ORDER_SEED) if train else [float("nan")]
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del pre, post
    torch.cuda.empty_cache()
    return net, {"pairs": NPAIRS, "pairgen_s": t_pairs, "epochs": EPOCHS, "batch": BATCH, "lr": LR,
                 "adam_steps": (NPAIRS // BATCH) * EPOCHS, "train_s": t_train,
                 "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1])}


def learned_variant(args, torch, lb, inputs, run, counts, nsites, shear_ref, rt_ref):
    """Train the network on the GPU (pairs, standardisation, Adam), then time
    the learned fused step on the shear wave and state its error against the
    FP64 run of the same number of steps."""
    from paper_1804_01918_amd.roofline import HBM_PEAK_GBS, bytes_per_site
    net, training = train_network(torch, lb)
    counts.clear()
    timed = ERR_STEPS_2048 - args.warmup
    dt, mom = run("f32s", "caosoa", timed, args.warmup, keep=True, net=net)
    m = nsites * timed / dt / 1e6
    v = {"mlups": m, "ms_per_step": dt / timed * 1e3, "timed_steps": timed, "threshold": THRESHOLD,
         "network_form": "first layer BF16 (v_mfma_f32_16x16x32_bf16); hidden activations, their GELU arithmetic "
                         "and the last two layers binary16 (v_mfma_f32_16x16x32_f16); FP32 accumulation",
         "fallback_fraction": counts.get("fallback_fraction"),
         "mfma_tflops": m * 1e6 * MLP_FLOP_PER_SITE / 1e12,
         "mfma_frac": m * 1e6 * MLP_FLOP_PER_SITE / 1e12 / BF16_PEAK_TFLOPS,
         "hbm_frac": m * 1e6 * bytes_per_site("f32") / (HBM_PEAK_GBS * 1e9),
         "hbm_traffic_bytes_per_launch": traffic_entry("k_step_learned_f32s_caosoa_2048x2048", nsites),
         "algorithmic_bytes_per_launch": bytes_per_site("f32") * nsites,
         "error_vs_f64_after_steps": ERR_STEPS_2048,
         "field_error_vs_f64": field_errors(shear_ref, mom) if shear_ref is not None else None,
         "training": training}
    if rt_ref is not None:
        rt = (LX, LY, [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(LX, LY, seed=0)])
        counts.clear()
        _, mom = run("f32s", "caosoa", timed, args.warmup, keep=True, state=rt, net=net)
        v["rayleigh_taylor_2048"] = {"error_vs_f64_after_steps": ERR_STEPS_2048,
                                     "fallback_fraction": counts.get("fallback_fraction"),
                                     "field_error_vs_f64": field_errors(rt_ref, mom)}
    # the same trained network with its hidden layer in FP8 (e4m3)
    net.set_precision("fp8")
    counts.clear()
    dt, mom = run("f32s", "caosoa", timed, args.warmup, keep=True, net=net)
    m8 = nsites * timed / dt / 1e6
    v8 = {"mlups": m8, "ms_per_step": dt / timed * 1e3, "threshold": THRESHOLD,
          "hidden_layer": "e4m3 inputs and weights, v_mfma_f32_16x16x32_fp8_fp8; first and last layers BF16",
          "fallback_fraction": counts.get("fallback_fraction"), "error_vs_f64_after_steps": ERR_STEPS_2048,
          "field_error_vs_f64": field_errors(shear_ref, mom) if shear_ref is not None else None}
    if rt_ref is not None:
        counts.clear()
        _, mom = run("f32s", "caosoa", timed, args.warmup, keep=True, state=rt, net=net)
        v8["rayleigh_taylor_2048"] = {"error_vs_f64_after_steps": ERR_STEPS_2048,
                                      "fallback_fraction": counts.get("fallback_fraction"),
                                      "field_error_vs_f64": field_errors(rt_ref, mom)}
    net.set_precision("f16")
    v["fp8_hidden_layer"] = v8
    return v, net


def time_calls(lat, torch, fn, n: int) -> float:
    """Seconds for n calls of fn on the lattice's stream (HIP events)."""
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(lat.stream)
    for _ in range(n):
        fn()
    stop.record(lat.stream)
    stop.synchronize()
    return start.elapsed_time(stop) / 1e3


# The paper's Table 1 (FP64, separate propagate and collide kernels,
# 1024 x 8192 lattice): T_prop and T_coll in ms per call.
TABLE1 = {"KNL 7230 flat/quad": (12.5, 50.3), "KNL 7230 cache/quad": (19.65, 51.42), "P100": (12.5, 24.1),
          "GK210": (32.3, 71.1), "KNC 7120P": (49.9, 180.9), "E5-2697v4": (98.06, 173.42)}


def table1_variant(args, torch, lb, inputs):
    """The paper's Table 1 workload shape on this GPU: FP64 CAoSoA,
    1024 x 8192, propagate and collide timed as separate kernels (as the
    paper does) and fused."""
    lx, ly = 1024, 8192
    n = lx * ly
    fields = [torch.from_numpy(a).cuda() for a in inputs.shear_wave(lx, ly, seed=0)]
    lat = lb.Lattice(lx, ly, TAU, fields, precision="f64", layout="caosoa")
    reps = max(10, args.variant_steps)
    for _ in range(args.warmup):
        lat.propagate()
        lat.collide()
    t_prop = time_calls(lat, torch, lat.propagate, reps) / reps
    t_coll = time_calls(lat, torch, lat.collide, reps) / reps
    t_step = time_calls(lat, torch, lambda: lat.step(1), reps) / reps
    lat.close()
    del lat, fields
    torch.cuda.empty_cache()
    return {"lattice": [lx, ly], "precision": "f64", "layout": "caosoa",
            "T_prop_ms": t_prop * 1e3, "T_coll_ms": t_coll * 1e3,
            "propagate_GBs": 2 * 37 * 8 * n / t_prop / 1e9, "collide_mlups": n / t_coll / 1e6,
            "split_step_mlups": n / (t_prop + t_coll) / 1e6, "fused_step_mlups": n / t_step / 1e6,
            "paper_table1_ms": {k: {"T_prop": a, "T_coll": b, "global_mlups_from_T": n / ((a + b) * 1e-3) / 1e6}
                                for k, (a, b) in TABLE1.items()}}


def graph_variant(args, torch, lb, inputs):
    """The small 128 x 64 lattice (8,192 sites: a few microseconds of GPU
    work per step, so launches dominate): FP64 CAoSoA steps launched one by
    one from the library's loop against the same steps captured once into a
    HIP graph (torch.cuda.CUDAGraph over lb_step) and replayed."""
    lx, ly, per, reps = 128, 64, 100, 20
    fields = [torch.from_numpy(a).cuda() for a in inputs.shear_wave(lx, ly, seed=0)]
    cap = torch.cuda.Stream()
    with torch.cuda.stream(cap):
        lat = lb.Lattice(lx, ly, TAU, fields, precision="f64", layout="caosoa")
        lat.step(10)
    torch.cuda.synchronize()
    t_eager = time_calls(lat, torch, lambda: lat.step(per), reps)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        lat.step(per)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(cap)
    for _ in range(reps):
        graph.replay()
    stop.record(cap)
    stop.synchronize()
    t_graph = start.elapsed_time(stop) / 1e3
    lat.close()
    del lat, graph
    torch.cuda.empty_cache()
    n = lx * ly * per * reps
    return {"lattice": [lx, ly], "precision": "f64", "layout": "caosoa", "steps": per * reps,
            "us_per_step_launched": t_eager / (per * reps) * 1e6, "us_per_step_graph": t_graph / (per * reps) * 1e6,
            "mlups_launched": n / t_eager / 1e6, "mlups_graph": n / t_graph / 1e6}


def energy_variant(args, torch, lb, fields, net):
    """Package power on the GPU's energy counter while a kernel loop runs
    (2048 x 2048 shear wave, about 3 s per loop), times the loop's GPU time:
    energy per lattice update of the fused step for each form and, as in the
    paper's energy figure, energy per iteration of the separate propagate
    and collide kernels for each FP64 layout."""
    from paper_1804_01918_amd.energy import EnergyMeter
    meter = EnergyMeter(0)
    out = {"available": meter.available, "reason": meter.reason or None,
           "method": "package power between energy-counter refreshes (about 1 s apart) inside the loop, "
                     "times GPU time per call; graphics clock and the share of the loop under "
                     "package-power throttling from the metrics table at the same refreshes",
           "power_cap_watts": meter.power_limit_watts(),
           "fused_step": {}, "f64_split_kernels_by_layout": {}}
    if not meter.available:
        return out

    def run_for(lat, fn, target_s):
        t = time_calls(lat, torch, fn, 20) / 20
        n = max(50, int(target_s / max(t, 1e-6)))
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()

        chunk = 10
        nchunks = (n + chunk - 1) // chunk
        n = nchunks * chunk
        state = {"i": 0}

        def launch_chunk():
            if state["i"] == 0:
                start.record(lat.stream)
            for _ in range(chunk):
                fn()
            state["i"] += 1
            if state["i"] == nchunks:
                stop.record(lat.stream)

        watts, span, refreshes = meter.power_during(launch_chunk, nchunks, stop.query)
        stop.synchronize()
        per_call = start.elapsed_time(stop) / 1e3 / n
        return {"calls": n, "gpu_s_per_call": per_call, "avg_watts": watts, "sampled_s": span,
                "counter_refreshes": refreshes, "J_per_call": watts * per_call if watts is not None else None,
                "gfxclk_mhz": meter.last_clock_mhz, "power_throttled_share": meter.last_power_throttled}

    forms = [("f64", None), ("f32s", None), ("f16s", None)] + ([("f32s", net)] if net is not None else [])
    for prec, nn in forms:
        lat = lb.Lattice(LX, LY, TAU, fields, precision=prec, layout="caosoa")
        if nn is not None:
            lat.set_surrogate(nn, THRESHOLD)
        lat.step(args.warmup)
        r = run_for(lat, lambda: lat.step(1), 3.5)
        r["nJ_per_lattice_update"] = r["J_per_call"] / (LX * LY) * 1e9 if r["J_per_call"] is not None else None
        out["fused_step"][("learned_" if nn is not None else "") + f"{prec}_caosoa"] = r
        lat.close()
        del lat
        torch.cuda.empty_cache()
    for layout in ("aos", "soa", "csoa", "caosoa"):
        lat = lb.Lattice(LX, LY, TAU, fields, precision="f64", layout=layout)
        out["f64_split_kernels_by_layout"][layout] = {
            "propagate": run_for(lat, lat.propagate, 2.5), "collide": run_for(lat, lat.collide, 2.5)}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    meter.close()
    return out


# Rayleigh-Taylor setting with gravity and walls: acceleration along -y
# (thermal units per step) and the walls at the two layers' temperatures.
RT_GRAVITY = (0.0, -1e-4)
RT_WALLS = dict(walls=True, t_bottom=1.05, t_top=0.95)


def gravity_walls_variant(args, torch, lb, inputs):
    """2048 x 2048 Rayleigh-Taylor-like state under gravity between diffuse
    walls (the paper's production setting), CAoSoA fused step in each
    precision: MLUPS, the FP64 mass audit over the run, and the shifted
    forms' field errors against the FP64 run after ERR_STEPS_2048 steps."""
    from paper_1804_01918_amd.roofline import HBM_PEAK_GBS, bytes_per_site
    fields = [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(LX, LY, seed=0)]
    timed = ERR_STEPS_2048 - args.warmup
    out = {"lattice": [LX, LY], "gravity": list(RT_GRAVITY), **RT_WALLS, "steps": ERR_STEPS_2048,
           "timed_steps": timed}
    ref = None
    for prec in ("f64", "f32s", "f16s"):
        lat = lb.Lattice(LX, LY, TAU, fields, precision=prec, layout="caosoa", audit=True, force=RT_GRAVITY,
                         **RT_WALLS)
        a0 = lat.audit()
        lat.step(args.warmup)
        dt = timed_steps(lat, torch, timed)
        a1 = lat.audit()
        mom = lat.moments()
        lat.close()
        del lat
        m = LX * LY * timed / dt / 1e6
        r = {"mlups": m, "hbm_frac": m * 1e6 * bytes_per_site(prec[:3]) / (HBM_PEAK_GBS * 1e9),
             "mass_drift_rel": float((a1[0] - a0[0]) / a0[0])}
        if prec == "f64":
            ref = mom
        else:
            r["field_error_vs_f64"] = field_errors(ref, mom)
            del mom
        out[prec] = r
        torch.cuda.empty_cache()
    del ref, fields
    torch.cuda.empty_cache()
    return out


def scale_variant(args, torch, inputs, run, counts, net):
    """8192 x 8192 Rayleigh-Taylor-like lattice: FP64, FP32-shifted and the
    learned collide on the same GPU, errors against the FP64 run."""
    n = 8192
    state = (n, n, [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(n, n, seed=0)])
    warm = args.warmup
    steps = args.scale_steps - warm
    out = {"lattice": [n, n], "steps": steps + warm, "error_vs_f64_after_steps": steps + warm,
           "timed_steps": steps}
    dt, ref = run("f64", "caosoa", steps, warm, keep=True, state=state)
    out["f64"] = {"mlups": n * n * steps / dt / 1e6,
                  "hbm_frac": n * n * steps / dt * 592 / 8e12}
    dt, mom = run("f32s", "caosoa", steps, warm, keep=True, state=state)
    out["f32s"] = {"mlups": n * n * steps / dt / 1e6, "field_error_vs_f64": field_errors(ref, mom)}
    dt, mom = run("f16s", "caosoa", steps, warm, keep=True, state=state)
    out["f16s"] = {"mlups": n * n * steps / dt / 1e6, "field_error_vs_f64": field_errors(ref, mom)}
    counts.clear()
    dt, mom = run("f32s", "caosoa", steps, warm, keep=True, state=state, net=net)
    out["learned_f32s"] = {"mlups": n * n * steps / dt / 1e6, "fallback_fraction": counts.get("fallback_fraction"),
                           "field_error_vs_f64": field_errors(ref, mom)}
    del state, ref, mom
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--variant-steps", type=int, default=200)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--threshold", type=float, default=None,
                    help="with --only learned: fallback threshold (default: the benchmark's)")
    ap.add_argument("--untrained", action="store_true",
                    help="with --only learned: skip the training (counter runs; HBM bytes do not depend on it)")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--scale-steps", type=int, default=ERR_STEPS_8192,
                    help="total steps (warm-up included) of the 8192 x 8192 runs")
    ap.add_argument("--only", default=None,
                    help="precision:layout[:split][:walls], 'learned' or 'learned_fp8', to time alone")
    ap.add_argument("--lattice", type=int, default=LX,
                    help="with --only: the lattice size N x N (the Rayleigh-Taylor-like state unless N is 2048)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run the library's copy kernel on buffers of this size (counter calibration)")
    ap.add_argument("--copy-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the lattice is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1804_01918_amd import inputs, lb
    from paper_1804_01918_amd.roofline import HBM_PEAK_GBS, bytes_per_site

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_bytes:
        gbs = copy_bandwidth(torch, lb, args.copy_bytes, reps=args.copy_reps)
        print(json.dumps({"copy_bytes": args.copy_bytes, "reps": args.copy_reps, "GB/s": gbs}))
        return
    fields = [torch.from_numpy(a).cuda() for a in inputs.shear_wave(LX, LY, seed=0)]
    nsites = LX * LY
    counts = {}

    def run(prec, layout, steps, warmup, split=False, keep=False, state=None, net=None, threshold=THRESHOLD,
            compensated=None, bc=None):
        lx, ly, flds = state if state is not None else (LX, LY, fields)
        lat = lb.Lattice(lx, ly, TAU, flds, precision=prec, layout=layout, audit=True, compensated=compensated,
                         **(bc or {}))
        if net is not None:
            lat.set_surrogate(net, threshold)
        if split:
            for _ in range(warmup):
                lat.propagate()
                lat.collide()
        else:
            lat.step(warmup)
        dt = timed_steps(lat, torch, steps, split=split)
        mom = lat.moments() if keep else None
        if net is not None:
            fb, tot = lat.surrogate_counts()
            counts["fallback_fraction"] = fb / max(tot, 1)
        lat.close()
        del lat
        torch.cuda.empty_cache()
        return dt, mom

    if args.only in ("learned", "learned_fp8"):
        net, _ = train_network(torch, lb, train=not args.untrained)
        if args.only == "learned_fp8":
            net.set_precision("fp8")
        # --lattice N other than 2048: the N x N Rayleigh-Taylor-like state
        n = args.lattice
        state = None if n == LX else (n, n, [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(n, n, seed=0)])
        dt, _ = run("f32s", "caosoa", args.steps, args.warmup, net=net, state=state,
                    threshold=THRESHOLD if args.threshold is None else args.threshold)
        print(json.dumps({"only": args.only, "lattice": [n, n], "mlups": n * n * args.steps / dt / 1e6,
                          "ms_per_step": dt / args.steps * 1e3, "fallback_fraction": counts.get("fallback_fraction")}))
        net.close()
        return
    if args.only:
        # precision:layout[:split][:walls]; "walls" runs the Rayleigh-Taylor-like
        # state under gravity between the diffuse walls; --lattice N times an
        # N x N lattice (the Rayleigh-Taylor-like state unless N is 2048)
        parts = args.only.split(":")
        walls = "walls" in parts[2:]
        n = args.lattice
        state = None
        if walls or n != LX:
            state = (n, n, [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(n, n, seed=0)])
        dt, _ = run(parts[0], parts[1], args.steps, args.warmup, split="split" in parts[2:], state=state,
                    bc=dict(force=RT_GRAVITY, **RT_WALLS) if walls else None)
        print(json.dumps({"only": args.only, "lattice": [n, n], "mlups": n * n * args.steps / dt / 1e6,
                          "ms_per_step": dt / args.steps * 1e3}))
        return

    # Headline: FP64 CAoSoA fused, the median of HEADLINE_REPEATS timed runs
    # of exactly --steps steps each (after --warmup untimed steps).
    lat = lb.Lattice(LX, LY, TAU, fields, precision="f64", layout="caosoa", audit=True)
    lat.step(args.warmup)
    head = sorted(timed_steps(lat, torch, args.steps) for _ in range(HEADLINE_REPEATS))
    lat.close()
    del lat
    torch.cuda.empty_cache()
    dt = head[HEADLINE_REPEATS // 2]
    mlups = nsites * args.steps / dt / 1e6
    t_launch = dt / args.steps
    alg_bytes = bytes_per_site("f64", fused=True) * nsites
    achieved = alg_bytes / t_launch / 1e9
    traffic = traffic_entry("k_step_f64_caosoa_2048x2048", nsites)

    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_launch * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "D2Q37 2048x2048 periodic shear wave (u_x=0.05 sin(2 pi y/LY) + 1e-4 noise), "
                               "FP64 populations, CAoSoA layout, fused propagate+collide, tau=0.8",
                   "lattice": [LX, LY], "precision": "f64", "layout": "caosoa", "fused": True, "tau": TAU,
                   "audit": "FP64 mass/momentum/energy sums fused into the last step of each timed run",
                   "value_is": f"median of {HEADLINE_REPEATS} timed runs of {args.steps} steps each"},
        "headline_repeats_mlups": [nsites * args.steps / d / 1e6 for d in head],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step<PrecF64, Layout<CAoSoA>> (fused propagate+collide)",
                     "algorithmic_bytes_per_site": bytes_per_site("f64", fused=True)},
        "collide_vector_flops": None,
    }

    fps = traffic_entry("k_step_f64_caosoa_2048x2048", nsites, "vector_flops_per_site")
    if fps:
        tf = fps * nsites / t_launch / 1e12
        out["collide_vector_flops"] = {"flops_per_site": fps, "achieved_tflops": tf, "fp64_vector_peak_tflops": 78.6,
                                       "frac": tf / 78.6, "source": "SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 counters"}
    # FP64 reference of the accuracy runs: the shear wave after exactly
    # ERR_STEPS_2048 steps (the workload's own count, whatever --steps is).
    err_timed = ERR_STEPS_2048 - args.warmup
    ref_mom = None
    if not (args.no_variants and args.no_learned):
        _, ref_mom = run("f64", "caosoa", err_timed, args.warmup, keep=True)
    rt_ref = None
    if not args.no_variants:
        variants = {}
        vs = args.variant_steps
        for prec in ("f32s", "f16s"):
            dtv, mom = run(prec, "caosoa", err_timed, args.warmup, keep=True)
            m = nsites * err_timed / dtv / 1e6
            variants[f"{prec}_caosoa_fused"] = {
                "compensated_moment_sums": prec == "f32s",
                "mlups": m, "ms_per_step": dtv / err_timed * 1e3, "timed_steps": err_timed,
                "hbm_frac": m * 1e6 * bytes_per_site(prec[:3]) / (HBM_PEAK_GBS * 1e9),
                "error_vs_f64_after_steps": ERR_STEPS_2048,
                "field_error_vs_f64": field_errors(ref_mom, mom),
                "hbm_traffic_bytes_per_launch": traffic_entry(f"k_step_{prec}_caosoa_2048x2048", nsites),
                "algorithmic_bytes_per_launch": bytes_per_site(prec[:3]) * nsites}
        # the same FP32 step with plain (uncompensated) moment sums
        dtv, mom = run("f32s", "caosoa", err_timed, args.warmup, keep=True, compensated=False)
        m = nsites * err_timed / dtv / 1e6
        variants["f32s_caosoa_fused_uncompensated"] = {
            "compensated_moment_sums": False, "mlups": m,
            "hbm_frac": m * 1e6 * bytes_per_site("f32") / (HBM_PEAK_GBS * 1e9),
            "error_vs_f64_after_steps": ERR_STEPS_2048, "field_error_vs_f64": field_errors(ref_mom, mom)}
        for layout in ("soa", "aos", "csoa"):
            dtv, _ = run("f64", layout, vs, args.warmup)
            m = nsites * vs / dtv / 1e6
            variants[f"f64_{layout}_fused"] = {"mlups": m, "hbm_frac": m * 1e6 * 592 / (HBM_PEAK_GBS * 1e9)}
        for layout in ("soa", "caosoa"):
            dtv, _ = run("f64", layout, vs, args.warmup, split=True)
            m = nsites * vs / dtv / 1e6
            variants[f"f64_{layout}_split"] = {"mlups": m, "hbm_frac": m * 1e6 * 1184 / (HBM_PEAK_GBS * 1e9)}
        cb = copy_bandwidth(torch, lb, alg_bytes // 2)
        variants["copy_kernel_gbs"] = cb
        out["roofline"]["frac_of_copy"] = achieved / cb

        variants["table1_1024x8192_f64"] = table1_variant(args, torch, lb, inputs)
        variants["graph_replay_128x64_f64"] = graph_variant(args, torch, lb, inputs)

        # Precision on the thermal Rayleigh-Taylor-like state.
        rt = (LX, LY, [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(LX, LY, seed=0)])
        _, rt_ref = run("f64", "caosoa", err_timed, args.warmup, keep=True, state=rt)
        variants["rayleigh_taylor_2048"] = {"error_vs_f64_after_steps": ERR_STEPS_2048}
        for prec in ("f32s", "f16s"):
            _, mom = run(prec, "caosoa", err_timed, args.warmup, keep=True, state=rt)
            variants["rayleigh_taylor_2048"][f"{prec}_field_error_vs_f64"] = field_errors(rt_ref, mom)
        _, mom = run("f32s", "caosoa", err_timed, args.warmup, keep=True, state=rt, compensated=False)
        variants["rayleigh_taylor_2048"]["f32s_uncompensated_field_error_vs_f64"] = field_errors(rt_ref, mom)
        variants["rayleigh_taylor_gravity_walls_2048"] = gravity_walls_variant(args, torch, lb, inputs)
        out["variants"] = variants

    if not args.no_learned:
        out["variants"] = out.get("variants", {})
        lv, net = learned_variant(args, torch, lb, inputs, run, counts, nsites, ref_mom, rt_ref)
        lv["mlups_vs_f32s_plain"] = (lv["mlups"] / out["variants"]["f32s_caosoa_fused"]["mlups"]
                                     if "f32s_caosoa_fused" in out["variants"] else None)
        out["variants"]["learned_f32s_caosoa_fused"] = lv
        if not args.no_scale:
            sv = scale_variant(args, torch, inputs, run, counts, net)
            out["variants"]["scale_8192_rayleigh_taylor"] = sv
            out["largest_single_gpu_config"] = {
                "workload": "D2Q37 8192x8192 periodic Rayleigh-Taylor-like state, FP64 populations, CAoSoA, "
                            "fused propagate+collide, tau=0.8",
                "steps": sv["steps"], "timed_steps": sv["timed_steps"], "f64_mlups": sv["f64"]["mlups"],
                "f64_hbm_frac": sv["f64"]["hbm_frac"], "f32s_mlups": sv["f32s"]["mlups"],
                "f16s_mlups": sv["f16s"]["mlups"], "learned_f32s_mlups": sv["learned_f32s"]["mlups"]}
        if not args.no_energy:
            out["variants"]["energy_2048"] = energy_variant(args, torch, lb, fields, net)
        net.close()

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
