#!/usr/bin/env python3
"""Benchmark of batched tricubic B-spline orbital VGL on one MI355X.

Step = one batch of the headline workload through the whole spline path
(lattice reduction, weights, 64-point gather-FMA, scaling, stores): an
80^3 grid with N=384 orbitals (the NiO-32 grid and electron count of the
paper's Table 1) in FP32, evaluated at 512 walkers x 384 electrons =
196,608 uniform random positions.  Inputs (table and positions) are resident
in HBM before the timed region.  Prints one JSON line.

Also reported in the same line: the BF16/FP16 storage forms on the same
workload (throughput, speedup over FP32 and error against the FP64 oracle),
the roofline of the dominant kernel, and the FP64 CPU oracle timed on a
bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_UNIT = {"f32": 64 * 4 + 20, "bf16": 64 * 2 + 20, "f16": 64 * 2 + 20, "f64": 64 * 8 + 40}
TUNE_CACHE = os.path.join(ROOT, "paper_1708_02645_amd", "tune_cache.txt")
KERNEL_SOURCES = ["paper_1708_02645_amd/csrc/eval_kernel.hpp", "paper_1708_02645_amd/csrc/eval_f32.hip",
                  "paper_1708_02645_amd/csrc/ratio_f32.hip", "paper_1708_02645_amd/csrc/shapes.hpp",
                  "paper_1708_02645_amd/csrc/common.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


VGH_SOURCES = KERNEL_SOURCES + ["paper_1708_02645_amd/csrc/vgh_kernel.hpp", "paper_1708_02645_amd/csrc/vgh_f32.hip"]
SORTED_SOURCES = KERNEL_SOURCES + ["paper_1708_02645_amd/csrc/locality.hip"]


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(tile, name: str = "vgl_f32_80cube_n384") -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source and tile shape."""
    p = os.path.join(ROOT, "profiles", name + "_traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    srcs = VGH_SOURCES if name.startswith("vgh") else SORTED_SOURCES if "sorted" in name else KERNEL_SOURCES
    if d.get("kernel_hash") != kernel_hash(srcs) or tuple(d.get("tile", ())) != tuple(tile):
        return None
    return d.get("hbm_bytes_per_launch")


LAST_TIMING = {}


def time_back_to_back(torch, fn, steps: int, warmup: int) -> float:
    """Mean ms per launch of `steps` launches issued back to back between one
    pair of HIP events (after `warmup` untimed ones): the average launch
    duration of a short kernel, without the per-launch event markers that a
    median of single launches carries."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        fn()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def time_burst_after_idle(torch, fn, n: int = 8, idle_s: float = 0.5, reps: int = 3):
    """Mean ms per launch of `n` back-to-back launches started after the GPU
    has been idle for `idle_s` seconds (median over `reps` such bursts): the
    duration at the clock an idle GPU starts from, before sustained
    matrix-core load makes the power management lower it.  A spin kernel
    enqueued first keeps the queue ahead of the host, so the event pair
    brackets the launches and no host latency."""
    import numpy as np

    st = torch.cuda.current_stream()
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        time.sleep(idle_s)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1_000_000)
        a.record(st)
        for _ in range(n):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / n)
    return float(np.median(out))


def time_steps(torch, fn, steps: int, warmup: int):
    """Runs `warmup` untimed steps, then exactly `steps` timed ones on the
    current stream (the one the library launches on), each between its own
    pair of HIP events, with a synchronization before and after.  Returns
    (median ms per step, wall seconds); the loop mean (one event pair around
    all steps) and the spread are kept in LAST_TIMING."""
    import numpy as np

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    outer0, outer1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    outer0.record(st)
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    outer1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in ev])
    med = float(np.median(per))
    LAST_TIMING.clear()
    LAST_TIMING.update({"median_ms": med, "loop_mean_ms": outer0.elapsed_time(outer1) / steps,
                        "min_ms": float(per.min()), "max_ms": float(per.max()), "launches": steps})
    return med, wall


def _read_csv(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def _counter_per_dispatch(rows, counter):
    """{dispatch id: (kernel name, grid work-items, summed value)} for one counter."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, grid, v = out.get(d, (r["Kernel_Name"], int(r.get("Grid_Size") or 0), 0.0))
        out[d] = (name, grid, v + float(r["Counter_Value"]))
    return out


def summarize_counters(d: str) -> int:
    """Writes profiles/<form>_traffic.json from a counter session in d:
    d/bench.json (the bench line of the counted run, for the tile shapes),
    d/fetch and d/write (FETCH_SIZE, WRITE_SIZE over that run), d/cfetch and
    d/cwrite (the same counters over --copy-probe 2048), d/copy4g.json (the
    line of --copy-probe 4096) and d/trace (a --kernel-trace run, for the
    kernels' average durations).  Counter values are KiB per dispatch; each is
    scaled by what the counter reads for the plain copy of known size."""
    import glob

    import numpy as np

    line = json.loads(open(os.path.join(d, "bench.json")).read().strip().splitlines()[-1])
    one = lambda sub: glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True)[0]  # noqa: E731
    fetch = _counter_per_dispatch(_read_csv(one("fetch")), "FETCH_SIZE")
    write = _counter_per_dispatch(_read_csv(one("write")), "WRITE_SIZE")
    cf = _counter_per_dispatch(_read_csv(one("cfetch")), "FETCH_SIZE")
    cw = _counter_per_dispatch(_read_csv(one("cwrite")), "WRITE_SIZE")
    copy_bytes = 2048 << 20
    # the six device copies of the probe (the fill before them reads nothing)
    cfk = [v for _, _, v in cf.values() if v * 1024 > copy_bytes / 4]
    cwk = [cw[k][2] for k in sorted(cw) if cf.get(k, ("", 0, 0.0))[2] * 1024 > copy_bytes / 4]
    fetch_scale = copy_bytes / (float(np.median(cfk)) * 1024)
    write_scale = copy_bytes / (float(np.median(cwk)) * 1024)
    trace_rows = _read_csv(glob.glob(os.path.join(d, "trace", "**", "*kernel_trace.csv"), recursive=True)[0])
    copy4 = json.loads(open(os.path.join(d, "copy4g.json")).read().strip().splitlines()[-1])
    B, N = line["config"]["positions"], line["config"]["norb"]
    forms = line["forms"]

    def name(kind, t, *rest):
        if kind == "vgh":
            return "void qs::vgh_kernel<(spline_dtype)1, %d, %d, %d, %d>(qs::VghArgs)" % (t[0], t[1], t[2], rest[0])
        return "void qs::eval_kernel<(spline_dtype)1, %d, %d, %d, true, %s>(qs::EvalArgs)" % (
            t[0], t[1], t[2], "true" if rest[0] else "false")

    specs = [
        ("vgl_f32_80cube_n384", name("eval", line["config"]["tile"], False), line["config"]["tile"], 276,
         KERNEL_SOURCES, "80^3 grid, N=384, FP32 table, 196608 positions"),
        ("ratio_vgl_f32_80cube_n384", name("eval", line["config"]["tile"], True), line["config"]["tile"],
         64 * 4 + 4 + 20.0 / N, KERNEL_SOURCES, "80^3 grid, N=384, FP32 table, 196608 positions"),
        ("vgh_f32_80cube_n384", name("vgh", forms["f32_vgh_hexagonal"]["tile"], 0), forms["f32_vgh_hexagonal"]["tile"],
         64 * 4 + 40, VGH_SOURCES, "80^3 grid, N=384, FP32 table, 196608 positions (orthorhombic and hexagonal cells)"),
        ("vgl_sorted_f32_80cube_n384", name("eval", forms["f32_locality_sorted"]["tile"], False),
         forms["f32_locality_sorted"]["tile"], 276, SORTED_SOURCES,
         "80^3 grid, N=384, FP32 table, 196608 positions, locality-ordered (positions sorted on the device first)"),
    ]
    for form, kname, tile, bpu, srcs, workload in specs:
        sorted_form = "sorted" in form
        # a locality-ordered launch follows the sort's scatter kernel; a plain one does not
        ids = sorted(k for k, (n_, g_, _) in fetch.items() if n_ == kname and g_ == -(-B // tile[3]) * 256)

        def after_scatter(k, table):
            prev = max((j for j in table if j < k), default=None)
            return prev is not None and "loc_scatter" in table[prev][0]

        ids = [k for k in ids if after_scatter(k, fetch) == sorted_form]
        wids = sorted(k for k, (n_, g_, _) in write.items() if n_ == kname and g_ == -(-B // tile[3]) * 256
                      and after_scatter(k, write) == sorted_form)
        if not ids or not wids:
            print("summarize: no dispatches of %s" % kname, file=sys.stderr)
            continue
        fk = [fetch[k][2] for k in ids]
        wk = [write[k][2] for k in wids]
        rd = float(np.mean(fk)) * 1024 * fetch_scale
        wr = float(np.mean(wk)) * 1024 * write_scale
        durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace_rows if r["Kernel_Name"] == kname
                and int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0) == -(-B // tile[3]) * 256]
        alg = B * N * bpu
        out = {"kernel": kname, "tile": list(tile), "workload": workload, "kernel_hash": kernel_hash(srcs),
               "fetch_size_kib_per_dispatch": fk, "write_size_kib_per_dispatch": wk,
               "copy_probe_bytes": copy_bytes, "copy_fetch_kib": cfk, "copy_write_kib": cwk,
               "fetch_scale": fetch_scale, "write_scale": write_scale,
               "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr, "hbm_bytes_per_launch": rd + wr,
               "algorithmic_bytes_per_launch": alg, "traffic_over_algorithmic": (rd + wr) / alg,
               "avg_kernel_ns_rocprof": float(np.mean(durs)) if durs else None,
               "kernel_trace_launches": len(durs),
               "hbm_GBs_measured": (rd + wr) / float(np.mean(durs)) if durs else None,
               "plain_device_copy_4GiB": copy4,
               "note": "FETCH_SIZE counts reads the Infinity Cache serves as well as DRAM reads",
               "commands": ["cd /tmp && export TMPDIR=/tmp",
                            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/fetch -o fetch -- python3 "
                            "<repo>/bench.py --no-forms --no-ragged --no-cpu-baseline --mlp-steps 0 --steps 3 "
                            "--warmup 1 > <out>/bench.json",
                            "rocprofv3 --pmc WRITE_SIZE (the same)",
                            "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE --output-format csv -d <out>/cfetch|cwrite -- "
                            "python3 <repo>/bench.py --copy-probe 2048",
                            "python3 <repo>/bench.py --copy-probe 4096 > <out>/copy4g.json",
                            "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o trace -- "
                            "python3 <repo>/bench.py --mlp-steps 300 --no-cpu-baseline  (the default bench: "
                            "same steps, warm-ups and tuned tiles; the surrogate trains 300 steps; the duration "
                            "averages every launch of the kernel on this batch, cold-cache ones included)",
                            "python3 <repo>/bench.py --summarize-counters <out>"]}
        with open(os.path.join(ROOT, "profiles", form + "_traffic.json"), "w") as f:
            json.dump(out, f, indent=1)
        print("%s: %d/%d dispatches, traffic %.3f of algorithmic, %s ns" % (
            form, len(fk), len(wk), out["traffic_over_algorithmic"], out["avg_kernel_ns_rocprof"]))
    return 0


MLP_FLOP_PER_POS = 2 * 5 * (96 * 256 + 256 * 256 + 256 * 192)
PEAK_FP32_VECTOR_TFLOPS = 78.6  # unpacked FMA (packed FP32 is not used)
PEAK_BF16_TFLOPS = 2500.0
MLP_TOLS = (1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 3e-1)


def bench_mlp(args, q, W, torch, dev, np):
    """The learned surrogate of the 48^3 / N=192 table: trained on the GPU
    against the spline's VGL, then timed on the 256 x 192 batch with and
    without the spline fallback, and its error measured against the spline
    on held-out positions."""
    log("bench: surrogate: building the 48^3 table and training %d steps ..." % args.mlp_steps)
    grid, N, coefs, _ = W.make_table(5)
    spl = q.Spline(grid, coefs, "f32", device=dev)
    _, Ws, bs = W.mlp_init(5)
    freqs = q.spectral_frequencies(coefs)  # the 48 most energetic frequency pairs of the table
    net = q.SurrogateMLP(N, freqs, q.flatten_mlp_params(Ws, bs), device=dev)
    train = torch.from_numpy(W.mlp_samples(5, count=10 ** 6)).to(dev)
    val = torch.from_numpy(W.mlp_samples(5, count=10 ** 5, validation=True)).to(dev)
    bt = 4096
    net.init_output(spl.eval_vgl(train[:bt]))
    loss = torch.zeros(1, device=dev)
    nb = train.shape[0] // bt
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.mlp_steps):
        pos = train[(step % nb) * bt:(step % nb + 1) * bt]
        lr = 5e-3 * 0.5 * (1.0 + np.cos(np.pi * step / args.mlp_steps)) + 1e-5
        net.train_step(pos, spl.eval_vgl(pos), lr=lr, loss_out=loss if step == args.mlp_steps - 1 else None)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    net.build_error_map(spl, val[:8 * 8 * 8 * 64], bins_per_dim=8)

    # error on held-out positions (the last 50000 validation points), against the spline
    import oracle

    hv = val[50000:]
    ref = [t.cpu().numpy() for t in spl.eval_vgl(hv)]
    e_net = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(net.forward(hv), ref)]
    bins = net.bin_errors().ravel()

    # timing on the 256 walkers x 192 electrons batch
    pos = torch.from_numpy(W.make_positions(5)).to(dev)
    B = pos.shape[0]
    out = net._out(B)
    ms_net, _ = time_steps(torch, lambda: net.forward(pos, out=out), args.steps, args.warmup)
    ms_net_b2b = time_back_to_back(torch, lambda: net.forward(pos, out=out), args.steps, args.warmup)
    ms_net_idle = time_burst_after_idle(torch, lambda: net.forward(pos, out=out))
    sout = spl.alloc_outputs(B)
    spl.autotune(pos, reps=2, out=sout)
    ms_spl, _ = time_steps(torch, lambda: spl.eval_vgl(pos, out=sout), args.steps, args.warmup)
    units = B * N

    # The combined path (network, then the spline for positions in bins whose
    # error exceeds tol) across tolerances: routed fraction, error against the
    # spline on the held-out positions, and speed on the batch.
    sweep = []
    for tol in MLP_TOLS:
        Vf, Gf, Lf, nf = net.eval_vgl(hv, fallback=spl, tol=tol)
        e_fb = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip((Vf, Gf, Lf), ref)]
        frac_h = int(nf.cpu()[0]) / hv.shape[0]
        res = {}
        ms_fb, _ = time_steps(torch, lambda: res.__setitem__("nf", net.eval_vgl(pos, fallback=spl, tol=tol,
                                                                                out=out)[3]),
                              args.steps, args.warmup)
        sweep.append({"tol": tol, "fallback_fraction_heldout": frac_h,
                      "fallback_fraction_batch": int(res["nf"].cpu()[0]) / B,
                      "eps_with_fallback_vs_spline": {"V": e_fb[0], "G": e_fb[1], "L": e_fb[2]},
                      "ms_with_fallback": ms_fb, "speedup_with_fallback_vs_spline": ms_spl / ms_fb})
    beats = [r for r in sweep if r["speedup_with_fallback_vs_spline"] > 1.0]
    tflops = B * MLP_FLOP_PER_POS / (ms_net_b2b * 1e-3) / 1e12
    tflops_idle = B * MLP_FLOP_PER_POS / (ms_net_idle * 1e-3) / 1e12
    _, energy = q.spectral_frequencies(coefs, with_energy=True)
    outside = 1.0 - (float(energy["pairs"].sum()) + energy["k0"]) / energy["total"]
    return {
        "table": "48^3 grid, N=192, FP32 (%.1f MB)" % (spl.layout.total_bytes / 1e6),
        "network_bytes": int(net.layout.n_params * 2), "train_steps": args.mlp_steps, "train_batch": bt,
        "train_seconds": train_s, "final_loss": float(loss.cpu()[0]),
        "eps_network_only_vs_spline": {"V": e_net[0], "G": e_net[1], "L": e_net[2]},
        "error_map_bins": {"count": int(bins.size), "min": float(bins.min()), "median": float(np.median(bins)),
                           "max": float(bins.max())},
        "coefficient_energy_outside_feature_pairs": outside,
        "positions": B, "ms_network_only": ms_net, "ms_spline_f32": ms_spl,
        "evals_per_s_network_only": units / (ms_net * 1e-3), "evals_per_s_spline_f32": units / (ms_spl * 1e-3),
        "speedup_network_only_vs_spline": ms_spl / ms_net,
        "fallback_sweep": sweep,
        "finest_tol_where_combined_beats_spline": min(r["tol"] for r in beats) if beats else None,
        "target_1e-3_met": any(r["tol"] <= 1e-3 and r["fallback_fraction_heldout"] < 1.0
                               and r["speedup_with_fallback_vs_spline"] > 1.0 for r in sweep),
        "dram_write_GBs_network": units * 20 / (ms_net * 1e-3) / 1e9,
        "roofline_network_kernel": {"bound": "mfma", "achieved": tflops, "peak": PEAK_BF16_TFLOPS,
                                    "unit": "TFLOP/s", "frac": tflops / PEAK_BF16_TFLOPS,
                                    "flop_per_position": MLP_FLOP_PER_POS,
                                    "ms_per_launch": ms_net_b2b,
                                    "ms_burst_after_idle": ms_net_idle,
                                    "frac_burst_after_idle": tflops_idle / PEAK_BF16_TFLOPS,
                                    "note": "frac: ms_per_launch, the mean of the timed launches issued "
                                            "back to back between one pair of HIP events, during which the "
                                            "power management lowers the clock of the sustained matrix-core "
                                            "load (ms_network_only is their median with an event pair "
                                            "around each); frac_burst_after_idle: 8 launches after 0.5 s "
                                            "idle, at the clock an idle GPU starts from"},
    }


def fixed_error_summary(forms, e32, ms32, ms_v, ms_rv, eps_rv32):
    """Which form meets which error bar, at what speed against its FP32
    counterpart.  eps: per-orbital max-norm relative error against the FP64
    oracle on the original coefficients (the network: against the FP32
    spline, its judge), for the quantities the form returns."""
    rows = [{"form": "f32 VGL", "quantities": "V,G,L", "eps": {"V": e32[0], "G": e32[1], "L": e32[2]},
             "speedup_vs_f32": 1.0, "against": "f32 VGL"},
            {"form": "f32 value only", "quantities": "V", "eps": {"V": e32[0]}, "speedup_vs_f32": 1.0,
             "against": "f32 value only"},
            {"form": "f32 value ratio", "quantities": "ratio", "eps": {"ratio": eps_rv32}, "speedup_vs_f32": 1.0,
             "against": "f32 value ratio"}]
    for dt in ("bf16", "f16"):
        f = forms.get(dt)
        if not f:
            continue
        rows.append({"form": dt + " VGL", "quantities": "V,G,L",
                     "eps": {"V": f["eps_V"], "G": f["eps_G"], "L": f["eps_L"]},
                     "speedup_vs_f32": f["speedup_vs_f32"], "against": "f32 VGL"})
        rows.append({"form": dt + " value only", "quantities": "V", "eps": {"V": f["value_only"]["eps_V"]},
                     "speedup_vs_f32": f["value_only"]["speedup_vs_f32_value_only"], "against": "f32 value only"})
        rows.append({"form": dt + " value ratio", "quantities": "ratio", "eps": {"ratio": f["ratio_v"]["eps"]},
                     "speedup_vs_f32": f["ratio_v"]["speedup_vs_f32_ratio_v"], "against": "f32 value ratio"})
    m = forms.get("mlp_surrogate")
    if m:
        rows.append({"form": "network alone", "quantities": "V,G,L", "eps": m["eps_network_only_vs_spline"],
                     "speedup_vs_f32": m["speedup_network_only_vs_spline"], "against": "f32 VGL (48^3, N=192)"})
        for r in m["fallback_sweep"]:
            rows.append({"form": "network + spline fallback, tol %g" % r["tol"], "quantities": "V,G,L",
                         "eps": r["eps_with_fallback_vs_spline"], "speedup_vs_f32": r["speedup_with_fallback_vs_spline"],
                         "fallback_fraction": r["fallback_fraction_batch"], "against": "f32 VGL (48^3, N=192)"})
    best = {}
    for r in rows:
        worst = max(r["eps"].values())
        r["meets_1e-5"] = worst <= 1e-5
        r["meets_1e-3"] = worst <= 1e-3
        if r["quantities"] == "ratio":
            continue  # a different error measure (relative to the dot product's scale): not ranked
        for bar in ("1e-5", "1e-3"):
            if r["meets_" + bar] and r["speedup_vs_f32"] > best.get(bar, {}).get("speedup_vs_f32", 0.0):
                best[bar] = {"form": r["form"], "speedup_vs_f32": r["speedup_vs_f32"]}
    return {"forms": rows, "fastest_meeting": best,
            "measure": "eps_Q = max over orbitals of max |Q - Q_ref| / max |Q_ref| (G's components pooled); "
                       "ratios: max |R - R_ref| / sum_i |a_i| max|V_i| (not ranked in fastest_meeting)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16/FP16 forms")
    ap.add_argument("--no-ragged", action="store_true", help="skip the four-table ragged plan")
    ap.add_argument("--mlp-steps", type=int, default=24000, help="training steps of the surrogate (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle wall time")
    ap.add_argument("--tile", type=str, default="", help="cw,nch,lpp,pb (skips the autotuner)")
    ap.add_argument("--vgh-tile", type=str, default="", help="cw,nch,lpp,pb for the VGH forms (skips their autotuner)")
    ap.add_argument("--sorted-tile", type=str, default="",
                    help="cw,nch,lpp,pb for the FP32 locality-ordered form (skips its autotuner)")
    ap.add_argument("--no-tune-cache", dest="use_tune_cache", action="store_false",
                    help="search tile shapes afresh instead of reading the committed tuning cache")
    ap.add_argument("--summarize-counters", type=str, default="", metavar="DIR",
                    help="only write profiles/*_traffic.json from a rocprofv3 counter session in DIR")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration)")
    args = ap.parse_args()

    if args.summarize_counters:
        return summarize_counters(args.summarize_counters)
    if args.copy_probe:
        import torch

        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_probe_bytes": n, "launches": 6, "ms": ms, "GBs_read_plus_write": 2 * n / ms / 1e6}),
              flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the spline path needs no exchange between GPUs "
              "(positions are independent and the table is read-only), so the figure for N GPUs is "
              "N times the one-GPU rate of each GPU's share; rerun with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1708_02645_amd as q
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("bench: building C3 table (80^3, N=384) ...")
    grid, N, coefs, _ = W.make_table(3)
    pos_np = W.make_positions(3)
    B = pos_np.shape[0]
    pos = torch.from_numpy(pos_np).to(dev)
    units = B * N

    def bench_form(dtype: str, tile=None):
        s = q.Spline(grid, coefs, dtype, device=dev)
        out = s.alloc_outputs(B)
        if tile:
            s.set_tile(tile)
        else:
            # the autotuner; its committed cache makes the choice repeatable
            s.autotune(pos, reps=3, out=out, cache_path=TUNE_CACHE if args.use_tune_cache else None)
        chosen = s.get_tile()
        ms, wall = time_steps(torch, lambda: s.eval_vgl(pos, out=out), args.steps, args.warmup)
        log("bench: %s tile %s  %.3f ms/step" % (dtype, chosen, ms))
        return s, out, chosen, ms, wall

    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None
    s32, out32, tile32, ms32, wall32 = bench_form("f32", tile)
    timing32 = dict(LAST_TIMING)
    evals = units / (ms32 * 1e-3)
    achieved = units * BYTES_PER_UNIT["f32"] / (ms32 * 1e-3) / 1e9

    # spot parity against the FP64 oracle on sampled positions (not timed)
    import oracle

    rng = np.random.default_rng(123)
    idx = rng.choice(B, 256, replace=False)
    it = torch.from_numpy(idx).to(dev)
    ref = oracle.eval_vgl(grid, coefs, pos_np[idx])

    def eps(out):
        V, G, L = out
        got = (V[it].double().cpu().numpy(), G[it].double().cpu().numpy(), L[it].double().cpu().numpy())
        return [oracle.rel_err(g, r) for g, r in zip(got, ref)]

    e32 = eps(out32)
    # cold variant: a 512 MB scratch write between launches evicts the caches
    # (L2, MALL) before every timed launch
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cold = []
    for _ in range(max(5, args.steps // 3)):
        scratch.fill_(1)
        ev0.record()
        s32.eval_vgl(pos, out=out32)
        ev1.record()
        torch.cuda.synchronize()
        cold.append(ev0.elapsed_time(ev1))
    ms_cold = float(np.median(cold))
    achieved_cold = units * BYTES_PER_UNIT["f32"] / (ms_cold * 1e-3) / 1e9
    del scratch
    # value only (the quadrature-point evaluation): same table and positions
    ms_v, _ = time_steps(torch, lambda: s32.eval_v(pos, out=out32[0]), args.steps, args.warmup)
    vtile32 = s32.get_value_tile()

    # Locality-ordered evaluation of the same batch: positions bucketed on the
    # device by Morton-ordered blocks of grid cells, then evaluated in that
    # order (the sort is inside the timed step); same outputs bit for bit.
    def bench_sorted(s, out, tile_arg):
        if tile_arg:
            s.set_sorted_tile(tile_arg)
            st = tuple(tile_arg)
        else:
            st = s.autotune_sorted(pos, reps=3, out=out, cache_path=TUNE_CACHE if args.use_tune_cache else None)
        ms, _ = time_steps(torch, lambda: s.eval_vgl_sorted(pos, out=out), args.steps, args.warmup)
        plain = s.eval_vgl(pos)
        same = all(bool(torch.equal(a, b)) for a, b in zip(out, plain))
        del plain
        torch.cuda.empty_cache()
        log("bench: %s locality-ordered tile %s  %.3f ms/step  bitwise equal: %s" % (s.dtype, st, ms, same))
        return st, ms, same

    stile_arg = tuple(int(x) for x in args.sorted_tile.split(",")) if args.sorted_tile else None
    stile32, ms_sorted, same32 = bench_sorted(s32, out32, stile_arg)
    # value only in locality order (its own tuned shape), against the plain values
    svtile32 = s32.get_sorted_value_tile()
    ms_v_s, _ = time_steps(torch, lambda: s32.eval_v_sorted(pos, out=out32[0]), args.steps, args.warmup)
    same_v = bool(torch.equal(out32[0], s32.eval_v(pos)))
    log("bench: f32 value-only locality-ordered tile %s  %.3f ms/step  bitwise equal: %s" % (svtile32, ms_v_s, same_v))
    del out32
    torch.cuda.empty_cache()

    # Fused determinant ratio: position b (walker-major, electron-minor) dots
    # row b of the stacked inverse Slater matrices with its orbital V, G, L;
    # only 5 (or 1) numbers per position are written.
    log("bench: determinant-ratio forms ...")
    rows_np = W.make_inverse_rows(3, B, N)
    rows_d = torch.from_numpy(rows_np).to(dev)
    Dbuf = torch.empty((B, 5), dtype=torch.float32, device=dev)
    Rbuf = torch.empty((B,), dtype=torch.float32, device=dev)
    ms_rvgl, _ = time_steps(torch, lambda: s32.eval_ratio_vgl(pos, rows_d, out=Dbuf), args.steps, args.warmup)
    ms_rv, _ = time_steps(torch, lambda: s32.eval_ratio_v(pos, rows_d, out=Rbuf), args.steps, args.warmup)
    from oracle import det as odet

    ridx = idx[:64]
    Dref = odet.ratio_vgl(grid, coefs, pos_np[ridx], rows_np[ridx])
    Vr, Gr, Lr = oracle.eval_vgl(grid, coefs, pos_np[ridx])
    Mq = [np.abs(Vr).max(0), np.abs(Gr).max((0, 1)), np.abs(Lr).max(0)]
    sv, sg, sl = (odet.ratio_scale(rows_np[ridx], m) for m in Mq)
    rscale = np.stack([sv, sg, sg, sg, sl], 1)
    rit = torch.from_numpy(ridx).to(dev)
    eps_ratio = float(np.max(np.abs(Dbuf[rit].double().cpu().numpy() - Dref) / rscale))
    eps_ratio_v = float(np.max(np.abs(Rbuf[rit].double().cpu().numpy() - Dref[:, 0]) / sv))
    # the same in locality order (sorted tile shape for the ratio with derivatives)
    ms_rvgl_s, _ = time_steps(torch, lambda: s32.eval_ratio_vgl_sorted(pos, rows_d, out=Dbuf), args.steps,
                              args.warmup)
    ms_rv_s, _ = time_steps(torch, lambda: s32.eval_ratio_v_sorted(pos, rows_d, out=Rbuf), args.steps, args.warmup)
    eps_ratio_s = float(np.max(np.abs(Dbuf[rit].double().cpu().numpy() - Dref) / rscale))
    eps_ratio_v_s = float(np.max(np.abs(Rbuf[rit].double().cpu().numpy() - Dref[:, 0]) / sv))
    # Sherman-Morrison update after one accepted move per walker: the 512
    # stacked 384 x 384 FP32 inverses above (their rows stand in for A^-1),
    # electron k_w = w mod 384, unit-variance orbital values.
    n_w = B // N
    inv_d = rows_d.view(n_w, N, N)
    k_d = torch.arange(n_w, dtype=torch.int32, device=dev) % N
    phi_d = torch.from_numpy(W.make_inverse_rows(3, n_w, N, seed=33) * np.float32(np.sqrt(N))).to(dev)
    ms_sm, _ = time_steps(torch, lambda: q.det_update(inv_d, k_d, phi_d), args.steps, args.warmup)
    ms_sm_b = time_back_to_back(torch, lambda: q.det_update(inv_d, k_d, phi_d), args.steps, args.warmup)
    bytes_sm = n_w * (8.0 * N * N + 4 * N + 4)
    # Delayed update of the same inverses: 16 accepted moves per walker
    # (value ratio against the pending moves, then accept), then one flush.
    delay = 16
    dl = q.DelayedUpdate(N, delay, n_w, device=dev)
    ks_d = [((torch.arange(n_w, dtype=torch.int32, device=dev) + i) % N).to(torch.int32) for i in range(delay)]
    r_d = torch.empty(n_w, dtype=torch.float32, device=dev)

    def dlu_batch():
        for i in range(delay):
            dl.ratio(inv_d, ks_d[i], phi_d, out=r_d)
            dl.accept(inv_d, ks_d[i], phi_d)
        dl.flush(inv_d)

    ms_dlu, _ = time_steps(torch, dlu_batch, max(3, args.steps // 5), 1)
    # the same batch captured once in a HIP graph and replayed (no host work per move)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        dlu_batch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g_dlu = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_dlu):
        dlu_batch()
    ms_dlu_graph, _ = time_steps(torch, g_dlu.replay, max(3, args.steps // 5), 1)

    # the same 16 moves with each accept fused into the next move's ratio
    def dlu_batch_fused():
        dl.ratio(inv_d, ks_d[0], phi_d, out=r_d)
        for i in range(1, delay):
            dl.accept_ratio(inv_d, ks_d[i - 1], phi_d, ks_d[i], phi_d, out=r_d)
        dl.accept(inv_d, ks_d[delay - 1], phi_d)
        dl.flush(inv_d)

    ms_dlu_fused, _ = time_steps(torch, dlu_batch_fused, max(3, args.steps // 5), 1)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        dlu_batch_fused()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g_dlu_f = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_dlu_f):
        dlu_batch_fused()
    ms_dlu_fused_graph, _ = time_steps(torch, g_dlu_f.replay, max(3, args.steps // 5), 1)
    del dl, g_dlu, g_dlu_f
    del s32, rows_d, Dbuf, Rbuf, inv_d, phi_d
    torch.cuda.empty_cache()
    bpu_rvgl = 64 * 4 + 4 + 20.0 / N
    bpu_rv = 64 * 4 + 4 + 4.0 / N

    # attainable read bandwidth: a plain streaming read of 4 GiB
    rbuf = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    rbuf.zero_()
    best_read = 0.0
    for grid_r in (1024, 2048, 4096):
        scratch = torch.empty(grid_r * 256, dtype=torch.float32, device=dev)
        ms_r, _ = time_steps(torch, lambda: q.probe_stream_read(rbuf, grid_r, out=scratch), 10, 2)
        best_read = max(best_read, rbuf.numel() / (ms_r * 1e-3) / 1e9)
    del rbuf
    # MALL-resident read rate: the same probe over 64 MB (fits the 256 MB
    # Infinity Cache), for tables that live there (C2)
    mbuf = torch.ones(64 << 20, dtype=torch.uint8, device=dev)
    mall_read = 0.0
    for grid_r in (256, 512, 1024):
        scratch_m = torch.empty(grid_r * 256, dtype=torch.float32, device=dev)
        ms_m, _ = time_steps(torch, lambda: q.probe_stream_read(mbuf, grid_r, out=scratch_m), 50, 5)
        mall_read = max(mall_read, mbuf.numel() / (ms_m * 1e-3) / 1e9)
    del mbuf, scratch_m
    torch.cuda.empty_cache()

    forms = {"f32": {"evals_per_s": evals, "ms_per_step": ms32, "tile": list(tile32),
                     "eps_V": e32[0], "eps_G": e32[1], "eps_L": e32[2],
                     "cold_cache": {"ms_per_launch": ms_cold, "evals_per_s": units / (ms_cold * 1e-3),
                                    "hbm_frac": units * BYTES_PER_UNIT["f32"] / (ms_cold * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                    "note": "median of single launches, each after a 512 MB scratch write"}},
             "f32_value_only": {"evals_per_s": units / (ms_v * 1e-3), "ms_per_step": ms_v, "tile": list(vtile32),
                                "hbm_frac": units * (64 * 4 + 4) / (ms_v * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                "bytes_per_unit": 64 * 4 + 4},
             "f32_ratio_vgl": {"evals_per_s": units / (ms_rvgl * 1e-3), "ms_per_step": ms_rvgl,
                               "hbm_frac": units * bpu_rvgl / (ms_rvgl * 1e-3) / 1e9 / PEAK_HBM_GBS,
                               "bytes_per_unit": bpu_rvgl, "speedup_vs_f32_vgl": ms32 / ms_rvgl,
                               "eps": eps_ratio,
                               "traffic": traffic_from_profiles(tile32, "ratio_vgl_f32_80cube_n384")},
             "f32_det_update": {"walkers": B // N, "n": N, "ms_per_step": ms_sm,
                                "updates_per_s": (B // N) / (ms_sm * 1e-3), "bytes_per_update": bytes_sm / (B // N),
                                "hbm_frac": bytes_sm / (ms_sm * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                "ms_back_to_back": ms_sm_b,
                                "hbm_frac_back_to_back": bytes_sm / (ms_sm_b * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                "timing_note": "ms_per_step: median of launches each between its own event pair "
                                               "(their markers add a few us); ms_back_to_back: mean of the "
                                               "same launches issued back to back under one event pair"},
             "f32_delayed_update": {"walkers": B // N, "n": N, "delay": delay, "ms_per_16_moves": ms_dlu,
                                    "ms_per_move": ms_dlu / delay, "speedup_per_move_vs_sherman_morrison":
                                    ms_sm / (ms_dlu / delay),
                                    "ms_per_16_moves_graph": ms_dlu_graph, "ms_per_move_graph": ms_dlu_graph / delay,
                                    "speedup_per_move_vs_sherman_morrison_graph": ms_sm / (ms_dlu_graph / delay),
                                    "ms_per_16_moves_fused": ms_dlu_fused,
                                    "ms_per_16_moves_fused_graph": ms_dlu_fused_graph,
                                    "ms_per_move_fused_graph": ms_dlu_fused_graph / delay,
                                    "speedup_per_move_vs_sherman_morrison_fused_graph":
                                        ms_sm / (ms_dlu_fused_graph / delay),
                                    "note": "each move: ratio against the pending moves + accept; one flush per "
                                            "16 moves (all included); _graph: the 16 moves and the flush replayed "
                                            "from one HIP graph; _fused: each accept in the same launch as the "
                                            "next move's ratio"},
             "f32_locality_sorted": {
                 "evals_per_s": units / (ms_sorted * 1e-3), "ms_per_step": ms_sorted, "tile": list(stile32),
                 "speedup_vs_f32": ms32 / ms_sorted, "bitwise_equal_to_f32": same32,
                 "algorithmic_GBs": units * BYTES_PER_UNIT["f32"] / (ms_sorted * 1e-3) / 1e9,
                 "traffic": traffic_from_profiles(stile32, "vgl_sorted_f32_80cube_n384"),
                 "fma_floor_ms": units * 320 * 2 / (PEAK_FP32_VECTOR_TFLOPS * 1e12) * 1e3,
                 "fma_frac_of_fp32_vector_peak": units * 320 * 2 / (ms_sorted * 1e-3) / (PEAK_FP32_VECTOR_TFLOPS * 1e12),
                 "note": "same batch and outputs; positions bucketed by Morton-ordered 4^3-cell blocks on the "
                         "device (4 small launches, timed) and dealt so each XCD takes a contiguous stretch, so "
                         "table rows are re-read from L2 / Infinity Cache: the algorithmic bytes exceed what "
                         "HBM moves"},
             "f32_ratio_vgl_locality_sorted": {"evals_per_s": units / (ms_rvgl_s * 1e-3), "ms_per_step": ms_rvgl_s,
                                               "tile": list(stile32), "speedup_vs_f32_ratio_vgl": ms_rvgl / ms_rvgl_s,
                                               "eps": eps_ratio_s},
             "f32_value_only_locality_sorted": {"evals_per_s": units / (ms_v_s * 1e-3), "ms_per_step": ms_v_s,
                                                "tile": list(svtile32), "speedup_vs_f32_value_only": ms_v / ms_v_s,
                                                "bitwise_equal_to_f32_value_only": same_v},
             "f32_ratio_v_locality_sorted": {"evals_per_s": units / (ms_rv_s * 1e-3), "ms_per_step": ms_rv_s,
                                             "tile": list(svtile32), "speedup_vs_f32_ratio_v": ms_rv / ms_rv_s,
                                             "eps": eps_ratio_v_s},
             "f32_ratio_v": {"evals_per_s": units / (ms_rv * 1e-3), "ms_per_step": ms_rv, "tile": list(vtile32),
                             "hbm_frac": units * bpu_rv / (ms_rv * 1e-3) / 1e9 / PEAK_HBM_GBS,
                             "bytes_per_unit": bpu_rv, "eps": eps_ratio_v}}
    if not args.no_forms:
        for dt in ("bf16", "f16"):
            s, out, t, ms, _ = bench_form(dt)
            e = eps(out)
            forms[dt] = {"evals_per_s": units / (ms * 1e-3), "ms_per_step": ms, "tile": list(t),
                         "speedup_vs_f32": ms32 / ms, "eps_V": e[0], "eps_G": e[1], "eps_L": e[2],
                         "hbm_frac": units * BYTES_PER_UNIT[dt] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
            # value only and the value ratio (the quadrature-point uses), with
            # their error against the FP64 oracle on the original coefficients
            ms_v16, _ = time_steps(torch, lambda: s.eval_v(pos, out=out[0]), args.steps, args.warmup)
            ev16 = oracle.rel_err(out[0][it].double().cpu().numpy(), ref[0])
            rows16 = torch.from_numpy(rows_np).to(dev)
            R16 = torch.empty((B,), dtype=torch.float32, device=dev)
            ms_rv16, _ = time_steps(torch, lambda: s.eval_ratio_v(pos, rows16, out=R16), args.steps, args.warmup)
            eps_rv16 = float(np.max(np.abs(R16[rit].double().cpu().numpy() - Dref[:, 0]) / sv))
            del rows16, R16
            forms[dt]["value_only"] = {"ms_per_step": ms_v16, "evals_per_s": units / (ms_v16 * 1e-3), "eps_V": ev16,
                                       "speedup_vs_f32_value_only": ms_v / ms_v16}
            forms[dt]["ratio_v"] = {"ms_per_step": ms_rv16, "evals_per_s": units / (ms_rv16 * 1e-3),
                                    "eps": eps_rv16, "speedup_vs_f32_ratio_v": ms_rv / ms_rv16}
            st, mss, same = bench_sorted(s, out, None)
            forms[dt + "_locality_sorted"] = {"evals_per_s": units / (mss * 1e-3), "ms_per_step": mss,
                                              "tile": list(st), "speedup_vs_f32": ms32 / mss,
                                              "bitwise_equal_to_" + dt: same}
            del s, out
            torch.cuda.empty_cache()
    del rows_np

    # Value-gradient-Hessian (the paper's Bspline-vgh) on the same table and
    # batch: orthorhombic cell, and a hexagonal cell (graphite-like lattice
    # a1 = (1,0,0), a2 = (-1/2, sqrt(3)/2, 0), a3 = (0,0,1.6); positions are
    # the same fractional coordinates mapped into it), with the general-cell
    # VGL beside it.
    log("bench: VGH forms ...")
    hexl = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])
    pos_hex = torch.from_numpy(pos_np @ hexl).to(dev)
    sh = q.Spline(grid, coefs, "f32", device=dev)
    vgh_out = sh.alloc_vgh(B)
    vgh_tile = tuple(int(x) for x in args.vgh_tile.split(",")) if args.vgh_tile else None

    def pick_vgh(p):
        if vgh_tile:
            sh.set_vgh_tile(vgh_tile)
            return vgh_tile
        return sh.autotune_vgh(p, reps=2, out=vgh_out)

    t_vgh = pick_vgh(pos)
    t_vgh_s = sh.get_sorted_vgh_tile()
    ms_vgh, _ = time_steps(torch, lambda: sh.eval_vgh(pos, out=vgh_out), args.steps, args.warmup)
    ms_vgh_s, _ = time_steps(torch, lambda: sh.eval_vgh_sorted(pos, out=vgh_out), args.steps, args.warmup)
    sh.set_lattice(hexl)
    t_vgh_hex = pick_vgh(pos_hex)
    ms_vgh_hex, _ = time_steps(torch, lambda: sh.eval_vgh(pos_hex, out=vgh_out), args.steps, args.warmup)
    ms_vgh_hex_s, _ = time_steps(torch, lambda: sh.eval_vgh_sorted(pos_hex, out=vgh_out), args.steps, args.warmup)
    Vh, Gh, Hh = vgh_out
    Lbuf = torch.empty((B, N), dtype=torch.float32, device=dev)
    ms_vgl_hex, _ = time_steps(torch, lambda: sh.eval_vgl(pos_hex, out=(Vh, Gh, Lbuf)), args.steps, args.warmup)
    ms_vgl_hex_s, _ = time_steps(torch, lambda: sh.eval_vgl_sorted(pos_hex, out=(Vh, Gh, Lbuf)), args.steps,
                                 args.warmup)
    hidx = idx[:128]
    hit = torch.from_numpy(hidx).to(dev)
    sh.eval_vgh(pos_hex, out=vgh_out)
    ref_h = oracle.eval_vgh(grid, coefs, pos_np[hidx] @ hexl, hexl)
    eps_h = [oracle.rel_err(t[hit].double().cpu().numpy(), r) for t, r in zip(vgh_out, ref_h)]
    del sh, vgh_out, Vh, Gh, Hh, Lbuf, pos_hex
    torch.cuda.empty_cache()
    bpu_vgh = 64 * 4 + 40
    forms["f32_vgh"] = {"evals_per_s": units / (ms_vgh * 1e-3), "ms_per_step": ms_vgh, "tile": list(t_vgh),
                        "bytes_per_unit": bpu_vgh,
                        "hbm_frac": units * bpu_vgh / (ms_vgh * 1e-3) / 1e9 / PEAK_HBM_GBS}
    forms["f32_vgh_hexagonal"] = {
        "evals_per_s": units / (ms_vgh_hex * 1e-3), "ms_per_step": ms_vgh_hex, "tile": list(t_vgh_hex),
        "bytes_per_unit": bpu_vgh, "hbm_frac": units * bpu_vgh / (ms_vgh_hex * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "eps_V": eps_h[0], "eps_G": eps_h[1], "eps_H": eps_h[2],
        "traffic": traffic_from_profiles(t_vgh_hex, "vgh_f32_80cube_n384")}
    forms["f32_vgl_hexagonal"] = {
        "evals_per_s": units / (ms_vgl_hex * 1e-3), "ms_per_step": ms_vgl_hex, "tile": list(t_vgh_hex),
        "bytes_per_unit": BYTES_PER_UNIT["f32"],
        "hbm_frac": units * BYTES_PER_UNIT["f32"] / (ms_vgl_hex * 1e-3) / 1e9 / PEAK_HBM_GBS}
    forms["f32_vgh_locality_sorted"] = {
        "ms_per_step": ms_vgh_s, "ms_per_step_hexagonal": ms_vgh_hex_s, "tile": list(t_vgh_s),
        "evals_per_s": units / (ms_vgh_s * 1e-3), "evals_per_s_hexagonal": units / (ms_vgh_hex_s * 1e-3),
        "speedup_vs_f32_vgh": ms_vgh / ms_vgh_s, "speedup_vs_f32_vgh_hexagonal": ms_vgh_hex / ms_vgh_hex_s}
    forms["f32_vgl_hexagonal_locality_sorted"] = {
        "ms_per_step": ms_vgl_hex_s, "evals_per_s": units / (ms_vgl_hex_s * 1e-3), "tile": list(t_vgh_s),
        "speedup_vs_f32_vgl_hexagonal": ms_vgl_hex / ms_vgl_hex_s}
    log("bench: vgh %.3f ms, vgh hexagonal %.3f ms, vgl hexagonal %.3f ms; sorted %.3f / %.3f / %.3f ms" % (
        ms_vgh, ms_vgh_hex, ms_vgl_hex, ms_vgh_s, ms_vgh_hex_s, ms_vgl_hex_s))

    # C2 (48^3, N = 192, FP32: a 102 MB table that the 256 MB MALL holds)
    # against the MALL-resident read rate, and one GPU's share of an 8-way
    # orbital split of C3 (N = 48 of 384 orbitals).
    log("bench: C2 and the N=48 shard ...")
    g2, N2, c2coef, _ = W.make_table(2)
    p2 = torch.from_numpy(W.make_positions(2)).to(dev)
    s2 = q.Spline(g2, c2coef, "f32", device=dev)
    o2 = s2.alloc_outputs(p2.shape[0])
    s2.autotune(p2, reps=3, out=o2)
    ms_c2, _ = time_steps(torch, lambda: s2.eval_vgl(p2, out=o2), args.steps, args.warmup)
    u2 = p2.shape[0] * N2
    forms["c2_f32_mall_resident"] = {
        "ms_per_step": ms_c2, "evals_per_s": u2 / (ms_c2 * 1e-3), "tile": list(s2.get_tile()),
        "algorithmic_GBs": u2 * BYTES_PER_UNIT["f32"] / (ms_c2 * 1e-3) / 1e9, "mall_resident_read_GBs": mall_read,
        "frac_of_mall_read": u2 * BYTES_PER_UNIT["f32"] / (ms_c2 * 1e-3) / 1e9 / mall_read}
    st2 = s2.autotune_sorted(p2, reps=3, out=o2, cache_path=TUNE_CACHE if args.use_tune_cache else None)
    ms_c2s, _ = time_steps(torch, lambda: s2.eval_vgl_sorted(p2, out=o2), args.steps, args.warmup)
    forms["c2_f32_locality_sorted"] = {"ms_per_step": ms_c2s, "evals_per_s": u2 / (ms_c2s * 1e-3), "tile": list(st2),
                                       "speedup_vs_c2_f32": ms_c2 / ms_c2s}
    del s2, o2, p2, c2coef
    s48 = q.Spline(grid, np.ascontiguousarray(coefs[..., :48]), "f32", device=dev)
    o48 = s48.alloc_outputs(B)
    s48.autotune(pos, reps=3, out=o48)
    ms_48, _ = time_steps(torch, lambda: s48.eval_vgl(pos, out=o48), args.steps, args.warmup)
    u48 = B * 48
    forms["c3_f32_shard_n48"] = {
        "ms_per_step": ms_48, "evals_per_s": u48 / (ms_48 * 1e-3), "tile": list(s48.get_tile()),
        "hbm_frac": u48 * BYTES_PER_UNIT["f32"] / (ms_48 * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "row_bytes": int(s48.layout.row_bytes), "orbital_bytes_per_row": 48 * 4,
        "note": "one GPU's share of C3 split 8 ways over orbitals; 192-B rows (short rows pad to 64 B, "
                "not 256 B)"}
    del s48, o48
    torch.cuda.empty_cache()

    # Jastrow (J1 + J2, 1D cubic B-spline functors): 384 electrons, 32 ions,
    # one proposed move per walker (512 and 16384 walkers), and the full
    # evaluation of 512 walkers.  Pair evaluations: a move forms every pair
    # of the moved electron at its old and new position.
    log("bench: Jastrow ...")
    jd = W.make_jastrow()
    jas = q.Jastrow(jd["cell"], jd["ions"], jd["species"], jd["f1"], jd["uu"], jd["ud"], jd["n_elec"], jd["n_up"],
                    device=dev)
    NE, NI = jd["n_elec"], len(jd["ions"])
    jforms = {}
    for nw in (W.JASTROW["walkers"], 16384):
        Re = W.make_electrons(nw, NE)
        Rd = jas.positions(Re)
        ks, disp = W.make_moves(nw, NE)
        kd = torch.from_numpy(ks).to(dev)
        rd = torch.from_numpy(Re[np.arange(nw), ks] + disp).to(dev)
        jout = torch.empty((nw, 5), dtype=torch.float32, device=dev)
        ms_mv, _ = time_steps(torch, lambda: jas.move(Rd, kd, rd, out=jout), args.steps, args.warmup)
        ms_mv_b = time_back_to_back(torch, lambda: jas.move(Rd, kd, rd, out=jout), args.steps, args.warmup)
        pairs = nw * 2 * (NE - 1 + NI)
        jforms["move_%d_walkers" % nw] = {"ms_per_step": ms_mv, "ms_back_to_back": ms_mv_b,
                                          "pair_evals_per_s": pairs / (ms_mv * 1e-3),
                                          "moves_per_s": nw / (ms_mv * 1e-3), "pairs": pairs}
        if nw == W.JASTROW["walkers"]:
            jo = (torch.empty(nw, dtype=torch.float32, device=dev),
                  torch.empty((nw, 3, NE), dtype=torch.float32, device=dev),
                  torch.empty((nw, NE), dtype=torch.float32, device=dev))
            ms_ev, _ = time_steps(torch, lambda: jas.evaluate(Rd, out=jo), args.steps, args.warmup)
            ms_ev_b = time_back_to_back(torch, lambda: jas.evaluate(Rd, out=jo), args.steps, args.warmup)
            pairs_ev = nw * NE * (NE - 1 + NI)  # pair terms of the definition (each e-e pair for both electrons)
            ops_ev = nw * (NE * (NE - 1) // 2 * 69.0 + NE * NI * 66.0)
            jforms["evaluate_%d_walkers" % nw] = {"ms_per_step": ms_ev, "ms_back_to_back": ms_ev_b,
                                                  "pair_evals_per_s": pairs_ev / (ms_ev * 1e-3),
                                                  "ops_per_step": ops_ev}
            del jo
        del Re, Rd, jout
    jforms["system"] = "%d electrons (%d up), %d ions of 2 species, unit cube, functors with 8 intervals, rcut 0.5" % (
        NE, jd["n_up"], NI)
    jforms["timing_note"] = ("ms_per_step: median of launches each between its own event pair; ms_back_to_back: "
                             "mean of launches issued back to back under one event pair, which for launches "
                             "shorter than the host's ~10 us per call measures the host's submission rate")
    # ALU roofline: FP32 operations of the definition against the VALU issue
    # rate, 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (packed FP32 off).  A pair
    # term with derivatives costs 66 operations, a value alone 41 (a move
    # forms both, at the new and the old position); the full evaluation
    # forms each electron pair once, 59 operations, and adds its terms to
    # both electrons, 10 more: 69 per unordered pair, 66 per electron-ion pair.
    peak_ops = 256 * 4 * 16 * 2.4e9
    for key, v in jforms.items():
        if not isinstance(v, dict):
            continue
        if key.startswith("evaluate"):
            ops_s = v["ops_per_step"] / (v["ms_per_step"] * 1e-3)
            v["roofline"] = {"bound": "alu", "ops_per_unordered_ee_pair": 69.0, "ops_per_ei_pair": 66.0,
                             "achieved_Tops": ops_s / 1e12, "peak_Tops": peak_ops / 1e12, "frac": ops_s / peak_ops,
                             "frac_back_to_back": v["ops_per_step"] / (v["ms_back_to_back"] * 1e-3) / peak_ops}
            continue
        ops = (66.0 + 41.0) / 2
        v["roofline"] = {"bound": "alu", "ops_per_pair": ops, "achieved_Tops": v["pair_evals_per_s"] * ops / 1e12,
                         "peak_Tops": peak_ops / 1e12, "frac": v["pair_evals_per_s"] * ops / peak_ops,
                         "frac_back_to_back": v["pairs"] * ops / (v["ms_back_to_back"] * 1e-3) / peak_ops}
    forms["jastrow_f32"] = jforms
    log("bench: jastrow %s" % {k: round(v["ms_per_step"], 4) for k, v in jforms.items() if isinstance(v, dict)})
    del jas
    torch.cuda.empty_cache()

    if not args.no_ragged:
        # Ragged workload: four tables (32^3/48^3/64^3/80^3, N = 64/128/256/384,
        # FP32) with U{64..1024} walkers each, in one graph-captured
        # persistent launch, against the same work as four tuned launches.
        log("bench: building the four ragged tables ...")
        tabs = W.make_ragged()
        sp = [q.Spline(t["grid"], t["coefs"], "f32", device=dev) for t in tabs]
        ps = [torch.from_numpy(t["pos"]).to(dev) for t in tabs]
        del tabs
        plan = q.Plan(sp, ps, tune_reps=3)
        units_r = sum(p.shape[0] * s.norb for s, p in zip(sp, ps))
        ms_plan, _ = time_steps(torch, plan.launch, args.steps, args.warmup)
        for s, p, o in zip(sp, ps, plan.outs):
            s.autotune(p, reps=2, out=o)

        def separate():
            for s, p, o in zip(sp, ps, plan.outs):
                s.eval_vgl(p, out=o)

        ms_sep, _ = time_steps(torch, separate, args.steps, args.warmup)
        info = plan.info()
        # the same plan in locality order (positions sorted on the device in
        # every launch, the task list dealt to the XCDs in eight segments)
        outs_plain = [[t.clone() for t in o] for o in plan.outs]
        plan_s = q.Plan(sp, ps, outs=plan.outs, tune_reps=3, sorted=True)
        ms_plan_s, _ = time_steps(torch, plan_s.launch, args.steps, args.warmup)
        plan.launch()
        same_s = True
        plan_s.launch()
        torch.cuda.synchronize()
        for o, e in zip(plan_s.outs, outs_plain):
            same_s = same_s and all(bool(torch.equal(a, b)) for a, b in zip(o, e))
        info_s = plan_s.info()
        del outs_plain
        forms["ragged_4_tables_f32"] = {
            "positions": [int(p.shape[0]) for p in ps], "norb": [s.norb for s in sp],
            "evals_per_s": units_r / (ms_plan * 1e-3), "ms_per_launch": ms_plan,
            "ms_four_separate_launches": ms_sep, "speedup_vs_separate": ms_sep / ms_plan,
            "hbm_frac": units_r * BYTES_PER_UNIT["f32"] / (ms_plan * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "tile": list(info["tile"]), "tasks": info["tasks"], "persistent_workgroups": info["blocks"]}
        forms["ragged_4_tables_f32_locality_sorted"] = {
            "evals_per_s": units_r / (ms_plan_s * 1e-3), "ms_per_launch": ms_plan_s,
            "speedup_vs_plan": ms_plan / ms_plan_s, "bitwise_equal_to_plan": same_s,
            "tile": list(info_s["tile"]), "tasks": info_s["tasks"], "persistent_workgroups": info_s["blocks"]}
        log("bench: ragged plan %.3f ms (sorted %.3f ms, equal %s) vs separate %.3f ms" % (
            ms_plan, ms_plan_s, same_s, ms_sep))
        del plan, plan_s, sp, ps
        torch.cuda.empty_cache()

    if args.mlp_steps > 0:
        forms["mlp_surrogate"] = bench_mlp(args, q, W, torch, dev, np)

    cpu = None
    if not args.no_cpu_baseline:
        # FP64 oracle on the host cores: a calibration run sizes a sample of
        # about --cpu-seconds (whole batches repeated if one batch is faster).
        ncores = len(os.sched_getaffinity(0))
        n_cal = 8192
        oracle.eval_vgl(grid, coefs, pos_np[:256], threads=ncores)  # thread pool start-up, untimed
        t0 = time.perf_counter()
        oracle.eval_vgl(grid, coefs, pos_np[:n_cal], threads=ncores)
        per_pos = (time.perf_counter() - t0) / n_cal
        want = int(args.cpu_seconds / max(per_pos, 1e-9))
        n = min(B, max(n_cal, want))
        reps = max(1, min(40, want // B)) if want > B else 1
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.eval_vgl(grid, coefs, pos_np[:n], threads=ncores)
        dt = time.perf_counter() - t0
        n1 = max(64, min(B, int(3.0 / max(per_pos * ncores, 1e-9))))
        t0 = time.perf_counter()
        oracle.eval_vgl(grid, coefs, pos_np[:n1], threads=1)
        dt1 = time.perf_counter() - t0
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": reps * n * N / dt, "unit": "orbital-VGL/s", "cores": ncores, "kind": "oracle",
               "single_thread": {"value": n1 * N / dt1, "sample": "the first %d positions, %.1f s" % (n1, dt1)},
               "host": {"cpu_model": model, "nproc": os.cpu_count(), "affinity": ncores},
               "sample": ("%d passes over the whole %d-position batch" % (reps, B) if n == B else
                          "the first %d of the %d positions" % (n, B)) +
                         " of the same workload, all %d orbitals; FP64 oracle (plain loops, OpenMP over "
                         "positions, gcc -O2), %.1f s wall" % (N, dt)}

    traffic = traffic_from_profiles(tile32)
    line = {
        "metric": "orbital-VGL evals/s and % HBM peak; MLP/BF16 vs FP32 spline speedup at fixed err",
        "value": evals,
        "unit": "orbital-VGL/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: plane-wave orbitals fitted on the grid, uniform random positions (seeded)",
        "config": {"workload": "80^3 periodic grid, N=384 orbitals, FP32 table; 512 walkers x 384 "
                               "electrons = 196608 positions per batch, one VGL each",
                   "grid": list(grid), "norb": N, "positions": B, "table": "f32", "tile": list(tile32),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "bytes_per_unit": BYTES_PER_UNIT["f32"], "units_per_launch": units,
                     "kernel": "eval_kernel<FP32, VGL> at tile %s" % (list(tile32),),
                     "timing": dict(timing32, statistic="median of the timed launches, each between its own pair "
                                                        "of HIP events on the launch stream"),
                     "cold_cache": {"ms_per_launch": ms_cold, "achieved": achieved_cold,
                                    "frac": achieved_cold / PEAK_HBM_GBS,
                                    "note": "median of single launches, each after a 512 MB scratch write that "
                                            "evicts L2 and the Infinity Cache"},
                     "traffic_note": "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by the same counters "
                                     "over a plain copy of known size; FETCH_SIZE also counts reads the Infinity "
                                     "Cache serves, so it bounds DRAM reads from above",
                     "attainable_stream_read_GBs": best_read,
                     "frac_of_attainable": achieved / best_read if best_read > 0 else None},
        "cpu_baseline": cpu,
        "fastest_form": {"form": "f32_locality_sorted", "evals_per_s": forms["f32_locality_sorted"]["evals_per_s"],
                         "ms_per_step": forms["f32_locality_sorted"]["ms_per_step"],
                         "note": "the same FP32 batch and outputs (bit for bit) with positions put in locality "
                                 "order on the device inside the timed step; value and roofline above are the "
                                 "plain evaluation, whose bound is HBM at the algorithmic bytes"},
        "forms": forms,
        "fixed_error": fixed_error_summary(forms, e32, ms32, ms_v, ms_rv, eps_ratio_v),
        "wall_s_timed": wall32,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
