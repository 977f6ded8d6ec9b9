"""Benchmark: particle x frequency-bin evaluations of the semi-coherent
statistic per second on one MI355X.

A step is one iteration of the search's hot path over the whole swarm: the
PSO move of 10^4 particles, the per-particle prologue (coefficients, support
window, equal-[h|h] edges), the generate-and-reduce over the data, the
finalize to Upsilon_N, and the best update.  Workload: 2^20 bins over
[0.016, 0.032) Hz (T_obs ~ 2.08 yr), A+E channels, two-component instrument
PSD, synthetic Gaussian noise plus a GW150914-like 3.5PN inspiral with the
low-frequency response at SNR 17, N = 1024 equal-[h|h] segments (node
stride 1024), particles uniform in the GW150914-like prior box.

Prints one JSON line.  value = in-support particle-bin evaluations per second
in FP64 (mixed precision reported beside it).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# FP64 operations per in-support particle-bin of the generate-and-reduce
# kernel, two channels, from its per-bin op list (a fused multiply-add counts
# 2, any other arithmetic op 1; roundings and conversions 0): bin coordinate
# 1 add; phase polynomial 5 FMA; split into table unit and remainder 3 add;
# remainder sin/cos: square 1 mul, sine 1 FMA + 1 mul, cosine 1 FMA; angle
# sum 2 FMA + 2 mul; response polynomials 20 FMA; data x conj(response)
# 6 FMA + 2 mul; Z rotate-and-accumulate 4 FMA; H 4 FMA + 2 mul.  Total
# 43 FMA + 12 other = 86 + 12 = 98 (the FP64 flop counter of rocprofv3 reads
# a few percent more per in-support evaluation: lanes idle at support edges
# and the per-block set-up).
FLOP_PER_EVAL_FP64 = 98
# The same with the sparse-grid template (cubic splines): the phase and the
# four response polynomials are cubic instead of quintic, 2 + 8 FMA fewer.
FLOP_PER_EVAL_FP64_SPLINE = 78
PEAK_FP64_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 64 lanes x 2
# FP32 operations per in-support particle-bin of the mixed-precision
# generate-and-reduce kernel, two channels, from its per-bin op list (same
# counting): bin coordinate 1 add; linear phase a1h j 1 mul, its fraction
# 1 op; residual cubic 3 FMA and 1 add; response cubics 4 x 3 FMA; data x
# conj(response) 6 FMA + 2 mul; Z rotate-and-accumulate 4 FMA; H 4 FMA +
# 2 mul.  Total 29 FMA + 8 other = 66, plus 2 hardware transcendentals
# (sin and cos of revolutions), counted apart.  The FP64 additions of the
# FP32 partial sums (3 per 32 bins) are left out.
FLOP_PER_EVAL_MIXED = 66
TRANS_PER_EVAL_MIXED = 2
# FP32 vector peak as published (256 CU x 2.4 GHz x 128 FMA lanes x 2), the
# rate of packed FP32 instructions, which the code does not use.  Non-packed
# FP32 instructions issue at up to 1.2x (three waves per SIMD) to 1.5x
# (eight waves, eight independent chains) the single-issue rate of 64 lanes
# per 4 cycles on gfx950; the library's peak probe measures the eight-wave
# figure (measured_peaks in the JSON line).  Transcendentals issue at a
# quarter of the FP32 rate.
PEAK_FP32_TFLOPS = 157.3
PEAK_TRANS_PER_S = 256 * 4 * 32 * 2.4e9 / 4  # 1.97e13 per second


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "k_main_multi_fp64_lisa1m.txt")
MIXED_PROFILE = os.path.join(ROOT, "profiles", "k_main_multi_mixed_lisa1m.txt")
STREAMS_PROFILE = os.path.join(ROOT, "profiles", "k_streams_lisa1m.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2408_13170_amd", "csrc", f)
                  for f in ("scs_kernels.hip", "scs_internal.hpp", "scs_math.hpp")]
LAUNCH_SOURCE = os.path.join(ROOT, "paper_2408_13170_amd", "csrc", "scs_host.hip")


def kernel_digest():
    """sha256 of the kernel sources and of the host code that sets the
    generate-and-reduce's launch shape (the marked regions of scs_host.hip)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    with open(LAUNCH_SOURCE) as fh:
        txt = fh.read()
    for part in re.findall(r"// ==== launch shape of the generate-and-reduce \(begin\)\n(.*?)"
                           r"// ==== launch shape of the generate-and-reduce \(end\)", txt, re.S):
        h.update(part.encode())
    return h.hexdigest()


def measured_traffic(path=PROFILE):
    """HBM bytes per launch of the profiled kernel (the FP64 generate-and-reduce
    by default) from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy), or None when the kernel sources or the
    host code that picks the generate-and-reduce's launch shape changed since
    it was taken."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256") != kernel_digest():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def n_eff(bounds):
    """Non-empty segments per row of edges [P, N+1]."""
    return np.sum(bounds[:, 1:] > bounds[:, :-1], axis=1)


def floored_err(got, ref, neff):
    """|got - ref| / max(|ref|, 2 N_eff): the relative error, floored at the
    statistic's noise mean (each non-empty segment adds chi^2 with two
    degrees of freedom)."""
    return np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 * np.maximum(neff, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--mode", choices=["step", "batched", "serve", "streams", "search", "peaks"], default="step",
                    help="step: PSO steps of one 10^4-particle swarm (default); batched: six swarms of the "
                         "hierarchy in one graph-captured persistent launch; serve: concurrent searches with "
                         "Poisson-arriving requests; streams: one theta against many noise realisations "
                         "(Sec 5.1), HBM-bound; search: the whole hierarchical multi-swarm search (Sec 3.2); "
                         "peaks: the device's measured FP64 / FP32 / sine / HBM ceilings")
    ap.add_argument("--max-iters", type=int, default=400, help="search: iteration cap per rung")
    ap.add_argument("--response", choices=["lf", "fd", "fd3"], default="lf",
                    help="step: LISA response model, low-frequency A+E (default), or the full frequency-domain "
                         "TDI response with its noise PSDs on A+E (fd) or A+E+T (fd3)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests per offered load")
    ap.add_argument("--realisations", type=int, default=1024,
                    help="streams: noise realisations held in HBM at once")
    ap.add_argument("--loads", type=str, default="0.5,0.8,0.95", help="serve: offered loads (x capacity)")
    ap.add_argument("--no-legs", action="store_true",
                    help="step: skip the short batched, served and 16384-bin legs of the default run")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="batched: autotuner cache file (read, then rewritten)")
    ap.add_argument("--sparse-stride", type=int, default=0,
                    help="step: evaluate the template on the sparse grid of Sec 4 (nodes every this many bins, "
                         "cubic splines onto every bin) instead of per bin; the paper's stride is 1000")
    args = ap.parse_args()
    if args.copy_probe_mib:
        import torch

        src = torch.ones(args.copy_probe_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the statistic shards by particle with no "
              "exchange, and that multi-GPU path is a design, not part of this library.", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "streams":
        return bench_streams(args)
    if args.mode == "search":
        return bench_search(args)
    if args.mode == "peaks":
        from paper_2408_13170_amd import B

        print(json.dumps({"measured_peaks": leg_peaks(B)}), flush=True)
        return

    import torch

    from paper_2408_13170_amd import B

    dev = torch.device("cuda:0")
    w = synth.workload("lisa1m")
    K = w.grid.K
    fd = args.response in ("fd", "fd3")
    psd = bench_psd(w, args.response)
    # --- data: noise + injection made with the library's own FP64 template
    ctx, d_ri = make_search(B, torch, w, dev, args.response, args.sparse_stride)
    resp = B.SCS_RESP_LISA_LF_AE if args.response == "lf" else B.SCS_RESP_LISA_FD_AE
    # --- swarm of 10^4 particles, first rung of the ladder (Table tab:PSO_hyperparams, N = 100 row)
    eps = [0.1, 0.05, 5e-8, 0.1, 0.1, 0.2, 0.1]  # Mc, eta, f_low, lambda, beta, iota, psi
    prm = B.pso_params(0.5, 0.2, 0.3, eps)
    stream = torch.cuda.current_stream()

    def run(prec, steps, warmup, swarm_seed):
        sw = B.scs_swarm_create(ctx, w.P, w.prior_lo, w.prior_hi, synth.PERIODIC, seed=swarm_seed, swarm_id=0)
        for _ in range(warmup):
            B.scs_pso_step(sw, prm, prec, stream)
        torch.cuda.synchronize()
        B.scs_ctx_stats(ctx, reset=True)
        B.scs_ctx_profile(ctx, 1)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(stream)
        for i in range(steps):
            B.scs_pso_step(sw, prm, prec, stream)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n_launch, main_ms = B.scs_ctx_profile(ctx, 0)
        ev_support, ev_band, unresolved = B.scs_ctx_stats(ctx, reset=True)
        step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        st = B.scs_swarm_read(sw, w.P)
        B.scs_swarm_destroy(sw)
        return {"wall_s": t1 - t0, "evals": ev_support, "unresolved": unresolved, "step_ms": step_ms,
                "main_ms": main_ms, "main_launches": n_launch, "gbest": st["gbest_val"]}

    r64 = run(B.SCS_PREC_FP64, args.steps, args.warmup, 101)
    log(f"fp64: {r64['evals'] / r64['wall_s']:.4g} evals/s, step p50 {np.median(r64['step_ms']):.3f} ms, "
        f"main kernel {r64['main_ms'] / max(r64['main_launches'], 1):.3f} ms/launch, best {r64['gbest']:.2f}")
    rmx = None
    if not args.no_mixed:
        rmx = run(B.SCS_PREC_MIXED, args.steps, args.warmup, 101)
        log(f"mixed: {rmx['evals'] / rmx['wall_s']:.4g} evals/s, step p50 {np.median(rmx['step_ms']):.3f} ms")
    # --- mixed vs FP64 on one fixed swarm position
    th = torch.tensor(synth.workload_particles(w, seed=w.seed + 7), device=dev)
    u64 = torch.empty(w.P, dtype=torch.float64, device=dev)
    u32 = torch.empty(w.P, dtype=torch.float64, device=dev)
    B.scs_evaluate(ctx, th, u64, B.SCS_PREC_FP64)
    torch.cuda.synchronize()
    neff = n_eff(B.scs_last_bounds(ctx, w.P, w.N)[1])
    B.scs_evaluate(ctx, th, u32, B.SCS_PREC_MIXED)
    torch.cuda.synchronize()
    a, b = u64.cpu().numpy(), u32.cpu().numpy()
    ok = np.isfinite(a)
    err = floored_err(b[ok], a[ok], neff[ok])
    # likelihood epilogue (Sec 2.1 - 2.2) on the same swarm: the same
    # generate-and-reduce with more sums in the epilogue, then log hat L_N and log L
    st = torch.empty((w.P, B.SCS_NSTATS), dtype=torch.float64, device=dev)
    amp = torch.ones(w.P, dtype=torch.float64, device=dev)
    ls, lc = torch.empty_like(amp), torch.empty_like(amp)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 3
    ev[0].record(stream)
    for _ in range(reps):
        B.scs_evaluate(ctx, th, u64, B.SCS_PREC_FP64)
    ev[1].record(stream)
    for _ in range(reps):
        B.scs_evaluate_stats(ctx, th, st, B.SCS_PREC_FP64)
    ev[2].record(stream)
    for _ in range(reps):
        B.scs_loglike(ctx, st, amp, None, ls, lc)
    ev[3].record(stream)
    torch.cuda.synchronize()
    epi = {"evaluate_ms": ev[0].elapsed_time(ev[1]) / reps, "evaluate_stats_ms": ev[1].elapsed_time(ev[2]) / reps,
           "loglike_ms": ev[2].elapsed_time(ev[3]) / reps,
           "what": "one FP64 evaluation of the fixed 10^4-particle swarm: Upsilon only, then with hat O_N, "
                   "<h|h>, <d|h> (Sec 2.1 - 2.2), then log hat L_N and log L from those rows"}
    log(f"likelihood epilogue: evaluate {epi['evaluate_ms']:.3f} ms, with statistics "
        f"{epi['evaluate_stats_ms']:.3f} ms, loglike {epi['loglike_ms']:.4f} ms")

    value = r64["evals"] / r64["wall_s"]
    ms_step = 1e3 * r64["wall_s"] / args.steps
    avg_main_ms = r64["main_ms"] / max(r64["main_launches"], 1)
    evals_per_launch = r64["evals"] / max(r64["main_launches"], 1)
    flop64 = FLOP_PER_EVAL_FP64_SPLINE if args.sparse_stride else FLOP_PER_EVAL_FP64
    achieved = evals_per_launch * flop64 / (avg_main_ms * 1e-3) / 1e12
    out = {
        "metric": "particle x freq-bin statistic evals/s (in-support), FP64; p50/p99 step latency; mixed vs FP64",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded Gaussian noise from the two-component LISA PSD + GW150914-like 3.5PN injection",
        "config": {"workload": "A+E, 2^20 bins over [0.016,0.032) Hz, T_obs 2.08 yr, N_seg 1024 (equal [h|h], "
                               "node stride 1024), 10^4 PSO particles in the GW150914-like prior box, one PSO "
                               "iteration per step", "particles": w.P, "bins": K, "N_seg": w.N,
                   "response": {"lf": "low-frequency A/E", "fd": "full frequency-domain TDI A/E (finite arm length)",
                                "fd3": "full frequency-domain TDI A/E/T (finite arm length)"}[args.response],
                   "template": (f"sparse grid, nodes every {args.sparse_stride} bins, cubic splines"
                                if args.sparse_stride else "per bin (block polynomials)")},
        "latency_ms": {"p50": float(np.median(r64["step_ms"])), "p99": float(np.quantile(r64["step_ms"], 0.99))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None if (fd or args.sparse_stride) else measured_traffic(),
                     "kernel": {"lf": "k_main_multi<2,false,1> (FP64 generate-and-reduce, low-frequency response)",
                                "fd": "k_main_multi<2,false,2> (FP64 generate-and-reduce, full response)",
                                "fd3": "k_main_multi<3,false,2> (FP64 generate-and-reduce, full response, A+E+T)"}[
                         args.response] + (", sparse-grid template" if args.sparse_stride else ""),
                     "avg_launch_ms": avg_main_ms, "flop_per_eval": flop64,
                     "evals_per_launch": evals_per_launch},
        "unresolved_particles": r64["unresolved"],
        "likelihood_epilogue": epi,
    }
    if rmx is not None:
        mx_launch_ms = rmx["main_ms"] / max(rmx["main_launches"], 1)
        mx_evals_per_launch = rmx["evals"] / max(rmx["main_launches"], 1)
        mx_rate = mx_evals_per_launch / (mx_launch_ms * 1e-3)
        mx_achieved = mx_rate * FLOP_PER_EVAL_MIXED / 1e12
        out["mixed"] = {"value": rmx["evals"] / rmx["wall_s"], "unit": "evals/s",
                        "roofline": {"bound": "alu", "achieved": mx_achieved, "peak": PEAK_FP32_TFLOPS,
                                     "unit": "TFLOP/s", "frac": mx_achieved / PEAK_FP32_TFLOPS,
                                     "traffic": None if (fd or args.sparse_stride)
                                     else measured_traffic(MIXED_PROFILE),
                                     "kernel": {"lf": "k_main_multi<2,true,1>", "fd": "k_main_multi<2,true,2>",
                                                "fd3": "k_main_multi<3,true,2>"}[args.response]
                                     + " (mixed-precision generate-and-reduce)",
                                     "avg_launch_ms": mx_launch_ms, "flop_per_eval": FLOP_PER_EVAL_MIXED,
                                     "evals_per_launch": mx_evals_per_launch,
                                     "transcendentals_per_eval": TRANS_PER_EVAL_MIXED,
                                     "transcendental_rate": mx_rate * TRANS_PER_EVAL_MIXED,
                                     "transcendental_peak": PEAK_TRANS_PER_S,
                                     "transcendental_frac": mx_rate * TRANS_PER_EVAL_MIXED / PEAK_TRANS_PER_S},
                        "ms_per_step": 1e3 * rmx["wall_s"] / args.steps,
                        "latency_ms": {"p50": float(np.median(rmx["step_ms"])),
                                       "p99": float(np.quantile(rmx["step_ms"], 0.99))},
                        "avg_main_launch_ms": rmx["main_ms"] / max(rmx["main_launches"], 1),
                        "speedup_vs_fp64": (rmx["evals"] / rmx["wall_s"]) / value,
                        "err_vs_fp64": {"median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                                        "max": float(err.max()),
                                        "measure": "|U_mixed - U_fp64| / max(U_fp64, 2 N_eff)"}}
    if not args.no_legs:
        pk = leg_peaks(B)
        out["measured_peaks"] = pk
        out["roofline"]["frac_of_measured_peak"] = achieved / pk["fp64_tflops"]
        if rmx is not None:
            out["mixed"]["roofline"]["frac_of_measured_peak"] = mx_achieved / pk["fp32_tflops"]
    if not args.no_legs and not args.sparse_stride:
        out["sparse_template"] = leg_sparse(B, ctx, w, resp, run, th, a, neff, args.no_mixed)
    if not args.no_legs:
        out["config1"] = leg_config1(B, torch, dev)
        out["batched"] = bench_batched_core(B, torch, dev, steps=5, warmup=2, tune_cache=args.tune_cache)
        out["served"] = bench_serve_core(B, torch, dev, n_requests=200, loads=[0.8])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, psd, d_ri.cpu().numpy(), args.cpu_seconds, fd)
    B.scs_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


def bench_psd(w, response="lf"):
    """PSDs of workload w: the low-frequency A/E model, or the TDI noise of
    the full response (its A and E rows, or A, E and T)."""
    if response == "lf":
        return synth.psd_arrays(w)
    return synth.lisa_tdi_psd(w.grid.freqs())[:3 if response == "fd3" else 2]


def make_search(B, torch, w, dev, response="lf", sparse_stride=0):
    """Context with seeded noise plus the injection of workload w at its SNR
    (template from the library's own FP64 per-bin waveform kernel); response
    selects the low-frequency or the full frequency-domain response (A+E or
    A+E+T); sparse_stride > 0 makes the context's template the sparse-grid one."""
    K, df, f_min = w.grid.K, w.grid.df, w.grid.f_min
    psd = bench_psd(w, response)
    nch = psd.shape[0]
    resp = B.SCS_RESP_LISA_LF_AE if response == "lf" else B.SCS_RESP_LISA_FD_AE
    noise = synth.noise(psd, df, w.seed)
    ctx = B.scs_ctx_create(0)
    B.scs_load_data(ctx, np.zeros((nch, K, 2)), psd, f_min, df)
    B.scs_set_model(ctx, w.pn_order, resp, B.SCS_SUPPORT_TOBS, w.grid.t_obs)
    h = torch.empty((nch, K, 2), dtype=torch.float64, device=dev)
    B.scs_waveform(ctx, torch.tensor(w.injection, device=dev), h)
    torch.cuda.synchronize()
    hc = torch.complex(h[..., 0], h[..., 1])
    S = torch.tensor(psd, device=dev)
    hh = float(4 * df * torch.sum(hc.abs() ** 2 / S))
    d = torch.tensor(noise, device=dev) + hc * (w.snr / math.sqrt(hh))
    d_ri = torch.stack([d.real, d.imag], -1).contiguous()
    B.scs_load_data(ctx, d_ri, S.contiguous(), f_min, df)
    B.scs_set_model(ctx, w.pn_order, resp, B.SCS_SUPPORT_TOBS, w.grid.t_obs, sparse_stride=sparse_stride)
    B.scs_define_segmentation(ctx, w.N, B.SCS_SEG_EQUAL_SNR, w.G)
    return ctx, d_ri


def bench_batched(args):
    import torch

    from paper_2408_13170_amd import B

    dev = torch.device("cuda:0")
    res = bench_batched_core(B, torch, dev, args.steps, args.warmup, args.tune_cache)
    out = {"metric": "particle x freq-bin statistic evals/s (in-support), batched hierarchy, FP64; mixed beside",
           "value": res["fp64"]["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["fp64"]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic: same data as the step benchmark",
           "config": {"workload": res["workload"]}}
    out.update({k: v for k, v in res.items() if k != "workload"})
    print(json.dumps(out), flush=True)


def bench_batched_core(B, torch, dev, steps, warmup, tune_cache=None):
    """Six swarms of the hierarchy, (N, P) = (4096, 16384) ... (1, 128), on the
    2^20-bin A+E data in ONE graph-captured batched launch (one persistent
    generate-and-reduce kernel over all tiles), FP64 and mixed, first with
    the default launch shapes, then with the shapes the batch autotuner picks
    (the launch occupancy and each swarm's LDS block and chunk, timed as the
    whole batched evaluation; cached in tune_cache when given); mixed error per level
    against FP64 (floored at 2 N_eff)."""
    w = synth.workload("lisa1m")
    ctx, _ = make_search(B, torch, w, dev)
    stream = torch.cuda.current_stream()
    items = []
    for i, (N, P) in enumerate(synth.LADDER_SWARMS):
        th = torch.tensor(synth.particles(w.prior_lo, w.prior_hi, P, w.seed + 700 + i), device=dev)
        items.append((ctx, N, th, torch.empty(P, dtype=torch.float64, device=dev)))

    def timed(prec):
        g = B.scs_graph_create(items, prec)
        for _ in range(warmup):
            B.scs_graph_launch(g, stream)
        torch.cuda.synchronize()
        B.scs_ctx_stats(ctx, reset=True)
        B.scs_ctx_profile(ctx, 1)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        evs[0].record(stream)
        for i in range(steps):
            B.scs_graph_launch(g, stream)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n_launch, main_ms = B.scs_ctx_profile(ctx, 0)
        ev_support, _, _ = B.scs_ctx_stats(ctx, reset=True)
        step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        B.scs_graph_destroy(g)
        return {"value": ev_support / (t1 - t0), "unit": "evals/s", "ms_per_batch": 1e3 * (t1 - t0) / steps,
                "latency_ms": {"p50": float(np.median(step_ms)), "p99": float(np.quantile(step_ms, 0.99))},
                "avg_main_launch_ms": main_ms / max(n_launch, 1), "evals_per_batch": ev_support / steps,
                "ups": [it[3].cpu().numpy().copy() for it in items]}

    res = {"default_shapes": {}}
    for prec, name in ((B.SCS_PREC_FP64, "fp64"), (B.SCS_PREC_MIXED, "mixed")):
        r = timed(prec)
        del r["ups"]
        res["default_shapes"][name] = r
        log(f"batched {name}, default shapes: {r['value']:.4g} evals/s, {r['ms_per_batch']:.2f} ms per batch")
    t0 = time.perf_counter()
    for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
        B.scs_autotune_batch(items, prec, tune_cache)
    tune_s = time.perf_counter() - t0
    for prec, name in ((B.SCS_PREC_FP64, "fp64"), (B.SCS_PREC_MIXED, "mixed")):
        res[name] = timed(prec)
        log(f"batched {name}, tuned shapes: {res[name]['value']:.4g} evals/s, "
            f"{res[name]['ms_per_batch']:.2f} ms per batch")
    per_level = []
    for (N, P), it, a, b in zip(synth.LADDER_SWARMS, items, res["fp64"]["ups"], res["mixed"]["ups"]):
        # edges of the level's particles (a solo evaluation gives the batched values bit for bit)
        B.scs_define_segmentation(ctx, N, B.SCS_SEG_EQUAL_SNR, w.G)
        B.scs_evaluate(ctx, it[2], torch.empty(P, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        neff = n_eff(B.scs_last_bounds(ctx, P, N)[1])
        ok = np.isfinite(a)
        e = floored_err(b[ok], a[ok], neff[ok])
        per_level.append({"N": N, "P": P, "median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)),
                          "max": float(e.max())})
    for r in (res["fp64"], res["mixed"]):
        del r["ups"]
    B.scs_ctx_destroy(ctx)
    res["mixed_speedup"] = res["mixed"]["value"] / res["fp64"]["value"]
    res["tuned_vs_default"] = {n: res[n]["value"] / res["default_shapes"][n]["value"] for n in ("fp64", "mixed")}
    res["tune_seconds"] = tune_s
    res["mixed_err_vs_fp64_per_level"] = per_level
    res["workload"] = ("six swarms (N, P) = " + str(synth.LADDER_SWARMS) + " on the 2^20-bin A+E data, one HIP "
                       "graph per precision, one persistent fused generate-and-reduce launch, autotuned shapes")
    return res


def leg_peaks(B):
    """The device's own ceilings (the library's peak microbenchmark): FP64
    and non-packed FP32 FMA chains, the FP32 hardware sine, and a streaming
    HBM copy; the published peaks stay the roofline's reference."""
    pk = B.scs_peak_probe(0)
    pk = {k: float(v) for k, v in pk.items()}
    pk["published"] = {"fp64_tflops": PEAK_FP64_TFLOPS, "fp32_tflops": PEAK_FP32_TFLOPS,
                       "sin32_per_s_1e12": PEAK_TRANS_PER_S / 1e12, "hbm_tbps": 8.0}
    log(f"measured peaks: FP64 {pk['fp64_tflops']:.1f} TFLOP/s, FP32 {pk['fp32_tflops']:.1f} TFLOP/s, "
        f"sine {pk['sin32_per_s_1e12']:.2f}e12/s, HBM copy {pk['hbm_copy_tbps']:.2f} TB/s")
    return pk


def leg_sparse(B, ctx, w, resp, run, th, ups_per_bin, neff, no_mixed, stride=1000, steps=10, warmup=2):
    """The step workload with the paper's sparse-grid template (Sec 4: nodes
    every 1000 bins, cubic splines onto every bin) on the same context: PSO
    steps in FP64 and mixed, and on the fixed swarm how far Upsilon_N moves
    from the per-bin template's (the interpolation's effect, second order)."""
    import torch

    B.scs_set_model(ctx, w.pn_order, resp, B.SCS_SUPPORT_TOBS, w.grid.t_obs, sparse_stride=stride)
    out = {"stride": stride, "flop_per_eval_fp64": FLOP_PER_EVAL_FP64_SPLINE}
    for prec, name in ((B.SCS_PREC_FP64, "fp64"), (B.SCS_PREC_MIXED, "mixed")):
        if no_mixed and prec == B.SCS_PREC_MIXED:
            continue
        r = run(prec, steps, warmup, 101)
        launch_ms = r["main_ms"] / max(r["main_launches"], 1)
        out[name] = {"value": r["evals"] / r["wall_s"], "unit": "evals/s",
                     "ms_per_step": 1e3 * r["wall_s"] / steps, "avg_main_launch_ms": launch_ms,
                     "latency_ms": {"p50": float(np.median(r["step_ms"])),
                                    "p99": float(np.quantile(r["step_ms"], 0.99))}}
        log(f"sparse-grid template {name}: {out[name]['value']:.4g} evals/s, main kernel {launch_ms:.3f} ms/launch")
    u = torch.empty(th.shape[0], dtype=torch.float64, device=th.device)
    B.scs_evaluate(ctx, th, u, B.SCS_PREC_FP64)
    torch.cuda.synchronize()
    us = u.cpu().numpy()
    ok = np.isfinite(ups_per_bin) & np.isfinite(us)
    dif = floored_err(us[ok], ups_per_bin[ok], neff[ok])
    out["ups_vs_per_bin_template"] = {"median": float(np.median(dif)), "max": float(dif.max()),
                                      "measure": "|U_sparse - U_per_bin| / max(U_per_bin, 2 N_eff), FP64"}
    return out


def leg_config1(B, torch, dev, reps=50):
    """The 16384-bin single-channel configuration: unit white PSD, 2PN
    injection (Mc 30, q 0.8) at SNR 20, N = 16, 64 particles in the
    Mc +-1% / q +-10% box, one evaluation per particle per call; FP64 and
    mixed call latency and throughput (a launch-bound size: 10^6
    particle-bins per call)."""
    w = synth.workload("white16k")
    K, df = w.grid.K, w.grid.df
    psd = synth.psd_arrays(w)
    ctx = B.scs_ctx_create(0)
    B.scs_load_data(ctx, np.zeros((1, K, 2)), psd, w.grid.f_min, df)
    B.scs_set_model(ctx, w.pn_order, B.SCS_RESP_NONE, B.SCS_SUPPORT_FULL, w.grid.t_obs)
    h = torch.empty((1, K, 2), dtype=torch.float64, device=dev)
    B.scs_waveform(ctx, torch.tensor(w.injection, device=dev), h)
    torch.cuda.synchronize()
    hc = torch.complex(h[..., 0], h[..., 1])
    hh = float(4 * df * torch.sum(hc.abs() ** 2))
    d = torch.tensor(synth.noise(psd, df, w.seed), device=dev) + hc * (w.snr / math.sqrt(hh))
    B.scs_load_data(ctx, torch.stack([d.real, d.imag], -1).contiguous(), torch.tensor(psd, device=dev),
                    w.grid.f_min, df)
    B.scs_set_model(ctx, w.pn_order, B.SCS_RESP_NONE, B.SCS_SUPPORT_FULL, w.grid.t_obs)
    B.scs_define_segmentation(ctx, w.N, B.SCS_SEG_EQUAL_SNR, w.G)
    th = torch.tensor(synth.workload_particles(w), device=dev)
    u = torch.empty(w.P, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    out = {"workload": "16384 bins over [0.016, 0.032) Hz, one channel, unit white PSD, 2PN, N_seg 16, "
                       "64 particles", "evals_per_call": w.P * K}
    for prec, name in ((B.SCS_PREC_FP64, "fp64"), (B.SCS_PREC_MIXED, "mixed")):
        for _ in range(5):
            B.scs_evaluate(ctx, th, u, prec)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record(stream)
        for i in range(reps):
            B.scs_evaluate(ctx, th, u, prec)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(reps)])
        out[name] = {"evals_per_s": w.P * K / (ms.mean() * 1e-3),
                     "latency_ms": {"p50": float(np.median(ms)), "p99": float(np.quantile(ms, 0.99))}}
        log(f"16384-bin configuration {name}: {out[name]['evals_per_s']:.3g} evals/s, "
            f"p50 {np.median(ms):.3f} ms per call")
    B.scs_ctx_destroy(ctx)
    return out


def bench_serve(args):
    import torch

    from paper_2408_13170_amd import B

    dev = torch.device("cuda:0")
    rep = bench_serve_core(B, torch, dev, args.requests, [float(x) for x in args.loads.split(",")])
    levels = rep["fp64"]["levels"]
    out = {"metric": "served statistic evaluations: p50/p99 request latency and throughput, FP64; mixed beside",
           "value": levels[-1]["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": len(levels),
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic: eight seeded searches",
           "config": {"workload": rep["workload"], **rep["server_shape"]},
           "capacity_rps": rep["fp64"]["capacity_rps"],
           "capacity_evals_per_s": rep["fp64"]["capacity_evals_per_s"], "levels": levels,
           "mixed": rep["mixed"], "equal_rate": rep.get("equal_rate"), "server": rep["server"]}
    print(json.dumps(out), flush=True)


def bench_serve_core(B, torch, dev, n_requests, loads, equal_rate=0.95):
    """Eight independent searches (2^19 - 2^21 bins, A+E, GW150914-like and
    GW190521-like injections at SNR 15 - 40) behind the native request loop.
    Requests of 256 - 16384 particles (log-uniform) at a segment count from
    the ladder arrive as a Poisson process at fractions of the measured
    capacity; p50 / p99 latency (submit to result) and throughput, FP64 and
    mixed; then the same requests at the same arrival times in both
    precisions, at equal_rate x the FP64 capacity (latency at equal offered
    traffic: each precision's loads above are fractions of its own capacity,
    and the mixed capacity is higher); mixed against FP64 on the same
    requests (floored at 2 N_eff)."""
    searches = []
    for w in synth.served_streams():
        ctx, _ = make_search(B, torch, w, dev)
        searches.append((w, ctx))
    torch.cuda.synchronize()
    ladder = [4096, 1024, 256, 64, 16]
    rng = np.random.default_rng(synth.BASE_SEED + 900)

    def make_requests(n):
        reqs = []
        for _ in range(n):
            si = int(rng.integers(len(searches)))
            w, ctx = searches[si]
            P = int(np.exp(rng.uniform(np.log(256), np.log(16384))))
            reqs.append((ctx, int(rng.choice(ladder)), synth.particles(w.prior_lo, w.prior_hi, P,
                                                                         int(rng.integers(1 << 30))), si))
        return reqs

    budget, inflight, n_streams = 64 << 30, 32, 4
    srv = B.scs_server_create(0, max_inflight=inflight, hbm_budget=budget, n_streams=n_streams)

    def run(reqs, arrivals, prec):
        outs = {}
        done = []
        t0 = time.perf_counter()
        k = 0
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while k < len(reqs) and (arrivals is None or arrivals[k] <= now):
                ctx, N, th, si = reqs[k]
                ups = np.empty(th.shape[0])
                rid = B.scs_server_submit(srv, ctx, N, th, ups, prec)
                outs[rid] = (ups, k)
                k += 1
            wait = 1 if k < len(reqs) else 20
            done += B.scs_server_poll(srv, max_out=1024, wait_ms=wait)
        t1 = time.perf_counter() - t0
        lat = np.array([d["t_done"] - d["t_submit"] for d in done]) * 1e3
        queue = np.array([d["t_launch"] - d["t_submit"] for d in done]) * 1e3
        assert all(d["status"] == 0 for d in done)
        results = [None] * len(reqs)
        for rid, (ups, i) in outs.items():
            results[i] = ups
        return t1, lat, queue, results

    burst = make_requests(max(32, n_requests // 8))
    run(burst[:16], None, B.SCS_PREC_FP64)  # warm-up: workspaces, slots
    run(burst[:16], None, B.SCS_PREC_MIXED)
    report = {}
    burst_out = {}
    for pname, prec in (("fp64", B.SCS_PREC_FP64), ("mixed", B.SCS_PREC_MIXED)):
        # capacity: a closed burst of requests
        for _, ctx in searches:
            B.scs_ctx_stats(ctx, reset=True)
        t_b, _, _, burst_out[pname] = run(burst, None, prec)
        ev_b = sum(B.scs_ctx_stats(ctx, reset=True)[0] for _, ctx in searches)
        capacity = len(burst) / t_b
        log(f"served {pname}: capacity {capacity:.1f} requests/s, {ev_b / t_b:.4g} evals/s")
        levels = []
        for load in loads:
            reqs = make_requests(n_requests)
            arrivals = np.cumsum(rng.exponential(1.0 / (load * capacity), len(reqs)))
            t, lat, queue, _ = run(reqs, arrivals, prec)
            ev = sum(B.scs_ctx_stats(ctx, reset=True)[0] for _, ctx in searches)
            levels.append({"offered_load": load, "offered_rps": load * capacity, "achieved_rps": len(reqs) / t,
                           "evals_per_s": ev / t, "requests": len(reqs),
                           "latency_ms": {"p50": float(np.median(lat)), "p99": float(np.quantile(lat, 0.99))},
                           "queue_ms": {"p50": float(np.median(queue)), "p99": float(np.quantile(queue, 0.99))}})
            log(f"served {pname} load {load}: {len(reqs) / t:.1f} req/s, p50 {np.median(lat):.1f} ms, "
                f"p99 {np.quantile(lat, 0.99):.1f} ms (queue p50 {np.median(queue):.1f} ms)")
        report[pname] = {"capacity_rps": capacity, "capacity_evals_per_s": ev_b / t_b, "levels": levels}
    if equal_rate:
        reqs = make_requests(n_requests)
        rate = equal_rate * report["fp64"]["capacity_rps"]
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
        eq = {"offered_rps": rate, "fraction_of_fp64_capacity": equal_rate, "requests": len(reqs)}
        for pname, prec in (("fp64", B.SCS_PREC_FP64), ("mixed", B.SCS_PREC_MIXED)):
            t, lat, queue, _ = run(reqs, arrivals, prec)
            for _, ctx in searches:
                B.scs_ctx_stats(ctx, reset=True)
            eq[pname] = {"achieved_rps": len(reqs) / t,
                         "latency_ms": {"p50": float(np.median(lat)), "p99": float(np.quantile(lat, 0.99))},
                         "queue_ms": {"p50": float(np.median(queue)), "p99": float(np.quantile(queue, 0.99))}}
            log(f"served {pname} at {rate:.1f} req/s (both precisions, same requests and arrivals): "
                f"p50 {np.median(lat):.1f} ms, p99 {np.quantile(lat, 0.99):.1f} ms")
        report["equal_rate"] = eq
    # mixed against FP64 on the burst's requests (each served in both precisions)
    errs = []
    for (ctx, N, th, si), a, b in zip(burst, burst_out["fp64"], burst_out["mixed"]):
        B.scs_define_segmentation(ctx, N, B.SCS_SEG_EQUAL_SNR, searches[si][0].G)
        B.scs_evaluate(ctx, torch.tensor(th, device=dev), torch.empty(th.shape[0], dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        neff = n_eff(B.scs_last_bounds(ctx, th.shape[0], N)[1])
        ok = np.isfinite(a)
        errs.append(floored_err(b[ok], a[ok], neff[ok]))
    err = np.concatenate(errs)
    report["mixed"]["err_vs_fp64"] = {"median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                                      "max": float(err.max()), "requests": len(burst),
                                      "measure": "|U_mixed - U_fp64| / max(U_fp64, 2 N_eff), same requests "
                                                 "served in both precisions"}
    log(f"served mixed vs fp64 on {len(burst)} requests: median {np.median(err):.3g}, max {err.max():.3g}")
    st = B.scs_server_stats(srv)
    B.scs_server_destroy(srv)
    for _, ctx in searches:
        B.scs_ctx_destroy(ctx)
    report["server"] = {k: int(v) for k, v in st.items()}
    report["server_shape"] = {"max_inflight": inflight, "streams": n_streams, "hbm_budget_gib": budget >> 30}
    report["workload"] = ("8 searches, K in {2^19, 2^20, 2^21}, A+E; requests of 256-16384 particles "
                          "(log-uniform), N in " + str(ladder) + ", Poisson arrivals")
    return report


def bench_streams(args):
    """Sec 5.1 experiment shape: the GW150914-like injection alone in the 2^20-bin
    A+E band at SNR 20, R noise realisations generated in HBM
    (scs_make_realisations), then Upsilon_N and the likelihood statistics of the
    injected theta against every realisation (scs_evaluate_streams) at
    N in {1, 10, 50, 100} (the Fig. fig:False_alarm_prob segment counts).  The
    streamed reduction reads each realisation's in-support bins once: HBM-bound."""
    import torch
    from scipy import stats as S

    from paper_2408_13170_amd import B

    dev = torch.device("cuda:0")
    w = synth.workload("lisa1m")
    K, df, f_min = w.grid.K, w.grid.df, w.grid.f_min
    snr = 20.0
    psd = synth.psd_arrays(w)
    ctx = B.scs_ctx_create(0)
    B.scs_load_data(ctx, np.zeros((w.n_chan, K, 2)), psd, f_min, df)
    B.scs_set_model(ctx, w.pn_order, B.SCS_RESP_LISA_LF_AE, B.SCS_SUPPORT_TOBS, w.grid.t_obs)
    h = torch.empty((w.n_chan, K, 2), dtype=torch.float64, device=dev)
    B.scs_waveform(ctx, torch.tensor(w.injection, device=dev), h)
    torch.cuda.synchronize()
    hc = torch.complex(h[..., 0], h[..., 1])
    Sd = torch.tensor(psd, device=dev)
    hh = float(4 * df * torch.sum(hc.abs() ** 2 / Sd))
    d = hc * (snr / math.sqrt(hh))
    B.scs_load_data(ctx, torch.stack([d.real, d.imag], -1).contiguous(), Sd.contiguous(), f_min, df)
    B.scs_set_model(ctx, w.pn_order, B.SCS_RESP_LISA_LF_AE, B.SCS_SUPPORT_TOBS, w.grid.t_obs)
    B.scs_define_segmentation(ctx, 1, B.SCS_SEG_EQUAL_SNR, w.G)
    B.scs_evaluate(ctx, torch.tensor(w.injection[None, :], device=dev), torch.empty(1, dtype=torch.float64,
                                                                                      device=dev))
    sup, _ = B.scs_last_bounds(ctx, 1, 1)
    nsup = int(sup[0, 1] - sup[0, 0])
    R = args.realisations
    streams = torch.empty((w.n_chan, K, R, 2), dtype=torch.float64, device=dev)
    st = torch.empty((R, B.SCS_NSTATS), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    B.scs_make_realisations(ctx, streams, synth.BASE_SEED + 51, 0, 1.0)  # warm-up
    torch.cuda.synchronize()
    ev[0].record(stream)
    B.scs_make_realisations(ctx, streams, synth.BASE_SEED + 51, 0, 1.0)
    ev[1].record(stream)
    torch.cuda.synchronize()
    gen_ms = ev[0].elapsed_time(ev[1])
    gen_bytes = streams.numel() * 8
    log(f"realisations: {R} x {w.n_chan} x {K} bins in {gen_ms:.2f} ms ({gen_bytes / gen_ms / 1e6:.0f} GB/s written)")
    levels = []
    read_bytes = R * nsup * w.n_chan * 16
    for N in (1, 10, 50, 100):
        B.scs_define_segmentation(ctx, N, B.SCS_SEG_EQUAL_SNR, w.G)
        B.scs_evaluate_streams(ctx, w.injection, streams, st)  # warm-up, sizes the workspace
        reps = max(1, args.steps // 4)
        t = []
        B.scs_ctx_profile(ctx, 1)
        for _ in range(reps):
            ev[0].record(stream)
            B.scs_evaluate_streams(ctx, w.injection, streams, st)
            ev[1].record(stream)
            torch.cuda.synchronize()
            t.append(ev[0].elapsed_time(ev[1]))
        n_k, k_ms = B.scs_ctx_profile(ctx, 0)
        call_ms = float(np.median(t))
        ms = k_ms / max(n_k, 1)  # the streamed reduction alone (HIP events on its stream)
        u = st[:, 0].cpu().numpy()
        law = S.ncx2(2 * N, snr ** 2)
        p = float(S.kstest(u, law.cdf).pvalue)
        levels.append({"N": N, "kernel_ms": ms, "call_ms": call_ms, "evals_per_s": R * nsup / (call_ms * 1e-3),
                       "stream_GBps": read_bytes / (ms * 1e-3) / 1e9,
                       "upsilon_mean": float(u.mean()), "law_mean": 2 * N + snr ** 2,
                       "upsilon_var": float(u.var()), "law_var": 4 * N + 4 * snr ** 2, "ks_p": p})
        log(f"N={N}: reduction {ms:.3f} ms ({read_bytes / (ms * 1e-3) / 1e9:.0f} GB/s of streams read), call "
            f"{call_ms:.3f} ms, {R} realisations, "
            f"mean {u.mean():.2f} vs {2 * N + snr ** 2}, KS p {p:.3g}")
    B.scs_ctx_destroy(ctx)
    best = max(lv["stream_GBps"] for lv in levels)
    out = {"metric": "realisation x freq-bin evaluations/s of one theta against noise realisations (Sec 5.1)",
           "value": max(lv["evals_per_s"] for lv in levels), "unit": "evals/s", "n_gpus": 1, "steps": len(levels),
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic: GW150914-like injection at SNR 20, Philox/Box-Muller noise in HBM",
           "config": {"workload": f"2^20-bin A+E band, {R} noise realisations ({gen_bytes / 1e9:.1f} GB in HBM), "
                                  f"{nsup} in-support bins, N in (1, 10, 50, 100)"},
           "roofline": {"bound": "hbm", "achieved": best, "peak": 8000.0, "unit": "GB/s", "frac": best / 8000.0,
                        "traffic": measured_traffic(STREAMS_PROFILE) if R == 1024 else None,
                        "kernel": "k_streams (streamed segmented reduction)",
                        "bytes_per_launch": read_bytes},
           "generate_ms": gen_ms, "generate_GBps_written": gen_bytes / gen_ms / 1e6, "levels": levels}
    print(json.dumps(out), flush=True)


# The rungs of the search ladder: (N, Omega, Phi_P, Phi_G, minimum speeds in
# the order Mc, eta, f_low, lambda, beta, iota, psi), Table tab:PSO_hyperparams.
SEARCH_LADDER = [(100, 0.5, 0.2, 0.3, [0.1, 0.05, 5e-8, 0.1, 0.1, 0.2, 0.1]),
                 (50, 0.5, 0.2, 0.4, [0.01, 0.05, 1e-8, 0.01, 0.01, 0.2, 0.1]),
                 (10, 0.3, 0.2, 0.5, [0.001, 0.05, 1e-8, 0.001, 0.001, 0.01, 0.1]),
                 (1, 0.72, 1.193, 1.193, [0.0] * 7)]


def bench_search(args):
    """The hierarchical search of Sec 3.2 as the paper runs it (app:PSO_params):
    6 swarms x 10^4 particles, ladder N = 100, 50, 10, 1 with the rung
    hyper-parameters of tab:PSO_hyperparams, convergence at a gain of at most
    2 over 50 iterations, k-means re-grouping between rungs; on the 2^20-bin
    A+E data of the step benchmark (GW150914-like injection at SNR 17),
    particles uniform in the GW150914-like prior box.  Every iteration steps
    all moving swarms with one batched generate-and-reduce."""
    import torch

    from paper_2408_13170_amd import B

    dev = torch.device("cuda:0")
    w = synth.workload("lisa1m")
    ctx, _ = make_search(B, torch, w, dev)
    B.scs_define_segmentation(ctx, 1, B.SCS_SEG_EQUAL_SNR, w.G)
    u = torch.empty(1, dtype=torch.float64, device=dev)
    B.scs_evaluate(ctx, torch.tensor(w.injection[None, :], device=dev), u)
    torch.cuda.synchronize()
    ups_inj = float(u[0])
    n_swarms, per = 6, 10000
    s = B.scs_search_create(ctx, n_swarms, per, w.prior_lo, w.prior_hi, synth.PERIODIC, G=w.G, conv_tol=2.0,
                            conv_window=50, kmeans_iters=100, seed=synth.BASE_SEED + 61)
    B.scs_ctx_stats(ctx, reset=True)
    rungs = []
    t0 = time.perf_counter()
    for N, om, pp, pg, eps in SEARCH_LADDER:
        rep = B.scs_search_run_rung(s, N, args.max_iters, B.pso_params(om, pp, pg, eps))
        sizes, best = B.scs_search_swarms(s)
        rep["sizes"] = [int(x) for x in sizes]
        rep["swarm_best"] = [float(x) for x in best[:, 7]]
        rungs.append(rep)
        log(f"rung N={N}: {rep['n_swarms']} swarms {rep['sizes']}, {rep['iterations']} iterations, "
            f"{rep['converged']} converged, best {rep['best_val']:.2f}, {rep['seconds']:.2f} s")
    wall = time.perf_counter() - t0
    ev_support, _, _ = B.scs_ctx_stats(ctx, reset=True)
    top = int(np.argmax(best[:, 7]))
    found = best[top, :7]
    B.scs_search_destroy(s)
    B.scs_ctx_destroy(ctx)
    iters = sum(r["iterations"] for r in rungs)
    out = {"metric": "particle x freq-bin statistic evals/s (in-support) over a whole hierarchical search, FP64",
           "value": ev_support / wall, "unit": "evals/s", "n_gpus": 1, "steps": iters, "warmup": 0,
           "ms_per_step": 1e3 * wall / max(iters, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic: same data as the step benchmark",
           "config": {"workload": f"{n_swarms} swarms x {per} particles, ladder N = (100, 50, 10, 1) "
                                  "(tab:PSO_hyperparams), convergence 2 over 50 iterations, cap "
                                  f"{args.max_iters} iterations per rung, 2^20-bin A+E data, GW150914-like "
                                  "injection at SNR 17"},
           "search_seconds": wall, "iterations": iters, "rungs": rungs,
           "best_upsilon_1": float(best[top, 7]), "upsilon_1_at_injection": ups_inj,
           "best_theta": [float(x) for x in found], "injection": [float(x) for x in w.injection]}
    print(json.dumps(out), flush=True)


def cpu_model():
    """The host CPU's model name and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(w, psd, d_ri, seconds, fd=False):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    particles from the same prior box, evaluated in batches on every host
    thread until about `seconds` of wall time, then a few particles on one
    thread."""
    import oracle as O

    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, psd.shape[0])
    m = O.Model(pn_order=w.pn_order, response=O.RESP_LISA_FD if fd else O.RESP_LISA_LF_AE,
                support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    th_all = synth.workload_particles(w, seed=w.seed + 11)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    evals, used, t = 0, 0, 0.0
    batch = max(threads, 8)
    while t < seconds and used + batch <= th_all.shape[0] and used < 512:
        th = th_all[used:used + batch]
        t0 = time.perf_counter()
        out = O.evaluate(g, m, d_ri, psd, th, w.N, O.SEG_EQUAL_SNR, w.G, n_threads=threads)
        t += time.perf_counter() - t0
        evals += int((out["support"][:, 1] - out["support"][:, 0]).sum())
        used += batch
    # one thread: particles one at a time until about a third of the budget
    e1, n1, t1 = 0, 0, 0.0
    while t1 < seconds / 3 and n1 < 64:
        th = th_all[used + n1:used + n1 + 1]
        t0 = time.perf_counter()
        out = O.evaluate(g, m, d_ri, psd, th, w.N, O.SEG_EQUAL_SNR, w.G, n_threads=1)
        t1 += time.perf_counter() - t0
        e1 += int(out["support"][0, 1] - out["support"][0, 0])
        n1 += 1
    # the 16384-bin single-channel configuration in full: 64 particles, one
    # thread, then every thread (data: the configuration's noise; the oracle's
    # cost does not depend on the values)
    w1 = synth.workload("white16k")
    g1 = O.Grid(w1.grid.K, w1.grid.k0, w1.grid.df, 1)
    m1 = O.Model(pn_order=w1.pn_order, response=O.RESP_NONE, support=O.SUPPORT_FULL, t_obs=w1.grid.t_obs)
    psd1 = synth.psd_arrays(w1)
    n1c = synth.noise(psd1, w1.grid.df, w1.seed)
    d1 = np.ascontiguousarray(np.stack([n1c.real, n1c.imag], -1))
    th1 = synth.workload_particles(w1)
    cfg1 = {}
    for nt, name in ((1, "single_core"), (threads, "all_cores")):
        t0 = time.perf_counter()
        O.evaluate(g1, m1, d1, psd1, th1, w1.N, O.SEG_EQUAL_SNR, w1.G, n_threads=nt)
        dt = time.perf_counter() - t0
        cfg1[name] = {"value": th1.shape[0] * w1.grid.K / dt, "unit": "evals/s", "threads": nt, "seconds": dt}
    model, ncpu = cpu_model()
    return {"value": evals / t, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{used} particles of the same workload (full 2^20-bin grid, N_seg 1024), {t:.1f} s "
                      f"on {threads} threads; {n1} more particles on one thread, {t1:.1f} s",
            "single_core": {"value": e1 / t1, "unit": "evals/s", "particles": n1, "seconds": t1},
            "cpu_model": model, "logical_cpus": ncpu,
            "config1": dict(cfg1, workload="16384 bins, one channel, unit white PSD, 2PN, N_seg 16, 64 particles "
                                           "(the whole configuration)")}


if __name__ == "__main__":
    main()
