"""Benchmark: exact binary64 sum throughput on one MI355X.

One step = one exact sum (one fused kernel launch: load, split, carry-free
add, block and grid merge, carry normalisation, rounding) of the default
workload, n = 2^31 doubles (17.2 GB): N(0,1) * 2^k with k uniform in
[-500, 500], one entry in 1000 a subnormal or +-DBL_MAX (signs of the
DBL_MAX entries balanced), resident in HBM before timing starts.

Prints one JSON line.  Besides the required fields it reports the roofline of
the accumulation kernel (HBM-bound), the same bytes read by a plain streaming
read with the kernel's access pattern (the measured ceiling), the sum from
cold caches, torch.sum on the same tensor (time and its error against the
exact result), and the CPU oracle timed on the host (all cores, and one core
on a bounded sample).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Other workloads (reported separately, not the headline line):
    python bench.py --workload single      2^28 binary64 cancelling pairs +
                                           1% perturbations (2 GiB)
    python bench.py --workload single --dtype f32
                                           the same 2 GiB as 2^29 binary32
    python bench.py --workload single --dtype bf16
                                           2 GiB as 2^30 bfloat16 (mixed signs)
    python bench.py --workload config1     10^6 binary64 (cache-resident)
    python bench.py --workload segmented   10^6 lognormal segments, mixed
                                           formats, one graph-captured launch
    python bench.py --workload serving     Poisson 2000 req/s for 60 s,
                                           continuous batching; p50/p99
"""

import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1605_05436_amd/csrc/xsum_kernels.hip",
                  "paper_1605_05436_amd/csrc/xsum_device.h",
                  "paper_1605_05436_amd/csrc/xsum_internal.h"]
TRAFFIC_PROFILE = "profiles/accumulate_f64_n2e28_hbm_counters.md"
TRAFFIC_PROFILES = {"f64": TRAFFIC_PROFILE,
                    "f32": "profiles/accumulate_f32_n2e29_hbm_counters.md",
                    "bf16": "profiles/accumulate_bf16_n2e30_hbm_counters.md"}
SEG_KERNEL_SOURCES = ["paper_1605_05436_amd/csrc/xsum_segmented.hip",
                      "paper_1605_05436_amd/csrc/xsum_segmented.h",
                      "paper_1605_05436_amd/csrc/xsum_plan.hip",
                      "paper_1605_05436_amd/csrc/xsum_device.h"]
SEG_TRAFFIC_PROFILE = "profiles/segmented_c4_1e6seg_hbm_counters.md"
TRUNC_KERNEL_SOURCES = ["paper_1605_05436_amd/csrc/xsum_truncated.hip",
                        "paper_1605_05436_amd/csrc/xsum_device.h"]
TRUNC_TRAFFIC_PROFILES = {"config3": "profiles/truncated_f64_n2e31_hbm_counters.md",
                          "config2": "profiles/truncated_f64_n2e28_hbm_counters.md"}


def measured_traffic(n, sources=KERNEL_SOURCES, profile=TRAFFIC_PROFILE, match=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source, this workload size n and (when
    given) the same plan settings; otherwise None."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in sources:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        text = open(os.path.join(ROOT, profile)).read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic-record:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_source_sha256") == h.hexdigest()[:16] and rec.get("n") == n \
                    and all(rec.get(k) == v for k, v in (match or {}).items()):
                return int(rec["traffic_bytes"])
    return None


def cpu_baseline_full(bits, fmt, terms=None, budget_s=3.0):
    """The cpu_baseline leg for one large sum: the oracle's binned sum over
    the whole input, repeated for about budget_s seconds (at least once), then
    rounded.  With terms, also checks the workload's closed form (the exact
    total equals the sum of terms).  Also gives log10 of the condition number
    sum|x| / |sum x| from one more exact sum over the magnitudes (None for an
    exact zero).  Returns ((bits, flags), closed form holds, threads, median
    seconds per run, runs, log10 condition number); the bench compares the
    GPU's bits with this result."""
    import math
    import oracle
    times = []
    acc = threads = None
    t_start = time.time()
    while not times or (time.time() - t_start < budget_s and len(times) < 50):
        t0 = time.time()
        acc, threads = oracle.exact_sum_binned(bits, fmt)
        times.append(time.time() - t0)
    times.sort()
    want = tuple(oracle.finish(acc, "f32" if fmt == "bf16" else fmt))
    closed = terms is None or oracle.exact_sum_binned(terms, fmt)[0].total == acc.total
    sign_bit = {"f64": np.uint64(1 << 63), "f32": np.uint32(1 << 31),
                "bf16": np.uint16(1 << 15)}[fmt]
    mag = oracle.exact_sum_binned(bits & ~sign_bit, fmt)[0].total
    cond = None if acc.total == 0 else round(math.log10(mag) - math.log10(abs(acc.total)), 2)
    return want, closed, threads, times[len(times) // 2], len(times), cond


def cpu_single_thread_refs(bits, want_bits, n_int, n_fsum):
    """Single-threaded CPU references on leading samples of a binary64
    input: the oracle's plain Python-int sum (n_int elements) and math.fsum
    (n_fsum elements, a correctly rounded library sum that the oracle's
    rounding must equal).  Returns a dict of rates; when the samples are the
    whole input, also whether fsum's result equals the oracle's bits."""
    import math
    import oracle
    m = min(len(bits), n_int)
    t0 = time.time()
    got_int = tuple(oracle.oracle_sum(bits[:m], "f64"))
    t_int = time.time() - t0
    f = min(len(bits), n_fsum)
    vals = bits[:f].view(np.float64).tolist()
    t0 = time.time()
    fs = math.fsum(vals)
    t_fs = time.time() - t0
    fs_bits = struct.unpack("<Q", struct.pack("<d", fs))[0]
    out = {"python_int": {"gelem_s": round(m / t_int / 1e9, 5), "elements": m,
                          "seconds": round(t_int, 3)},
           "math_fsum": {"gelem_s": round(f / t_fs / 1e9, 5), "elements": f,
                         "seconds": round(t_fs, 3)}}
    if m == len(bits):
        out["python_int"]["same_bits_as_binned"] = got_int[0] == want_bits
    if f == len(bits):
        out["math_fsum"]["same_bits_as_oracle"] = fs_bits == want_bits
    return out


def cpu_baseline_sample(pieces, threads=16):
    """The cpu_baseline leg for many sums: the oracle on a bounded sample of
    (bit-pattern array, format) pieces, timed.  Returns (results, elements,
    seconds, threads); the bench also checks the GPU's bits against them."""
    import oracle
    t0 = time.time()
    results = [tuple(oracle.oracle_sum_binned(b, fmt, threads=threads)) for b, fmt in pieces]
    secs = time.time() - t0
    return results, sum(len(b) for b, _ in pieces), secs, threads


def ulps_between(a, b, fmt="f64"):
    """Distance between a and b in units in the last place of b, where b is a
    binary64 (fmt "f64") or binary32 (fmt "f32") value."""
    if a == b:
        return 0.0
    if b == 0 or not math.isfinite(a) or not math.isfinite(b):
        return float("inf")
    if fmt == "f64":
        return abs(a - b) / math.ulp(b)
    e = max(math.frexp(b)[1] - 1, -126)          # binary32 exponent of b
    return abs(a - b) / math.ldexp(1.0, e - 23)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--log2n", type=int, default=28,
                    help="size of the 'single' workload (2^log2n binary64)")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16"],
                    help="input format of the 'single' workload (2 GiB each: "
                         "2^28 binary64, 2^29 binary32, 2^30 bfloat16)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-torch-sum", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the read-probe and cold-cache legs")
    ap.add_argument("--workload", default="config3",
                    choices=["config3", "single", "config1", "segmented", "serving",
                             "truncated"])
    ap.add_argument("--trunc-input", default="config3", choices=["config3", "config2"],
                    help="input of the 'truncated' workload: the 2^31 binary64 "
                         "headline input, or the 2^28 cancelling-pairs input")
    ap.add_argument("--nseg", type=int, default=1_000_000)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="segmented workload: use the library's default tuning")
    ap.add_argument("--clock-trace", type=int, default=0, metavar="LAUNCHES",
                    help="single workloads: after an idle pause, time LAUNCHES "
                         "back-to-back launches one by one while a one-wave "
                         "kernel on a second stream samples the shader clock")
    ap.add_argument("--seg-lanes", type=int, default=0, choices=[0, 1, 2, 4, 8, 16],
                    help="segmented workload: give every lane-group segment "
                         "this many lanes (no autotuning); 0 = tuned")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run one device copy of the input "
                         "(a plain copy kernel of known size, for scaling "
                         "profiler byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the exact sum runs on a single "
              "MI355X here; multi-GPU sharding is a design note, not measured "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "segmented":
        return bench_segmented(args)
    if args.workload == "config1":
        return bench_config1(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "truncated":
        return bench_truncated(args)
    return bench_single(args)


def timed_launches(step, stream, warmup, steps):
    """W untimed launches, then K launches bracketed by HIP events on the
    launch stream (synchronised on both sides).  Returns ms per launch."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def cold_median_ms(step, stream, flush_buf, reps=20):
    """Median of reps single launches, each after a 1 GiB buffer fill that
    evicts the input from the caches; only the launch is timed."""
    import torch
    import paper_1605_05436_amd as xs
    sh = xs.stream_handle(stream)
    times = []
    for i in range(reps):
        xs.xsum_probe_flush(flush_buf.data_ptr(), flush_buf.numel(), i, sh)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def clock_trace(step, stream, launches, est_ms, idle_s=3.0, interval_ticks=5000):
    """Per-launch times of `launches` back-to-back launches from an idle GPU,
    with the shader clock sampled every interval_ticks of the 100 MHz
    counter (50 us by default) by xsum_probe_clock on a second stream.
    Returns launch-time means over ranges of launches, the clock per 5 ms of
    the run, and the clock before the first launch."""
    import torch
    import paper_1605_05436_amd as xs
    torch.cuda.synchronize()
    time.sleep(idle_s)
    sh = xs.stream_handle(stream)
    side = torch.cuda.Stream()
    # sample from 5 ms before the first launch until well past the last
    # (est_ms: the launch time measured before; at most 10 s)
    span_us = 5000.0 + 2.0 * launches * est_ms * 1e3 + 50_000.0
    nsamp = int(min(200_000, span_us * 100.0 / interval_ticks))
    samples = torch.zeros(2 * nsamp, dtype=torch.int64, device="cuda")
    marks = torch.zeros(4, dtype=torch.int64, device="cuda")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
    xs.xsum_probe_clock(samples.data_ptr(), nsamp, interval_ticks, xs.stream_handle(side))
    time.sleep(0.005)           # a few idle samples first
    xs.xsum_probe_clock(marks.data_ptr(), 1, 1, sh)
    for i in range(launches):
        evs[i].record(stream)
        step()
    evs[launches].record(stream)
    xs.xsum_probe_clock(marks[2:].data_ptr(), 1, 1, sh)
    torch.cuda.synchronize()
    d = np.array([evs[i].elapsed_time(evs[i + 1]) * 1e3 for i in range(launches)])
    s = samples.cpu().numpy().reshape(-1, 2).astype(np.float64)
    m = marks.cpu().numpy().astype(np.float64)
    rt, ck = s[:, 0], s[:, 1]
    mhz = np.diff(ck) / np.diff(rt) * 100.0
    t_us = (rt[1:] - m[0]) / 100.0                 # since the first launch
    end_us = (m[2] - m[0]) / 100.0
    ranges = {}
    for a, b in ((0, 5), (5, 25), (25, 50), (50, 100), (100, 200), (200, 400),
                 (400, launches)):
        if a < min(b, launches):
            seg = d[a:b]
            ranges["%d-%d" % (a + 1, min(b, launches))] = [
                round(float(seg.mean()), 1), round(float(seg.min()), 1),
                round(float(seg.max()), 1)]
    buckets = []
    for b0 in np.arange(0.0, end_us, 5000.0):
        sel = (t_us >= b0) & (t_us < b0 + 5000.0)
        if sel.any():
            buckets.append([round(b0 / 1e3, 1), round(float(mhz[sel].mean())),
                            round(float(mhz[sel].min()))])
    before = mhz[t_us < 0]
    out = {"launches": launches, "span_ms": round(end_us / 1e3, 2),
           "launch_us_mean_min_max": ranges,
           "clock_mhz_per_5ms": buckets,
           "clock_mhz_before": round(float(before.mean())) if len(before) else None,
           "first_launches_us": [round(float(v), 1) for v in d[:30]]}
    log("clock trace: %d launches over %.1f ms, clock before %s MHz"
        % (launches, end_us / 1e3, out["clock_mhz_before"]))
    for k, v in ranges.items():
        log("  launches %-9s mean %.1f us (min %.1f, max %.1f)" % (k, *v))
    for t0, c, cmin in buckets:
        log("  t %6.1f ms: clock %d MHz (min %d)" % (t0, c, cmin))
    return out


def bench_single(args):
    """One exact sum per step over an input resident in HBM.

    config3 (default): 2^31 binary64 N(0,1) * 2^k, k uniform in [-500, 500],
    one subnormal or +-DBL_MAX (signs balanced) per 1000 elements: 17.2 GB.
    single: the cancelling-pairs workload of 2 GiB (2^28 binary64, or the
    same bytes as binary32 / bfloat16 with --dtype)."""
    import torch
    import paper_1605_05436_amd as xs
    import workloads

    fmt = "f64" if args.workload == "config3" else args.dtype
    code = {"f64": xs.F64, "f32": xs.F32, "bf16": xs.BF16}[fmt]
    esize = {"f64": 8, "f32": 4, "bf16": 2}[fmt]
    t0 = time.time()
    terms = None
    if args.workload == "config3":
        n = 1 << 31
        log("generating config: n=2^31 binary64 N(0,1)*2^k with specials")
        bits = workloads.config3(n=n, seed=args.seed)
        workload = ("single exact sum, n=2^31 binary64 N(0,1)*2^k, k in [-500,500], "
                    "0.1% subnormal/+-DBL_MAX (balanced)")
        traffic_profile = "profiles/accumulate_f64_n2e31_hbm_counters.md"
    else:
        n = (1 << args.log2n) * 8 // esize      # the same bytes in every format
        traffic_profile = TRAFFIC_PROFILES[fmt]
        if fmt == "f64":
            log("generating config: n=2^%d binary64 cancelling pairs + perturbations"
                % args.log2n)
            bits, terms = workloads.config2(log2n=args.log2n, seed=args.seed)
            workload = ("single exact sum, n=2^%d binary64, cancelling pairs + 1%% "
                        "perturbations, seeded shuffle" % args.log2n)
        elif fmt == "f32":
            log("generating %d binary32 cancelling pairs + perturbations" % n)
            bits = workloads.serving_payload(n, "f32", seed=args.seed)
            workload = ("single exact sum, n=2^%d binary32, cancelling pairs + 1%% "
                        "perturbations, seeded shuffle" % (args.log2n + 1))
        else:
            log("generating %d bfloat16 values, mixed signs, exponents in [-50, 50]" % n)
            piece = min(n, 1 << 26)     # generated in pieces to bound host memory
            bits = np.concatenate([workloads.family("mixed", piece, 100,
                                                    seed=args.seed * 4096 + i, fmt="bf16")
                                   for i in range(n // piece)])
            workload = ("single exact sum, n=2^%d bfloat16, mixed signs, exponents in "
                        "[-50, 50]" % (args.log2n + 2))
    log("generated in %.1f s" % (time.time() - t0))

    signed = {8: np.int64, 4: np.int32, 2: np.int16}[esize]
    x = torch.from_numpy(bits.view(signed)).to("cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    scratch = xs.new_states(1)
    stream = torch.cuda.current_stream()
    sh = xs.stream_handle(stream)
    torch.cuda.synchronize()

    def step():
        xs.xsum_exact_sum_async(x.data_ptr(), n, code, xs.SAME, out.data_ptr(),
                                flags.data_ptr(), scratch.data_ptr(), sh)

    ms_per_step = timed_launches(step, stream, args.warmup, args.steps)
    gelem_s = n / (ms_per_step * 1e-3) / 1e9
    out_fmt = "f64" if fmt == "f64" else "f32"
    result_bits = int(out.cpu().numpy().view(np.uint64)[0]) & \
        ((1 << (8 * (8 if out_fmt == "f64" else 4))) - 1)
    result_flags = int(flags.cpu()[0])
    log("exact sum: %.3f ms/step, %.1f Gelem/s" % (ms_per_step, gelem_s))

    alg_bytes = n * esize
    probe = None
    if not args.no_probe:
        # the plain read of the same bytes with the binary64 kernel's access
        # pattern, timed the same way (the practical ceiling), and the exact
        # sum once more from cold caches, median of 20
        sink = torch.zeros(4, dtype=torch.int32, device="cuda")
        probe_ms = timed_launches(
            lambda: xs.xsum_probe_read(x.data_ptr(), alg_bytes, sink.data_ptr(), sh),
            stream, args.warmup, args.steps)
        flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        cold_ms = cold_median_ms(step, stream, flush)
        del flush
        probe = {"read_probe_ms": round(probe_ms, 4),
                 "read_probe_gb_s": round(alg_bytes / (probe_ms * 1e-3) / 1e9, 1),
                 "frac_of_read_probe": round(probe_ms / ms_per_step, 4),
                 "cold_median_ms": round(cold_ms, 4),
                 "cold_gelem_s": round(n / (cold_ms * 1e-3) / 1e9, 2)}
        log("read probe: %.3f ms (%.1f GB/s); cold median %.3f ms"
            % (probe_ms, probe["read_probe_gb_s"], cold_ms))

    # parity of the timed result against the oracle (config 2: also the
    # closed form, the sum of the replaced pairs equals the sum of everything)
    (want_bits, want_flags), closed, threads, cpu_s, cpu_runs, log10_cond = \
        cpu_baseline_full(bits, fmt, terms)
    bit_exact = (result_bits, result_flags) == (want_bits, want_flags) and closed
    if out_fmt == "f64":
        exact_val = struct.unpack("<d", struct.pack("<Q", want_bits))[0]
    else:
        exact_val = float(struct.unpack("<f", struct.pack("<I", want_bits))[0])
    log("oracle: %.3f s per run (median of %d) on %d threads, bit_exact=%s"
        % (cpu_s, cpu_runs, threads, bit_exact))
    trace = (clock_trace(step, stream, args.clock_trace, ms_per_step)
             if args.clock_trace else None)
    if trace is not None:
        # the traced launches wrote the same result
        trace["same_result"] = (int(out.cpu().numpy().view(np.uint64)[0]) &
                                ((1 << (8 * (8 if out_fmt == "f64" else 4))) - 1),
                                int(flags.cpu()[0])) == (result_bits, result_flags)

    achieved = alg_bytes / (ms_per_step * 1e-3) / 1e9
    metric = ("exact FP64 sum Gelem/s + % HBM roofline vs torch.sum on same GPU (bit-exact)"
              if fmt == "f64" else
              "exact %s sum Gelem/s + %% roofline vs torch.sum on same GPU (bit-exact)"
              % {"f32": "binary32", "bf16": "bfloat16"}[fmt])
    rec = {
        "metric": metric,
        "value": round(gelem_s, 2),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n": n, "input_dtype": fmt, "out_dtype": out_fmt,
                   "seed": args.seed},
        "bit_exact": bit_exact,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(n, profile=traffic_profile)},
    }
    if probe:
        rec["measured_peak"] = probe
    if trace is not None:
        rec["clock_trace"] = trace

    if not args.no_torch_sum:
        xf = x.view({"f64": torch.float64, "f32": torch.float32,
                     "bf16": torch.bfloat16}[fmt])
        sum_dtype = torch.float32 if fmt == "bf16" else None
        res = []
        tms = timed_launches(lambda: res.append(torch.sum(xf, dtype=sum_dtype)),
                             stream, args.warmup, args.steps)
        tval = float(res[-1].cpu())
        del res
        rec["torch_sum"] = {"ms_per_step": round(tms, 4),
                            "gelem_s": round(n / (tms * 1e-3) / 1e9, 2),
                            "value": tval, "exact_rounded": exact_val,
                            "error_ulps": ulps_between(tval, exact_val, out_fmt),
                            "log10_condition_number": log10_cond,
                            "rel_error": (abs(tval - exact_val) / abs(exact_val)
                                          if exact_val and math.isfinite(tval) else None)}

    if args.copy_calibration:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = {"read": n * esize, "write": n * esize}
        del y

    if not args.no_cpu_baseline:
        # the same oracle on one host core, over a bounded leading sample
        import oracle
        m1 = min(n, 1 << 26)
        t1 = time.time()
        oracle.exact_sum_binned(bits[:m1], fmt, threads=1)
        one_s = time.time() - t1
        rec["cpu_baseline"] = {"value": round(n / cpu_s / 1e9, 4),
                               "unit": "Gelem/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the full n=%d input, median of %d runs "
                                         "(exponent-binned 128-bit C accumulation + "
                                         "big-int fold + RNE rounding)" % (n, cpu_runs),
                               "value_1core": round(m1 / one_s / 1e9, 4),
                               "sample_1core": "the first %d elements on 1 thread, "
                                               "accumulation only" % m1}
        if args.workload == "single" and fmt == "f64":
            # the oracle's plain Python-int sum and math.fsum, single-threaded,
            # on leading samples (the whole input would take minutes)
            rec["cpu_baseline"]["single_thread"] = cpu_single_thread_refs(
                bits, want_bits, 1 << 20, 1 << 24)
    print(json.dumps(rec), flush=True)


def bench_truncated(args):
    """Section 4's condition-number-sensitive iteration on one large input
    resident in HBM: each pass (r = 2, 4, 16) timed on its own with HIP events,
    then the whole blocking iteration (passes until one certifies, else the
    exact kernel), whose result is checked against the oracle."""
    import torch
    import paper_1605_05436_amd as xs
    import workloads
    import oracle

    t0 = time.time()
    terms = None
    if args.trunc_input == "config3":
        n = 1 << 31
        bits = workloads.config3(n=n, seed=args.seed)
        workload = ("Section 4 iteration, n=2^31 binary64 N(0,1)*2^k, k in [-500,500], "
                    "0.1% subnormal/+-DBL_MAX (balanced)")
    else:
        n = 1 << 28
        bits, terms = workloads.config2(log2n=28, seed=args.seed)
        workload = ("Section 4 iteration, n=2^28 binary64, cancelling pairs + 1% "
                    "perturbations, seeded shuffle")
    log("generated %d elements in %.1f s" % (n, time.time() - t0))
    x = torch.from_numpy(bits.view(np.int64)).to("cuda")
    wsb = xs.xsum_truncated_workspace_size()
    ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
    rec = torch.zeros(256, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sh = xs.stream_handle(stream)
    torch.cuda.synchronize()
    passes = {}
    for r in (2, 4, 16):
        ms = timed_launches(lambda: xs.xsum_truncated_round(
            x.data_ptr(), n, xs.F64, xs.F64, r, rec.data_ptr(), ws.data_ptr(), wsb, sh),
            stream, max(1, args.warmup // 4), max(1, args.steps // 4))
        root = xs.read_trunc_root(rec)
        passes[r] = {"ms": round(ms, 4), "gb_s": round(n * 8 / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(n * 8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "certified": bool(root.certified), "root_entries": int(root.count),
                     "bound_log2": (None if root.bound_value == 0 else
                                    32 * root.bound_index - 1074 +
                                    root.bound_value.bit_length() - 1)}
        log("pass r=%d: %.3f ms, certified=%s" % (r, ms, passes[r]["certified"]))
    # the blocking iteration, end to end (host reads each pass's record)
    times, res = [], None
    for i in range(max(3, args.steps // 8)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = xs.xsum_exact_sum_truncated(x.data_ptr(), n, xs.F64, xs.F64, ws.data_ptr(),
                                          wsb, sh)
        times.append((time.perf_counter() - t1) * 1e3)
    times.sort()
    ms = times[len(times) // 2]
    state = xs.new_states(1)
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    exact_ms = timed_launches(lambda: xs.xsum_exact_sum_async(
        x.data_ptr(), n, xs.F64, xs.F64, out.data_ptr(), out.data_ptr() + 8,
        state.data_ptr(), sh), stream, max(1, args.warmup // 4), max(1, args.steps // 4))
    log("iteration: %.3f ms (median of %d), r=%d; exact kernel %.3f ms" % (ms, len(times), res[2], exact_ms))
    (want_bits, want_flags), closed, threads, cpu_s, cpu_runs, log10_cond = \
        cpu_baseline_full(bits, "f64", terms)
    bit_exact = (res[0], res[1]) == (want_bits, want_flags) and closed
    # the oracle's own Section 4 iteration (pure Python) on a bounded prefix
    sample = 1 << 14
    t1 = time.time()
    o_res, o_passes, o_r = oracle.adaptive_sum(bits[:sample], "f64")
    o_s = time.time() - t1
    o_ok = tuple(o_res) == tuple(oracle.oracle_sum(bits[:sample], "f64"))
    dominant = max(passes, key=lambda k: passes[k]["ms"] if (k <= (res[2] or 16)) else 0)
    dp = passes[dominant]
    if args.copy_calibration:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del y
    rec_out = {
        "metric": "exact FP64 sum Gelem/s, Section 4 condition-number-sensitive iteration (bit-exact)",
        "value": round(n / (ms * 1e-3) / 1e9, 2), "unit": "Gelem/s", "n_gpus": 1,
        "steps": len(times), "warmup": 1, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": workload, "n": n, "bytes": n * 8, "seed": args.seed},
        "bit_exact": bool(bit_exact), "certified_r": res[2],
        "passes": {str(k): v for k, v in passes.items()},
        "exact_kernel_ms": round(exact_ms, 4), "log10_condition_number": log10_cond,
        "copy_calibration_bytes": ({"read": n * 8, "write": n * 8}
                                   if args.copy_calibration else None),
        "cpu_baseline": {"value": round(sample / o_s / 1e9, 6), "unit": "Gelem/s", "cores": 1,
                         "kind": "oracle",
                         "sample": "first %d elements through the oracle's Section 4 "
                                   "iteration (pure Python, balanced tree): %d passes, "
                                   "r=%d, result equals the exact oracle: %s" % (
                                       sample, o_passes, o_r, o_ok),
                         "full_input_exact_oracle_s": round(cpu_s, 3),
                         "full_input_exact_oracle_threads": threads},
        "roofline": {"bound": "hbm", "achieved": dp["gb_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dp["frac_hbm"],
                     "traffic": measured_traffic(n, TRUNC_KERNEL_SOURCES,
                                                 TRUNC_TRAFFIC_PROFILES[args.trunc_input],
                                                 {"r": dominant}),
                     "kernel": "truncated_kernel r=%d" % dominant},
    }
    print(json.dumps(rec_out), flush=True)


def bench_config1(args):
    """10^6 binary64 values, exponents in [-50, 50] (8 MB): small enough to
    stay in the 256 MB last-level cache, so a sum is bound by launch and
    finish latency.  Warm: one captured graph of 100 back-to-back sums,
    replayed.  Cold: a 1 GiB buffer is rewritten before each single sum, and
    only the sum is timed."""
    import torch
    import paper_1605_05436_amd as xs
    import workloads

    n = 1_000_000
    bits = workloads.config1(n, seed=args.seed)
    x = torch.from_numpy(bits.view(np.int64)).to("cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    scratch = xs.new_states(1)
    s = torch.cuda.Stream()
    sh = xs.stream_handle(s)

    def one():
        xs.xsum_exact_sum_async(x.data_ptr(), n, xs.F64, xs.F64, out.data_ptr(),
                                flags.data_ptr(), scratch.data_ptr(), sh)

    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(10):
            one()
    torch.cuda.synchronize()
    per_graph = 100
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(per_graph):
            one()
    replays = max(1, args.steps // 10)
    with torch.cuda.stream(s):
        for _ in range(max(1, args.warmup // 10)):
            g.replay()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(replays):
            g.replay()
        ev1.record(s)
    torch.cuda.synchronize()
    warm_us = ev0.elapsed_time(ev1) * 1e3 / (replays * per_graph)
    got_warm = (int(out.cpu().numpy().view(np.uint64)[0]), int(flags.cpu()[0]))
    # cold: evict the input from the caches before every timed sum
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    cold = []
    with torch.cuda.stream(s):
        for i in range(30):
            flush.fill_(i & 0xff)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            one()
            e1.record(s)
            e1.synchronize()
            cold.append(e0.elapsed_time(e1) * 1e3)
    cold.sort()
    cold_us = cold[len(cold) // 2]
    got = (int(out.cpu().numpy().view(np.uint64)[0]), int(flags.cpu()[0]))
    want, _, threads, cpu_s, cpu_runs, log10_cond = cpu_baseline_full(bits, "f64")
    rec = {"metric": "exact FP64 sum Gelem/s (bit-exact), 10^6 elements, graph-replayed",
           "value": round(n / (warm_us * 1e-6) / 1e9, 2), "unit": "Gelem/s", "n_gpus": 1,
           "steps": replays * per_graph, "warmup": max(1, args.warmup // 10) * per_graph,
           "ms_per_step": round(warm_us * 1e-3, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "single exact sum, n=10^6 binary64, exponents in [-50, 50]",
                      "n": n, "seed": args.seed},
           "bit_exact": got == want and got_warm == want,
           "warm_us_per_sum": round(warm_us, 2), "cold_us_per_sum": round(cold_us, 2),
           "cold_gelem_s": round(n / (cold_us * 1e-6) / 1e9, 2),
           "roofline": {"bound": "latency", "achieved": round(n * 8 / (warm_us * 1e-6) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(n * 8 / (warm_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": None},
           "cpu_baseline": {"value": round(n / cpu_s / 1e9, 4), "unit": "Gelem/s",
                            "cores": threads, "kind": "oracle",
                            "sample": "the full 10^6 input, median of %d runs" % cpu_runs}}
    if not args.no_cpu_baseline:
        # single-threaded references over the whole input
        rec["cpu_baseline"]["single_thread"] = cpu_single_thread_refs(bits, want[0], n, n)
    print(json.dumps(rec), flush=True)


def bench_segmented(args):
    """10^6 segments, lognormal lengths (median 256, sigma 2, clipped to
    [1, 2^20]), 50% binary64 / 37.5% binary32 / 12.5% bfloat16, replayed
    from one captured graph of one persistent launch."""
    import torch
    import paper_1605_05436_amd as xs
    import workloads

    t0 = time.time()
    buf, desc = workloads.config4(nseg=args.nseg, seed=args.seed)
    log("generated %d segments, %.2f GB in %.1f s" % (len(desc), buf.nbytes / 1e9,
                                                       time.time() - t0))
    nel = int(desc["length"].sum())
    nbytes = int((desc["length"] * np.array([8, 4, 2])[desc["dtype"]]).sum())
    dbuf = torch.from_numpy(buf).to("cuda")
    # the autotuner times candidate plans (all must agree bit for bit) and
    # picks the fastest for this batch: global knobs, then lanes per segment
    # and vectors in flight per format and size bucket
    from paper_1605_05436_amd import autotune
    t0 = time.time()
    if args.seg_lanes:
        # every lane-group segment gets the same number of lanes
        g = args.seg_lanes
        best = autotune._full(autotune.DEFAULT_CANDIDATES[0])[:7] + \
            (tuple(tuple(g for _ in range(autotune.NB)) for _ in range(3)),
             autotune.EMPTY_TABLE)
        table = []
    elif args.no_autotune:
        best, table = autotune._full(autotune.DEFAULT_CANDIDATES[0]), []
    else:
        best, table = autotune.tune_segmented(desc, dbuf, use_cache=False)
    tune_s = time.time() - t0
    log("autotune done in %.1f s" % tune_s)
    t0 = time.time()
    ss = xs.SegmentedSum(desc, tuning=autotune.tuning_struct(best))
    plan_s = time.time() - t0
    out = torch.zeros(len(desc), dtype=torch.int64, device="cuda")
    fl = torch.zeros(len(desc), dtype=torch.int32, device="cuda")
    graph = ss.capture(dbuf, out, fl)
    stream = torch.cuda.current_stream()
    sh = xs.stream_handle(stream)
    steps = max(1, args.steps // 2)
    ms = timed_launches(lambda: xs.xsum_graph_launch(graph, sh), stream, args.warmup, steps)
    res = out.cpu().numpy().view(np.uint64)
    rf = fl.cpu().numpy().view(np.uint32)
    # the binary64 segments alone, same buffer and tuning, also one graph
    f64_desc = desc[desc["dtype"] == 0]
    f64_bytes = int(f64_desc["length"].sum()) * 8
    ss64 = xs.SegmentedSum(f64_desc, tuning=autotune.tuning_struct(best))
    out64 = torch.zeros(len(f64_desc), dtype=torch.int64, device="cuda")
    fl64 = torch.zeros(len(f64_desc), dtype=torch.int32, device="cuda")
    g64 = ss64.capture(dbuf, out64, fl64)
    ms64 = timed_launches(lambda: xs.xsum_graph_launch(g64, sh), stream, args.warmup, steps)
    same64 = np.array_equal(out64.cpu().numpy().view(np.uint64),
                            res[desc["dtype"] == 0])
    xs.xsum_graph_destroy(g64)
    ss64.close()
    # parity of every segment: the oracle's per-segment sums over the whole
    # buffer (exponent bins and a wide-integer fold in C, rounding in Python),
    # which is also the timed cpu_baseline leg
    import oracle
    t0 = time.time()
    wants = oracle.segmented_oracle_sums(buf, desc["byte_offset"], desc["length"],
                                         desc["dtype"])
    cpu_s = time.time() - t0
    cpu_threads = oracle.binned.default_threads()
    wb = np.array([w[0] for w in wants], dtype=np.uint64)
    wf = np.array([w[1] for w in wants], dtype=np.uint32)
    bad = np.nonzero((wb != res) | (wf != rf))[0]
    ok = bad.size == 0
    log("oracle over all %d segments: %.1f s, mismatches %d" % (len(desc), cpu_s, bad.size))
    xs.xsum_graph_destroy(graph)
    info = ss.info
    ss.close()
    copy_note = None
    if args.copy_calibration:
        y = torch.empty_like(dbuf)
        y.copy_(dbuf)
        torch.cuda.synchronize()
        copy_note = {"read": int(dbuf.numel()), "write": int(dbuf.numel())}
        del y
    achieved = nbytes / (ms * 1e-3) / 1e9
    rec = {"metric": "segmented exact sums Gelem/s + % HBM roofline (bit-exact)",
           "value": round(nel / (ms * 1e-3) / 1e9, 2), "unit": "Gelem/s",
           "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "1e6 segments, lognormal lengths (median 256, sigma 2, "
                                  "clip [1, 2^20]), f64/f32/bf16 50/37.5/12.5, one graph launch",
                      "segments": len(desc), "elements": nel, "bytes": nbytes,
                      "seed": args.seed,
                      "lanes_per_segment": args.seg_lanes or "planner/autotuner"},
           "bit_exact": ok, "checked_segments": int(len(desc)),
           "cpu_baseline": {"value": round(nel / cpu_s / 1e9, 4), "unit": "Gelem/s",
                            "cores": cpu_threads, "kind": "oracle",
                            "sample": "all %d segments (%d elements): exponent-binned C "
                                      "sums with a wide-integer fold, then big-int RNE "
                                      "rounding per segment" % (len(desc), nel)},
           "plan_seconds": round(plan_s, 3), "autotune_seconds": round(tune_s, 1),
           "autotune": {"chosen": autotune._as_list(best),
                        "candidates_ms": [round(m, 4) for _, m in table]},
           "f64_segments": {"segments": int(len(f64_desc)), "bytes": f64_bytes,
                            "ms_per_step": round(ms64, 4),
                            "gb_s": round(f64_bytes / (ms64 * 1e-3) / 1e9, 1),
                            "frac": round(f64_bytes / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "same_bits_as_mixed_run": bool(same64)},
           "plan": {k: info[k] for k in
                                                       ("lane_segments", "wave_segments",
                                                        "chunked_segments", "work_items")},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(
                            nel, SEG_KERNEL_SOURCES, SEG_TRAFFIC_PROFILE,
                            {"tuning": autotune._as_list(best)})}}
    if copy_note:
        rec["copy_calibration_bytes"] = copy_note
    print(json.dumps(rec), flush=True)


def bench_serving(args):
    """Poisson arrivals at --rate req/s for --duration s; sizes log-uniform in
    [1e3, 1e8]; binary64 or binary32 with equal probability; values shaped like
    the cancelling-pairs workload.  Payloads are slices of two device pools,
    copied into the server's arena on admission."""
    import torch
    import workloads
    from paper_1605_05436_amd.serve import ExactSumServer, Request, run_trace, latency_stats

    t0 = time.time()
    npool = 100_000_000
    host = {0: workloads.serving_payload(npool, "f64", seed=args.seed + 1),
            1: workloads.serving_payload(npool, "f32", seed=args.seed + 2)}
    dev = {0: torch.from_numpy(host[0].view(np.int64)).to("cuda"),
           1: torch.from_numpy(host[1].view(np.int32)).to("cuda")}
    t, size, dt = workloads.serving_trace(seed=args.seed, rate=args.rate,
                                         duration=args.duration)
    rng = np.random.default_rng(args.seed + 3)
    offs = [int(rng.integers(0, npool - int(n) + 1)) for n in size]
    reqs = [Request(rid=i, src=dev[int(d)][o:o + int(n)], n=int(n), dtype=int(d),
                    arrival=float(a))
            for i, (a, n, d, o) in enumerate(zip(t, size, dt, offs))]
    torch.cuda.synchronize()
    log("serving: %d requests, %.2e elements, pools ready in %.1f s"
        % (len(reqs), float(size.sum()), time.time() - t0))
    # warm up the server (and the GPU clocks) with a short burst
    srv = ExactSumServer(arena_bytes=16 << 30, slots=4096)
    run_trace(srv, [Request(rid=-1 - i, src=dev[0][:1 << 20], n=1 << 20, dtype=0)
                    for i in range(50)], realtime=False)
    srv.completed.clear()
    srv.gpu_time_ms = 0.0
    srv.elements = 0
    srv.batches = 0
    w0 = time.perf_counter()
    done = run_trace(srv, reqs)
    wall = time.perf_counter() - w0
    st = latency_stats(done)
    # parity on a sample of requests
    sample = rng.choice(len(reqs), size=min(200, len(reqs)), replace=False)
    byid = {r.rid: r for r in done}
    pieces = [(host[reqs[i].dtype][offs[i]:offs[i] + reqs[i].n],
               "f64" if reqs[i].dtype == 0 else "f32") for i in sample.tolist()]
    wants, cpu_elems, cpu_s, cpu_threads = cpu_baseline_sample(pieces)
    ok = all((byid[reqs[i].rid].bits, byid[reqs[i].rid].flags) == w
             for i, w in zip(sample.tolist(), wants))
    elems = float(sum(r.n for r in done))
    rec = {"metric": "exact-sum serving: aggregate Gelem/s with p50/p99 latency (bit-exact)",
           "value": round(elems / wall / 1e9, 3), "unit": "Gelem/s", "n_gpus": 1,
           "steps": len(done), "warmup": 50, "ms_per_step": round(st["mean_ms"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": "Poisson %.0f req/s x %.0f s, sizes log-uniform [1e3, 1e8], "
                                  "f64/f32 50/50" % (args.rate, args.duration),
                      "requests": len(reqs), "elements": elems},
           "latency_ms": {k: round(v, 3) for k, v in st.items() if k != "count"},
           "gpu_busy_gelem_s": round(elems / (srv.gpu_time_ms * 1e-3) / 1e9, 1)
           if srv.gpu_time_ms else None,
           "gpu_busy_fraction": round(srv.gpu_time_ms * 1e-3 / wall, 4),
           "batches": srv.batches, "bit_exact_sample": ok,
           "sample_requests": int(len(sample)),
           "cpu_baseline": {"value": round(cpu_elems / cpu_s / 1e9, 4), "unit": "Gelem/s",
                            "cores": cpu_threads, "kind": "oracle",
                            "sample": "%d sampled requests (%d elements), one oracle sum each"
                                      % (len(sample), cpu_elems)}}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
