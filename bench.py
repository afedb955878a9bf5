#!/usr/bin/env python3
"""Benchmark: the 1-D complex FFT size sweep on one MI355X.

Workload (one "step"): for each length n in {2^10, 2^16, 2^20, 2^24, 3*2^18, 5*2^16,
7*3^9}, complex64 and complex128, forward and inverse, one transform of a batch
sized to ~1 GiB of input (batch = floor(2^30 / (n * element bytes))), inputs
complex N(0,1) from a seed, already resident in HBM.  28 plan executions per step.

Metric: nominal GFLOP/s = sum(5 * n * log2(n) * batch) / time (the FFT community's
convention, also for non-powers of two), plus the fraction of the HBM roofline:
algorithmic bytes (one read of the input + one write of the output per call) over
time, against the 8 TB/s peak.

roofline: the dominant kernel family (the complex Stockham pass kernels of the dtype
with the most time in the step).  A call of p passes over k batch chunks is p * k
launches, and its algorithmic bytes (2 * batch * n * element bytes: input read once,
output written once) are shared by those launches; achieved = the family's
algorithmic bytes / its event-timed duration on the stream the kernels run on, i.e.
the per-call fraction of the roofline.  The per-pass streaming rate (each pass
credited with the bytes it must stream, 2 * batch * n * element bytes) is reported
beside it as pass_stream_frac.  traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE per
launch (calibrated against a plain copy), recorded under profiles/, null when the
kernel sources changed since; traffic_per_call = traffic * launches per call.

forms: the split-BF16 matrix-core forms against the FP32 kernels on 64 x 2^20
complex64, with each form's error against the FP64 oracle.  check: sampled
transforms of every sweep case against the oracle.  also: the other benchmark
configurations (complex128 4096 x 64, 512^3 r2c and 4096^2 c2c, the 20,000-length
ragged batch, DCT-II/III, the spectral Laplacian), timed briefly.

cpu_baseline: the FP64 oracle, untuned, on this host's cores (all available physical
cores, and one thread), over a bounded sample, in the same nominal GFLOP/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1707_03776_amd/csrc/pass_device.h", "paper_1707_03776_amd/csrc/pass_f32_plain.hip",
                  "paper_1707_03776_amd/csrc/pass_f64_plain.hip", "paper_1707_03776_amd/csrc/dft_small.h",
                  "paper_1707_03776_amd/csrc/fft_args.h", "paper_1707_03776_amd/csrc/planner.cpp",
                  "paper_1707_03776_amd/csrc/shapes.h", "paper_1707_03776_amd/csrc/api.cpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def plan_launches(desc: str):
    """(passes per batch chunk, ops per chunk, kernel dispatches per call) of a plan's
    out-of-place op list as fft_plan_describe prints it: a plan that runs its batch in
    k chunks dispatches its op list once per chunk (a shorter last chunk has its own,
    listed after "last chunk:")."""
    import re
    main, _, last = desc.partition("  last chunk:")
    def count(part):
        lines = [l.strip() for l in part.splitlines()]
        return (sum(1 for l in lines if l.startswith("op") and " pass " in l),
                sum(1 for l in lines if l.startswith("op")))
    npass, nops = count(main)
    m = re.search(r"chunks of \d+ transforms \((\d+) chunks", desc)
    k = int(m.group(1)) if m else 1
    if last:
        lp, _ = count(last)
        return npass, nops, npass * (k - 1) + lp
    return npass, nops, npass * k


def nominal_flops(n: int, batch: int) -> float:
    return 5.0 * n * math.log2(n) * batch


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sizes", type=str, default="", help="comma list of lengths (default: the whole sweep)")
    ap.add_argument("--dtypes", type=str, default="c64,c128")
    ap.add_argument("--dirs", type=str, default="fwd,inv")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle comparison")
    ap.add_argument("--only-sweep", action="store_true", help="skip the forms and the other configurations")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--workload", choices=["sweep", "c128", "multidim", "precision", "ragged", "copy", "laplace",
                                           "dct"],
                    default="sweep",
                    help="sweep (default, the headline line); c128: 64 x 4096 complex128; multidim: 512^3 r2c and "
                         "4096^2 c2c; precision: 64 x 2^20 complex64 in FP32 and the split-BF16 MFMA forms; "
                         "ragged: 20,000 uneven lengths in one graph launch; copy: the plain 1 GiB device copy "
                         "the roofline and the traffic counters are calibrated with; laplace: the pseudo-spectral "
                         "Laplacian of a 512^3 field in float32 and float64; dct: DCT-II and DCT-III of 128 x 2^20 "
                         "float32 and 64 x 2^20 float64")
    return ap.parse_args()


def time_plan(plan_fn, reps=10, warmup=3):
    """Median ms of plan_fn() over reps, HIP events on torch's current stream."""
    import numpy as np
    import torch
    for _ in range(warmup):
        plan_fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan_fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def line_base(args, metric, value, unit, ms, dtype, workload, **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
         "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic, seeded, resident in HBM", "config": {"workload": workload}}
    d.update(extra)
    return d


def workload_c128(args):
    """64 transforms of 4096 complex128 points, forward; all 64 checked against the oracle."""
    import numpy as np
    import torch
    import oracle
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    n, b = 4096, 64
    rng = np.random.default_rng(inputs.seed_for(1, 1))
    x = inputs.complex_normal(rng, (b, n), np.complex128)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    plan = mf.Plan((n,), b, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F64)
    ms = time_plan(lambda: plan(xd, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
    err = oracle.rel_l2(yd.cpu().numpy(), oracle.c2c(x, (n,)))
    gf = nominal_flops(n, b) / (ms * 1e-3) / 1e9
    return line_base(args, "FFT GFLOP/s (5N*log2N/t) + % HBM peak", round(gf, 1), "GFLOP/s", ms, "f64",
                     "64 x 4096 complex128 c2c forward (8 MiB; cache-resident, launch-bound)",
                     hbm_frac=round(2 * x.nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     rel_l2_max=float(err.max()), rel_l2_median=float(np.median(err)), plan=plan.describe())


def workload_precision(args):
    """64 x 2^20 complex64 forward: FP32 vector kernels versus the split-BF16 MFMA forms;
    every transform checked against the FP64 oracle."""
    import numpy as np
    import torch
    import oracle
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    n, b = 1 << 20, 64
    rng = np.random.default_rng(inputs.seed_for(4, 1))
    x = inputs.complex_normal(rng, (b, n), np.complex64)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ref = oracle.c2c(x, (n,))
    forms = {}
    for name, dt in [("f32", mf.FFT_F32), ("bf16x2", mf.FFT_F32_BF16X2), ("bf16x3", mf.FFT_F32_BF16X3)]:
        plan = mf.Plan((n,), b, mf.FFT_C2C, mf.FFT_FORWARD, dt)
        ms = time_plan(lambda: plan(xd, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
        e = oracle.rel_l2(yd.cpu().numpy(), ref)
        forms[name] = {"ms": round(ms, 4), "gflops": round(nominal_flops(n, b) / (ms * 1e-3) / 1e9, 1),
                       "hbm_frac": round(2 * x.nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "rel_l2_max": float(e.max()), "rel_l2_median": float(np.median(e)),
                       "rel_l2_per_transform": [float(v) for v in e]}
        plan.close()
    f = forms["bf16x3"]
    return line_base(args, "FFT GFLOP/s (5N*log2N/t) + % HBM peak", f["gflops"], "GFLOP/s", f["ms"],
                     "f32 (bf16 MFMA operands)", "64 x 2^20 complex64 c2c forward: FP32 vs split-BF16 MFMA",
                     forms=forms)


def workload_multidim(args):
    """3-D r2c float32 512^3 and 2-D c2c complex64 4096^2, inputs uniform[-1,1) plus three
    pure tones at seeded frequencies; each tone's spike is checked in the output."""
    import numpy as np
    import torch
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    out = {}
    # (i) 3-D r2c
    dims = (512, 512, 512)
    rng = np.random.default_rng(inputs.seed_for(3, 1))
    x, freqs, phases, _ = inputs.real_with_tones(rng, dims, 3, np.float32)
    xd = torch.from_numpy(x).cuda()
    plan = mf.Plan(dims, 1, mf.FFT_R2C, mf.FFT_FORWARD, mf.FFT_F32)
    yd = torch.empty((1, 512, 512, 257), dtype=torch.complex64, device="cuda")
    ms = time_plan(lambda: plan(xd, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
    N = float(np.prod(dims))
    spikes = [complex(yd[0, k[0], k[1], k[2]].item()) / (N / 2) * np.exp(-1j * ph) for k, ph in zip(freqs, phases)]
    alg = x.nbytes + yd.numel() * 8
    out["r2c_512^3"] = {"ms": round(ms, 4), "gflops": round(2.5 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                        "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "tone_spike_ratio": [round(abs(v), 6) for v in spikes], "plan": plan.describe()}
    plan.close()
    del xd, yd
    # (ii) 2-D c2c
    dims = (4096, 4096)
    rng = np.random.default_rng(inputs.seed_for(3, 2))
    x, freqs, phases, _ = inputs.complex_with_tones(rng, dims, 3, np.complex64)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    plan = mf.Plan(dims, 1, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
    ms2 = time_plan(lambda: plan(xd, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
    N = float(np.prod(dims))
    spikes = [complex(yd[k[0], k[1]].item()) / N * np.exp(-1j * ph) for k, ph in zip(freqs, phases)]
    out["c2c_4096^2"] = {"ms": round(ms2, 4), "gflops": round(5 * N * math.log2(N) / (ms2 * 1e-3) / 1e9, 1),
                         "hbm_frac": round(2 * x.nbytes / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "tone_spike_ratio": [round(abs(v), 6) for v in spikes], "plan": plan.describe()}
    plan.close()
    tot_ms = ms + ms2
    flops = 2.5 * 512 ** 3 * 27 + 5 * 4096 ** 2 * 24
    return line_base(args, "FFT GFLOP/s (5N*log2N/t; 2.5N*log2N for r2c) + % HBM peak",
                     round(flops / (tot_ms * 1e-3) / 1e9, 1), "GFLOP/s", tot_ms, "f32",
                     "3-D r2c 512^3 float32 + 2-D c2c 4096^2 complex64", cases=out)


def host_cpu():
    """lscpu's model, sockets and cores, and the CPUs this process may run on."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass

    def num(key):
        try:
            return int(info.get(key, ""))
        except ValueError:
            return None
    sockets, cps, tpc = num("Socket(s)"), num("Core(s) per socket"), num("Thread(s) per core")
    return {"model": info.get("Model name"), "sockets": sockets, "cores_per_socket": cps, "threads_per_core": tpc,
            "physical_cores": sockets * cps if sockets and cps else None,
            "cpus_available": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _oracle_rate(inputs_by_case, sizes, threads, per_thread):
    """Oracle GFLOP/s over min(per_thread * threads, batch) transforms of each length."""
    import numpy as np
    import oracle
    oracle.set_threads(threads)
    flops = secs = 0.0
    parts = []
    for n in sizes:
        x_dev, batch = inputs_by_case[(n, "c64")]
        k = min(per_thread * threads, batch)
        x = x_dev[:k].cpu().numpy().astype(np.complex128)
        t0 = time.perf_counter()
        oracle.c2c(x, (n,))
        secs += time.perf_counter() - t0
        flops += nominal_flops(n, k)
        parts.append(f"{k}x{n}")
    return flops / secs / 1e9, secs, parts


def cpu_baseline(inputs_by_case, sizes):
    """The oracle on all available physical cores (several transforms per thread of each
    length) and on one thread (one transform of each length); complex64 sweep inputs
    upcast, forward; about 10-30 s of CPU work together."""
    import oracle
    host = host_cpu()
    avail = oracle.max_threads()  # honours OMP_NUM_THREADS (the host's CPU share)
    threads = min(avail, host["physical_cores"] or avail)
    v_all, s_all, parts = _oracle_rate(inputs_by_case, sizes, threads, 2)
    v_one, s_one, parts1 = _oracle_rate(inputs_by_case, sizes, 1, 1)
    oracle.set_threads(avail)
    return {"value": round(v_all, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "forward c2c, FP64 oracle (recursive Cooley-Tukey), one call per length over " +
                      ", ".join(parts) + f" transforms of the sweep's complex64 inputs (upcast), OpenMP over "
                      f"the transforms of a call; {s_all:.1f} s wall time",
            "single_thread": {"value": round(v_one, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": ", ".join(parts1) + f" transforms; {s_one:.1f} s"},
            "host": host}


def workload_ragged(args):
    """20,000 complex64 transforms, lengths log-uniform in [64, 65536] snapped to 7-smooth
    sizes, 5% primes (Bluestein): one hipGraph launch of the ragged plan (a few phase
    kernels), versus one fft_execute per transform (plans cached per length), both end to
    end on one stream."""
    import numpy as np
    import torch
    import oracle
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    lengths = inputs.ragged_lengths()
    data, offs = inputs.ragged_inputs(lengths)
    xd = torch.from_numpy(data).cuda()
    yd = torch.empty_like(xd)
    yb = torch.empty_like(xd)
    offs_l = [int(o) for o in offs[:-1]]
    t0 = time.perf_counter()
    plan = mf.fft_plan_create_many(lengths, offs_l, offs_l, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
    plan_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream().cuda_stream
    ms = time_plan(lambda: mf.fft_execute(plan, xd.data_ptr(), yd.data_ptr(), stream), reps=max(args.steps, 10),
                   warmup=args.warmup)
    # baseline: one execute per transform
    lib = mf.load_library()
    plans = {}
    for n in sorted(set(lengths)):
        plans[n] = mf.fft_plan_create(1, (n,), 1, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
    xp, yp = xd.data_ptr(), yb.data_ptr()

    def per_transform():
        for t, n in enumerate(lengths):
            o = offs_l[t] * 8
            lib.fft_execute(plans[n], xp + o, yp + o, stream)
    ms_base = time_plan(per_transform, reps=3, warmup=1)
    # parity: every transform of the ragged plan equals the per-transform form to
    # rounding, and a sample against the oracle
    y1 = yd.cpu().numpy()
    y2 = yb.cpu().numpy()
    diff = 0.0
    errs = []
    rng = np.random.default_rng(5)
    sample = set(int(t) for t in rng.choice(len(lengths), 64, replace=False))
    for t, n in enumerate(lengths):
        a, b = y1[offs[t]:offs[t + 1]], y2[offs[t]:offs[t + 1]]
        diff = max(diff, float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)))
        if t in sample:
            ref = oracle.c2c(data[offs[t]:offs[t + 1]][None], (n,))[0]
            errs.append(float(np.linalg.norm(a - ref) / np.linalg.norm(ref)))
    for p in plans.values():
        mf.fft_plan_destroy(p)
    desc = "\n".join(l for l in mf.fft_plan_describe(plan).splitlines()
                     if l.startswith("mifft") or "schedule:" in l or "block=" in l and "op" not in l)
    mf.fft_plan_destroy(plan)
    flops = sum(5.0 * n * math.log2(n) for n in lengths)
    by = 2 * data.nbytes
    return line_base(args, "FFT GFLOP/s (5N*log2N/t) + % HBM peak", round(flops / (ms * 1e-3) / 1e9, 1), "GFLOP/s",
                     ms, "f32", "20,000 ragged complex64 c2c (lengths log-uniform 64..65536, 5% primes)",
                     hbm_frac=round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     per_transform_launches={"ms": round(ms_base, 3),
                                             "gflops": round(flops / (ms_base * 1e-3) / 1e9, 1)},
                     speedup_vs_per_transform=round(ms_base / ms, 2), plan_create_s=round(plan_s, 2),
                     distinct_lengths=len(set(lengths)), total_points=int(offs[-1]),
                     max_rel_diff_vs_per_transform=diff, sample_rel_l2_max=max(errs), plan=desc)


def workload_laplace(args):
    """Pseudo-spectral Laplacian of one 512^3 periodic field (uniform[-1,1) plus three
    tones), float32 and float64: r2c, the -|kappa|^2 multiply, c2r.  The r2c and c2r
    plans are also timed alone, so the multiply's share is the difference."""
    import numpy as np
    import torch
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    dims, L = (512, 512, 512), (1.0, 1.0, 1.0)
    N = float(np.prod(dims))
    rng = np.random.default_rng(inputs.seed_for(6, 1))
    x32, _, _, _ = inputs.real_with_tones(rng, dims, 3, np.float32)
    forms = {}
    for name, dt, npdt, cdt in [("f32", mf.FFT_F32, np.float32, torch.complex64),
                                ("f64", mf.FFT_F64, np.float64, torch.complex128)]:
        xd = torch.from_numpy(x32.astype(npdt)).cuda().reshape(1, *dims)
        yd = torch.empty_like(xd)
        lap = mf.Laplacian(dims, 1, L, dt)
        ms = time_plan(lambda: lap(xd, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
        lap.close()
        fwd = mf.Plan(dims, 1, mf.FFT_R2C, mf.FFT_FORWARD, dt)
        inv = mf.Plan(dims, 1, mf.FFT_C2R, mf.FFT_INVERSE, dt)
        spec = torch.empty((1, 512, 512, 257), dtype=cdt, device="cuda")
        ms_f = time_plan(lambda: fwd(xd, out=spec), reps=max(args.steps, 10), warmup=args.warmup)
        ms_i = time_plan(lambda: inv(spec, out=yd), reps=max(args.steps, 10), warmup=args.warmup)
        fwd.close()
        inv.close()
        spec_bytes = spec.numel() * spec.element_size()
        # algorithmic bytes of the whole operator: field in, field out, plus the
        # half spectrum written, read and written by the multiply, read by c2r
        alg = 2 * xd.numel() * xd.element_size() + 4 * spec_bytes
        forms[name] = {"ms": round(ms, 4), "r2c_ms": round(ms_f, 4), "c2r_ms": round(ms_i, 4),
                       "multiply_ms_est": round(ms - ms_f - ms_i, 4),
                       "gpoints_per_s": round(N / (ms * 1e-3) / 1e9, 2),
                       "gflops": round(2 * 2.5 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                       "alg_hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del xd, yd, spec
    f = forms["f32"]
    return line_base(args, "Laplacian grid points/s (512^3, one application)", f["gpoints_per_s"], "Gpoints/s",
                     f["ms"], "f32", "pseudo-spectral Laplacian of one 512^3 periodic field: r2c, -|kappa|^2, c2r",
                     forms=forms)


def workload_dct(args):
    """DCT-II and DCT-III of 2^20-point real lines (128 float32 / 64 float64 lines, 512 MiB
    each way): the element-wise prologue, the 2^20-point real transform and the
    element-wise epilogue; the real and the complex FFT of the same lines are timed alone
    beside it."""
    import numpy as np
    import torch
    import paper_1707_03776_amd as mf
    n = 1 << 20
    forms = {}
    for name, dt, b, rdt, cdt in [("f32", mf.FFT_F32, 128, torch.float32, torch.complex64),
                                  ("f64", mf.FFT_F64, 64, torch.float64, torch.complex128)]:
        g = torch.Generator(device="cuda").manual_seed(6000 + dt)
        x = torch.randn((b, n), dtype=rdt, device="cuda", generator=g)
        y = torch.empty_like(x)
        row = {}
        for kname, kind in (("dct2", mf.FFT_DCT2), ("dct3", mf.FFT_DCT3)):
            plan = mf.Plan((n,), b, kind, mf.FFT_FORWARD, dt)
            ms = time_plan(lambda: plan(x, out=y), reps=max(args.steps, 10), warmup=args.warmup)
            plan.close()
            alg = 2 * x.numel() * x.element_size()
            row[kname] = {"ms": round(ms, 4), "gflops": round(2.5 * n * math.log2(n) * b / (ms * 1e-3) / 1e9, 1),
                          "alg_hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # the real-input transform of the same lines (what DCT-II adds its reorder and
        # rotation to) and the complex one
        yh = torch.empty((b, n // 2 + 1), dtype=cdt, device="cuda")
        plan = mf.Plan((n,), b, mf.FFT_R2C, mf.FFT_FORWARD, dt)
        row["r2c_same_lines_ms"] = round(time_plan(lambda: plan(x, out=yh), reps=max(args.steps, 10),
                                                   warmup=args.warmup), 4)
        plan.close()
        del yh
        xc = torch.empty((b, n), dtype=cdt, device="cuda")
        yc = torch.empty_like(xc)
        plan = mf.Plan((n,), b, mf.FFT_C2C, mf.FFT_FORWARD, dt)
        row["c2c_same_lines_ms"] = round(time_plan(lambda: plan(xc, out=yc), reps=max(args.steps, 10),
                                                   warmup=args.warmup), 4)
        plan.close()
        forms[name] = row
        del x, y, xc, yc
    f = forms["f32"]["dct2"]
    return line_base(args, "DCT GFLOP/s (2.5N*log2N/t per real line) + % HBM peak", f["gflops"], "GFLOP/s", f["ms"],
                     "f32", "DCT-II / DCT-III of 2^20-point real lines: 128 float32, 64 float64", forms=forms)


def workload_copy(args):
    """Calibration: torch's device copy of a 1 GiB complex64 tensor (2^27 elements), 20 times
    per step.  Its rate is the practical read+write bandwidth the pass kernels compete with,
    and its FETCH_SIZE / WRITE_SIZE counters scale the kernels' traffic figures."""
    import torch
    x = torch.randn(1 << 27, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)

    def step():
        for _ in range(20):
            y.copy_(x)
    ms = time_plan(step, reps=max(args.steps, 3), warmup=args.warmup) / 20
    by = 2 * x.numel() * 8
    return line_base(args, "device copy GB/s (read + write)", round(by / (ms * 1e-3) / 1e9, 1), "GB/s", ms, "c64",
                     "plain 1 GiB complex64 device copy (torch copy_), calibration only",
                     hbm_frac=round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), copies_per_step=20)


def main():
    args = parse()
    if args.gpus == 1 and args.workload != "sweep":
        import torch
        import paper_1707_03776_amd as mf
        if not os.path.exists(mf.LIB_PATH):
            from paper_1707_03776_amd import build as b
            b.build()
        torch.cuda.set_device(0)
        fn = {"c128": workload_c128, "precision": workload_precision, "multidim": workload_multidim,
              "ragged": workload_ragged, "copy": workload_copy, "laplace": workload_laplace, "dct": workload_dct}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this "
                                   "build (the batch would shard by transform with no communication)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs

    if not os.path.exists(mf.LIB_PATH):
        from paper_1707_03776_amd import build as b
        b.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    sizes = [int(s) for s in args.sizes.split(",") if s] or list(inputs.SWEEP_LENGTHS)
    dts = [d for d in args.dtypes.split(",") if d]
    dirs = [d for d in args.dirs.split(",") if d]
    tmap = {"c64": (np.complex64, torch.complex64, mf.FFT_F32, 8),
            "c128": (np.complex128, torch.complex128, mf.FFT_F64, 16)}

    # inputs (seeded, on the GPU), one output buffer per dtype, plans
    inputs_by_case = {}
    for n in sizes:
        for d in dts:
            npdt, tdt, _, eb = tmap[d]
            batch = inputs.sweep_batch(n, npdt)
            seed = inputs.seed_for(2, inputs.sweep_case_index(n, npdt))
            inputs_by_case[(n, d)] = (inputs.device_complex_normal((batch, n), npdt, seed, dev), batch)
    outs = {}
    for d in dts:
        npdt, tdt, _, eb = tmap[d]
        need = max(inputs.sweep_batch(n, npdt) * n for n in sizes)
        outs[d] = torch.empty(need, dtype=tdt, device=dev)
    cases = []
    for n in sizes:
        for d in dts:
            for r in dirs:
                npdt, tdt, fdt, eb = tmap[d]
                x, batch = inputs_by_case[(n, d)]
                plan = mf.Plan((n,), batch, mf.FFT_C2C, mf.FFT_FORWARD if r == "fwd" else mf.FFT_INVERSE, fdt)
                desc = plan.describe().split("  in place")[0]  # the out-of-place op list
                npass, nops, launches = plan_launches(desc)
                cases.append(dict(n=n, dtype=d, dir=r, batch=batch, plan=plan, x=x,
                                  y=outs[d][:batch * n].view(batch, n), passes=npass, eb=eb, ops=nops,
                                  launches=launches))
                if args.verbose:
                    print(desc, flush=True)

    stream = torch.cuda.current_stream(dev)

    def step(events=None):
        for i, c in enumerate(cases):
            if events is not None:
                events[i][0].record(stream)
            mf.fft_execute(c["plan"].handle, c["x"].data_ptr(), c["y"].data_ptr(), stream.cuda_stream)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    case_ms = [sum(events[s][i][0].elapsed_time(events[s][i][1]) for s in range(args.steps)) / args.steps
               for i in range(len(cases))]
    ms_per_step = wall * 1e3 / args.steps

    total_flops = sum(nominal_flops(c["n"], c["batch"]) for c in cases)
    gflops = total_flops / (ms_per_step * 1e-3) / 1e9

    per_case = []
    fam = {}
    for c, ms in zip(cases, case_ms):
        alg_bytes = 2 * c["batch"] * c["n"] * c["eb"]
        per_case.append({"n": c["n"], "dtype": c["dtype"], "dir": c["dir"], "batch": c["batch"],
                         "passes": c["passes"], "launches": c["launches"], "ms": round(ms, 4),
                         "gflops": round(nominal_flops(c["n"], c["batch"]) / (ms * 1e-3) / 1e9, 1),
                         "hbm_frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        if c["ops"] == c["passes"]:  # cases made only of Stockham passes
            f = fam.setdefault(c["dtype"], {"bytes": 0.0, "stream_bytes": 0.0, "ms": 0.0, "launches": 0,
                                            "calls": 0})
            f["bytes"] += alg_bytes             # the call's in + out, shared by its launches
            f["stream_bytes"] += alg_bytes * c["passes"]  # what the passes stream between them
            f["ms"] += ms
            f["launches"] += c["launches"]      # kernel dispatches: passes x batch chunks
            f["calls"] += 1
    kname = {"c64": "k_pass_fixed<float, PRO_PLAIN, EPI_PLAIN, radices...> (complex64 Stockham passes)",
             "c128": "k_pass_fixed<double, PRO_PLAIN, EPI_PLAIN, radices...> (complex128 Stockham passes)"}
    dom = max(fam, key=lambda d: fam[d]["ms"]) if fam else None
    roofline = None
    if dom:
        f = fam[dom]
        avg_ms = f["ms"] / f["launches"]
        achieved = f["bytes"] / (f["ms"] * 1e-3) / 1e9
        traffic = None
        try:
            with open(TRAFFIC_FILE) as fh:
                tr = json.load(fh)
            if tr.get("kernel_hash") == kernel_hash() and tr.get("dtype") == dom:
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError):
            pass
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_per_call": (round(traffic * f["launches"] / f["calls"]) if traffic else None),
                    "kernel": kname[dom], "launches_per_step": f["launches"], "calls_per_step": f["calls"],
                    "avg_launch_ms": round(avg_ms, 4),
                    "alg_bytes_per_launch": round(f["bytes"] / f["launches"]),
                    "alg_bytes_per_call": round(f["bytes"] / f["calls"]),
                    "pass_stream_frac": round(f["stream_bytes"] / (f["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    check = None
    if not args.no_check:
        check = sweep_check(cases, stream)

    cpu = None
    if not args.no_cpu_baseline and "c64" in dts:
        cpu = cpu_baseline(inputs_by_case, sizes)

    dtype_str = "+".join({"c64": "f32", "c128": "f64"}[d] for d in dts)
    line = {
        "metric": "FFT GFLOP/s (5N*log2N/t) + % HBM peak",
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_str,
        "data": "synthetic: complex N(0,1) from a seed (torch Philox on the GPU), resident in HBM",
        "config": {"workload": "1-D c2c sweep: n in {2^10,2^16,2^20,2^24,3*2^18,5*2^16,7*3^9}, "
                               "complex64 and complex128, forward and inverse, batch ~1 GiB of input each",
                   "sizes": sizes, "dtypes": dts, "dirs": dirs, "executions_per_step": len(cases),
                   "hbm_frac_whole_step": round(sum(2 * c["batch"] * c["n"] * c["eb"] for c in cases)
                                                / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_case": per_case,
    }
    if check is not None:
        line["check"] = check
    for c in cases:
        c["plan"].close()
    cases.clear()
    inputs_by_case.clear()
    outs.clear()
    torch.cuda.empty_cache()
    if not args.only_sweep:
        brief = argparse.Namespace(**vars(args))
        brief.steps, brief.warmup = 5, 2
        line["forms"] = forms_line(brief)
        also = {}
        for name, fn in (("c128_4096x64", workload_c128), ("multidim", workload_multidim),
                         ("ragged", workload_ragged), ("dct", workload_dct), ("laplace", workload_laplace)):
            r = fn(brief)
            also[name] = _brief({k: v for k, v in r.items() if k not in ("n_gpus", "steps", "warmup",
                                                                        "higher_is_better", "scaling",
                                                                        "vs_baseline", "data")})
            torch.cuda.empty_cache()
        line["also"] = also
    print(json.dumps(line), flush=True)


def _brief(d):
    """A workload's result without plan descriptions and per-transform error lists."""
    if isinstance(d, dict):
        return {k: _brief(v) for k, v in d.items() if k not in ("plan", "rel_l2_per_transform")}
    return d


def sweep_check(cases, stream):
    """First and last transform of every sweep case against the oracle: the largest
    relative L2 and element error (|y - ref| / rms(ref)) of each case."""
    import numpy as np
    import torch
    import oracle
    import paper_1707_03776_amd as mf
    worst = {}
    for c in cases:
        b = c["batch"]
        rows = sorted({0, b - 1})
        xs = c["x"][rows].cpu().numpy()
        mf.fft_execute(c["plan"].handle, c["x"].data_ptr(), c["y"].data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        ys = c["y"][rows].cpu().numpy()
        ref = oracle.c2c(xs, (c["n"],), inverse=c["dir"] == "inv")
        worst[f'{c["n"]}/{c["dtype"]}/{c["dir"]}'] = {
            "rel_l2": float(np.max(oracle.rel_l2(ys, ref))),
            "max_elem_over_rms": float(np.max(oracle.max_elem_err(ys, ref))), "transforms": rows}
    return worst


def forms_line(args):
    """64 x 2^20 complex64 forward: the FP32 kernels and the split-BF16 MFMA forms, each
    with its error against the FP64 oracle on 8 seeded transforms."""
    import numpy as np
    import torch
    import oracle
    import paper_1707_03776_amd as mf
    from paper_1707_03776_amd import inputs
    n, b = 1 << 20, 64
    x = inputs.device_complex_normal((b, n), np.complex64, inputs.seed_for(4, 1))
    y = torch.empty_like(x)
    rows = sorted({0, b - 1} | set(int(v) for v in np.random.default_rng(4001).integers(0, b, 6)))
    ref = oracle.c2c(x[rows].cpu().numpy(), (n,))
    forms = {}
    for name, dt in [("f32", mf.FFT_F32), ("bf16x2", mf.FFT_F32_BF16X2), ("bf16x3", mf.FFT_F32_BF16X3)]:
        plan = mf.Plan((n,), b, mf.FFT_C2C, mf.FFT_FORWARD, dt)
        ms = time_plan(lambda: plan(x, out=y), reps=max(args.steps, 10), warmup=args.warmup)
        ys = y[rows].cpu().numpy()
        e = oracle.rel_l2(ys, ref)
        forms[name] = {"ms": round(ms, 4), "gflops": round(nominal_flops(n, b) / (ms * 1e-3) / 1e9, 1),
                       "hbm_frac": round(2 * x.numel() * 8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "rel_l2_max": float(e.max()), "rel_l2_median": float(np.median(e)),
                       "max_elem_over_rms": float(np.max(oracle.max_elem_err(ys, ref)))}
        plan.close()
    return {"workload": "64 x 2^20 complex64 c2c forward", "oracle_transforms": rows, **forms}


if __name__ == "__main__":
    main()
