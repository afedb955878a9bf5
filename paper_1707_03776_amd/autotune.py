"""Autotuner: picks pass splits, radix orders and tile/workgroup shapes by timing
candidate plans on the GPU, and writes the winners as a tuning table
(``fft_tune_set`` format) that the planner reads at plan creation.

Knobs (see ``include/mifft.h``, ``fft_tune_set``):

* split key  ``<dt>:n<n>:S1:split = s<L1>.<L2>...`` - how a 1-D axis splits into passes;
* radix key  ``<dt>:L<L>:radix = r<r1>.<r2>...``   - stage radices of a length-L pass;
* pass key   ``<dt>:L<L>:<radices>:<map>:tw<k> = c<cols>,t<threads>,p<pitch>`` - columns per
  workgroup (tile width), minimum workgroup size and LDS column pitch;
* chunk key  ``<dt>:<kind>:<dims>:chunk = b<bytes>`` - input bytes per batch chunk of a
  multi-pass plan (``b0``: the whole batch at once);
* ``rag:schedule = w<parts>`` - how many parts a ragged transform may have and still run
  whole in one workgroup.

Ragged plans have their own keys (prefix ``rag:``), tuned per size class on the ragged
workload itself.  The search is greedy coordinate descent: splits first, then the batch
chunk size, then the radix order of each pass length, then the tile shape of each pass;
a candidate replaces the incumbent only if it is at least ``gain`` faster (median of
``reps`` timed runs).

Usage (on a GPU):  ``python -m paper_1707_03776_amd.autotune --out FILE [--workload ...]``
"""
from __future__ import annotations

import argparse
import itertools
import math
import re
import sys
import time

import numpy as np

import paper_1707_03776_amd as mf
from paper_1707_03776_amd import inputs

# ----------------------------------------------------------------------------- candidates

def factor7(n: int):
    """Exponents of 2, 3, 5, 7 in n, or None if n is not 7-smooth."""
    e = {}
    for p in (2, 3, 5, 7):
        e[p] = 0
        while n % p == 0:
            n //= p
            e[p] += 1
    return e if n == 1 else None


def divisors7(n: int):
    e = factor7(n)
    if e is None:
        return []
    out = []
    for a in range(e[2] + 1):
        for b in range(e[3] + 1):
            for c in range(e[5] + 1):
                for d in range(e[7] + 1):
                    out.append(2 ** a * 3 ** b * 5 ** c * 7 ** d)
    return sorted(out)


def candidate_splits(n: int, limit: int = 10, max_len: int = 8192):
    """Ordered factorisations of n into 1-3 pass lengths, most balanced first."""
    if factor7(n) is None:
        return []
    cands = set()
    if n <= max_len:
        cands.add((n,))
    divs = [d for d in divisors7(n) if 16 <= d <= max_len]
    for a in divs:
        b = n // a
        if 16 <= b <= max_len:
            cands.add((a, b))
        for c in divs:
            if b % c == 0 and 16 <= b // c <= max_len:
                cands.add((a, c, b // c))
    # prefer fewer passes, then balance (max/min ratio)
    ranked = sorted(cands, key=lambda s: (len(s), max(s) / min(s)))
    out = []
    for s in ranked:
        if len(out) >= limit:
            break
        if len(s) > 1 and max(s) / min(s) > 64:
            continue
        out.append(s)
    return out


def candidate_radices(L: int, default, limit: int = 8):
    """Radix sequences for a length-L pass: orders of the default multiset, and the
    power-of-two part regrouped into the same number of stages."""
    e = factor7(L)
    if e is None or L < 2:
        return []
    odd = [r for r in default if r in (3, 9, 5, 7)]
    pow2_default = [r for r in default if r in (2, 4, 8, 16)]
    groups = {tuple(sorted(pow2_default, reverse=True))}
    a2, s = e[2], len(pow2_default)
    if s > 0:
        for combo in itertools.combinations_with_replacement((16, 8, 4, 2), s):
            if sum(int(math.log2(r)) for r in combo) == a2:
                groups.add(tuple(sorted(combo, reverse=True)))
    seqs = []
    for g in groups:
        for perm in set(itertools.permutations(list(g) + odd)):
            seqs.append(perm)
    seqs = sorted(set(seqs), key=lambda q: (q != tuple(default), q))
    return seqs[:limit]


# ----------------------------------------------------------------------------- plan parsing

PASS_RE = re.compile(r" pass \S+ L=(\d+) radices=([\dx]+) \S+ c=(\d+) T=(\d+) .* key=(\S+)")


def plan_passes(desc: str):
    """(L, radices, c, T, key) of every pass of the out-of-place op list (of a chunk,
    for a plan that runs its batch in chunks)."""
    out = []
    for line in desc.split("  in place")[0].split("  last chunk")[0].splitlines():
        m = PASS_RE.search(line)
        if m:
            out.append((int(m.group(1)), tuple(int(r) for r in m.group(2).split("x")), int(m.group(3)),
                        int(m.group(4)), m.group(5)))
    return out


def dt_name(dtype: int, ragged: bool = False) -> str:
    base = {mf.FFT_F32: "f32", mf.FFT_F64: "f64", mf.FFT_F32_BF16X2: "bf2", mf.FFT_F32_BF16X3: "bf3"}[dtype]
    return ("rag:" if ragged else "") + base


# ----------------------------------------------------------------------------- timing

def fastest(ts, k: int = 3) -> float:
    """Mean of the k fastest of repeated timings (robust to interference)."""
    return float(np.mean(sorted(ts)[:k]))


class Problem:
    """A plan request plus device buffers, timed with HIP events on the current stream."""

    def __init__(self, dims, batch, kind=mf.FFT_C2C, dtype=mf.FFT_F32, direction=mf.FFT_FORWARD):
        import torch
        self.dims, self.batch, self.kind, self.dtype, self.direction = tuple(dims), batch, kind, dtype, direction
        f64 = dtype == mf.FFT_F64
        n = int(np.prod(dims))
        if kind == mf.FFT_R2C:
            self.x = torch.randn((batch, n), dtype=torch.float64 if f64 else torch.float32, device="cuda")
            half = int(np.prod(dims[:-1])) * (dims[-1] // 2 + 1)
            self.y = torch.empty((batch, half), dtype=torch.complex128 if f64 else torch.complex64, device="cuda")
        else:
            self.x = inputs.device_complex_normal((batch, n), np.complex128 if f64 else np.complex64, 1)
            self.y = torch.empty_like(self.x)
        self.label = f"{'x'.join(map(str, dims))} b={batch} kind={kind} dtype={dtype}"

    def describe(self) -> str:
        return mf.fft_plan_inspect(len(self.dims), self.dims, self.batch, self.kind, self.direction, self.dtype)

    def time(self, reps: int = 10, warmup: int = 3) -> float:
        import torch
        try:
            plan = mf.fft_plan_create(len(self.dims), self.dims, self.batch, self.kind, self.direction, self.dtype)
        except mf.MifftError:
            return math.inf
        try:
            s = torch.cuda.current_stream().cuda_stream
            for _ in range(warmup):
                mf.fft_execute(plan, self.x.data_ptr(), self.y.data_ptr(), s)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mf.fft_execute(plan, self.x.data_ptr(), self.y.data_ptr(), s)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return fastest(ts)
        finally:
            mf.fft_plan_destroy(plan)

    def close(self):
        del self.x, self.y


class RaggedProblem:
    """A ragged batch (fft_plan_create_many), packed contiguously."""

    def __init__(self, lengths, dtype=mf.FFT_F32, direction=mf.FFT_FORWARD):
        import torch
        self.lengths = [int(n) for n in lengths]
        self.dtype, self.direction = dtype, direction
        offs = np.zeros(len(self.lengths) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(self.lengths)
        self.offs = offs[:-1]
        npdt = np.complex128 if dtype == mf.FFT_F64 else np.complex64
        self.x = inputs.device_complex_normal((int(offs[-1]),), npdt, 1)
        self.y = torch.empty_like(self.x)
        self.label = f"ragged count={len(self.lengths)} dtype={dtype}"

    def describe(self) -> str:
        return mf.fft_plan_inspect_many(self.lengths, mf.FFT_C2C, self.direction, self.dtype)

    def time(self, reps: int = 10, warmup: int = 3) -> float:
        import torch
        try:
            plan = mf.fft_plan_create_many(self.lengths, self.offs, self.offs, mf.FFT_C2C, self.direction,
                                           self.dtype)
        except mf.MifftError:
            return math.inf
        try:
            s = torch.cuda.current_stream().cuda_stream
            for _ in range(warmup):
                mf.fft_execute(plan, self.x.data_ptr(), self.y.data_ptr(), s)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mf.fft_execute(plan, self.x.data_ptr(), self.y.data_ptr(), s)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return fastest(ts)
        finally:
            mf.fft_plan_destroy(plan)

    def close(self):
        del self.x, self.y


# ----------------------------------------------------------------------------- search

class Tuner:
    def __init__(self, gain: float = 0.03, verbose: bool = True):
        self.gain = gain
        self.verbose = verbose
        self.entries = {}  # key -> value (the winners so far)

    def log(self, *a):
        if self.verbose:
            print(*a, flush=True)

    def _apply(self, extra=None):
        items = dict(self.entries)
        if extra:
            items.update(extra)
        mf.fft_tune_set("\n".join(f"{k}={v}" for k, v in items.items() if v), replace=True)

    def _try(self, prob, key, values, best=None):
        """Time each value of key against a fresh timing of the incumbent table; adopt
        the fastest if it wins by the gain margin twice (once in the sweep, once in a
        confirming head-to-head).  Values that leave the plan unchanged are skipped."""
        self._apply()
        inc_desc = prob.describe()
        inc_t = prob.time()
        incumbent = self.entries.get(key)
        best_v, best_t = None, inc_t
        for v in values:
            if v == incumbent:
                continue
            self._apply({key: v})
            try:
                if prob.describe() == inc_desc:
                    continue
            except mf.MifftError:
                continue
            t = prob.time()
            self.log(f"    {key}={v}: {t * 1e3:9.1f} us (incumbent {inc_t * 1e3:.1f})" if math.isfinite(t)
                     else f"    {key}={v}: no plan")
            if t < best_t:
                best_v, best_t = v, t
        if best_v is not None and best_t < inc_t * (1.0 - self.gain):
            self._apply({key: best_v})
            t1 = prob.time()
            self._apply()
            t0 = prob.time()
            if t1 < t0 * (1.0 - self.gain):
                self.entries[key] = best_v
                self.log(f"    adopt {key}={best_v}: {t0 * 1e3:.1f} -> {t1 * 1e3:.1f} us")
                inc_t = t1
        self._apply()
        return inc_t

    def tune(self, prob, splits=True, radices=True, tiles=True, max_passes=None):
        self._apply()
        best = prob.time()
        self.log(f"  {prob.label}: incumbent table {best * 1e3:.1f} us")
        dt = dt_name(prob.dtype, isinstance(prob, RaggedProblem))
        if splits and isinstance(prob, Problem) and len(prob.dims) == 1 and prob.kind == mf.FFT_C2C:
            n = prob.dims[0]
            key = f"{dt}:n{n}:S1:split"
            vals = ["s" + ".".join(map(str, s)) for s in candidate_splits(n)]
            best = self._try(prob, key, vals, best)
        if isinstance(prob, Problem) and prob.batch > 1 and len(plan_passes(prob.describe())) > 1:
            kind = {mf.FFT_C2C: "c2c", mf.FFT_R2C: "r2c", mf.FFT_C2R: "c2r"}[prob.kind]
            key = f"{dt}:{kind}:{'x'.join(map(str, prob.dims))}:chunk"
            best = self._try(prob, key, [f"b{v << 20}" for v in (0, 64, 128, 256, 512)], best)
        passes = plan_passes(prob.describe())
        if max_passes is not None:
            passes = passes[:max_passes]
        if radices:
            seen = set()
            for L, rad, _, _, _ in passes:
                if L in seen or L < 8:
                    continue
                seen.add(L)
                key = f"{dt}:L{L}:radix"
                vals = ["r" + ".".join(map(str, q)) for q in candidate_radices(L, rad)]
                best = self._try(prob, key, vals, best)
            passes = plan_passes(prob.describe())
            if max_passes is not None:
                passes = passes[:max_passes]
        if tiles:
            for L, rad, c, T, key in dict.fromkeys(passes):
                cvals = [f"c{v}" for v in (c // 2, c * 2, c * 4, c * 8) if 1 <= v <= 64]
                best = self._try(prob, key, cvals, best)
                base = self.entries.get(key, f"c{c}")
                tvals = [f"{base},t{v}" for v in (T * 2,) if v <= 1024]
                best = self._try(prob, key, tvals, best)
                base = self.entries.get(key, f"c{c}")
                pvals = [f"{base},p{v}" for v in (4, 8)]
                best = self._try(prob, key, pvals, best)
        # final head-to-head of the planner defaults against the tuned table
        saved = dict(self.entries)
        self.entries = {}
        self._apply()
        t_def = prob.time()
        self.entries = saved
        self._apply()
        t_tuned = prob.time()
        self.log(f"  {prob.label}: default {t_def * 1e3:.1f} us, tuned {t_tuned * 1e3:.1f} us "
                 f"({t_def / t_tuned:.3f}x)")
        return t_def, t_tuned

    def text(self, header: str = "") -> str:
        lines = [f"# {h}" for h in header.splitlines()] if header else []
        lines += [f"{k}={v}" for k, v in sorted(self.entries.items()) if v]
        return "\n".join(lines) + "\n"


# ----------------------------------------------------------------------------- workloads

SWEEP = [1 << 10, 1 << 16, 1 << 20, 1 << 24, 3 << 18, 5 << 16, 7 * 3 ** 9]


def sweep_problems(dtypes=(mf.FFT_F32, mf.FFT_F64)):
    for dtype in dtypes:
        eb = 16 if dtype == mf.FFT_F64 else 8
        for n in SWEEP:
            yield (n,), max(1, (1 << 30) // (n * eb)), mf.FFT_C2C, dtype


def other_problems():
    yield (4096,), 64, mf.FFT_C2C, mf.FFT_F64
    yield (512, 512, 512), 1, mf.FFT_R2C, mf.FFT_F32
    yield (4096, 4096), 1, mf.FFT_C2C, mf.FFT_F32
    yield (1 << 20,), 64, mf.FFT_C2C, mf.FFT_F32_BF16X2
    yield (1 << 20,), 64, mf.FFT_C2C, mf.FFT_F32_BF16X3


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="tuning file to write")
    ap.add_argument("--workload", default="all", choices=["sweep", "other", "ragged", "all"])
    ap.add_argument("--gain", type=float, default=0.03, help="minimum relative improvement to adopt a candidate")
    ap.add_argument("--ragged-keys", type=int, default=12, help="heaviest ragged passes to tune")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the autotuner times plans on a GPU"
    mf.fft_tune_set("", replace=True)
    tuner = Tuner(gain=args.gain)
    t0 = time.time()
    summary = []
    probs = []
    if args.workload in ("sweep", "all"):
        probs += list(sweep_problems())
    if args.workload in ("other", "all"):
        probs += list(other_problems())
    for dims, batch, kind, dtype in probs:
        p = Problem(dims, batch, kind, dtype)
        tuner.tune(p, splits=(kind == mf.FFT_C2C and len(dims) == 1 and dtype in (0, 1)))
        p.close()
    # every problem again with the final table (keys are shared between problems)
    final = dict(tuner.entries)
    for dims, batch, kind, dtype in probs:
        p = Problem(dims, batch, kind, dtype)
        tuner.entries = {}
        tuner._apply()
        a = p.time()
        tuner.entries = final
        tuner._apply()
        b = p.time()
        summary.append(f"{p.label}: default {a * 1e3:.1f} us, tuned {b * 1e3:.1f} us ({a / b:.3f}x)")
        tuner.log(summary[-1])
        p.close()
    if args.workload in ("ragged", "all"):
        p = RaggedProblem(inputs.ragged_lengths())
        # size classes: the heaviest pass keys of the ragged plan (by points they process)
        passes = plan_passes_ragged(p.describe(), args.ragged_keys, p.dtype)
        a = p.time()
        best = a
        tuner.log(f"  {p.label}: default {a * 1e3:.1f} us; tuning {len(passes)} size classes")
        dt = dt_name(p.dtype, True)
        best = tuner._try(p, "rag:schedule", [f"w{v}" for v in (2, 4, 8, 32)], best)
        for L in dict.fromkeys(L for L, _, _, _ in passes):
            rad = [r for L2, r, _, _ in passes if L2 == L][0]
            best = tuner._try(p, f"{dt}:L{L}:radix", ["r" + ".".join(map(str, q))
                                                       for q in candidate_radices(L, rad, limit=4)], best)
        for L, rad, c, key in plan_passes_ragged(p.describe(), args.ragged_keys, p.dtype):
            best = tuner._try(p, key, [f"c{v}" for v in (c // 2, c * 2) if 1 <= v <= 64], best)
        saved = dict(tuner.entries)
        tuner.entries = {k: v for k, v in saved.items() if not k.startswith("rag:")}
        tuner._apply()
        a = p.time()
        tuner.entries = saved
        tuner._apply()
        best = p.time()
        summary.append(f"{p.label}: default {a * 1e3:.1f} us, tuned {best * 1e3:.1f} us ({a / best:.3f}x)")
        tuner.log(summary[-1])
        p.close()
    header = ("MI355X (gfx950) tuning table written by paper_1707_03776_amd.autotune\n"
              f"workload={args.workload} gain={args.gain} elapsed={time.time() - t0:.0f}s\n" + "\n".join(summary))
    with open(args.out, "w") as f:
        f.write(tuner.text(header))
    print("\n".join(summary), flush=True)
    print(f"wrote {args.out} ({len(tuner.entries)} entries)", flush=True)


RAG_RE = re.compile(r"^\s+n=(\d+) count=(\d+)")
RAG_PASS_RE = re.compile(r"op\d+ pass \S+ L=(\d+) radices=([\dx]+) \S+ c=(\d+) T=(\d+) lds=\d+ tiles=(\d+) cols=(\d+)"
                         r" rin=(\d+) rout=(\d+) map=(\w+)(?: twN=\d+)?")


def plan_passes_ragged(desc: str, top: int, dtype: int = mf.FFT_F32):
    """Heaviest ragged pass keys (L, radices, c, key) of a ragged plan description,
    weighted by the points they process over the whole batch."""
    weights = {}
    count = 1
    for line in desc.splitlines():
        m = RAG_RE.match(line)
        if m:
            count = int(m.group(2))
            continue
        m = RAG_PASS_RE.search(line)
        if m:
            L, rad, c = int(m.group(1)), m.group(2), int(m.group(3))
            cols, mp = int(m.group(6)), m.group(9)
            tw = 1 if "twN=" in line else 0
            key = f"{dt_name(dtype, True)}:L{L}:{rad}:{mp}:tw{tw}"
            w, _, _ = weights.get(key, (0, L, c))
            weights[key] = (w + count * cols * L, (L, tuple(int(r) for r in rad.split("x"))), c)
    ranked = sorted(weights.items(), key=lambda kv: -kv[1][0])[:top]
    return [(v[1][0], v[1][1], v[2], k) for k, v in ranked]


if __name__ == "__main__":
    sys.exit(main())
