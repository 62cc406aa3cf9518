"""Throughput of the BLDTT compute phase on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload cube1e7] [--mode both|plain|fp32|tuned]
    python bench.py --sweep plain|tuned        # choose the operating points
    python bench.py --workload batch256        # 256 problems in one persistent graph launch

One step is one bldtt_compute: host traversal and list packing, upward pass,
PP/PC/CP/CC sums, downward pass and the scatter to caller order, with the
particles already resident in HBM.  The tree build (bldtt_setup) is outside
the timed region and reported as setup_ms.  The accuracy of each timed form
is measured afterwards against the direct sum on a random 0.1% of the targets
(GPU compensated direct sum, spot-checked against the CPU oracle).

Forms timed on the same particles:
  plain  FP64 evaluation, one degree n for every pair: the paper's method and
         arithmetic.  `value`, `dtype` and `roofline` are this form's.
  tuned  FP32 evaluation with every term added to FP64 sums, and a per-pair
         degree chosen by the GPU-trained model (models/coulomb_degree.bin);
         reported under forms.tuned with tuned_over_plain.
The other workloads of the build (1E6 cube in three forms, the unequal
Yukawa sets, the 256-problem batch, 1E8 with the learned degree) follow
under `extras` with a few steps each (--no-extras skips them).  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s (compute phase) at rel L2 err 1e-6, plain vs tuned BLDTT, N=1E7"
TARGET_ERR = 1e-6
FP64_VALU_PEAK = 78.6          # TFLOP/s, MI355X vector FP64
FP32_VALU_PEAK = 157.3         # TFLOP/s, MI355X vector FP32 (packed)
FLOPS_PER_EVAL = {"coulomb": 11, "yukawa": 15, "oscillatory": 15, "regcoulomb": 12, "poly": 8}
KERNEL_SOURCES = ("kernels.hip", "device.hpp", "batch.hip")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the interaction kernels' sources,
    without their `//` comments and trailing blanks (a comment edit leaves the
    code, and so the counter records, valid)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2012_06925_amd", "csrc", name), encoding="utf-8") as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _profile_record(name: str):
    """A committed rocprofv3 counter record, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec if rec.get("kernel_source_sha256_16") == kernel_source_hash() else None


def traffic_for(kernel_name: str, mode: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of the pass."""
    rec = _profile_record(f"traffic_{kernel_name}_{mode}.txt")
    return rec.get("bytes_per_launch") if rec else None


def counters_for(kernel_name: str, mode: str):
    """Counter-based vector/matrix FLOPs per launch of the pass (SQ_INSTS_VALU_*)."""
    rec = _profile_record(f"counters_{kernel_name}_{mode}.json")
    return rec.get("per_launch") if rec else None


# rocprofv3 counter passes: SQ_INSTS_VALU_FLOPS_* count wave instructions (x64
# lanes); SQ_INSTS_VALU_MFMA_MOPS_F64 counts FP64 matrix ops in units of 512.
PMC_PASSES = {
    "A": "SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU_FLOPS_FP64_TRANS "
         "SQ_INSTS_VALU_FLOPS_FP32_TRANS SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_F64 SQ_INSTS_VALU "
         "SQ_INSTS_VALU_CVT",
    "B": "SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_VALU_MFMA_BUSY_CYCLES SQ_VALU_MFMA_COEXEC_CYCLES SQ_WAVE_CYCLES "
         "SQ_WAVES SQ_INSTS_LDS SQ_ACTIVE_INST_LDS",
    "C": "FETCH_SIZE",
    "D": "WRITE_SIZE",
}
# the symmetric passes of the two timed forms, by kernel; where one kernel runs
# two passes, its dispatch groups (by grid) are told apart by duration, longest first
PMC_PASS_NAMES = {
    "plain": {"k_sym<false, false>": ("pp_sym", "pp_self"), "k_sym<false, true>": ("cc_sym",)},
    "tuned": {"k_sym_mfma<false, false>": ("pp_sym",), "k_sym_mfma<false, true>": ("pp_sym", "pp_self"),
              "k_sym_mfma<true, false>": ("cc_sym",)},
    "batch": {},                # the configuration of the last k_batch dispatch (the timed one)
}
# kernels whose records are kept, per mode (batch: every k_batch instance)
PMC_BATCH_PREFIX = "k_batch<"


def summarize_markers(db: str) -> None:
    """Markdown table of the library's host ranges (roctx) in a rocprofv3
    --marker-trace database: calls and durations per range name."""
    import collections
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select extdata, start, end from regions where category like '%MARKER%'").fetchall()
    agg = collections.defaultdict(list)
    for ext, t0, t1 in rows:
        agg[json.loads(ext).get("message", "?")].append((t1 - t0) / 1e6)
    print("| host range | calls | avg ms | min ms | max ms |")
    print("|---|---:|---:|---:|---:|")
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{name}` | {len(v)} | {sum(v) / len(v):.3f} | {min(v):.3f} | {max(v):.3f} |")


def summarize_pmc(prefix: str, mode: str) -> None:
    """Turn the four counter passes of `bench.py --mode MODE` (rocprofv3 output
    under PREFIX_A .. PREFIX_D, counters as PMC_PASSES) into the per-launch
    records the roofline reads (profiles/counters_<pass>_<prec>.json and
    profiles/traffic_<pass>_<prec>.txt), and print a table of the kernels."""
    import collections
    import re
    import sqlite3

    def short(n):
        n = re.sub(r"bldtt::\(anonymous namespace\)::", "", n)
        return re.sub(r"\(.*", "", n).replace("void ", "")

    groups = collections.defaultdict(lambda: collections.defaultdict(list))
    copy = {}
    last_batch = (-1, None)
    for tag in PMC_PASSES:
        con = sqlite3.connect(f"{prefix}_{tag}/pmc_results.db")
        rows = con.execute("select dispatch_id, kernel_name, grid_size, counter_name, value, duration "
                           "from counters_collection").fetchall()
        per = collections.defaultdict(dict)
        meta = {}
        for d, k, g, c, v, dur in rows:
            per[d][c] = per[d].get(c, 0.0) + v
            meta[d] = (short(k), g // 256, dur / 1e6)
        for d, cs in per.items():
            k, g, dur = meta[d]
            if k.startswith(PMC_BATCH_PREFIX) and d > last_batch[0]:
                last_batch = (d, (k, g))
            groups[(k, g)]["duration_ms"].append(dur)
            for c, v in cs.items():
                groups[(k, g)][c].append(v)
                if k == "__amd_rocclr_copyBuffer" and c in ("FETCH_SIZE", "WRITE_SIZE"):
                    copy[c] = max(copy.get(c, 0.0), v)
    avg = {key: {c: sum(v) / len(v) for c, v in r.items()} for key, r in groups.items()}
    calib_kib = (1 << 30) / 1024.0          # the 1024 MiB copy of --copy-calib-mib 1024
    scale = {c: calib_kib / copy[c] for c in ("FETCH_SIZE", "WRITE_SIZE")}
    prec = "fp64" if mode in ("plain", "batch") else "fp32"
    src_hash = kernel_source_hash()

    def derived(a):
        dur = a["duration_ms"]
        f64 = 64.0 * a.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
        f64t = 64.0 * a.get("SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0)
        f32 = 64.0 * (a.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0) + a.get("SQ_INSTS_VALU_FLOPS_FP32_TRANS", 0.0))
        mf = 512.0 * a.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        hbm = 1024.0 * (a["FETCH_SIZE"] * scale["FETCH_SIZE"] + a["WRITE_SIZE"] * scale["WRITE_SIZE"])
        return {"duration_ms": round(dur, 4), "valu_fp64_flops": f64, "valu_fp64_trans_flops": f64t,
                "valu_fp32_flops": f32, "mfma_f64_flops": mf,
                "fp64_tflops": round((f64 + f64t + mf) / dur / 1e9, 3),
                "fp64_frac_of_peak": round((f64 + f64t + mf) / dur / 1e9 / FP64_VALU_PEAK, 4),
                "fp32_tflops": round(f32 / dur / 1e9, 3),
                "hbm_bytes": hbm, "hbm_gb_per_s": round(hbm / dur / 1e6, 1),
                "raw": {c: v for c, v in sorted(a.items()) if c != "duration_ms"}}

    passes = collections.defaultdict(list)
    if mode == "batch" and last_batch[1]:
        passes["batch"].append(last_batch[1])
    for kname, names in PMC_PASS_NAMES[mode].items():
        keys = sorted((k for k in avg if k[0] == kname), key=lambda k: -avg[k]["duration_ms"])
        for name, key in zip(names, keys):
            passes[name].append(key)
    run = "--workload batch256 --steps 2 --warmup 1 --no-cpu" if mode == "batch" else \
        f"--mode {mode} --steps 2 --warmup 1 --no-cpu --no-extras"
    cmd = (f"python3 bench.py --summarize-pmc {prefix} --mode {mode}  (after: cd /tmp && timeout -s KILL 240 "
           f"rocprofv3 --pmc <PMC_PASSES[X]> -d {prefix}_X -o pmc -- python3 $R/bench.py {run} "
           f"[--copy-calib-mib 1024 for C, D], X = A B C D)")
    for name, keys in passes.items():
        tot = collections.Counter()
        for k in keys:
            tot.update(avg[k])
        rec = derived(dict(tot))
        raw = rec.pop("raw")
        with open(os.path.join(ROOT, "profiles", f"counters_{name}_{prec}.json"), "w") as f:
            json.dump({"pass": name, "mode": prec, "kernels": [f"{k}, grid {g} workgroups" for k, g in keys],
                       "kernel_source_sha256_16": src_hash, "command": cmd, "per_launch": rec,
                       "raw_counters_per_launch": raw}, f, indent=1)
        with open(os.path.join(ROOT, "profiles", f"traffic_{name}_{prec}.txt"), "w") as f:
            json.dump({"pass": name, "mode": prec, "kernel_source_sha256_16": src_hash,
                       "bytes_per_launch": rec["hbm_bytes"], "fetch_kib": tot["FETCH_SIZE"],
                       "write_kib": tot["WRITE_SIZE"], "fetch_scale": scale["FETCH_SIZE"],
                       "write_scale": scale["WRITE_SIZE"], "command": cmd}, f, indent=1)
    print(f"| kernel | grid (workgroups) | dispatches | avg ms | FP64 TFLOP/s (VALU + trans + MFMA) | "
          f"FP32 TFLOP/s | HBM GB/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for key in sorted(avg, key=lambda k: -avg[k]["duration_ms"] * len(groups[k]["duration_ms"]))[:10]:
        if "FETCH_SIZE" not in avg[key] or "SQ_INSTS_VALU" not in avg[key]:
            continue
        d = derived(avg[key])
        print(f"| `{key[0]}` | {key[1]} | {len(groups[key]['duration_ms']) // len(PMC_PASSES)} | "
              f"{d['duration_ms']:.3f} | {d['fp64_tflops']:.2f} | {d['fp32_tflops']:.2f} | {d['hbm_gb_per_s']:.0f} |")
    print(f"calibration: FETCH_SIZE x {scale['FETCH_SIZE']:.4f}, WRITE_SIZE x {scale['WRITE_SIZE']:.4f}; "
          f"passes {dict((k, [f'{a}@{b}' for a, b in v]) for k, v in passes.items())}")


def cpu_baseline(p, kernel, theta, degree, leaf, stride) -> dict:
    """The CPU oracle's compute phase on the benchmark's own particles: the
    traversal, upward and downward passes in full, the interaction sums on the
    leaves and clusters whose index is 0 modulo `stride` (a bounded sample),
    scaled by `stride`.  The oracle's tree build is setup and is not timed."""
    from oracle import core
    run = core.Run(p, p, kernel=kernel, theta=theta, degree=degree, leaf=leaf)
    t0 = time.perf_counter()
    run.traverse()
    t1 = time.perf_counter()
    run.upward()
    t2 = time.perf_counter()
    t_int = run.interact_sample(stride)
    t3 = time.perf_counter()
    run.downward()
    t4 = time.perf_counter()
    total = (t1 - t0) + (t2 - t1) + stride * t_int + (t4 - t3)
    return {"value": p.n / total, "unit": "particles/s", "cores": core.num_threads(), "kind": "oracle",
            "sample": f"the same {p.n} particles ({kernel}, theta={theta}, n={degree}, leaf={leaf}, FP64): traversal, "
                      f"upward and downward timed in full; PP/PC/CP/CC sums timed on every {stride}th leaf and "
                      f"cluster ({t_int:.2f} s) and scaled by {stride}; estimated compute phase {total:.1f} s",
            "phase_s": {"traverse": round(t1 - t0, 4), "upward": round(t2 - t1, 4),
                        "interact_sampled": round(t_int, 4), "interact_scaled": round(stride * t_int, 3),
                        "downward": round(t4 - t3, 4)}}


class Bench:
    """Timed forms of one particle problem: targets None (= sources) or (x, y, z)."""

    def __init__(self, args, kernel, leaf, tgt, src, seed, fraction=1e-3, minimum=1000):
        import torch
        from paper_2012_06925_amd import api, inputs
        self.torch, self.api = torch, api
        self.args, self.kernel, self.leaf, self.tgt, self.src = args, kernel, leaf, tgt, src
        self.M = (src if tgt is None else tgt)[0].numel()
        dev = src[0].device
        self.sel = inputs.error_sample(self.M, seed, fraction=fraction, minimum=min(self.M, minimum))
        sel_t = torch.from_numpy(self.sel).to(dev)
        t3 = src[:3] if tgt is None else tgt
        self.ds = api.direct_sum(t3, src, kernel=kernel, sel=sel_t).cpu().numpy()
        self.out = torch.empty(self.M, dtype=torch.float64, device=dev)
        self.model = None

    def plan(self, mode, theta, degree, tau=None, profile=False):
        from paper_2012_06925_amd import _lib
        flags = _lib.PROFILE if profile else 0
        if self.args.valu_passes:
            flags |= _lib.VALU_PASSES
        if self.args.mfma_leaf:
            flags |= _lib.MFMA_LEAF
        if self.args.device_traversal:
            flags |= _lib.DEVICE_TRAVERSAL
        if not self.args.host_tree:
            flags |= _lib.DEVICE_TREE
        if mode in ("fp32", "tuned"):
            flags |= _lib.FP32_EVAL
        if mode == "tuned":
            flags |= _lib.LEARNED_DEGREE
        t0 = time.perf_counter()
        plan = self.api.Plan(self.tgt, self.src, kernel=self.kernel, theta=theta, degree=degree, leaf=self.leaf,
                             flags=flags)
        setup_ms = (time.perf_counter() - t0) * 1e3
        if mode == "tuned":
            if self.model is None:
                from paper_2012_06925_amd.train_degree_model import load_model
                self.model = load_model(self.args.model)
            plan.set_degree_model(self.model, fallback=degree, tau=tau)
        return plan, setup_ms

    def error(self) -> float:
        phi = self.out.cpu().numpy()
        return float(np.sqrt(np.sum((phi[self.sel] - self.ds) ** 2) / np.sum(self.ds ** 2)))

    def time_plan(self, plan, steps, warmup):
        torch = self.torch
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            plan.compute(self.out)
        torch.cuda.synchronize()
        base = plan.stats()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            plan.compute(self.out)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - w0) * 1e3 / steps
        ms = ev0.elapsed_time(ev1) / steps
        st = plan.stats()
        n_prof = st["profiled_computes"] - base["profiled_computes"]
        phase = {k: (st["phase_ms"][k] - base["phase_ms"][k]) / max(1, n_prof) for k in st["phase_ms"]}
        return ms, wall_ms, phase, st

    def form(self, mode, theta, degree, tau=None, steps=None, warmup=None):
        steps = self.args.steps if steps is None else steps
        warmup = self.args.warmup if warmup is None else warmup
        plan, setup_ms = self.plan(mode, theta, degree, tau, profile=True)
        ms, wall_ms, phase, st = self.time_plan(plan, steps, warmup)
        err = self.error()
        plan.close()
        rec = {"mode": mode, "theta": theta, "degree": degree, "particles_per_s": self.M / (ms * 1e-3),
               "ms_per_step": round(ms, 3), "wall_ms_per_step": round(wall_ms, 3), "steps": steps,
               "error_vs_direct": err, "setup_ms": round(setup_ms, 1),
               "phase_ms": {k: round(v, 4) for k, v in phase.items()},
               "traverse_ms": round(st["traverse_ms"], 3), "host_marks_ms": [round(v, 3) for v in st["host_marks_ms"]],
               "interactions": st["interactions"], "n_entries": st["n_entries"],
               "roofline": roofline(mode, self.kernel, st, phase)}
        if mode != "plain":
            rec["fp64_close_pairs"] = st["fp64_close_pairs"]
        if mode == "tuned":
            rec.update(tau=tau, sep_pairs=st["sep_pairs"], sep_direct=st["sep_direct"],
                       sep_fallback=st["sep_fallback"], pairs_per_degree=st["pairs_per_degree"],
                       down_degree=st["down_degree"])
        log(f"{mode}: {ms:.2f} ms/step err {err:.3e} phases {rec['phase_ms']}")
        return rec

    def sweep(self, mode):
        rows = []
        leaves = self.args.sweep_leaves or [self.leaf]
        if mode == "plain":
            grid = [(lf, th, n, None) for lf in leaves for th in self.args.sweep_thetas for n in self.args.sweep_degrees]
        else:
            grid = [(lf, th, self.args.tuned_fallback, tau) for lf in leaves for th in self.args.sweep_thetas
                    for tau in self.args.sweep_taus]
        for lf, th, n, tau in grid:
            self.leaf = lf
            plan, _ = self.plan("tuned" if mode == "tuned" else "plain", th, n, tau)
            ms, wall, _, st = self.time_plan(plan, self.args.steps, 1)
            err = self.error()
            plan.close()
            row = {"leaf": lf, "theta": th, "degree": n, "tau": tau, "ms": round(ms, 2), "err": err,
                   "particles_per_s": self.M / (ms * 1e-3), "interactions": st["interactions"]}
            if mode == "tuned":
                row.update(sep_direct=st["sep_direct"], pairs_per_degree=st["pairs_per_degree"])
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
        ok = [r for r in rows if r["err"] <= TARGET_ERR]
        best = min(ok, key=lambda r: r["ms"]) if ok else None
        return {"sweep": mode, "workload": self.args.workload, "M": self.M, "best": best, "rows": rows}


def roofline(mode, kernel, st, phase) -> dict:
    """Roofline of the dominant pass.  `achieved` is algorithmic: the pass's
    kernel terms from the lists (both directions of a symmetric pair, the
    method's count) x the flops per term, over the pass's duration (HIP events
    on the pass's own stream).  `evaluated_per_s` counts the kernel values the
    pass computes (a symmetric pass computes one value for two terms), and
    `counters` holds the rocprofv3 instruction-counter figures of the pass
    when they were taken on the current kernel source."""
    inter = st["interactions"]
    fl = FLOPS_PER_EVAL[kernel]
    # the particle pass (near-field PP in the per-pair degree form), its second
    # pass (separated pairs' PP/PC), the symmetric PP pass, the proxy pass, and
    # the pass over each leaf with itself that runs before the traversal
    terms = {"pp_pc": st["pass_interactions"][0], "pp_pc_sep": st["pass_interactions"][1],
             "pp_sym": st["pass_interactions"][2], "cp_cc": inter["CP"] + inter["CC"],
             "pp_self": st["pass_interactions"][4]}
    dom = max(terms, key=lambda k: phase[k])
    sec = phase[dom] * 1e-3
    achieved = terms[dom] * fl / sec / 1e12
    fp32 = mode != "plain"
    peak = FP32_VALU_PEAK if fp32 else FP64_VALU_PEAK
    prec = "fp32" if fp32 else "fp64"
    values = terms[dom] / (2.0 if dom == "pp_sym" else 1.0)
    return {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic_for(dom, prec),
            "flops_per_launch": terms[dom] * fl, "launch_ms": round(phase[dom], 4), "flops_per_term": fl,
            "terms_per_s": round(terms[dom] / sec, 1), "evaluated_per_s": round(values / sec, 1),
            "counters": counters_for(dom, prec)}


BATCH_METRIC = "particles/s (compute phase), 256 uneven problems in one persistent graph launch"


def batch_bench(args, wl, name, steps, warmup, with_cpu=True) -> dict:
    """One graph launch of the batched persistent kernel per step, against the
    same problems run one after another (bldtt_compute each)."""
    import tempfile

    import torch
    from paper_2012_06925_amd import _lib, api, inputs
    dev = torch.device("cuda:0")
    theta = args.theta if args.theta is not None and args.workload == name else wl["theta"]
    degree = args.degree if args.degree is not None and args.workload == name else wl["degree"]
    leaf = args.leaf if args.leaf is not None and args.workload == name else wl["leaf"]
    probs = inputs.batch_problems(count=wl["count"], seed=inputs.workload_seed(name), lo_exp=wl["lo_exp"],
                                  hi_exp=wl["hi_exp"])
    sets = [p for _, p in probs]
    total = sum(p.n for p in sets)
    log(f"{len(sets)} problems, {total} particles")
    dsets = [(None, tuple(torch.from_numpy(a).to(dev) for a in (p.x, p.y, p.z, p.q))) for p in sets]
    kw = dict(kernel=wl["kernel"], theta=theta, degree=degree, leaf=leaf)
    outs = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in sets]
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # the same problems one after another (plans built outside the timed region)
    plans = [api.Plan(t, s, **kw) for t, s in dsets]
    for pl, o in zip(plans, outs):
        pl.compute(o)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for pl, o in zip(plans, outs):
        pl.compute(o)
    ev1.record(stream)
    torch.cuda.synchronize()
    seq_wall = (time.perf_counter() - w0) * 1e3
    seq_ms = ev0.elapsed_time(ev1)
    seq_traverse = sum(pl.stats()["traverse_ms"] for pl in plans)
    seq_phi = [o.clone() for o in outs]
    for pl in plans:
        pl.close()
    log(f"sequential: {seq_ms:.2f} ms (wall {seq_wall:.2f}, host traversal {seq_traverse:.2f})")

    # the batch: autotuned tile, one graph launch per step
    cache = args.tune_cache or os.path.join(tempfile.gettempdir(), "bldtt_tune_cache.txt")
    api.set_tune_cache(cache)
    t0 = time.perf_counter()
    b = api.Batch(dsets, flags=_lib.AUTOTUNE, **kw)
    setup_ms = (time.perf_counter() - t0) * 1e3
    st = b.stats()
    log(f"batch setup {setup_ms:.0f} ms, tile tpt={st['tpt']} groups/CU={st['groups_per_cu']} "
        f"(tuned={st['tuned']}), {st['n_tasks']} tasks")
    for _ in range(warmup):
        b.compute(outs)
    b.check()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        b.compute(outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) * 1e3 / steps
    ms = ev0.elapsed_time(ev1) / steps
    b.check()
    parity = max(float((o - r).abs().max() / r.abs().max()) for o, r in zip(outs, seq_phi))
    # accuracy against the direct sum on 0.1% of each problem's targets (at least 8)
    num = den = 0.0
    worst = 0.0
    for i, (p, o) in enumerate(zip(sets, outs)):
        sel = inputs.error_sample(p.n, inputs.workload_seed(name) + 7 * i, fraction=1e-3, minimum=min(p.n, 8))
        src = dsets[i][1]
        ds = api.direct_sum(src[:3], src, kernel=wl["kernel"], sel=torch.from_numpy(sel).to(dev)).cpu().numpy()
        got = o.cpu().numpy()[sel]
        e2, d2 = float(np.sum((got - ds) ** 2)), float(np.sum(ds ** 2))
        num, den = num + e2, den + d2
        worst = max(worst, np.sqrt(e2 / d2))
    err = float(np.sqrt(num / den))
    inter = st["interactions"]
    fl = FLOPS_PER_EVAL[wl["kernel"]]
    work = sum(inter.values()) * fl
    achieved = work / (ms * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": "k_batch (every phase, one launch)", "achieved": round(achieved, 3),
            "peak": FP64_VALU_PEAK, "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK, 4),
            "traffic": traffic_for("batch", "fp64"), "flops_per_launch": work, "launch_ms": round(ms, 4),
            "flops_per_term": fl, "counters": counters_for("batch", "fp64")}
    b.close()
    cpu = None
    if with_cpu:
        k = args.cpu_problems
        from oracle import core
        t0 = time.perf_counter()
        for p in sets[:k]:
            core.Run(p, p, kernel=wl["kernel"], theta=theta, degree=degree, leaf=leaf).run_all()
        wall_cpu = time.perf_counter() - t0
        n_cpu = sum(p.n for p in sets[:k])
        cpu = {"value": n_cpu / wall_cpu, "unit": "particles/s", "cores": core.num_threads(), "kind": "oracle",
               "sample": f"the first {k} of the {len(sets)} problems ({n_cpu} particles), one after another, "
                         f"FP64 ({wall_cpu:.2f} s)"}
    return {
        "metric": BATCH_METRIC, "value": total / (ms * 1e-3), "unit": "particles/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "problems": len(sets), "particles": total, "kernel": wl["kernel"],
                   "theta": theta, "degree": degree, "leaf": leaf},
        "error_vs_direct": err, "worst_problem_error": worst, "batch_vs_sequential_maxrel": parity,
        "wall_ms_per_step": round(wall, 3), "setup_ms": round(setup_ms, 1),
        "tile": {"tpt": st["tpt"], "groups_per_cu": st["groups_per_cu"], "grid": st["grid"], "tuned": st["tuned"],
                 "tune_ms": round(st["tune_ms"], 1)},
        "n_tasks": st["n_tasks"], "interactions": inter,
        "sequential": {"ms": round(seq_ms, 3), "wall_ms": round(seq_wall, 3), "host_traversal_ms": round(seq_traverse, 3),
                       "particles_per_s": total / (seq_ms * 1e-3)},
        "batch_over_sequential": seq_ms / ms,
        "roofline": roof, "cpu_baseline": cpu,
    }


def _dev_set(p, dev, charges=True):
    import torch
    arrays = (p.x, p.y, p.z, p.q) if charges else (p.x, p.y, p.z)
    return tuple(torch.from_numpy(a).to(dev) for a in arrays)


def ablation(args) -> dict:
    """Sec. 4.3's ablation: the BLDTT with all four interaction types against
    the variant that keeps only CC and PP (PC/CP pairs become PP), plain
    FP64, on a uniform and a Gaussian set: per-type list entries, kernel
    evaluations (the pointwise-interaction counts), compute time and error."""
    from paper_2012_06925_amd import _lib, inputs
    dev = __import__("torch").device("cuda:0")
    n = args.n or 1_000_000
    theta = args.theta if args.theta is not None else 0.7
    degree = args.degree if args.degree is not None else 8
    leaf = args.leaf if args.leaf is not None else 2000
    out = {"M": n, "theta": theta, "degree": degree, "leaf": leaf}
    for dist in ("uniform", "gaussian"):
        seed = inputs.BASE_SEED + 400 + (dist == "gaussian")
        p = inputs.particles(n, dist, seed=seed)
        b = Bench(args, "coulomb", leaf, None, _dev_set(p, dev), seed)
        rows = {}
        for name, extra in (("all_four", 0), ("pp_cc_only", _lib.PP_CC_ONLY)):
            from paper_2012_06925_amd import api
            flags = _lib.PROFILE | extra
            pl = api.Plan(None, b.src, kernel="coulomb", theta=theta, degree=degree, leaf=leaf, flags=flags)
            ms, _, phase, st = b.time_plan(pl, args.steps, args.warmup)
            err = b.error()
            pl.close()
            rows[name] = {"ms_per_step": round(ms, 3), "particles_per_s": n / (ms * 1e-3), "error_vs_direct": err,
                          "n_entries": st["n_entries"], "interactions": st["interactions"],
                          "total_interactions": sum(st["interactions"].values()),
                          "phase_ms": {k: round(v, 3) for k, v in phase.items()}}
            log(f"ablation {dist} {name}: {ms:.2f} ms err {err:.2e} interactions {rows[name]['interactions']}")
        rows["speedup_all_four"] = rows["pp_cc_only"]["ms_per_step"] / rows["all_four"]["ms_per_step"]
        rows["interaction_ratio"] = rows["pp_cc_only"]["total_interactions"] / rows["all_four"]["total_interactions"]
        out[dist] = rows
    return {"ablation": out}


def treecodes(args) -> dict:
    """Sec. 4.5's comparison on unequal uniform sets, (a) M = 2E7 targets with
    N = 2E6 sources and (b) M = 2E6 with N = 2E7: the BLDTT against the
    particle-cluster treecode BLTC (Sec. 2.8) and the cluster-particle treecode
    CP-BLTC, plain FP64, one (theta, n) per --treecode-grid entry: compute
    time, error against the direct sum and per-type interaction counts."""
    from paper_2012_06925_amd import _lib, api, inputs
    dev = __import__("torch").device("cuda:0")
    leaf = args.leaf if args.leaf is not None else 2000
    grid = [(float(a), int(b)) for a, b in (e.split(":") for e in args.treecode_grid.split(","))]
    out = {"leaf": leaf, "grid": grid}
    for name, M, N in (("a_M2e7_N2e6", 20_000_000, 2_000_000), ("b_M2e6_N2e7", 2_000_000, 20_000_000)):
        seed = inputs.BASE_SEED + 500 + (name[0] == "b")
        t, s = inputs.unequal_sets(M, "uniform", N, "uniform", seed=seed)
        b = Bench(args, "coulomb", leaf, _dev_set(t, dev, charges=False), _dev_set(s, dev), seed)
        del t, s
        rows = []
        for theta, degree in grid:
            for method, flag in (("bldtt", 0), ("bltc", _lib.BLTC), ("cp_bltc", _lib.CP_BLTC)):
                pl = api.Plan(b.tgt, b.src, kernel="coulomb", theta=theta, degree=degree, leaf=leaf,
                              flags=_lib.PROFILE | flag)
                ms, _, phase, st = b.time_plan(pl, args.steps, args.warmup)
                err = b.error()
                pl.close()
                rows.append({"method": method, "theta": theta, "degree": degree, "ms_per_step": round(ms, 3),
                             "error_vs_direct": err, "interactions": st["interactions"],
                             "n_entries": st["n_entries"], "phase_ms": {k: round(v, 3) for k, v in phase.items()}})
                log(f"treecodes {name} {method} theta={theta} n={degree}: {ms:.2f} ms err {err:.2e}")
        out[name] = rows
    return {"treecodes": out}


def extras(args) -> dict:
    """The build's other workloads, a few steps each: the 1E6 cube in its three
    forms, the unequal Yukawa sets, the 256-problem batch and 1E8 with the
    learned degree (the workload's theta 0.8 and the faster 0.87)."""
    import torch
    from paper_2012_06925_amd import inputs
    dev = torch.device("cuda:0")
    steps, warmup = args.extra_steps, 1
    out = {}

    def guarded(name, fn):
        t0 = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as e:      # an extra never hides the headline; its failure is reported
            traceback.print_exc()
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"extra {name} done in {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    def cube1e6():
        wl = inputs.WORKLOADS["cube1e6"]
        seed = inputs.workload_seed("cube1e6")
        p = inputs.particles(wl["M"], "uniform", seed=seed)
        b = Bench(args, "coulomb", wl["leaf"], None, _dev_set(p, dev), seed)
        r = {"M": wl["M"], "N": wl["M"]}
        for mode in ("plain", "fp32", "tuned"):
            r[mode] = b.form(mode, wl["theta"], wl["degree"], wl.get("tau") if mode == "tuned" else None, steps, warmup)
        r["fp32_over_plain"] = r["fp32"]["particles_per_s"] / r["plain"]["particles_per_s"]
        r["tuned_over_plain"] = r["tuned"]["particles_per_s"] / r["plain"]["particles_per_s"]
        return r

    def unequal():
        name = "sphere2e6_gauss1e7"
        wl = inputs.WORKLOADS[name]
        seed = inputs.workload_seed(name)
        t, s = inputs.unequal_sets(wl["M"], wl["tdist"], wl["N"], wl["sdist"], seed=seed)
        b = Bench(args, wl["kernel"], wl["leaf"], _dev_set(t, dev, False), _dev_set(s, dev), seed)
        r = {"M": wl["M"], "N": wl["N"], "kernel": wl["kernel"]}
        for mode in ("fp32", "plain"):
            r[mode] = b.form(mode, wl["theta"], wl["degree"], None, steps, warmup)
        r["fp32_over_plain"] = r["fp32"]["particles_per_s"] / r["plain"]["particles_per_s"]
        return r

    def batch():
        name = "batch256"
        return batch_bench(args, inputs.WORKLOADS[name], name, steps, warmup, with_cpu=False)

    def cube1e8():
        name = "cube1e8"
        wl = inputs.WORKLOADS[name]
        seed = inputs.workload_seed(name)
        p = inputs.particles(wl["M"], "uniform", seed=seed)
        src = _dev_set(p, dev)
        del p
        b = Bench(args, "coulomb", wl["leaf"], None, src, seed, fraction=1e-4, minimum=1000)
        r = {"M": wl["M"], "N": wl["M"]}
        r["tuned"] = b.form("tuned", wl["theta"], wl["tuned_fallback"], wl["tau"], 1, 1)
        r["tuned_fast"] = b.form("tuned", wl["tuned_theta"], wl["tuned_fallback"], wl["tau"], 1, 1)
        r["plain"] = b.form("plain", wl["theta"], wl["degree"], None, 1, 1)
        r["tuned_over_plain"] = r["tuned_fast"]["particles_per_s"] / r["plain"]["particles_per_s"]
        return r

    guarded("cube1e6", cube1e6)
    guarded("sphere2e6_gauss1e7", unequal)
    guarded("batch256", batch)
    if not args.no_1e8:
        guarded("cube1e8", cube1e8)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube1e7")
    ap.add_argument("--n", type=int, default=None, help="override the particle count")
    ap.add_argument("--mode", default="both", choices=("both", "plain", "fp32", "tuned", "batch"),
                    help="batch: only with --summarize-pmc")
    ap.add_argument("--theta", type=float, default=None, help="plain form")
    ap.add_argument("--degree", type=int, default=None, help="plain form")
    ap.add_argument("--tuned-theta", type=float, default=None)
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--tuned-fallback", type=int, default=None)
    ap.add_argument("--leaf", type=int, default=None)
    ap.add_argument("--model", default=None)
    ap.add_argument("--cpu-stride", type=int, default=32,
                    help="CPU baseline: interaction sums timed on every k-th leaf and cluster, scaled by k")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-1e8", action="store_true", help="skip the 1E8 workload among the extras")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--sweep", choices=("plain", "tuned"), default=None)
    ap.add_argument("--ablation", action="store_true",
                    help="all four interaction types vs PP + CC only (plain FP64, uniform and Gaussian)")
    ap.add_argument("--summarize-pmc", default=None, metavar="PREFIX",
                    help="write the profiles/ counter records from rocprofv3 passes PREFIX_A .. PREFIX_D of --mode")
    ap.add_argument("--summarize-markers", default=None, metavar="DB",
                    help="print the host ranges of a rocprofv3 --marker-trace database as a table")
    ap.add_argument("--treecodes", action="store_true",
                    help="Sec. 4.5: BLDTT vs BLTC vs CP-BLTC on unequal uniform sets (2E7/2E6 and 2E6/2E7)")
    ap.add_argument("--treecode-grid", default="0.7:8", help="comma list of theta:degree for --treecodes")
    ap.add_argument("--sweep-thetas", default="0.5,0.6,0.7,0.8,0.9")
    ap.add_argument("--sweep-degrees", default="4,5,6,7,8,9,10")
    ap.add_argument("--sweep-taus", default="3e-8,1e-7,3e-7,1e-6,3e-6")
    ap.add_argument("--sweep-leaves", default=None, help="comma list; default: the workload's leaf size")
    ap.add_argument("--valu-passes", action="store_true",
                    help="run the up/down transfers on the vector ALUs instead of the matrix cores")
    ap.add_argument("--device-traversal", action="store_true", help="build the lists on the GPU (BLDTT_DEVICE_TRAVERSAL)")
    ap.add_argument("--host-tree", action="store_true",
                    help="build the trees on the host at setup (default: on the GPU, BLDTT_DEVICE_TREE)")
    ap.add_argument("--mfma-leaf", action="store_true",
                    help="run the leaf contractions on the matrix cores instead of the vector ALUs")
    ap.add_argument("--cpu-problems", type=int, default=16, help="batch workloads: problems in the CPU sample")
    ap.add_argument("--tune-cache", default=None, help="batch workloads: autotune cache file")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    args.sweep_thetas = [float(x) for x in args.sweep_thetas.split(",")]
    args.sweep_degrees = [int(x) for x in args.sweep_degrees.split(",")]
    args.sweep_taus = [float(x) for x in args.sweep_taus.split(",")]
    args.sweep_leaves = [int(x) for x in args.sweep_leaves.split(",")] if args.sweep_leaves else None

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        return 2
    if args.summarize_markers:
        summarize_markers(args.summarize_markers)
        return 0

    import torch
    from paper_2012_06925_amd import inputs
    from paper_2012_06925_amd.train_degree_model import DEFAULT_MODEL

    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.mode)
        return 0
    args.model = args.model or DEFAULT_MODEL
    if args.ablation:
        print(json.dumps(ablation(args)), flush=True)
        return 0
    if args.treecodes:
        print(json.dumps(treecodes(args)), flush=True)
        return 0
    wl = dict(inputs.WORKLOADS[args.workload])
    dev = torch.device("cuda:0")
    if args.copy_calib_mib:
        a = torch.empty(args.copy_calib_mib * 2 ** 20 // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calib_mib} MiB done")
        del a, b
    if "count" in wl:
        print(json.dumps(batch_bench(args, wl, args.workload, args.steps, args.warmup, not args.no_cpu)), flush=True)
        return 0
    if "dist" not in wl:
        raise SystemExit("the headline workloads are targets = sources; unequal sets run among the extras")
    M = args.n or wl["M"]
    args.theta = args.theta if args.theta is not None else wl["theta"]
    args.degree = args.degree if args.degree is not None else wl["degree"]
    args.leaf = args.leaf if args.leaf is not None else wl["leaf"]
    args.tuned_theta = args.tuned_theta if args.tuned_theta is not None else wl.get("tuned_theta", args.theta)
    args.tau = args.tau if args.tau is not None else wl.get("tau", 3e-7)
    args.tuned_fallback = args.tuned_fallback if args.tuned_fallback is not None else wl.get("tuned_fallback", 8)
    seed = inputs.workload_seed(args.workload)

    log(f"generating {M} {wl['dist']} particles")
    p = inputs.particles(M, wl["dist"], seed=seed)
    src = _dev_set(p, dev)
    torch.cuda.synchronize()
    bench = Bench(args, wl["kernel"], args.leaf, None, src, seed)

    if args.sweep:
        print(json.dumps(bench.sweep(args.sweep)), flush=True)
        return 0

    forms = {}
    if args.mode in ("both", "plain"):
        forms["plain"] = bench.form("plain", args.theta, args.degree)
    if args.mode == "fp32":
        forms["fp32"] = bench.form("fp32", args.theta, args.degree)
    if args.mode in ("both", "tuned"):
        forms["tuned"] = bench.form("tuned", args.tuned_theta, args.tuned_fallback, args.tau)

    # spot check of the GPU direct sum against the CPU oracle's compensated direct sum
    ds_check = None
    if not args.no_cpu:
        from oracle import core
        ref = core.direct_sum(p, p, kernel=wl["kernel"], sel=bench.sel[:8])
        ds_check = float(np.max(np.abs(bench.ds[:8] - ref) / np.abs(ref)))

    head = forms.get("plain") or next(iter(forms.values()))
    cpu = None
    if not args.no_cpu:
        log(f"CPU oracle baseline on the same {M} particles (interaction sums sampled 1/{args.cpu_stride})")
        cpu = cpu_baseline(p, wl["kernel"], args.theta, args.degree, args.leaf, args.cpu_stride)
        log(f"CPU oracle: {cpu['value']:.3e} particles/s on {cpu['cores']} threads")
    del p
    ext = None
    if not args.no_extras:
        del bench
        torch.cuda.empty_cache()
        ext = extras(args)

    dtype = {"plain": "f64", "fp32": "f32-eval/f64-acc", "tuned": "f32-eval/f64-acc"}[head["mode"]]
    res = {
        "metric": METRIC, "value": head["particles_per_s"], "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "M": M, "N": M, "distribution": wl["dist"], "kernel": wl["kernel"],
                   "leaf": args.leaf, "mode": head["mode"], "theta": head["theta"], "degree": head["degree"],
                   "tau": head.get("tau")},
        "error_vs_direct": head["error_vs_direct"], "direct_sum_cpu_check_maxrel": ds_check,
        "roofline": head["roofline"], "cpu_baseline": cpu, "setup_ms": head["setup_ms"],
        "forms": forms,
        "tuned_over_plain": (forms["tuned"]["particles_per_s"] / forms["plain"]["particles_per_s"]
                             if "tuned" in forms and "plain" in forms else None),
        "extras": ext,
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
