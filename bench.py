#!/usr/bin/env python3
"""Throughput of the LiFE hot path on one MI355X.

A step is one SBB-NNLS iteration (Algorithm 1) through the C ABI: two DSC
(y = M w), one or two WC (g = M^T y; two on even iterations) and the step
glue, on the synthetic full-scale connectome (N_theta = 96, N_a = 1057,
~300k voxels, 1.5M fascicles, ~90M nonzeros) with every input resident in HBM.
The plan (restructuring) is built once before the timed region.

Output: one JSON line.  ``value`` = Phi nonzeros per second per DSC+WC pair:
nnz * (DSC calls + WC calls) / 2 / wall time of the K timed iterations (glue
included).  ``roofline`` covers the kernel with the largest share of the time,
from HIP events recorded around every launch of the timed region on the
launch stream; ``cpu_baseline`` times the FP64 oracle (DSC + WC) on a bounded
random sample of the same nonzeros.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the multi-threaded CPU oracle keeps its threads on neighbouring cores (read when
# the OpenMP runtime starts, so set before anything loads it)
os.environ.setdefault("OMP_PROC_BIND", "close")

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# what the path computes in: float32 data and sums; the dense projections inside WC
# are exact integer sums of 8-bit digit products on the matrix cores, rounded once
ARITHMETIC = "f32; WC projections exact int8-MFMA digit products of 30-bit fixed-point D and y, rounded once"
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector; a plain v_fma_f32 loop reached 132 TFLOP/s here


# rocprofv3 commands whose outputs --summarize reads (run from /tmp with
# TMPDIR=/tmp; the synthetic connectome cached through LIFE_SYNTH_CACHE)
# SQ counters, two passes (at most 8 SQ counters per run)
SQ_PASS1 = ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU",
            "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_MISC")
SQ_PASS2 = ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_SALU",
            "SQ_LDS_IDX_ACTIVE", "SQ_WAVES", "SQ_INSTS_MFMA")


def profile_commands(config: str) -> dict:
    """The rocprofv3 runs behind profiles/<config>_*: a kernel trace, then FETCH_SIZE,
    WRITE_SIZE and the L2 hit counters in runs of their own, and the copy probe that
    calibrates the byte counters."""
    cfg = "" if config == "full" else f" --config {config}"
    out = "$R/gpurun_out/prof" + ("" if config == "full" else f"_{config}")
    run = f"python3 $R/bench.py{cfg}"
    short = f"{run} --steps 2 --warmup 1 --no-cpu-baseline --no-extras"
    return {
        "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d {out}/trace -o run -- "
                 f"{run} --steps 6 --warmup 2 --no-cpu-baseline --no-extras",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/fetch -o run -- {short}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/write -o run -- {short}",
        "tcc": f"rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --output-format csv -d {out}/tcc -o run -- {short}",
        "sq1": f"rocprofv3 --pmc {' '.join(SQ_PASS1)} --output-format csv -d {out}/sq1 -o run -- {short}",
        "sq2": f"rocprofv3 --pmc {' '.join(SQ_PASS2)} --output-format csv -d {out}/sq2 -o run -- {short}",
        "copyf": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/copyf -o run -- "
                 "python3 $R/bench.py --copy-probe",
        "copyw": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/copyw -o run -- "
                 "python3 $R/bench.py --copy-probe",
    }


PROFILE_COMMANDS = profile_commands("full")
KIND_KERNELS = {"dsc": ("k_dsc_chunk", "k_dsc"), "wc_z": ("k_wcr_mfma", "k_wc_z"), "wc_sum": ("k_wc_sum",)}
# profiling classes launched by the same kernel (the second WC of even iterations)
KIND_GROUPS = {"dsc": ("dsc",), "wc_z": ("wc_z", "wc_z_2nd"), "wc_sum": ("wc_sum", "wc_sum_2nd")}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """SHA-256 of the library sources: counters recorded for other sources are stale."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1905_06234_amd", "csrc", "*"))) + \
        [os.path.join(ROOT, "include", "life.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name: str) -> str:
    m = re.search(r"(k_[a-z_0-9]+(<\d+>)?|__amd_rocclr_\w+)", name)
    return m.group(1) if m else name[:40]


def _counter_means(d: str):
    """{kernel: (dispatches, mean value)} over the counter rows of a rocprofv3 csv run."""
    acc = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            k = (_short(r["Kernel_Name"]), r["Counter_Name"])
            n, t = acc.get(k, (0, 0.0))
            acc[k] = (n + 1, t + float(r["Counter_Value"]))
    return {k: (n, t / n) for k, (n, t) in acc.items()}


def summarize(prof_dir: str, workload: str):
    """Turn the rocprofv3 outputs of PROFILE_COMMANDS into profiles/<workload>_*.{md,json}."""
    stats = {}
    for path in glob.glob(os.path.join(prof_dir, "trace", "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            stats[_short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]))
    fetch, write = _counter_means(os.path.join(prof_dir, "fetch")), _counter_means(os.path.join(prof_dir, "write"))
    tcc = _counter_means(os.path.join(prof_dir, "tcc"))
    cf, cw = _counter_means(os.path.join(prof_dir, "copyf")), _counter_means(os.path.join(prof_dir, "copyw"))
    copy_bytes = 256 << 20

    def copy_kib(m, counter):
        vals = [v for (k, c), (n, v) in m.items() if c == counter and "copyBuffer" in k]
        return max(vals) if vals else None
    ckf, ckw = copy_kib(cf, "FETCH_SIZE"), copy_kib(cw, "WRITE_SIZE")
    ff = copy_bytes / (ckf * 1024) if ckf else None
    fw = copy_bytes / (ckw * 1024) if ckw else None
    kernels = {}
    for name in sorted({k for (k, c) in fetch} | set(stats)):
        if not name.startswith("k_"):
            continue
        e = {"calls_traced": stats.get(name, (0, 0))[0], "avg_us": round(stats.get(name, (0, 0.0))[1] / 1e3, 2)}
        if (name, "FETCH_SIZE") in fetch and (name, "WRITE_SIZE") in write and ff and fw:
            fk, wk = fetch[(name, "FETCH_SIZE")][1], write[(name, "WRITE_SIZE")][1]
            e.update({"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                      "hbm_bytes": int(fk * 1024 * ff + wk * 1024 * fw)})
        if (name, "TCC_HIT_sum") in tcc and (name, "TCC_MISS_sum") in tcc:
            hit, miss = tcc[(name, "TCC_HIT_sum")][1], tcc[(name, "TCC_MISS_sum")][1]
            e["l2_hit_rate"] = round(hit / max(hit + miss, 1.0), 4)
        kernels[name] = e
    rec = {"workload": workload, "source_sha256": source_hash(),
           "copy_probe": {"bytes_each_way": copy_bytes, "fetch_kib": ckf, "write_kib": ckw,
                          "fetch_factor": ff, "write_factor": fw},
           "kernels": kernels, "commands": profile_commands(workload)}
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"{workload}_counters.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# Kernel times and HBM traffic, {workload} synthetic connectome", "",
             "Per-dispatch averages. Times: `rocprofv3 --kernel-trace --stats`. Bytes: `FETCH_SIZE` and",
             "`WRITE_SIZE` (KiB per dispatch, separate runs), scaled by what the same counters read for a",
             (f"plain 256 MiB device copy (`bench.py --copy-probe`): fetch x{ff:.3f}, write x{fw:.3f}." if ff and fw
              else "plain 256 MiB device copy (`bench.py --copy-probe`): calibration missing."), "",
             "| kernel | calls (trace) | avg us | FETCH KiB | WRITE KiB | HBM GB (scaled) | L2 hit |",
             "|---|---|---|---|---|---|---|"]
    for name, e in kernels.items():
        gb = f"{e['hbm_bytes'] / 1e9:.3f}" if "hbm_bytes" in e else "-"
        lines.append(f"| `{name}` | {e['calls_traced']} | {e['avg_us']} | {e.get('fetch_kib', '-')} | "
                     f"{e.get('write_kib', '-')} | {gb} | {e.get('l2_hit_rate', '-')} |")
    lines += ["", f"Library source SHA-256: `{rec['source_sha256']}`", "",
              "Commands (repository root `$R`; run from `/tmp` with `TMPDIR=/tmp`,",
              "`LIFE_SYNTH_CACHE=/tmp/life_synth`), then "
              f"`python3 bench.py{'' if workload == 'full' else ' --config ' + workload} --summarize "
              f"$R/gpurun_out/prof{'' if workload == 'full' else '_' + workload}`:", ""]
    lines += [f"    {c}" for k, c in profile_commands(workload).items() if not k.startswith("sq")]
    with open(os.path.join(out_dir, f"{workload}_kernels.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    sq = {}
    for d in ("sq1", "sq2"):
        sq.update(_counter_means(os.path.join(prof_dir, d)))
    if sq:
        names = sorted({k for (k, c) in sq if k.startswith("k_")})
        cols = [c for c in SQ_PASS1 + SQ_PASS2 if any((n, c) in sq for n in names)]
        frac = {"SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_MISC"}
        sl = [f"# SQ counters, {workload} synthetic connectome", "",
              "Per-dispatch means. Columns marked `/wave` are divided by `SQ_WAVE_CYCLES` (the share of",
              "wave-cycles spent waiting or issuing); `LDS_BANK_CONFLICT` is also given as a share of",
              "`SQ_LDS_IDX_ACTIVE`. Taken on the library sources of the same SHA-256 as",
              f"`{workload}_kernels.md`.", "",
              "| kernel | " + " | ".join(c.replace("SQ_", "") + (" /wave" if c in frac else "") for c in cols)
              + " | bank conflict share |",
              "|---" * (len(cols) + 2) + "|"]
        for n in names:
            wc = sq.get((n, "SQ_WAVE_CYCLES"), (0, 0.0))[1]
            row = []
            for c in cols:
                v = sq.get((n, c))
                if v is None:
                    row.append("-")
                elif c in frac and wc > 0:
                    row.append(f"{v[1] / wc:.3f}")
                else:
                    row.append(f"{v[1]:.3g}")
            bc, act = sq.get((n, "SQ_LDS_BANK_CONFLICT")), sq.get((n, "SQ_LDS_IDX_ACTIVE"))
            share = f"{bc[1] / act[1]:.3f}" if bc and act and act[1] > 0 else "-"
            sl.append(f"| `{n}` | " + " | ".join(row) + f" | {share} |")
        sl += ["", "Commands (as for the kernel table):", ""]
        sl += [f"    {profile_commands(workload)[k]}" for k in ("sq1", "sq2")]
        with open(os.path.join(out_dir, f"{workload}_sq_counters.md"), "w") as fh:
            fh.write("\n".join(sl) + "\n")
    print(json.dumps({"summarized": workload, "kernels": list(kernels)}))


def recorded_traffic(workload: str, kind: str):
    """HBM bytes per launch of the kernel class from profiles/, or None when the
    record is missing or was taken on other library sources (the records are taken
    with the default Morton voxel order)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_hash():
        return None
    for name, e in rec["kernels"].items():
        if "hbm_bytes" in e and re.sub(r"<\d+>$", "", name) in KIND_KERNELS[kind][:1]:
            return e["hbm_bytes"]
    for name, e in rec["kernels"].items():
        if "hbm_bytes" in e and re.sub(r"<\d+>$", "", name) in KIND_KERNELS[kind]:
            return e["hbm_bytes"]
    return None


def algorithmic(kind: str, d) -> tuple[float, float]:
    """(bytes, flops) the method must move / compute per launch of a kernel class."""
    nnz, nt, nv, nf, na = d.nnz, d.n_theta, d.n_voxels, d.n_fascicles, d.n_atoms
    if kind == "dsc":      # sorted (atom, fascicle, phi) streams, w gathered once, y written once, D once
        return 10.0 * nnz + 4.0 * nt * nv + 4.0 * nf + 4.0 * nt * na + 4.0 * (nv + 1), (2.0 * nt + 1) * nnz
    if kind == "wc_z":     # (atom, phi) streams, y read once, D once, one z per nonzero written
        return 10.0 * nnz + 4.0 * nt * nv + 4.0 * nt * na + 4.0 * (nv + 1), (2.0 * nt + 1) * nnz
    if kind == "wc_sum":   # permutation and z read, g written
        return 8.0 * nnz + 4.0 * nf + 4.0 * (nf + 1), 1.0 * nnz
    return 0.0, 0.0


def pair_bytes(d) -> float:
    """Algorithmic bytes of one DSC plus one WC: the sorted streams, each dense vector
    once, D once."""
    nnz, nt, nv, nf, na = d.nnz, d.n_theta, d.n_voxels, d.n_fascicles, d.n_atoms
    b_dsc = 10.0 * nnz + 4.0 * nt * nv + 4.0 * nf + 4.0 * nt * na + 4.0 * (nv + 1)
    b_wc = 10.0 * nnz + 4.0 * nt * nv + 4.0 * nf + 4.0 * nt * na + 4.0 * (nf + 1)
    return b_dsc + b_wc


def cold_mall_kernels(plan, D, b, w, state, steps: int) -> dict:
    """Per-kernel times of SBB steps with a 512 MB device copy between steps, so each
    step starts with the Infinity Cache (256 MB) holding none of its data.  Only the
    library's own launches are timed (the copy is outside their events)."""
    import torch
    src = torch.empty(64 << 20, dtype=torch.float32, device=D.device)
    dst = torch.empty_like(src)
    plan.profile_read()
    for _ in range(steps):
        dst.copy_(src)
        plan.profile_enable(True)
        plan.sbbnnls_step(D, b, w, state)
        plan.profile_enable(False)
    torch.cuda.synchronize()
    ms, cnt = plan.profile_read()
    del src, dst
    avg = {k: (ms[k] / cnt[k] if cnt[k] else 0.0) for k in ms}
    t = avg["dsc"] + avg["wc_z"] + avg["wc_sum"]
    return {"kernel_avg_ms": {k: round(v, 4) for k, v in avg.items() if cnt[k]},
            "pair_kernel_nnz_per_s": round(plan.dims.nnz / (t / 1e3), 1) if t > 0 else None, "steps": steps}


def cpu_baseline(c, seq_seconds: float):
    """FP64 oracle DSC + WC on the host's cores: the multi-threaded oracle (bit-equal
    to the sequential one) over the whole operator, median of 3 runs; plus the
    sequential oracle on one core over a bounded random sample of the nonzeros."""
    import numpy as np
    import oracle

    op = oracle.Operator.from_connectome(c)
    t0 = time.perf_counter()
    par = op.parallel()
    t_group = time.perf_counter() - t0
    w = c.w0.astype(np.float64)
    y = c.noise.astype(np.float64)
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        par.dsc(w)
        t1 = time.perf_counter()
        par.wc(y)
        t2 = time.perf_counter()
        runs.append((t2 - t0, t1 - t0, t2 - t1))
    par.close()
    runs.sort()
    t_pair, t_dsc, t_wc = runs[1]
    threads = oracle.par_threads()
    out = {"value": round(c.nnz / t_pair, 1), "unit": "nnz/s", "cores": threads, "kind": "oracle",
           "sample": f"whole operator ({c.nnz} nonzeros): one DSC ({t_dsc:.3f} s) + one WC ({t_wc:.3f} s), "
                     f"median of 3, multi-threaded C oracle ({threads} OpenMP threads, "
                     f"OMP_PROC_BIND={os.environ.get('OMP_PROC_BIND', '')}), float64; grouping the "
                     f"nonzeros by voxel and by fascicle took {t_group:.1f} s (not timed)"}
    if seq_seconds > 0:
        def run(n):
            sub = oracle.Operator(c.atom[:n], c.voxel[:n], c.fascicle[:n], c.phi[:n], c.D, c.n_voxels,
                                  c.n_fascicles)
            t0 = time.perf_counter()
            sub.dsc(w)
            t1 = time.perf_counter()
            sub.wc(y)
            return t1 - t0, time.perf_counter() - t1

        probe = min(c.nnz, 500_000)
        a, b = run(probe)
        n = int(min(c.nnz, max(probe, probe * seq_seconds / max(a + b, 1e-9))))
        a, b = run(n) if n != probe else (a, b)
        out["one_core"] = {"value": round(n / (a + b), 1), "unit": "nnz/s", "cores": 1,
                           "sample": f"first {n} nonzeros (input order is a seeded random permutation), "
                                     f"sequential C oracle, one DSC + one WC"}
    return out


def plan_build_times(c, morton: bool) -> dict:
    """Restructuring times after the first build of the process (warm): from host
    COO arrays (copied to the device inside the call), from COO arrays already on
    the device, and the host builder once (the reference, only below 20M nonzeros)."""
    import numpy as np
    import torch
    from paper_1905_06234_amd import life

    xyz = c.voxel_xyz if morton else None
    out = {}
    args = (c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi)
    t0 = time.perf_counter()
    life.Plan.build(*args, voxel_xyz=xyz).close()
    out["host_input"] = round((time.perf_counter() - t0) * 1e3, 1)
    coo = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.atom, c.voxel, c.fascicle, c.phi)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    life.Plan.build(*args[:4], *coo, voxel_xyz=xyz).close()
    out["device_input"] = round((time.perf_counter() - t0) * 1e3, 1)
    del coo
    if c.nnz < 20_000_000:
        t0 = time.perf_counter()
        life.Plan.build(*args, voxel_xyz=xyz, host_build=True).close()
        out["host_builder"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def _time_ms(fn, reps: int) -> float:
    """Wall milliseconds per call of fn (device-synchronized bracket)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def bench_solve(args):
    """A whole SBB-NNLS solve: --iterations iterations (default 500, the paper's run
    length) from w0 on the chosen connectome, timed end to end on the device, with
    the objective read back after the first iteration and every 50 (outside the
    timed stretches); the state after iteration i holds f(w) = 1/2 ||M w - b||^2 at
    the iterate that iteration started from."""
    import numpy as np
    import torch

    import synth
    from paper_1905_06234_amd import life

    life.load()
    dev = torch.device("cuda:0")
    c = synth.make(args.config)
    plan = life.Plan.from_connectome(c, morton=args.voxel_order == "morton")
    D = torch.from_numpy(c.D.ravel()).to(dev)
    y_true = plan.dsc(D, torch.from_numpy(c.w_true).to(dev))
    rms = torch.sqrt(torch.mean(y_true.double() ** 2)).float()
    b = y_true + 0.05 * rms * torch.from_numpy(c.noise).to(dev)
    del y_true
    w = torch.from_numpy(c.w0).to(dev)
    state = life.new_state(dev)
    torch.cuda.synchronize()
    trace, elapsed, done = [], 0.0, 0
    while done < args.iterations:
        k = min(1 if done == 0 else 50 - done % 50, args.iterations - done)
        t0 = time.perf_counter()
        for _ in range(k):
            plan.sbbnnls_step(D, b, w, state)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        done += k
        st = life.read_state(state)
        trace.append((done, st["obj"]))
        log(f"{done} iterations: f(w) = {st['obj']:.6e}, {elapsed * 1e3:.1f} ms")
    wn = w.cpu().numpy()
    plan.close()
    print(json.dumps({
        "metric": "SBB-NNLS solve: wall time per iteration (2 DSC + 1 or 2 WC + glue, all on the device)",
        "value": round(elapsed * 1e3 / args.iterations, 4), "unit": "ms/iteration", "higher_is_better": False,
        "n_gpus": 1, "iterations": args.iterations, "total_s": round(elapsed, 4), "dtype": ARITHMETIC,
        "data": "synthetic", "config": {"workload": f"{args.config} synthetic connectome", "nnz": c.nnz,
                                        "voxel_order": args.voxel_order},
        "objective": {"at_w0": trace[0][1], "last": trace[-1][1], "trace": trace},
        "zero_weights_fraction": round(float(np.mean(wn == 0.0)), 4),
    }), flush=True)


def bench_adam(args):
    """Joint (w, D) Adam on ||y_obs - M(D) w||^2 through the library's
    differentiable DSC (forward DSC; backward WC + dictionary gradient), timed
    against plain DSC+WC pairs on the same plan (mid synthetic connectome)."""
    import numpy as np
    import torch

    import synth
    from paper_1905_06234_amd import autograd, life

    life.load()
    dev = torch.device("cuda:0")
    c = synth.make("mid")
    plan = life.Plan.from_connectome(c)
    log(f"adam: mid nnz={c.nnz}, plan built")
    D0 = torch.from_numpy(c.D).to(dev)
    w0 = torch.from_numpy(c.w0).to(dev)
    y_obs = plan.dsc(D0, torch.from_numpy(c.w_true).to(dev))
    y_obs += 0.05 * torch.sqrt(torch.mean(y_obs.double() ** 2)).float() * torch.from_numpy(c.noise).to(dev)
    D = D0.clone().requires_grad_(True)
    w = w0.clone().requires_grad_(True)
    opt = torch.optim.Adam([D, w], lr=1e-3)

    def adam_step():
        opt.zero_grad(set_to_none=False)
        L = autograd.loss(plan, D, w, y_obs)
        L.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(min=0.0)
        return L

    y = torch.empty(plan.n_signal, device=dev)
    g = torch.empty(plan.dims.n_fascicles, device=dev)

    def pair():
        plan.dsc(D0, w0, y)
        plan.wc(D0, y_obs, g)

    for _ in range(args.warmup):
        adam_step()
        pair()
    L0 = float(autograd.loss(plan, D, w, y_obs))
    plan.profile_read()
    plan.profile_enable(True)
    t_adam = _time_ms(adam_step, args.adam_steps)
    plan.profile_enable(False)
    ms, cnt = plan.profile_read()
    L1 = float(autograd.loss(plan, D, w, y_obs))
    t_pair = _time_ms(pair, args.steps)
    avg = {k: round(ms[k] / cnt[k], 4) for k in ms if cnt[k]}
    out = {"metric": "joint (w, D) Adam step on ||y_obs - M(D)w||^2 / plain DSC+WC pair time",
           "value": round(t_adam / t_pair, 4), "unit": "ratio", "higher_is_better": False, "n_gpus": 1,
           "steps": args.adam_steps, "warmup": args.warmup, "ms_per_adam_step": round(t_adam, 4),
           "ms_per_dsc_wc_pair": round(t_pair, 4), "dtype": ARITHMETIC, "data": "synthetic",
           "loss_before": L0, "loss_after": L1, "kernel_avg_ms": avg,
           "config": {"workload": "mid synthetic connectome, dictionary learning", "n_theta": c.n_theta,
                      "n_atoms": c.n_atoms, "n_voxels": c.n_voxels, "n_fascicles": c.n_fascicles, "nnz": c.nnz}}
    plan.close()
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """32 uneven instances sharing one dictionary: one batched SBB-NNLS iteration
    over all of them (eager, and replayed from a hipGraph) against the 32
    single-instance plans stepped one after another."""
    import numpy as np
    import torch

    import synth
    from paper_1905_06234_amd import life

    life.load()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    inst = synth.make_batch(args.instances, seed=7, scale=args.batch_scale)
    nnz = sum(c.nnz for c in inst)
    log(f"batched: {len(inst)} instances, nnz {nnz} ({time.perf_counter() - t0:.0f} s)")
    D = torch.from_numpy(inst[0].D.ravel()).to(dev)
    t0 = time.perf_counter()
    bp = life.Plan.autotune(inst, D, reps=3)
    t_tune = time.perf_counter() - t0
    singles = [life.Plan.from_connectome(c) for c in inst]
    log(f"plans built; batched plan autotuned in {t_tune:.2f} s: {bp.tile_atoms} atoms per tile, "
        f"schedule {bp.policy}")
    bs, ws = [], []
    for c, sp in zip(inst, singles):
        y = sp.dsc(D, torch.from_numpy(c.w_true).to(dev))
        bs.append(y + 0.05 * torch.sqrt(torch.mean(y.double() ** 2)).float() * torch.from_numpy(c.noise).to(dev))
        ws.append(torch.from_numpy(c.w0).to(dev))
    b_all = torch.cat(bs)
    w_all = torch.cat(ws)
    states = life.new_state(dev, n=len(inst))
    policy = bp.policy

    def batched():
        bp.sbbnnls_step_batch(D, b_all, w_all, states)

    single_states = [life.new_state(dev) for _ in inst]

    def sequential():
        for sp, b, w, st in zip(singles, bs, ws, single_states):
            sp.sbbnnls_step(D, b, w, st)

    for _ in range(args.warmup):
        batched()
        sequential()
    t_batched = _time_ms(batched, args.steps)
    t_seq = _time_ms(sequential, args.steps)
    # the same iteration captured once and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched()
    t_graph = _time_ms(graph.replay, args.steps)

    # time inside the library's launches (events around each launch group), per step
    def kernel_ms(plans, fn):
        for p in plans:
            p.profile_read()
            p.profile_enable(True)
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        tot = 0.0
        for p in plans:
            p.profile_enable(False)
            tot += sum(p.profile_read()[0].values())
        return tot / args.steps
    k_batched = kernel_ms([bp], batched)
    k_seq = kernel_ms(singles, sequential)
    log(f"kernel time per step: batched {k_batched:.3f} ms, sequential plans {k_seq:.3f} ms")
    out = {"metric": "Phi nonzeros/s for one batched SBB-NNLS iteration over all instances (hipGraph replay)",
           "value": round(nnz * 3.5 / 2 / (t_graph / 1e3), 1), "unit": "nnz/s", "higher_is_better": True,
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_graph, 4), "ms_per_step_eager": round(t_batched, 4),
           "ms_per_step_sequential_plans": round(t_seq, 4), "speedup_vs_sequential": round(t_seq / t_graph, 3),
           "kernel_ms_per_step_batched": round(k_batched, 4), "kernel_ms_per_step_sequential": round(k_seq, 4),
           "schedule": policy, "tile_atoms": bp.tile_atoms, "autotune_s": round(t_tune, 3),
           "dtype": ARITHMETIC, "data": "synthetic",
           "config": {"workload": f"{len(inst)} uneven synthetic connectomes sharing D", "nnz": nnz,
                      "n_voxels": [c.n_voxels for c in inst], "n_fascicles": [c.n_fascicles for c in inst],
                      "scale": args.batch_scale}}
    for sp in singles:
        sp.close()
    bp.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--config", default="full", choices=["tiny", "mid", "full"])
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target time of the one-core sequential oracle sample (0: skip it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plan-builder timings and the DSC timings at sparse weights (profiler runs)")
    ap.add_argument("--voxel-order", default="morton", choices=["morton", "index"],
                    help="voxel processing order of the plan: Morton order of the grid coordinates, or voxel index")
    ap.add_argument("--mall-flush", action="store_true",
                    help="also time the kernels with a 512 MB copy between steps (cold Infinity Cache)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (calibrates the HBM byte counters)")
    ap.add_argument("--workload", default="sbb", choices=["sbb", "adam", "batched", "solve"],
                    help="sbb: the headline SBB-NNLS iteration; adam: dictionary learning steps on the mid "
                         "connectome; batched: uneven instances sharing D; solve: a whole SBB-NNLS solve")
    ap.add_argument("--autotune", action="store_true",
                    help="sbb: time the plan geometry chosen by life_plan_autotune instead of the default one")
    ap.add_argument("--iterations", type=int, default=500, help="iterations of --workload solve")
    ap.add_argument("--adam-steps", type=int, default=200)
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--batch-scale", type=float, default=1.0, help="size factor of the batched instances")
    ap.add_argument("--summarize", metavar="PROF_DIR",
                    help="only summarize rocprofv3 outputs (trace/, fetch/, write/, tcc/, copyf/, copyw/) into profiles/")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize, args.config)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the voxel-sharded "
              "design is documented, not implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "adam":
        bench_adam(args)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "solve":
        bench_solve(args)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "launches": 5}), flush=True)
        return

    import numpy as np
    import torch

    import synth
    from paper_1905_06234_amd import life

    life.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    c = synth.make(args.config)
    log(f"generated {args.config}: nnz={c.nnz} Nv={c.n_voxels} Nf={c.n_fascicles} ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    plan = life.Plan.from_connectome(c, morton=args.voxel_order == "morton")
    plan_ms = (time.perf_counter() - t0) * 1e3
    log(f"plan built in {plan_ms:.0f} ms (first build of the process)")
    d = plan.dims
    plan_times = None if args.no_extras else plan_build_times(c, args.voxel_order == "morton")
    log(f"plan builds: {plan_times}")

    D = torch.from_numpy(c.D.ravel()).to(dev)
    tuned = None
    if args.autotune:
        plan.close()
        t0 = time.perf_counter()
        plan = life.Plan.autotune([c], D, reps=3, morton=args.voxel_order == "morton")
        tuned = {"seconds": round(time.perf_counter() - t0, 3), "tile_atoms": plan.tile_atoms,
                 "schedule": plan.policy}
        log(f"autotuned plan: {tuned}")
    w = torch.from_numpy(c.w0).to(dev)
    # b = M w_true + 5% noise, formed with the library's own DSC (input preparation)
    y_true = plan.dsc(D, torch.from_numpy(c.w_true).to(dev))
    rms = torch.sqrt(torch.mean(y_true.double() ** 2)).float()
    b = y_true + 0.05 * rms * torch.from_numpy(c.noise).to(dev)
    del y_true
    state = life.new_state(dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        plan.sbbnnls_step(D, b, w, state)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    # the headline: K steps with nothing but the library's own launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.sbbnnls_step(D, b, w, state)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = life.read_state(state)
    w_zero = float((w == 0).float().mean().item())
    log(f"timed {args.steps} steps: {wall * 1e3:.2f} ms; f={st['obj']:.6e} alpha={st['alpha']:.3e}; "
        f"zero weights {w_zero:.3f}")
    # per-kernel times from a separate pass of K steps with every launch bracketed by events
    plan.profile_read()                 # drop anything recorded so far
    plan.profile_enable(True)
    for _ in range(args.steps):
        plan.sbbnnls_step(D, b, w, state)
    torch.cuda.synchronize()
    plan.profile_enable(False)
    ms, cnt = plan.profile_read()
    log(f"profiled pass: kernel ms {ms}")

    # DSC and WC per step: 2 DSC; 1 WC, plus the second on even iterations (Algorithm 1)
    evens = sum(1 for i in range(args.warmup, args.warmup + args.steps) if i % 2 == 0)
    n_dsc = 2 * args.steps
    n_wc = args.steps + evens
    pairs = (n_dsc + n_wc) / 2.0
    value = d.nnz * pairs / wall
    avg = {k: (ms[k] / cnt[k] if cnt[k] else 0.0) for k in ms}
    t_dsc = avg["dsc"]
    t_wc = avg["wc_z"] + avg["wc_sum"]

    # the kernel with the largest total time over the timed steps
    tot = {k: sum(ms[x] for x in g) for k, g in KIND_GROUPS.items()}
    launches = {k: sum(cnt[x] for x in g) for k, g in KIND_GROUPS.items()}
    dom = max(tot, key=lambda k: tot[k])
    dom_ms = tot[dom] / max(launches[dom], 1)
    by, fl = algorithmic(dom, d)
    t_s = dom_ms / 1e3
    bw = by / t_s / 1e9
    tf = fl / t_s / 1e12
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": round(tf, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(bw, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(bw / HBM_PEAK_GBS, 4)}
    # DSC alone at growing fractions of zero weights (the zero-weight skip, Sec. 6.6)
    rng = np.random.default_rng(11)
    y_buf = torch.empty(d.n_theta * d.n_voxels, dtype=torch.float32, device=dev)
    dsc_zero = {}
    for frac in () if args.no_extras else (0.0, 0.5, 0.9, 0.99):
        wz = torch.from_numpy(np.where(rng.random(d.n_fascicles) < frac, 0.0, c.w0).astype(np.float32)).to(dev)
        plan.dsc(D, wz, y_buf)
        dsc_zero[str(frac)] = round(_time_ms(lambda: plan.dsc(D, wz, y_buf), 10), 4)
    del y_buf
    log(f"DSC ms by fraction of zero weights: {dsc_zero}")
    # achievable stream bandwidth on this GPU: a plain 1 GiB device copy (read + write)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    t_copy = _time_ms(lambda: dst.copy_(src), 5)
    copy_gbs = 2.0 * src.numel() * 4 / (t_copy / 1e3) / 1e9
    del src, dst
    traffic = recorded_traffic(args.config, dom) if args.voxel_order == "morton" else None
    roof.update({"traffic": traffic, "kernel": dom, "avg_ms": round(dom_ms, 4),
                 "achievable_copy_GBs": round(copy_gbs, 1),
                 "algorithmic_bytes": int(by), "algorithmic_flops": int(fl),
                 "hbm_GBs": round(bw, 1), "hbm_frac": round(bw / HBM_PEAK_GBS, 4)})

    out = {
        "metric": "Phi nonzeros/s for DSC (Mw)+WC (M^T y) per SBB-NNLS iteration; % HBM peak",
        "value": round(value, 1), "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ARITHMETIC, "data": "synthetic",
        "config": {"workload": f"{args.config} synthetic connectome", "n_theta": d.n_theta, "n_atoms": d.n_atoms,
                   "n_voxels": d.n_voxels, "n_fascicles": d.n_fascicles, "nnz": d.nnz,
                   "voxel_order": args.voxel_order,
                   "step": "one SBB-NNLS iteration (2 DSC + 1 or 2 WC + glue)"},
        "pair_kernel_nnz_per_s": round(d.nnz / ((t_dsc + t_wc) / 1e3), 1) if t_dsc + t_wc > 0 else None,
        # algorithmic bytes of one DSC plus one WC over their kernel times, against 8 TB/s
        "pair_hbm_frac": round(pair_bytes(d) / ((t_dsc + t_wc) / 1e3) / (HBM_PEAK_GBS * 1e9), 4)
        if t_dsc + t_wc > 0 else None,
        "kernel_avg_ms": {k: round(v, 4) for k, v in avg.items()},
        "kernel_launches": cnt,
        "w_zero_fraction_after_timed_steps": round(w_zero, 4), "dsc_ms_by_zero_fraction": dsc_zero,
        "plan_ms": round(plan_ms, 1), "plan_build_ms": plan_times, "tile_atoms": plan.tile_atoms,
        "roofline": roof,
    }
    if tuned:
        out["autotune"] = tuned
    if args.mall_flush:
        out["cold_mall"] = cold_mall_kernels(plan, D, b, w, state, args.steps)
        log(f"cold-MALL kernel times: {out['cold_mall']}")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
