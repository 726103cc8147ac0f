"""Host-side checks of bench.py's measurement plumbing (no GPU): the one-GPU
refusal, the arithmetic of the rocprofv3 summaries (counter scaling by the copy
probe, L2 hit rate), the staleness rule of recorded traffic, the per-config
profiling commands, and the algorithmic byte and flop counts of DSC and WC."""
import csv
import importlib.util
import json
import os
import subprocess
import sys
from types import SimpleNamespace

from conftest import ROOT


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_summary_scales_counters_by_the_copy_probe(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "prof"
    dsc = "void (anonymous namespace)::k_dsc_chunk<3>(int const*, float*)"
    _csv(str(prof / "trace" / "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
         [[dsc, 4, 1_250_000.0], ["void (anonymous namespace)::k_wc_sum(int const*)", 2, 500_000.0]])
    cols = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _csv(str(prof / "fetch" / "run_counter_collection.csv"), cols,
         [[dsc, "FETCH_SIZE", 1000.0], [dsc, "FETCH_SIZE", 3000.0]])           # mean 2000 KiB
    _csv(str(prof / "write" / "run_counter_collection.csv"), cols, [[dsc, "WRITE_SIZE", 500.0]])
    _csv(str(prof / "tcc" / "run_counter_collection.csv"), cols,
         [[dsc, "TCC_HIT_sum", 90.0], [dsc, "TCC_MISS_sum", 10.0]])
    # a 256 MiB copy read as 128 MiB by FETCH_SIZE (factor 2) and 256 MiB by WRITE_SIZE (factor 1)
    _csv(str(prof / "copyf" / "run_counter_collection.csv"), cols, [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072.0]])
    _csv(str(prof / "copyw" / "run_counter_collection.csv"), cols, [["__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144.0]])
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "source_hash", lambda: "sources-a")
    b.summarize(str(prof), "full")
    rec = json.load(open(tmp_path / "profiles" / "full_counters.json"))
    e = rec["kernels"]["k_dsc_chunk<3>"]
    assert e["calls_traced"] == 4 and e["avg_us"] == 1250.0
    assert e["hbm_bytes"] == 2000 * 1024 * 2 + 500 * 1024 * 1
    assert e["l2_hit_rate"] == 0.9
    assert "hbm_bytes" not in rec["kernels"]["k_wc_sum"]          # no counters recorded for it
    md = (tmp_path / "profiles" / "full_kernels.md").read_text()
    assert "k_dsc_chunk<3>" in md and "sources-a" in md and "fetch x2.000, write x1.000" in md
    # the bench line uses the record only while the library sources are the same
    assert b.recorded_traffic("full", "dsc") == e["hbm_bytes"]
    monkeypatch.setattr(b, "source_hash", lambda: "sources-b")
    assert b.recorded_traffic("full", "dsc") is None
    assert b.recorded_traffic("mid", "dsc") is None                # no record for mid here


def test_profile_commands_per_config():
    b = _bench()
    full, mid = b.profile_commands("full"), b.profile_commands("mid")
    assert full == b.PROFILE_COMMANDS
    assert set(full) == {"trace", "fetch", "write", "tcc", "sq1", "sq2", "copyf", "copyw"}
    # each SQ pass stays within the 8 SQ counters one run can collect
    for k in ("sq1", "sq2"):
        pmc = full[k].split("--pmc ")[1].split(" --")[0].split()
        assert 0 < len(pmc) <= 8 and all(c.startswith("SQ_") for c in pmc)
        assert "--kernel-trace" not in full[k] and "--sys-trace" not in full[k]
    assert "--config" not in full["trace"] and "gpurun_out/prof/" in full["trace"]
    assert all("gpurun_out/prof_mid/" in c for c in mid.values())
    assert all("--config mid" in mid[k] for k in ("trace", "fetch", "write", "tcc", "sq1", "sq2"))
    # counters never share a run with the trace, and one counter block per run
    assert all("--pmc" not in full[k] for k in ("trace",)) and "--kernel-trace" not in full["fetch"]


def test_algorithmic_counts_closed_form():
    b = _bench()
    d = SimpleNamespace(nnz=10, n_theta=2, n_voxels=3, n_fascicles=4, n_atoms=5)
    # DSC: sorted (atom, fascicle, phi) streams, y written once, w, D and the segment pointers once
    assert b.algorithmic("dsc", d) == (10 * 10 + 4 * 2 * 3 + 4 * 4 + 4 * 2 * 5 + 4 * (3 + 1), (2 * 2 + 1) * 10)
    # WC pass 1: (atom, phi) streams, one z per nonzero, y read once, D once, the voxel pointers
    assert b.algorithmic("wc_z", d) == (10 * 10 + 4 * 2 * 3 + 4 * 2 * 5 + 4 * (3 + 1), (2 * 2 + 1) * 10)
    assert b.algorithmic("wc_sum", d) == (8 * 10 + 4 * 4 + 4 * (4 + 1), 10)
    assert b.pair_bytes(d) == (100 + 24 + 16 + 40 + 16) + (100 + 24 + 16 + 40 + 20)
