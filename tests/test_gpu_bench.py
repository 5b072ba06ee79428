"""The benchmark's JSON line on a small mesh: every field of the contract is
present and the reported errors are the FP64 oracle's (run as a child
process, as the benchmark is run)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_json_line_small_mesh():
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--n", "8", "--steps", "3", "--warmup", "1",
           "--no-batched", "--no-reacting", "--no-hex", "--long-steps", "5", "--cpu-threads", "2"]
    print("running", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "euler_vortex_pert_p3_8cubed" and d["config"]["elements"] == 8 ** 3 * 6
    rf = d["roofline"]
    assert rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["flops_per_elem"] == 26400 and rf["bytes_per_elem"] == 1832
    assert rf["traffic"] is None  # the stored counters belong to the 48^3 workload
    sp = d["ms_per_step_spread"]
    assert sp["min"] <= sp["median"] <= sp["max"] and sp["launches_per_batch"] == 3
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] in (1, 2) and cb["value"] > 0 and "3071" in cb["sample"]
    assert set(cb["by_threads"]) == {"1", "2"} and cb["cpu_model"]
    for field, e in d["error_vs_oracle"].items():
        assert e["l2"] <= 1e-12, (field, e)
        assert e["max_err_over_T_in_u"] <= e["bar_in_u"], (field, e)
    ls = d["after_steps"]
    assert ls["steps"] == 5 and ls["fp64_finite"]
    for mode, bound in (("fp32", 1e-4), ("split_bf16", 1e-2)):
        for field, e in ls[mode].items():
            assert e["l2"] <= bound, (mode, field, e)
    for mode, bound in (("fp32", 1e-4), ("split_bf16", 1e-2)):
        v = d["variants"][mode]
        assert v["value"] > 0
        for field, e in v["error_vs_oracle"].items():
            assert e["l2"] <= bound, (mode, field, e)
