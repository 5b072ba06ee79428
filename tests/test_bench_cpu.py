"""Host-side pieces of the benchmark contract (no GPU): the one-GPU guard,
the per-element algorithmic counts the roofline uses, and the gate that
drops the stored HBM traffic once the kernel's sources differ from the ones
the counters were taken on."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_counts_at_p3():
    # the roofline's per-element figures: 12.0k volume + 1.8k metric + 0.6k
    # flux + 4.0k surface + 8.0k lift flops; bytes: state in and rhs out
    # (2 * 5 * 20 * 8) + 200 (affine geometry) + 32 (connectivity)
    assert bench.algorithmic_counts(3) == (12000 + 1800 + 600 + 4000 + 8000, 2 * 5 * 20 * 8 + 200 + 32)
    for p in (1, 2, 3, 4):
        Np = (p + 1) * (p + 2) * (p + 3) // 6
        assert bench.algorithmic_counts(p)[1] == 2 * 5 * Np * 8 + 232


def test_kernel_counts_at_p3():
    # 2 nf Np (3 Np + 4 Nfp) = 2 * 5 * 20 * 100 = 20,000 contraction flops,
    # 52 * 20 pointwise and 80 * 40 face-flux flops; bytes: 2 * 5 * 20 * 8 +
    # 72 (metric) + 32 (connectivity)
    assert bench.kernel_counts(3) == (20000 + 1040 + 3200, 1704)
    assert bench.kernel_counts(1) == (2 * 5 * 4 * (12 + 12) + 52 * 4 + 80 * 12, 2 * 5 * 4 * 8 + 104)


def test_iteration_histogram():
    h = bench.iteration_histogram(np.array([3, 5, 5, -1, 3, 3]))
    assert h == {"-1": 1, "3": 3, "5": 2}


def test_entry_ratios_units():
    """Errors are quoted in units of u relative to each entry's magnitude."""
    u = 2.0 ** -53
    ref = np.ones((5, 2, 20))
    mag = np.full_like(ref, 4.0)
    got = ref + 8 * u  # 8 u absolute on a magnitude of 4: 2 u
    r = bench.entry_ratios(got, ref, mag, 3)
    assert abs(r["rho"]["max_err_over_T_in_u"] - 2.0) < 1e-9 and r["E"]["bar_in_u"] == 100
    assert r["rho"]["max_rhs_over_max_T"] == 0.25


def test_stored_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """A counter summary names the sha256 of the kernel sources it was taken
    on; the stored traffic is used only while the sources are unchanged."""
    summary = tmp_path / "pmc.txt"
    summary.write_text(f"kernel_source_sha256: {bench.kernel_source_sha()}\ntraffic_bytes_per_launch: 1234.0\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(summary))
    assert bench.stored_traffic() == 1234.0
    copies = []
    for i, f in enumerate(bench.KERNEL_SRCS):
        dst = tmp_path / f"src{i}"
        shutil.copy(f, dst)
        copies.append(dst)
    monkeypatch.setattr(bench, "KERNEL_SRCS", [str(c) for c in copies])
    assert bench.stored_traffic() == 1234.0
    for c in copies:  # a change to any one source drops the stored figure
        original = c.read_bytes()
        c.write_bytes(original + b"\n// changed\n")
        assert bench.stored_traffic() is None
        c.write_bytes(original)
        assert bench.stored_traffic() == 1234.0


def test_stored_counters_follow_the_launch_shape(tmp_path, monkeypatch):
    """Counters taken in one launch shape are not reported for another: the
    XCD run length changes the L2 reuse and with it the traffic."""
    summary = tmp_path / "pmc.txt"
    summary.write_text(f"kernel_source_sha256: {bench.kernel_source_sha()}\nlaunch_waves_per_block: 4\n"
                       "launch_lds_stage: 1\nlaunch_xcd_run: 27\ntraffic_bytes_per_launch: 99.0\n"
                       "mfma_busy_frac: 0.5\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(summary))
    same = dict(waves_per_block=4, rk_fused=0, lds_stage=1, xcd_run=27)
    assert bench.stored_counters(same) == {"traffic": 99.0, "mfma_busy": 0.5}
    for k, v in (("waves_per_block", 2), ("lds_stage", 0), ("xcd_run", 9)):
        assert bench.stored_counters(dict(same, **{k: v})) == {}, k


def test_launch_option_parses_four_integers():
    assert bench.parse_launch(bench.DEFAULT_LAUNCH) == [4, 1, 1, 27]
    assert bench.parse_launch("2,0,1,9") == [2, 0, 1, 9]
    for bad in ("4,1,1", "4,1,1,27,3", "a,b,c,d"):
        with pytest.raises(ValueError):
            bench.parse_launch(bad)


def test_committed_counter_summary_matches_the_sources():
    """The committed FP64 counter summary was taken on the current kernel
    sources (else the bench line would report no traffic)."""
    assert bench.stored_counters().get("traffic", 0) > 0


def test_paper_context_quotes_the_papers_figures():
    """The bench line quotes the paper's RHS throughputs (Sec. 5.3) with
    their hardware, and the closest leg measured here in the same unit."""
    import bench
    ctx = bench.paper_context({"shock": {"hex_shock_slab_p1_120cubed": {"elements": 1000, "ms_rhs_with_av": 2.0}}})
    hw = {(f["system"], f["hardware"]): f["value"] for f in ctx["figures"]}
    assert hw[("MIRGE-Com", "AMD MI300A")] == 100.4e6
    assert hw[("MIRGE-Com", "Apple M2 (CPU)")] == 1.6e6
    assert ctx["closest_here"]["value"] == 8000 / 2e-3
    assert "closest_here" not in bench.paper_context({})
