"""Benchmark: DG Euler right-hand-side throughput on one MI355X.

Workload: periodic box [0,10]^3, 48^3 cubes x 6 = 663,552 affine tets with
seeded 3 % vertex jitter, order p = 3 (20 nodes per tet), 5 conserved fields,
isentropic vortex plus a seeded entropy perturbation of the density
(amplitude 1e-2, wavenumbers 1..4) — synthetic stand-in for the paper's
periodic isentropic-vortex Euler benchmark (Sec. 5.2).

A step is one evaluation of the full right-hand side (volume divergence, face
gather with the Lax-Friedrichs flux, lift and inverse mass) over the whole
mesh; the state is resident in HBM before timing starts.  Throughput is
GDOF.fields/s = E * Np * nf * steps / time / 1e9.

Prints ONE JSON line.  Also reports the roofline of the RHS kernel (its
launch duration measured with HIP events on the stream it runs on) and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG RHS GDOF·fields/s at p=3 (FP64 vs FP32/split-BF16), error vs FP64 oracle"
WORKLOAD = dict(name="euler_vortex_pert_p3_48cubed", n=48, order=3, jitter=0.03, mesh_seed=1002, pert_seed=2002)
NF = 5
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "rhs_euler_fp64_p3_48cubed_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2512_17101_amd", "csrc", "rhs_euler.hip")


def algorithmic_counts(p: int):
    """Per-element FP64 flops and HBM bytes the RHS must move at minimum.

    flops: contractions 2 nf Np (3 Np + 4 Nfp) + pointwise flux 52 Np + face
    flux 80 (4 Nfp).  bytes: state in and rhs out (2 nf Np 8), 9 metric terms
    (72) and 4 faces x (neighbour id, face/permutation code) (32)."""
    Np = (p + 1) * (p + 2) * (p + 3) // 6
    Nfp = (p + 1) * (p + 2) // 2
    flops = 2 * NF * Np * (3 * Np + 4 * Nfp) + 52 * Np + 80 * 4 * Nfp
    bytes_ = 2 * NF * Np * 8 + 72 + 32
    return flops, bytes_


def stored_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    kv = {}
    for line in open(PMC_SUMMARY):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(xyz, vid, q_np, p, sample_elems):
    """Oracle RHS timed on a contiguous sample of elements (BLAS limited to one
    thread, so one core does the work)."""
    from threadpoolctl import threadpool_limits

    from oracle import euler as oe, mesh as om, reference_element as ore
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    idx = np.arange(min(sample_elems, xyz.shape[0]))
    with threadpool_limits(limits=1):
        oe.rhs(ops, geo, conn, q_np, elems=idx[:1024])
        t0 = time.perf_counter()
        oe.rhs(ops, geo, conn, q_np, elems=idx)
        t = time.perf_counter() - t0
    Np = ops["Np"]
    return {"value": len(idx) * Np * NF / t / 1e9, "unit": "GDOF·fields/s", "cores": 1, "kind": "oracle",
            "sample": f"one RHS over elements 0..{len(idx) - 1} of the {xyz.shape[0]}-tet mesh "
                      f"({t:.1f} s, NumPy FP64, 1 thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "split_bf16"])
    ap.add_argument("--cpu-sample", type=int, default=262144, help="elements in the CPU-baseline sample (0: skip)")
    ap.add_argument("--n", type=int, default=WORKLOAD["n"], help="cubes per side (default: the 48^3 workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path shards by element "
              "partition across GPUs, which this build does not run)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_17101_amd import dg, workload as wl
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": n * 8, "launches": 5}), flush=True)
        return
    p = WORKLOAD["order"]
    xyz, vid = wl.kuhn_box_mesh(args.n, 10.0, WORKLOAD["jitter"], WORKLOAD["mesh_seed"])
    mesh = dg.Mesh(p, xyz, vid, 0)
    X = mesh.nodes()
    q_np = wl.vortex_state(X, pert=wl.density_perturbation(WORKLOAD["pert_seed"]))
    q = torch.from_numpy(q_np).to(dev)
    out = torch.empty_like(q)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            dg.rhs(mesh, q, out, args.precision, stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            dg.rhs(mesh, q, out, args.precision, stream=stream)
        e1.record(stream)
        stream.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps  # one launch per step: this is the kernel's average duration
    E, Np = mesh.E, mesh.Np
    value = E * Np * NF / (ms * 1e-3) / 1e9
    flops, bytes_ = algorithmic_counts(p)
    achieved_tf = flops * E / (ms * 1e-3) / 1e12
    achieved_gbs = bytes_ * E / (ms * 1e-3) / 1e9
    traffic = stored_traffic()
    roofline = {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                "kernel": f"rhs_euler_fp64_kernel<{p}>", "flops_per_elem": flops, "bytes_per_elem": bytes_,
                "hbm_view": {"achieved": round(achieved_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": round(achieved_gbs / PEAK_HBM_GBS, 4)}}
    rec = {"metric": METRIC, "value": round(value, 3), "unit": "GDOF·fields/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WORKLOAD["name"] if args.n == WORKLOAD["n"] else f"euler_vortex_pert_p3_{args.n}cubed",
                      "elements": E, "order": p, "nodes_per_element": Np, "fields": NF,
                      "contraction_precision": args.precision},
           "roofline": roofline}
    if args.cpu_sample > 0:
        rec["cpu_baseline"] = cpu_baseline(xyz, vid, q_np, p, args.cpu_sample)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
