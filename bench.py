"""Benchmark: DG Euler right-hand-side throughput on one MI355X.

Workload: periodic box [0,10]^3, 48^3 cubes x 6 = 663,552 affine tets with
seeded 3 % vertex jitter, order p = 3 (20 nodes per tet), 5 conserved fields,
isentropic vortex plus a seeded entropy perturbation of the density
(amplitude 1e-2, wavenumbers 1..4) — synthetic stand-in for the paper's
periodic isentropic-vortex Euler benchmark (Sec. 5.2).

A step is one evaluation of the full right-hand side (volume divergence, face
gather with the Lax-Friedrichs flux, lift and inverse mass) over the whole
mesh; the state is resident in HBM before timing starts.  Throughput is
GDOF.fields/s = E * Np * nf * steps / time / 1e9.  The reported value is the
FP64 form; the FP32 and split-BF16 contraction forms are timed the same way
and listed under "variants" with their per-field errors against the oracle.

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
# device sources of the FP64 RHS kernel (the kernel file, then its tile helpers)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2512_17101_amd", "csrc", f) for f in ("rhs_euler.hip", "euler_point.hpp")]


# Algorithmic work per element of one Euler RHS evaluation, by order: flops
# (volume contraction + metric + pointwise flux + surface flux + lift) and
# the minimum HBM bytes (FP64 state in and rhs out, 200 B of affine geometry,
# 32 B of face connectivity).  These are the figures the roofline fraction is
# quoted against; the kernel's own count (below) is lower because it stores
# 72 B of geometry and folds the metric into the flux.
ALGORITHMIC = {1: (2640, 552), 2: (9000, 1032), 3: (26400, 1832), 4: (67950, 3032)}


# The paper's own right-hand-side throughputs (Sec. 5.3, the shock wave /
# boundary layer interaction case: 2-D, degree-1 tensor-product elements,
# full compressible Navier-Stokes; "DOFs" counted per scalar field).  Quoted
# as context with the hardware the paper names: none of them is this
# workload, and the paper states no precision for them.
PAPER_FIGURES = [
    {"system": "MIRGE-Com", "value": 1.6e6, "unit": "DOFs/s (per field)", "hardware": "Apple M2 (CPU)"},
    {"system": "Ryujin (comparison code)", "value": 3.8e6, "unit": "DOFs/s (per field)", "hardware": "Apple M2 (CPU)"},
    {"system": "MIRGE-Com", "value": 100.4e6, "unit": "DOFs/s (per field)", "hardware": "AMD MI300A"},
]


def paper_context(rec):
    """The paper's figures beside the closest leg measured here (the p = 1
    hexahedron shock slab: RHS with artificial viscosity, 3-D Euler), in the
    paper's unit (nodes x RHS evaluations per second, per field)."""
    out = {"source": "Sec. 5.3 (shock wave / boundary layer interaction, 2-D, degree-1 TPEs, Navier-Stokes)",
           "figures": PAPER_FIGURES}
    sh = rec.get("shock", {}).get("hex_shock_slab_p1_120cubed")
    if sh:
        nodes = sh["elements"] * 8
        out["closest_here"] = {"leg": "hex_shock_slab_p1_120cubed (RHS with artificial viscosity, 3-D Euler)",
                               "value": round(nodes / (sh["ms_rhs_with_av"] * 1e-3), 1),
                               "unit": "DOFs/s (per field)", "hardware": "AMD MI355X (one GPU)"}
    return out


def algorithmic_counts(p: int):
    """(flops, bytes) per element of one Euler RHS (the table above)."""
    return ALGORITHMIC[p]


def kernel_counts(p: int):
    """Per-element FP64 flops and HBM bytes of this library's RHS kernel.

    flops: contractions 2 nf Np (3 Np + 4 Nfp) + pointwise flux 52 Np + face
    flux 80 (4 Nfp).  bytes: state in and rhs out (2 nf Np 8), 9 metric terms
    (72) and 4 faces x (neighbour id, face/permutation code) (32)."""
    Np = (p + 1) * (p + 2) * (p + 3) // 6
    Nfp = (p + 1) * (p + 2) // 2
    flops = 2 * NF * Np * (3 * Np + 4 * Nfp) + 52 * Np + 80 * 4 * Nfp
    bytes_ = 2 * NF * Np * 8 + 72 + 32
    return flops, bytes_


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def stored_counters(launch=None):
    """Figures per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and, given `launch` (a launch
    configuration dict), in the same launch shape (tiles per block, LDS
    staging, XCD run length): HBM traffic in bytes
    (traffic_bytes_per_launch) and the matrix-core busy fraction
    (mfma_busy_frac).  Empty otherwise."""
    if not os.path.exists(PMC_SUMMARY):
        return {}
    kv = {}
    for line in open(PMC_SUMMARY):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha():
        return {}
    if launch is not None:
        for k in ("waves_per_block", "lds_stage", "xcd_run"):
            if kv.get("launch_" + k) != str(launch[k]):
                return {}
    out = {}
    if "traffic_bytes_per_launch" in kv:
        out["traffic"] = float(kv["traffic_bytes_per_launch"])
    if "mfma_busy_frac" in kv:
        out["mfma_busy"] = float(kv["mfma_busy_frac"])
    return out


def stored_traffic():
    """HBM bytes per launch from the committed counter summary, or None."""
    return stored_counters().get("traffic")


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo) and the cores this
    process may run on."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def cpu_baseline(xyz, vid, q_np, p, sample_elems, threads):
    """Oracle RHS timed on a contiguous sample of elements, once with BLAS on
    one thread and once on `threads` threads (the NumPy oracle's contractions
    are BLAS calls; its pointwise work runs on one core either way).  q_np
    maps node coordinates [E, Np, 3] to the state.  Returns (record, element
    ids, oracle RHS on them, oracle term magnitudes on them)."""
    from threadpoolctl import threadpool_limits

    from oracle import euler as oe, mesh as om, reference_element as ore
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    idx = np.arange(xyz.shape[0] if sample_elems < 0 else min(sample_elems, xyz.shape[0]))
    # the oracle's own nodes: the same smooth state evaluated there (it agrees
    # with the library's nodes to rounding), so no oracle input comes from the library
    q_np = q_np(om.node_coordinates(xyz, ops["rst"]))
    times = {}
    for nt in (1, threads):
        with threadpool_limits(limits=nt):
            oe.rhs(ops, geo, conn, q_np, elems=idx[:1024])
            t0 = time.perf_counter()
            ref = oe.rhs(ops, geo, conn, q_np, elems=idx)
            times[nt] = time.perf_counter() - t0
    with threadpool_limits(limits=threads):
        mag = oe.rhs_term_magnitude(ops, geo, conn, q_np, elems=idx)
    Np = ops["Np"]
    model, ncpu = cpu_model()
    rate = lambda t: len(idx) * Np * NF / t / 1e9
    best = min(times, key=times.get)
    rec = {"value": rate(times[best]), "unit": "GDOF·fields/s", "cores": best, "kind": "oracle",
           "sample": f"one RHS over elements 0..{len(idx) - 1} of the {xyz.shape[0]}-tet mesh "
                     f"({times[best]:.1f} s, NumPy FP64, BLAS on {best} threads)",
           "cpu_model": model, "cpus_available": ncpu,
           "by_threads": {str(nt): {"seconds": round(t, 2), "value": rate(t)} for nt, t in times.items()}}
    return rec, idx, ref, mag


FIELDS = ("rho", "rho_u", "rho_v", "rho_w", "E")


def entry_ratios(got, ref, mag, p):
    """Per field: the largest |gpu_i - oracle_i| / T_i over the sample, in
    units of u = 2^-53, with T_i the oracle's term magnitude of entry i (the
    scale of the rounding of a computed sum of products), the per-entry bar
    K = 3 Np + 4 Nfp it is held to in the tests, and max|rhs_f| / max T_f
    (how far the field's terms cancel)."""
    u = 2.0 ** -53
    Np = (p + 1) * (p + 2) * (p + 3) // 6
    Nfp = (p + 1) * (p + 2) // 2
    K = 3 * Np + 4 * Nfp
    r = (np.abs(got - ref) / mag).max(axis=(1, 2)) / u
    c = np.abs(ref).max(axis=(1, 2)) / mag.max(axis=(1, 2))
    return {nm: {"max_err_over_T_in_u": round(float(r[f]), 3), "bar_in_u": K, "max_rhs_over_max_T": float(c[f])}
            for f, nm in enumerate(FIELDS)}


def long_run_errors(dg, mesh, q, q_np, work, modes, steps, stream):
    """Per-field errors of the reduced-precision forms against the FP64 form
    after `steps` LSRK steps from the same state, CFL 0.2 on the cube size
    (dt = 0.2 h / ((p + 1)^2 max(|u| + c)) from the initial state)."""
    import torch
    rho = q_np[0]
    vel = np.sqrt(q_np[1] ** 2 + q_np[2] ** 2 + q_np[3] ** 2) / rho
    pres = (1.4 - 1.0) * (q_np[4] - 0.5 * rho * vel ** 2)
    vmax = float((vel + np.sqrt(1.4 * pres / rho)).max())
    h = 10.0 / round((mesh.E / 6) ** (1.0 / 3.0))
    dt = 0.2 * h / ((mesh.order + 1) ** 2 * vmax)
    finals = {}
    with torch.cuda.stream(stream):
        for mode in modes:
            qs = q.clone()
            for _ in range(steps):
                dg.rk_step(mesh, qs, work, 0.0, dt, mode, stream=stream)
            stream.synchronize()
            finals[mode] = qs.cpu().numpy()
    ref = finals["fp64"]
    out = {"steps": steps, "dt": dt, "t_final": steps * dt, "reference": "GPU FP64 form"}
    for mode in modes:
        if mode != "fp64":
            out[mode] = field_errors(finals[mode], ref)
    out["fp64_finite"] = bool(np.isfinite(ref).all())
    return out


def field_errors(got, ref):
    """Per-field relative L2 and Linf errors (momentum components scaled by the
    momentum vector's magnitude)."""
    d = got - ref
    l2 = np.sqrt((d ** 2).sum(axis=(1, 2)))
    n2 = np.sqrt((ref ** 2).sum(axis=(1, 2)))
    li = np.abs(d).max(axis=(1, 2))
    ni = np.abs(ref).max(axis=(1, 2))
    n2[1:4] = n2[1:4].max()
    ni[1:4] = ni[1:4].max()
    return {nm: {"l2": float(l2[f] / n2[f]), "linf": float(li[f] / ni[f])} for f, nm in enumerate(FIELDS)}


# Launch shape of the single-mesh legs: four tiles per block, fused stages,
# LDS DMA staging, XCD runs of 27 blocks (the autotuner's usual choice on
# the 48^3 workload; fixed so that every run times the same kernels)
DEFAULT_LAUNCH = "4,1,1,27"


def parse_launch(text):
    vals = [int(v) for v in text.split(",")]
    if len(vals) != 4:
        raise ValueError(f"--launch wants four integers or 'auto', got {text!r}")
    return vals


SETTLE_S = 0.5  # seconds of untimed launches before the first timed batch (clocks ramp up)
REPEATS = 5    # batches of `steps` launches timed after the reported one, for the spread


def time_rhs(dg, mesh, q, out, precision, steps, warmup, stream):
    """Average duration of one dg_rhs launch, HIP events on its stream: a
    settle phase of SETTLE_S seconds of launches, `warmup` launches, then one
    timed batch of exactly `steps` launches (the reported figure), then
    REPEATS more batches of the same size for the spread."""
    import torch
    launch = lambda: dg.rhs(mesh, q, out, precision, stream=stream)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < SETTLE_S:
            for _ in range(50):
                launch()
            stream.synchronize()
        for _ in range(warmup):
            launch()
        stream.synchronize()
        batches = [_time_ms(stream, launch, steps) for _ in range(1 + REPEATS)]
    return batches[0], {"median": round(float(np.median(batches)), 5), "min": round(min(batches), 5),
                        "max": round(max(batches), 5), "batches": len(batches), "launches_per_batch": steps}


def time_rk_step(dg, mesh, q, work, dt, precision, steps, stream):
    """Average duration of one dg_rk_step (five stages), HIP events on its
    stream: SETTLE_S / 2 seconds of untimed steps, then 1 + REPEATS batches of
    `steps` steps; the first batch is the reported figure, all of them the
    spread."""
    import torch
    launch = lambda: dg.rk_step(mesh, q, work, 0.0, dt, precision, stream=stream)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < SETTLE_S / 2:
            for _ in range(10):
                launch()
            stream.synchronize()
        batches = [_time_ms(stream, launch, steps) for _ in range(1 + REPEATS)]
    return batches[0], {"median": round(float(np.median(batches)), 4), "min": round(min(batches), 4),
                        "max": round(max(batches), 4), "batches": len(batches), "steps_per_batch": steps}


def batched_leg(dg, wl, dev, stream, steps):
    """Batched workload: 64 independent periodic vortex boxes of seeded size
    (4..40 cubes per side) and order (1..4), FP32 contractions, FP64 state.
    Times one LSRK step of all meshes as the tuned, graph-captured batch (one
    mixed-order launch per stage, or one per order present) and as 64 separate
    single-mesh steps."""
    import torch
    specs = wl.batch_specs()
    meshes, qs, works, dts = [], [], [], []
    t0 = time.perf_counter()
    for s in specs:
        xyz, vid = wl.kuhn_box_mesh(s["n"], 10.0, s["jitter"], s["mesh_seed"])
        m = dg.Mesh(s["order"], xyz, vid, 0)
        q_np = wl.vortex_state(m.nodes(), beta=s["beta"], center=s["center"])
        rho = q_np[0]
        vel = np.sqrt((q_np[1] ** 2 + q_np[2] ** 2 + q_np[3] ** 2)) / rho
        pres = (wl.GAMMA - 1.0) * (q_np[4] - 0.5 * rho * vel ** 2)
        vmax = float((vel + np.sqrt(wl.GAMMA * pres / rho)).max())
        dts.append(0.2 * (10.0 / s["n"]) / ((s["order"] + 1) ** 2 * vmax))  # CFL 0.2 on the cube size
        meshes.append(m)
        qs.append(torch.from_numpy(q_np).to(dev))
        works.append(torch.empty((2,) + q_np.shape, dtype=torch.float64, device=dev))
    setup_s = time.perf_counter() - t0
    dt = torch.tensor(dts, dtype=torch.float64, device=dev)
    batch = dg.Batch(meshes, "fp32")
    batch.bind(qs, works, dt)
    with torch.cuda.stream(stream):
        cfg, tune_ms = batch.autotune(trials=2, stream=stream)
        batch.rk_step(use_graph=True, stream=stream)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            batch.rk_step(use_graph=True, stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_graph = e0.elapsed_time(e1) / steps
        # each launch mode at its default shape, for the record
        mode_ms = {}
        for name, c in (("mixed_4x2", (4, 2, 0, 0, 0)), ("per_order_forked", (4, 2, 0, 0, 1)),
                        ("per_order_serial", (4, 2, 0, 0, 2))):
            batch.set_config(*c)
            batch.rk_step(use_graph=True, stream=stream)
            e0.record(stream)
            for _ in range(steps):
                batch.rk_step(use_graph=True, stream=stream)
            e1.record(stream)
            stream.synchronize()
            mode_ms[name] = round(e0.elapsed_time(e1) / steps, 4)
        batch.set_config(**cfg)
        batch.rk_step(use_graph=True, stream=stream)
        for m, q, w, d in zip(meshes, qs, works, dts):
            dg.rk_step(m, q, w, 0.0, d, "fp32", stream=stream)
        stream.synchronize()
        e0.record(stream)
        for _ in range(steps):
            for m, q, w, d in zip(meshes, qs, works, dts):
                dg.rk_step(m, q, w, 0.0, d, "fp32", stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_sep = e0.elapsed_time(e1) / steps
    info = batch.info()
    batch_cfg = cfg
    # the same workload with split-BF16 contractions, for comparison
    sb = dg.Batch(meshes, "split_bf16")
    sb.bind(qs, works, dt)
    with torch.cuda.stream(stream):
        cfg_s, _ = sb.autotune(trials=2, stream=stream)
        sb.rk_step(use_graph=True, stream=stream)
        stream.synchronize()
        e0.record(stream)
        for _ in range(steps):
            sb.rk_step(use_graph=True, stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_split = e0.elapsed_time(e1) / steps
    sb.close()
    cfg = batch_cfg
    dof_fields = sum(m.E * m.Np for m in meshes) * NF
    finite = all(bool(torch.isfinite(q).all()) for q in qs)
    out = {"workload": "batch64_vortex_n4to40_p1to4", "meshes": len(meshes), "elements": info["n_elem"],
           "dofs": dof_fields // NF, "work_items": info["n_items"], "contraction_precision": "fp32",
           "orders": {str(p): sum(1 for m in meshes if m.order == p) for p in range(1, 5)},
           "value": round(5 * dof_fields / (ms_graph * 1e-3) / 1e9, 3), "unit": "GDOF·fields/s (RHS evaluations)",
           "ms_per_step": round(ms_graph, 4), "separate_ms_per_step": round(ms_sep, 4),
           "separate_launches_per_step": 6 * len(meshes),
           "speedup_vs_separate": round(ms_sep / ms_graph, 3),
           "launches_per_stage": (info["graph_kernel_nodes"] - 1) // 5 if cfg["per_order"] != 1
           else info["graph_kernel_nodes"] // 6,
           "graph_kernel_nodes_per_step": info["graph_kernel_nodes"], "autotuned": cfg, "mode_ms_per_step": mode_ms,
           "autotune_best_ms": round(tune_ms, 4),
           "split_bf16": {"ms_per_step": round(ms_split, 4),
                          "value": round(5 * dof_fields / (ms_split * 1e-3) / 1e9, 3), "autotuned": cfg_s},
           "steps": steps, "state_finite": finite,
           "host_setup_s": round(setup_s, 1)}
    batch.close()
    return out


def copy_bandwidth(dev, stream, mib: int = 1024, reps: int = 20):
    """Measured HBM bandwidth of a plain device copy (torch's copy kernel,
    MIB MiB read and MIB MiB written per call, HIP events on the stream): the
    second denominator beside the 8 TB/s datasheet peak."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()  # src was filled on the default stream; the copies run on `stream`
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
        stream.synchronize()
        ms = _time_ms(stream, lambda: dst.copy_(src), reps)
    del src, dst
    return {"bytes_per_copy": 2 * n * 8, "ms_per_copy": round(ms, 5), "gbs": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}


def _time_ms(stream, fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / reps


def reacting_leg(dg, wl, dev, stream, steps):
    """Reacting Navier-Stokes with BR1 viscous terms: periodic [0, 1 cm]^3,
    32^3 cubes x 6 = 196,608 tets, 3 % jitter, p = 3, 7 species, seeded
    300-2200 K fronts.  Times the temperature Newton (plain 1000 K start),
    the gradient + right-hand-side passes and one fused LSRK step."""
    import torch
    n, p = 32, 3
    xyz, vid = wl.kuhn_box_mesh(n, 0.01, 0.03, 1003)
    mesh = dg.Mesh(p, xyz, vid, 0)
    X = mesh.nodes().reshape(-1, 3)
    q_np = wl.reacting_state(X, seed=3005, L=0.01, n_cells=n).reshape(12, mesh.E, mesh.Np)
    TH, MECH = wl.synthetic_thermo(3003), wl.synthetic_mechanism(3004)
    th = dg.Thermo(TH["W"], TH["a"])
    mk = dg.Mechanism(th, MECH["A"], MECH["Ea"], MECH["nu_r"], MECH["nu_p"])
    q = torch.from_numpy(np.ascontiguousarray(q_np)).to(dev)
    nn = mesh.E * mesh.Np
    T = torch.empty((mesh.E, mesh.Np), dtype=torch.float64, device=dev)
    it = torch.empty((mesh.E, mesh.Np), dtype=torch.int32, device=dev)
    sig = torch.empty((mesh.E, mesh.Np, 33), dtype=torch.float64, device=dev)
    out = torch.empty_like(q)
    with torch.cuda.stream(stream):
        dg.temperature(th, q, T, it, stream=stream)
        dg.ns_rhs(mesh, th, q, T, sig, out, mech=mk, stream=stream)
        stream.synchronize()
        ms_T = _time_ms(stream, lambda: dg.temperature(th, q, T, it, stream=stream), steps)
        omega = torch.empty((th.ns, mesh.E, mesh.Np), dtype=torch.float64, device=dev)
        ms_src = _time_ms(stream, lambda: dg.sources(mk, q, T, omega, stream=stream), steps)
        ms_rhs = _time_ms(stream, lambda: dg.ns_rhs(mesh, th, q, T, sig, out, mech=mk, stream=stream), steps)
        work = torch.empty(dg.NS_WORK_PER_NODE * nn, dtype=torch.float64, device=dev)
        qs, Ts = q.clone(), T.clone()
        # the seeded rates are stiff (A up to 1e12 SI): a stable explicit step is tiny
        dt_rk = 1e-14
        dg.ns_rk_step(mesh, th, qs, Ts, work, dt_rk, mech=mk, stream=stream)
        stream.synchronize()
        ms_rk = _time_ms(stream, lambda: dg.ns_rk_step(mesh, th, qs, Ts, work, dt_rk, mech=mk, stream=stream),
                         max(2, steps // 5))
    iters = it.cpu().numpy()
    finite = bool(torch.isfinite(out).all()) and bool(torch.isfinite(qs).all())
    dof_f = nn * 12
    rec = {"workload": "reacting_ns_p3_32cubed", "elements": mesh.E, "order": p, "fields": 12, "species": 7,
           "mu": dg.MU, "Pr": dg.PR, "Sc": dg.SC,
           "ns_rhs_ms": round(ms_rhs, 4), "value": round(dof_f / (ms_rhs * 1e-3) / 1e9, 3),
           "unit": "GDOF·fields/s (gradient + right-hand side, sources included)",
           "temperature_ms": round(ms_T, 4), "sources_ms": round(ms_src, 4),
           # HBM bytes per node: Newton reads 12 fields, writes T and the iteration count (108 B);
           # the sources read 7 species and T and write 7 rates (120 B)
           "temperature_gbs": round(108 * nn / (ms_T * 1e-3) / 1e9, 1),
           "sources_gbs": round(120 * nn / (ms_src * 1e-3) / 1e9, 1),
           "newton_mean_iters_from_1000K": round(float(iters.mean()), 3),
           "newton_iters_histogram": iteration_histogram(iters),
           "newton_failures": int((iters < 0).sum()), "rk_step_ms": round(ms_rk, 4), "rk_dt": dt_rk,
           "finite": finite}
    return rec


LEARNED_DT = 2e-9     # s: LSRK step of the snapshot run (acoustic CFL about 0.1 on the 32^3 p = 3 mesh)
LEARNED_STEPS = 100   # steps of the snapshot run
LEARNED_EVERY = 10    # a snapshot every this many steps (steps 0, 10, ..., 100)
LEARNED_STATES = 2_000_000
LEARNED_HELD_OUT = 0.1
LEARNED_EPOCHS = 20
LEARNED_BATCH = 4096


def learned_leg(dg, wl, dev, stream, X48):
    """Learned temperature guess: the 9-64-64-64-1 network trained on the GPU
    (BF16 matrix cores, FP32 masters, Adam, lr 1e-3) on states the reacting
    solver produces: the 32^3 p = 3 reacting run (seeded fronts, sources off,
    LSRK steps of LEARNED_DT) snapshotted every LEARNED_EVERY steps, targets
    from plain-guess Newton; 2M states sampled without replacement (seed
    4001), 10 % held out; init seed 4002, shuffle seed 4003.  Then evaluated
    inside Newton on the 48^3 p = 3 mesh's 13.27M nodes carrying reacting
    fields (coordinates scaled to the 1 cm box).  Plain Newton from 1000 K is
    the reference."""
    import torch
    TH = wl.synthetic_thermo(3003)
    th = dg.Thermo(TH["W"], TH["a"])
    n32, p = 32, 3
    xyz, vid = wl.kuhn_box_mesh(n32, 0.01, 0.03, 1003)
    m32 = dg.Mesh(p, xyz, vid, 0)
    nn = m32.E * m32.Np
    q = torch.from_numpy(wl.reacting_state(m32.nodes().reshape(-1, 3), seed=3005, L=0.01, n_cells=n32)
                         .reshape(12, m32.E, m32.Np)).to(dev)
    T = torch.empty((m32.E, m32.Np), dtype=torch.float64, device=dev)
    it = torch.empty((m32.E, m32.Np), dtype=torch.int32, device=dev)
    work = torch.empty(dg.NS_WORK_PER_NODE * nn, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        dg.temperature(th, q, T, it, stream=stream)
        snaps = [q.reshape(12, nn).clone()]
        for step in range(1, LEARNED_STEPS + 1):
            dg.ns_rk_step(m32, th, q, T, work, LEARNED_DT, mech=None, stream=stream)
            if step % LEARNED_EVERY == 0:
                snaps.append(q.reshape(12, nn).clone())
        dg.synchronize(0, stream)
    run_s = time.perf_counter() - t0
    del work, T, it
    qtr = torch.cat(snaps, dim=1).contiguous()
    del snaps
    ntr = qtr.shape[1]
    Ttr = torch.empty(ntr, dtype=torch.float64, device=dev)
    itr = torch.empty(ntr, dtype=torch.int32, device=dev)
    dg.temperature(th, qtr, Ttr, itr)
    pick = torch.randperm(ntr, generator=torch.Generator().manual_seed(4001))[:LEARNED_STATES].to(dev)
    n_val = int(LEARNED_HELD_OUT * LEARNED_STATES)
    val, train = pick[:n_val].contiguous(), pick[n_val:].contiguous()
    net = dg.MLP(seed=4002)
    net.fit_normalization(qtr, train, Ttr)
    gen = torch.Generator().manual_seed(4003)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    batch = LEARNED_BATCH
    nb = train.numel() // batch

    def held_out_loss():
        acc, cnt = 0.0, 0
        for b in range(0, val.numel(), batch):
            sl = val[b:b + batch]
            net.loss_grad(qtr, sl, Ttr, loss=loss, stream=stream)
            stream.synchronize()
            acc += loss.item() * sl.numel()
            cnt += sl.numel()
        return acc / cnt

    torch.cuda.synchronize()  # the training set and loss were made on the default stream
    t0 = time.perf_counter()
    epoch_loss = []
    with torch.cuda.stream(stream):
        for ep in range(LEARNED_EPOCHS):
            perm = train[torch.randperm(train.numel(), generator=gen).to(dev)]
            for b in range(nb):
                net.train_step(qtr, perm[b * batch:(b + 1) * batch], Ttr, lr=1e-3, loss=loss, stream=stream)
            if ep in (0, LEARNED_EPOCHS // 2 - 1, LEARNED_EPOCHS - 1):
                epoch_loss.append((ep + 1, loss.item()))
        stream.synchronize()
    train_s = time.perf_counter() - t0
    with torch.cuda.stream(stream):
        val_loss = held_out_loss()
        qv = qtr.index_select(1, val).contiguous()
        Tv_pred = torch.empty(n_val, dtype=torch.float64, device=dev)
        net.predict(qv, Tv_pred, stream=stream)
        stream.synchronize()
    val_rms = float(((Tv_pred - Ttr.index_select(0, val)) ** 2).mean().sqrt().item())
    del qtr, Ttr, itr, pick, qv
    # evaluation on the 48^3 mesh's nodes
    q = torch.from_numpy(wl.reacting_state(X48.reshape(-1, 3) * 1e-3, seed=3005, L=0.01, n_cells=48)).to(dev)
    n = q.shape[1]
    Tp, ip = torch.empty(n, dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.int32, device=dev)
    Tl, il = torch.empty_like(Tp), torch.empty_like(ip)
    fb = torch.zeros(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()  # fb was cleared on the default stream
    with torch.cuda.stream(stream):
        dg.temperature(th, q, Tp, ip, stream=stream)
        dg.temperature_learned(th, net, q, Tl, il, fallback_count=fb, stream=stream)
        stream.synchronize()
        ms_p = _time_ms(stream, lambda: dg.temperature(th, q, Tp, ip, stream=stream), 10)
        fb.zero_()
        ms_l = _time_ms(stream, lambda: dg.temperature_learned(th, net, q, Tl, il, fallback_count=fb,
                                                               stream=stream), 10)
    fallbacks = fb.item() / 10  # counted over the 10 timed calls
    Tpred = torch.empty_like(Tp)
    net.predict(q, Tpred)
    torch.cuda.synchronize()
    ipn, iln = ip.cpu().numpy(), il.cpu().numpy()
    return {"workload": "reacting_fields_on_48cubed_p3_nodes", "nodes": n,
            "train": {"source": f"32^3 p=3 reacting NS run (sources off), dt {LEARNED_DT:g} s, snapshots every "
                                f"{LEARNED_EVERY} of {LEARNED_STEPS} steps", "pool_states": ntr,
                      "states": LEARNED_STATES, "held_out": n_val, "batch": batch, "epochs": LEARNED_EPOCHS,
                      "adam_steps": LEARNED_EPOCHS * nb, "batch_loss_by_epoch": epoch_loss,
                      "held_out_loss": round(val_loss, 8), "held_out_rms_error_K": round(val_rms, 4),
                      "run_seconds": round(run_s, 2), "train_seconds": round(train_s, 2),
                      "samples_per_s": round(LEARNED_EPOCHS * nb * batch / train_s, 1)},
            "plain": {"ms": round(ms_p, 4), "mean_iters": round(float(ipn.mean()), 3),
                      "failures": int((ipn < 0).sum()), "iters_histogram": iteration_histogram(ipn)},
            "learned": {"ms": round(ms_l, 4), "mean_iters": round(float(iln.mean()), 3),
                        "fallbacks": fallbacks, "fallback_rate": fallbacks / n,
                        "iters_histogram": iteration_histogram(iln),
                        "max_abs_dT_vs_plain_K": float((Tl - Tp).abs().max().item()),
                        "guess_rms_error_K": float(((Tpred - Tp) ** 2).mean().sqrt().item())},
            "speedup_vs_plain": round(ms_p / ms_l, 3)}


HEX_WORKLOADS = (("hex_vortex_pert_p4_48cubed", 48, 4), ("hex_vortex_pert_p1_120cubed", 120, 1))


def hex_oi_flops(p: int) -> int:
    """FP64 flops per element of the overintegrated RHS: interpolation to
    the nq^3 points (3 passes x 5 fields), fluxes (about 33 flop per point
    and field triple), projection back (3 directions x 3 passes x 5 fields),
    and per face two interpolations and two projections of 5 fields, the
    Lax-Friedrichs flux (about 80 flop per face point) and the lift."""
    n, q = p + 1, -(-3 * (p + 1) // 2)
    interp = 5 * 2 * (n * n * q * n + n * q * q * n + q * q * q * n)
    flux = 5 * 3 * 11 * q ** 3
    proj = 5 * 3 * 2 * (q * q * n * q + q * n * n * q + n ** 3 * q)
    face = 6 * (2 * 5 * 2 * (n * q * n + q * q * n) + 80 * q * q + 5 * 2 * (q * n * q + n * n * q) + 5 * 2 * n ** 3)
    return interp + flux + proj + face


def hex_leg(dg, hexdg, wl, dev, stream, steps, warmup):
    """Tensor-product hexahedra (the element of the paper's own vortex
    benchmark): periodic rectilinear [0,10]^3 boxes with 5 % grid-line
    jitter, vortex plus the seeded density perturbation, at p = 4 (48^3
    cells) and p = 1 (120^3 cells), 13.8M nodes each.  Times the
    sum-factorised FP64 RHS (settle, warm-up, one batch of `steps` launches
    and five more for the spread) and the LSRK step; the roofline is HBM:
    the state in and the rhs out, 2 x 5 x Np x 8 bytes per element."""
    import torch
    out = {}
    for name, n, p in HEX_WORKLOADS:
        lines = wl.rectilinear_box(n, 10.0, 0.05, 1002)
        m = hexdg.HexMesh(p, *lines)
        q = torch.from_numpy(wl.vortex_state(m.nodes(), pert=wl.density_perturbation(2002))).to(dev)
        r = torch.empty_like(q)
        launch = lambda: hexdg.rhs(m, q, r, stream=stream)
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < SETTLE_S:
                for _ in range(50):
                    launch()
                stream.synchronize()
            for _ in range(warmup):
                launch()
            stream.synchronize()
            batches = [_time_ms(stream, launch, steps) for _ in range(1 + REPEATS)]
            work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
            qs = q.clone()
            hexdg.rk_step(m, qs, work, 0.0, 1e-4, stream=stream)
            stream.synchronize()
            ms_rk = _time_ms(stream, lambda: hexdg.rk_step(m, qs, work, 0.0, 1e-4, stream=stream), max(2, steps // 10))
        dg.synchronize(0, stream)
        ms = batches[0]
        bytes_el = 2 * 5 * m.Np * 8
        gbs = bytes_el * m.E / (ms * 1e-3) / 1e9
        # overintegrated form, same workload: FP64-pipe bound
        with torch.cuda.stream(stream):
            launch_oi = lambda: hexdg.rhs_oi(m, q, r, stream=stream)
            for _ in range(max(warmup, 5)):
                launch_oi()
            stream.synchronize()
            ms_oi = _time_ms(stream, launch_oi, steps)
            qs2 = q.clone()
            ms_oi_rk = _time_ms(stream, lambda: hexdg.rk_step(m, qs2, work, 0.0, 1e-4, overintegrate=True,
                                                              stream=stream), max(2, steps // 10))
        dg.synchronize(0, stream)
        fl = hex_oi_flops(p)
        tf = fl * m.E / (ms_oi * 1e-3) / 1e12
        oi_rec = {"gauss_points_per_direction": -(-3 * (p + 1) // 2), "ms_per_rhs": round(ms_oi, 5),
                  "value": round(m.E * m.Np * NF / (ms_oi * 1e-3) / 1e9, 3), "unit": "GDOF·fields/s",
                  "roofline": {"bound": "fp64", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(tf / PEAK_FP64_TFLOPS, 4), "flops_per_elem": fl,
                               "kernel": f"hex_oi_kernel<{p}>"},
                  "lsrk_step_ms": round(ms_oi_rk, 4), "cost_vs_collocated": round(ms_oi / ms, 3)}
        del qs2
        out[name] = {"elements": m.E, "order": p, "nodes_per_element": m.Np, "ms_per_rhs": round(ms, 5),
                     "ms_per_rhs_spread": {"median": round(float(np.median(batches)), 5),
                                           "min": round(min(batches), 5), "max": round(max(batches), 5)},
                     "value": round(m.E * m.Np * NF / (ms * 1e-3) / 1e9, 3), "unit": "GDOF·fields/s",
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_elem": bytes_el,
                                  "kernel": "hex_rhs_tile_kernel<1, 4, 4, 2>" if p == 1 else f"hex_rhs_kernel<{p}>"},
                     "lsrk_step_ms": round(ms_rk, 4), "overintegrated": oi_rec}
        del q, r, work, qs
        m.close()
    return out


SHOCK_WORKLOADS = (("hex_shock_slab_p1_120cubed", 120, 1), ("hex_shock_slab_p4_48cubed", 48, 4))


def shock_leg(dg, hexdg, wl, dev, stream, steps, warmup):
    """Shock capturing on the hexahedra: the density slab at rest (ratio 100,
    p = rho / gamma, rippled interfaces) on periodic rectilinear [0,10]^3
    boxes with 5 % grid-line jitter, p = 1 (120^3 cells, the paper's shock
    cases use degree-1 tensor-product elements) and p = 4 (48^3).  Times
    the indicator + viscous-flux kernel, the RHS with artificial viscosity,
    the limiter, and the LSRK step with viscosity and stage limiting against
    the plain step (timed on gas at rest: without shock capturing the slab
    loses positivity within a few steps)."""
    import torch
    out = {}
    for name, n, p in SHOCK_WORKLOADS:
        lines = wl.rectilinear_box(n, 10.0, 0.05, 1002)
        m = hexdg.HexMesh(p, *lines)
        q = torch.from_numpy(wl.shock_slab_state(m.nodes())).to(dev)
        r = torch.empty_like(q)
        nn = m.E * m.Np
        G = torch.empty((3, 5, m.E, m.Np), dtype=torch.float64, device=dev)
        eps = torch.empty(m.E, dtype=torch.float64, device=dev)
        work = torch.empty(hexdg.SHOCK_STEP_WORK * nn + 2 * m.E, dtype=torch.float64, device=dev)
        wplain = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
        av = hexdg.av_params(p)
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                hexdg.av_rhs(m, q, r, work, av, stream=stream)
            stream.synchronize()
            ms_flux = _time_ms(stream, lambda: hexdg.av_viscosity(m, q, G, None, eps, av, stream=stream), steps)
            ms_rhs = _time_ms(stream, lambda: hexdg.av_rhs(m, q, r, work, av, stream=stream), steps)
            ms_plain = _time_ms(stream, lambda: hexdg.rhs(m, q, r, stream=stream), steps)
            ql = q.clone()
            ms_lim = _time_ms(stream, lambda: hexdg.limit(m, ql, av, stream=stream), steps)
            qs = q.clone()
            dt = 1e-4
            ms_step = _time_ms(stream, lambda: hexdg.shock_rk_step(m, qs, work, 0.0, dt, av, stream=stream),
                               max(2, steps // 10))
            dg.synchronize(0, stream)
            # the plain step has no shock capturing: on the slab it loses
            # positivity within a few steps, so it is timed on gas at rest
            # (its cost does not depend on the values)
            qp = torch.zeros_like(q)
            qp[0] = 1.2
            qp[4] = 1.2 / (1.4 * 0.4)
            ms_pstep = _time_ms(stream, lambda: hexdg.rk_step(m, qp, wplain, 0.0, dt, stream=stream), max(2, steps // 10))
        dg.synchronize(0, stream)
        viscous = int((eps > 0).sum().item())
        # algorithmic bytes of the two passes per element: the state read by
        # both, the rhs written, indicator and viscosity (16 + 8 B), and for
        # the viscous elements G (3 x 5 x Np doubles) written once, read once
        bytes_av = m.E * (120 * m.Np + 24) + viscous * 240 * m.Np
        gbs_av = bytes_av / (ms_rhs * 1e-3) / 1e9
        out[name] = {"elements": m.E, "order": p, "viscous_elements": viscous,
                     "ms_indicator_and_viscous_flux": round(ms_flux, 4), "ms_rhs_with_av": round(ms_rhs, 4),
                     "ms_rhs_plain": round(ms_plain, 4), "ms_limiter": round(ms_lim, 4),
                     "ms_step_with_av_and_limiter": round(ms_step, 4), "ms_step_plain": round(ms_pstep, 4),
                     "value": round(nn * NF / (ms_rhs * 1e-3) / 1e9, 3),
                     "unit": "GDOF·fields/s (RHS with artificial viscosity)",
                     "roofline": {"bound": "hbm", "achieved": round(gbs_av, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": round(gbs_av / PEAK_HBM_GBS, 4), "bytes": int(bytes_av),
                                  "kernels": ("hex_av_flux_tile_kernel + hex_rhs_tile_kernel (viscous variant)" if p == 1
                                              else "hex_av_flux_kernel + hex_rhs_kernel (viscous variant)")},
                     "state_finite": bool(torch.isfinite(qs).all()), "min_density_after_steps": float(qs[0].min())}
        del q, r, G, eps, work, wplain, ql, qs, qp
        m.close()
    return out


def iteration_histogram(iters):
    """{iterations: node count} of a Newton solve (-1 = failed)."""
    vals, counts = np.unique(iters, return_counts=True)
    return {str(int(v)): int(c) for v, c in zip(vals, counts)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="all", choices=["all", "fp64", "fp32", "split_bf16"],
                    help="contraction precision; 'all' times FP64 (the reported value) then FP32 and split BF16")
    ap.add_argument("--no-rk", action="store_true", help="skip the LSRK step timing")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="elements in the CPU-baseline sample (-1: the whole mesh, 0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="BLAS threads of the CPU baseline's second timing (the first uses one)")
    ap.add_argument("--long-steps", type=int, default=100,
                    help="LSRK steps of the reduced-precision forms against the FP64 form (0: skip)")
    ap.add_argument("--n", type=int, default=WORKLOAD["n"], help="cubes per side (default: the 48^3 workload)")
    ap.add_argument("--launch", default=DEFAULT_LAUNCH,
                    help="launch shape of the single-mesh legs, 'waves_per_block,rk_fused,lds_stage,xcd_run' "
                         "for every precision, or 'auto' for the autotuner's choice per precision")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-mesh batched leg")
    ap.add_argument("--no-hex", action="store_true", help="skip the hexahedron leg")
    ap.add_argument("--no-shock", action="store_true", help="skip the shock-capturing leg")
    ap.add_argument("--hex-only", action="store_true", help="run only the hexahedron leg")
    ap.add_argument("--batched-only", action="store_true", help="run only the 64-mesh batched leg")
    ap.add_argument("--no-reacting", action="store_true", help="skip the reacting NS and learned-guess legs")
    ap.add_argument("--reacting-only", action="store_true", help="run only the reacting NS and learned-guess legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the method would shard by "
              "element partition across GPUs with a face-trace exchange per stage; only one GPU is run)",
              file=sys.stderr)
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
    if args.hex_only:
        from paper_2512_17101_amd import hexdg
        stream = torch.cuda.Stream(device=dev)
        rec = {"hex": hex_leg(dg, hexdg, wl, dev, stream, args.steps, args.warmup)}
        if not args.no_shock:
            rec["shock"] = shock_leg(dg, hexdg, wl, dev, stream, args.steps, args.warmup)
        print(json.dumps(rec), flush=True)
        return
    if args.batched_only:
        stream = torch.cuda.Stream(device=dev)
        print(json.dumps({"batched": batched_leg(dg, wl, dev, stream, max(2, args.steps // 10))}), flush=True)
        return
    if args.reacting_only:
        stream = torch.cuda.Stream(device=dev)
        xyz, vid = wl.kuhn_box_mesh(WORKLOAD["n"], 10.0, WORKLOAD["jitter"], WORKLOAD["mesh_seed"])
        X48 = dg.Mesh(WORKLOAD["order"], xyz, vid, 0).nodes()
        rec = {"reacting": reacting_leg(dg, wl, dev, stream, max(2, args.steps // 5))}
        print(json.dumps(rec), flush=True)
        rec["learned_guess"] = learned_leg(dg, wl, dev, stream, X48)
        print(json.dumps(rec), flush=True)
        return
    p = WORKLOAD["order"]
    xyz, vid = wl.kuhn_box_mesh(args.n, 10.0, WORKLOAD["jitter"], WORKLOAD["mesh_seed"])
    mesh = dg.Mesh(p, xyz, vid, 0)
    X = mesh.nodes()
    q_np = wl.vortex_state(X, pert=wl.density_perturbation(WORKLOAD["pert_seed"]))
    q = torch.from_numpy(q_np).to(dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    E, Np = mesh.E, mesh.Np
    modes = ["fp64", "fp32", "split_bf16"] if args.precision == "all" else [args.precision]
    outs, ms, spread, tuned = {}, {}, {}, {}
    for mode in modes:
        # the launch shape (tiles per block, fused or split stages, LDS
        # staging, XCD run length): fixed, so that runs and profiles of the
        # bench time the same kernels, or the autotuner's choice (it times
        # whole Runge-Kutta steps of this mesh, and candidates within its
        # noise may win)
        if args.launch == "auto":
            with torch.cuda.stream(stream):
                mesh.autotune(mode, trials=3, stream=stream)
        else:
            mesh.set_launch(mode, *parse_launch(args.launch))
        tuned[mode] = mesh.get_launch(mode)
        outs[mode] = torch.empty_like(q)
        ms[mode], spread[mode] = time_rhs(dg, mesh, q, outs[mode], mode, args.steps, args.warmup, stream)
    torch.cuda.synchronize()
    head = modes[0]
    value = E * Np * NF / (ms[head] * 1e-3) / 1e9
    flops, bytes_ = algorithmic_counts(p)
    kflops, kbytes = kernel_counts(p)
    achieved_tf = flops * E / (ms[head] * 1e-3) / 1e12
    achieved_gbs = bytes_ * E / (ms[head] * 1e-3) / 1e9
    # the stored counters describe the FP64 kernel on the 48^3 workload only
    on_workload = args.n == WORKLOAD["n"]
    counters = stored_counters(tuned[head]) if head == "fp64" and on_workload else {}
    copy_bw = copy_bandwidth(dev, stream)  # measured after the timed launches
    hbm_view = {"achieved": round(achieved_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / PEAK_HBM_GBS, 4), "measured_copy_gbs": copy_bw["gbs"],
                "frac_of_measured_copy": round(achieved_gbs / copy_bw["gbs"], 4)}
    if head == "fp64":
        roofline = {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4), "traffic": counters.get("traffic"),
                    "kernel": f"rhs_euler_fp64_kernel<{p}>", "flops_per_elem": flops, "bytes_per_elem": bytes_,
                    "kernel_flops_per_elem": kflops, "kernel_bytes_per_elem": kbytes,
                    "mfma_busy": counters.get("mfma_busy"), "hbm_view": hbm_view}
    else:
        # reduced-precision contractions: the FP64 pipe keeps only the
        # pointwise work, and the kernel's bound is HBM
        roofline = dict(hbm_view, bound="hbm", traffic=None, kernel=f"rhs_euler_lowp_kernel<{p}>",
                        flops_per_elem=flops, bytes_per_elem=bytes_)
    rec = {"metric": METRIC, "value": round(value, 3), "unit": "GDOF·fields/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms[head], 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16x3-f32acc"}[head], "data": "synthetic",
           "config": {"workload": WORKLOAD["name"] if on_workload else f"euler_vortex_pert_p3_{args.n}cubed",
                      "elements": E, "order": p, "nodes_per_element": Np, "fields": NF,
                      "contraction_precision": head},
           "roofline": roofline, "ms_per_step_spread": spread[head], "copy_bandwidth": copy_bw,
           "launch": tuned[head]}
    variants = {}
    for mode in modes[1:]:
        gbs = bytes_ * E / (ms[mode] * 1e-3) / 1e9
        variants[mode] = {"value": round(E * Np * NF / (ms[mode] * 1e-3) / 1e9, 3), "ms_per_step": round(ms[mode], 5),
                          "ms_per_step_spread": spread[mode], "speedup_vs_fp64": round(ms[head] / ms[mode], 3),
                          "launch": tuned[mode],
                          "hbm_view": {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                       "frac": round(gbs / PEAK_HBM_GBS, 4), "measured_copy_gbs": copy_bw["gbs"],
                                       "frac_of_measured_copy": round(gbs / copy_bw["gbs"], 4)}}
    if not args.no_rk:
        work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
        qs = q.clone()
        torch.cuda.synchronize()  # qs was written on the default stream; the steps run on `stream`
        for mode in modes:
            t_rk, sp_rk = time_rk_step(dg, mesh, qs, work, 1e-4, mode, max(2, args.steps // 10), stream)
            (rec if mode == head else variants[mode])["lsrk_step_ms"] = round(t_rk, 4)
            (rec if mode == head else variants[mode])["lsrk_step_ms_spread"] = sp_rk
        dg.synchronize(0, stream)  # raises if a step produced a non-finite state
        if len(modes) > 1 and args.long_steps > 0:
            rec["after_steps"] = long_run_errors(dg, mesh, q, q_np, work, modes, args.long_steps, stream)
            dg.synchronize(0, stream)
        del work, qs
    if args.cpu_sample != 0:
        state = lambda Xn: wl.vortex_state(Xn, pert=wl.density_perturbation(WORKLOAD["pert_seed"]))
        cpu, idx, ref, mag = cpu_baseline(xyz, vid, state, p, args.cpu_sample, args.cpu_threads)
        rec["cpu_baseline"] = cpu
        idx_t = torch.from_numpy(idx).to(dev)
        for mode in modes:
            got = outs[mode].index_select(1, idx_t).cpu().numpy()
            errs = field_errors(got, ref)
            if mode == "fp64":
                ratio = entry_ratios(got, ref, mag, p)
                for f, nm in enumerate(FIELDS):
                    errs[nm].update(ratio[nm])
            if mode == head:
                rec["error_vs_oracle"] = errs
            else:
                variants[mode]["error_vs_oracle"] = errs
    if variants:
        rec["variants"] = variants
    if not args.no_hex:
        from paper_2512_17101_amd import hexdg
        torch.cuda.empty_cache()
        rec["hex"] = hex_leg(dg, hexdg, wl, dev, stream, args.steps, args.warmup)
        if not args.no_shock:
            rec["shock"] = shock_leg(dg, hexdg, wl, dev, stream, args.steps, args.warmup)
    if not args.no_batched:
        del outs
        torch.cuda.empty_cache()
        rec["batched"] = batched_leg(dg, wl, dev, stream, max(2, args.steps // 10))
    if not args.no_reacting:
        torch.cuda.empty_cache()
        rec["reacting"] = reacting_leg(dg, wl, dev, stream, max(2, args.steps // 5))
        rec["learned_guess"] = learned_leg(dg, wl, dev, stream, X)
    rec["paper_context"] = paper_context(rec)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
