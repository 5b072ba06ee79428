"""GPU batched stepping of many meshes of mixed order, through the C ABI.

Bar: every mesh of a batch after batched LSRK steps is bitwise the state the
single-mesh step gives it at the same precision and time step, for every
launch shape of both launch modes, with and without the captured graph
(whose kernel nodes are five stages and one copy, once in the mixed-order
mode and with the stages once per order present in the per-order modes),
after tuning; and
the batched state tracks the oracle's FP64 steps within the
reduced-precision bar of the single-mesh tests."""
import json

import numpy as np
import pytest

from oracle import euler as oe, lsrk as olsrk, mesh as om, precision as opr, reference_element as ore
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (cubes per side, order): tile counts with ragged tails (6 n^3 = 162, 384, 750)
SHAPES = [(3, 1), (3, 4), (4, 2), (3, 3), (5, 1), (3, 2), (4, 4)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _problem(shapes=SHAPES, seed=77):
    dev = _dev()
    meshes, q0, dts, host = [], [], [], []
    rng = np.random.default_rng(seed)
    for i, (n, p) in enumerate(shapes):
        xyz, vid = wl.kuhn_box_mesh(n, 10.0, 0.05, 900 + i)
        m = dg.Mesh(p, xyz, vid)
        ops = ore.operators(p)
        geo = om.geometry(xyz)
        q = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]), beta=rng.uniform(3, 5),
                            center=tuple(rng.uniform(3, 7, 2)))
        q = q * (1.0 + 1e-3 * rng.standard_normal(q.shape))  # jumping face traces
        dt = oe.cfl_dt(ops, geo, q, 0.2)
        meshes.append(m)
        q0.append(q)
        dts.append(dt)
        host.append((xyz, vid, ops, geo))
    return dev, meshes, q0, np.array(dts), host


def _single(meshes, q0, dts, steps, mode, dev):
    out = []
    for m, q_np, dt in zip(meshes, q0, dts):
        q = torch.from_numpy(q_np).to(dev)
        work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
        for s in range(steps):
            dg.rk_step(m, q, work, s * dt, dt, mode)
        out.append(q)
    torch.cuda.synchronize()
    return [q.cpu().numpy() for q in out]


def _bound(batch, q0, dev, dts):
    qs = [torch.from_numpy(q).to(dev) for q in q0]
    works = [torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev) for q in qs]
    dt = torch.tensor(dts, dtype=torch.float64, device=dev)
    batch.bind(qs, works, dt)
    return qs, works, dt


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
@pytest.mark.parametrize("per_order", [0, 1, 2])
def test_batch_equals_single_mesh_bitwise(mode, per_order):
    dev, meshes, q0, dts, _ = _problem()
    steps = 3
    ref = _single(meshes, q0, dts, steps, mode, dev)
    b = dg.Batch(meshes, mode)
    b.set_config(per_order=per_order)
    info = b.info()
    assert info["n_elem"] == sum(6 * n ** 3 for n, _ in SHAPES)
    assert info["n_items"] == sum((6 * n ** 3 + 15) // 16 for n, _ in SHAPES)
    for use_graph in (False, True):
        qs, works, dt = _bound(b, q0, dev, dts)
        for _ in range(steps):
            b.rk_step(use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (q, r) in enumerate(zip(qs, ref)):
            assert np.array_equal(q.cpu().numpy(), r), f"mesh {i} (n, p) = {SHAPES[i]} graph={use_graph}"
    # five stages + one copy per step; per order present (1..4) in the per-order modes
    assert b.info()["graph_kernel_nodes"] == {0: 6, 1: 24, 2: 21}[per_order]


@pytest.mark.parametrize("shapes", [[(3, 2), (4, 2), (3, 2)], [(4, 1), (3, 3)]])
def test_per_order_mode_with_fewer_orders(shapes):
    """One order (no stream fork) and two orders (one side stream)."""
    dev, meshes, q0, dts, _ = _problem(shapes=shapes, seed=83)
    ref = _single(meshes, q0, dts, 2, "split_bf16", dev)
    b = dg.Batch(meshes, "split_bf16")
    assert b.get_config()["per_order"] == 1
    qs, _, _ = _bound(b, q0, dev, dts)
    b.rk_step(use_graph=False)
    b.rk_step(use_graph=True)
    torch.cuda.synchronize()
    for q, r in zip(qs, ref):
        assert np.array_equal(q.cpu().numpy(), r)
    assert b.info()["graph_kernel_nodes"] == 6 * len({p for _, p in shapes})


@pytest.mark.parametrize("cfg", [(2, 1, 0, 0, 0), (8, 1, 1, 1, 0), (4, 4, 1, 0, 0), (2, 3, 0, 1, 0), (2, 1, 1, 1, 1),
                                 (4, 2, 0, 0, 2)])
def test_every_launch_shape_gives_the_same_bits(cfg):
    dev, meshes, q0, dts, _ = _problem(seed=78)
    ref = _single(meshes, q0, dts, 2, "fp32", dev)
    b = dg.Batch(meshes, "fp32")
    b.set_config(*cfg)
    assert b.get_config() == dict(waves_per_block=cfg[0], blocks_per_cu=cfg[1], order=cfg[2], xcd_chunks=cfg[3],
                                  per_order=cfg[4])
    qs, _, _ = _bound(b, q0, dev, dts)
    for _ in range(2):
        b.rk_step(use_graph=True)
    torch.cuda.synchronize()
    for q, r in zip(qs, ref):
        assert np.array_equal(q.cpu().numpy(), r)


def test_graph_replays_see_new_time_steps_and_eager_work():
    """dt is read from device memory on every replay: changing it between
    replays (with eager work in between) changes the step like the single-mesh
    call with the new dt; every replay is checked."""
    dev, meshes, q0, dts, _ = _problem(shapes=SHAPES[:4], seed=79)
    b = dg.Batch(meshes, "fp32")
    qs, _, dt = _bound(b, q0, dev, dts)
    ref_q = [torch.from_numpy(q).to(dev) for q in q0]
    ref_w = [torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev) for q in ref_q]
    for rep in range(4):
        scale = 1.0 - 0.2 * rep
        dt.copy_(torch.tensor(dts * scale, dtype=torch.float64))
        _ = torch.ones(1000, device=dev).sum()  # unrelated eager work between replays
        b.rk_step(use_graph=True)
        for m, q, w, d in zip(meshes, ref_q, ref_w, dts):
            dg.rk_step(m, q, w, 0.0, d * scale, "fp32")
        torch.cuda.synchronize()
        for i, (a, r) in enumerate(zip(qs, ref_q)):
            assert torch.equal(a, r), f"replay {rep} mesh {i}"


def test_batch_tracks_oracle_steps():
    """Two batched FP32 steps per mesh stay within 1e-5 (relative, per field)
    of the oracle's FP32-emulating steps and within 1e-4 of its FP64 steps."""
    dev, meshes, q0, dts, host = _problem(shapes=[(3, 1), (3, 2), (3, 3), (3, 4)], seed=80)
    b = dg.Batch(meshes, "fp32")
    qs, _, _ = _bound(b, q0, dev, dts)
    for _ in range(2):
        b.rk_step()
    torch.cuda.synchronize()
    for (xyz, vid, ops, geo), m, q_init, q, dt in zip(host, meshes, q0, qs, dts):
        conn = om.connectivity(vid, m.order)
        f32 = lambda qq, tt: opr.rhs(ops, geo, conn, qq, "fp32")[0]
        f64 = lambda qq, tt: oe.rhs(ops, geo, conn, qq)
        qe, qd = q_init.copy(), q_init.copy()
        for s in range(2):
            qe, _ = olsrk.lsrk_step(f32, qe, s * dt, dt)
            qd, _ = olsrk.lsrk_step(f64, qd, s * dt, dt)
        scale = np.abs(qd).max(axis=(1, 2))
        scale[1:4] = scale[1:4].max()
        got = q.cpu().numpy()
        e32 = np.abs(got - qe).max(axis=(1, 2)) / scale
        e64 = np.abs(got - qd).max(axis=(1, 2)) / scale
        print(f"p={m.order} E={m.E}: rel diff vs FP32 emulation {e32}, vs FP64 {e64}")
        assert np.all(e32 <= 1e-5) and np.all(e64 <= 1e-4)


def test_autotune_restores_state_and_uses_cache(tmp_path):
    dev, meshes, q0, dts, _ = _problem(seed=81)
    b = dg.Batch(meshes, "fp32")
    qs, _, _ = _bound(b, q0, dev, dts)
    cache = tmp_path / "tune.json"
    cfg, ms = b.autotune(cache_path=cache, trials=2)
    torch.cuda.synchronize()
    assert ms > 0
    assert cfg == b.get_config()
    for q, r in zip(qs, q0):
        assert np.array_equal(q.cpu().numpy(), r)  # state as it was
    doc = json.loads(cache.read_text())
    (key, entry), = doc["entries"].items()
    assert {k: entry[k] for k in cfg} == cfg
    # a second batch of the same meshes takes the cached choice without timing
    b2 = dg.Batch(meshes, "fp32")
    _bound(b2, q0, dev, dts)
    cfg2, ms2 = b2.autotune(cache_path=cache, trials=2)
    assert cfg2 == cfg and ms2 < 0
    # and the tuned batch still steps bitwise like the single-mesh call
    ref = _single(meshes, q0, dts, 1, "fp32", dev)
    b.rk_step()
    torch.cuda.synchronize()
    for q, r in zip(qs, ref):
        assert np.array_equal(q.cpu().numpy(), r)


def test_batch_error_paths():
    dev, meshes, q0, dts, _ = _problem(shapes=SHAPES[:2], seed=82)
    with pytest.raises(dg.DGError, match="UNSUPPORTED"):
        dg.Batch(meshes, "fp64")
    b = dg.Batch(meshes, "fp32")
    with pytest.raises(dg.DGError, match="no state bound"):
        b.rk_step()
    with pytest.raises(dg.DGError, match="waves_per_block"):
        b.set_config(3, 1, 0, 0)
    with pytest.raises(dg.DGError):
        b.set_config(4, 5, 0, 0)
    with pytest.raises(dg.DGError, match="per_order"):
        b.set_config(4, 2, 0, 0, 3)
    qs = [torch.from_numpy(q).to(dev) for q in q0]
    big = [torch.empty(3 * q.numel(), dtype=torch.float64, device=dev) for q in qs]
    overl = [w[q.numel() // 2:] for w, q in zip(big, qs)]  # work overlapping its q
    fake_q = [w[: q.numel()].view(q.shape) for w, q in zip(big, qs)]
    with pytest.raises(dg.DGError, match="overlaps"):
        b.bind(fake_q, overl, torch.tensor(dts, dtype=torch.float64, device=dev))
    assert b.get_config() == dict(waves_per_block=4, blocks_per_cu=2, order=0, xcd_chunks=0, per_order=1)


def test_full_size_batch_equals_separate_steps():
    """The benchmark's batched workload in full: 64 boxes of 4^3..40^3 cubes
    (7.22M tets, 153.3M nodes), p = 1..4 mixed, FP32 contractions.  One
    graph-replayed batched step in each per-order mode equals 64 separate
    single-mesh steps bitwise (compared on the device)."""
    dev = _dev()
    specs = wl.batch_specs()
    meshes, q0, dts = [], [], []
    for s in specs:
        xyz, vid = wl.kuhn_box_mesh(s["n"], 10.0, s["jitter"], s["mesh_seed"])
        m = dg.Mesh(s["order"], xyz, vid)
        q0.append(torch.from_numpy(wl.vortex_state(m.nodes(), beta=s["beta"], center=s["center"])).to(dev))
        meshes.append(m)
        dts.append(0.2 * (10.0 / s["n"]) / ((s["order"] + 1) ** 2 * 2.0))
    assert sum(m.E for m in meshes) == 7218618
    ref = []
    for m, q, d in zip(meshes, q0, dts):
        r = q.clone()
        w = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
        dg.rk_step(m, r, w, 0.0, d, "fp32")
        ref.append(r)
        del w
    b = dg.Batch(meshes, "fp32")
    dt = torch.tensor(dts, dtype=torch.float64, device=dev)
    for per_order in (1, 2):
        b.set_config(per_order=per_order)
        qs = [q.clone() for q in q0]
        works = [torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev) for q in qs]
        b.bind(qs, works, dt)
        b.rk_step(use_graph=True)
        torch.cuda.synchronize()
        for i, (a, r) in enumerate(zip(qs, ref)):
            assert torch.equal(a, r), f"per_order={per_order} mesh {i} (n, p) = ({specs[i]['n']}, {specs[i]['order']})"
        del qs, works
    b.close()
