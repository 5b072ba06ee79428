"""GPU parity of the HIP DG Euler path against the FP64 oracle, through the
C ABI.

Bar (FP64), per entry i of every field: |gpu_i - oracle_i| <= K u T_i with
u = 2^-53, K = 3 Np + 4 Nfp the number of products summed into the entry and
T_i the sum of their absolute values before any cancellation (Higham's
bound gamma_K T_i of a computed sum of products; the oracle's own error
against extended precision is about one u T_i, so the bar leaves the GPU
the same worst case as one side).  For every field that is not a
near-cancellation (max|rhs_f| >= 1e-2 max T_f, where K u T <= 1e-12 max|rhs|
holds) also max|gpu - oracle| <= 1e-12 max|rhs_f|.  Summation order
differs between the two sides, so bit equality is not expected."""
import itertools
import math

import numpy as np
import pytest

from oracle import euler as oe, lsrk as olsrk, mesh as om, reference_element as ore
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(order, dims, lengths=(10.0, 10.0, 10.0), jitter=0.05, seed=1001, pert_seed=None, state="vortex"):
    xyz, vid = wl.kuhn_mesh(dims, lengths, jitter, seed)
    ops = ore.operators(order)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, order)
    X = om.node_coordinates(xyz, ops["rst"])
    if state == "vortex":
        pert = wl.density_perturbation(pert_seed) if pert_seed is not None else None
        q = wl.vortex_state(X, pert=pert)
    else:
        q = wl.constant_state(X.shape[:2])
    return dict(xyz=xyz, vid=vid, ops=ops, geo=geo, conn=conn, X=X, q=q)


def _gpu_rhs(mesh, q_np):
    q = torch.from_numpy(q_np).to(_dev())
    out = torch.empty_like(q)
    dg.rhs(mesh, q, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _assert_parity(got, ref, T, p, label=""):
    K = oe.contraction_length(p)
    u = 2.0 ** -53
    d = np.abs(got - ref)
    ratio = (d / np.maximum(T, 1e-300)).max(axis=(1, 2))
    err = d.max(axis=(1, 2))
    sT = T.max(axis=(1, 2))
    sR = np.abs(ref).max(axis=(1, 2))
    strict = sR >= 1e-2 * sT
    print(f"{label} max_i err_i/T_i in u: {np.array2string(ratio / u, precision=2)} (bar K = {K}); "
          f"err/max|rhs| {np.array2string(err / np.maximum(sR, 1e-300), precision=2)}; "
          f"max|rhs|/max T {np.array2string(sR / sT, precision=2)}")
    assert np.all(np.isfinite(got))
    assert np.all(ratio <= K * u)
    assert np.all(err[strict] <= TOL * sR[strict])


def _check(c, got, elems=None, label=""):
    ref = oe.rhs(c["ops"], c["geo"], c["conn"], c["q"], elems=elems)
    T = oe.rhs_term_magnitude(c["ops"], c["geo"], c["conn"], c["q"], elems=elems)
    _assert_parity(got if elems is None else got[:, elems], ref, T, c["ops"]["p"], label=label)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mesh_nodes_and_face_map_match_oracle(p):
    _dev()
    c = _case(p, (3, 4, 5))
    mesh = dg.Mesh(p, c["xyz"], c["vid"])
    np.testing.assert_allclose(mesh.nodes(), c["X"], atol=1e-13)
    ne, nn = mesh.face_map()
    assert np.array_equal(ne, c["conn"]["mapP_elem"])
    assert np.array_equal(nn, c["conn"]["mapP_node"])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_rhs_parity_ragged_mesh(p):
    # 3 x 4 x 5 cells = 360 tets: 22 full tiles of 16 plus a ragged tail of 8
    _dev()
    c = _case(p, (3, 4, 5), pert_seed=7)
    mesh = dg.Mesh(p, c["xyz"], c["vid"])
    _check(c, _gpu_rhs(mesh, c["q"]), label=f"p={p} E={mesh.E}")


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_rhs_parity_discontinuous_traces(p):
    """Per-node noise (1 %) makes every face trace jump, so the face flux, the
    Lax-Friedrichs term and the normal of every face enter the result (a
    smooth state sampled at nodes has no jumps and leaves the surface term
    zero whatever the normals)."""
    _dev()
    c = _case(p, (3, 4, 5), pert_seed=7)
    c["q"] = np.ascontiguousarray(c["q"] * (1.0 + 0.01 * np.random.default_rng(p).standard_normal(c["q"].shape)))
    mesh = dg.Mesh(p, c["xyz"], c["vid"])
    _check(c, _gpu_rhs(mesh, c["q"]), label=f"p={p} E={mesh.E} noisy")


def test_rhs_parity_vortex_p2_4cubed():
    """384 tets, p = 2, +-5 % jitter, isentropic vortex (the small workload)."""
    _dev()
    c = _case(2, (4, 4, 4), seed=1001)
    mesh = dg.Mesh(2, c["xyz"], c["vid"])
    _check(c, _gpu_rhs(mesh, c["q"]), label="vortex p2 4^3")


def test_rhs_parity_multi_tile_p3():
    _dev()
    c = _case(3, (8, 8, 8), jitter=0.03, seed=5, pert_seed=2002)
    mesh = dg.Mesh(3, c["xyz"], c["vid"])
    _check(c, _gpu_rhs(mesh, c["q"]), label="p3 8^3")


def test_rhs_free_stream_p3():
    _dev()
    c = _case(3, (4, 5, 3), state="const")
    mesh = dg.Mesh(3, c["xyz"], c["vid"])
    got = _gpu_rhs(mesh, c["q"])
    S = oe.max_wave_speed(c["q"]) * np.abs(c["q"]).max() * c["geo"]["Fscale"].max()
    assert np.abs(got).max() <= TOL * S


def test_rhs_full_size_p3_48cubed():
    """663,552 tets, p = 3, 3 % jitter, perturbed vortex: the full workload in
    the launch configuration the benchmark times, every entry of the whole
    mesh against the oracle (evaluated in chunks of elements)."""
    _dev()
    import bench
    xyz, vid = wl.kuhn_box_mesh(48, 10.0, 0.03, 1002)
    mesh = dg.Mesh(3, xyz, vid)
    mesh.set_launch("fp64", *bench.parse_launch(bench.DEFAULT_LAUNCH))
    ops = ore.operators(3)
    q_np = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]), pert=wl.density_perturbation(2002))
    got = _gpu_rhs(mesh, q_np)
    geo, conn = om.geometry(xyz), om.connectivity(vid, 3)
    E = xyz.shape[0]
    ref = np.empty_like(q_np)
    T = np.empty_like(q_np)
    for c0 in range(0, E, 65536):
        idx = np.arange(c0, min(E, c0 + 65536))
        ref[:, idx] = oe.rhs(ops, geo, conn, q_np, elems=idx)
        T[:, idx] = oe.rhs_term_magnitude(ops, geo, conn, q_np, elems=idx)
    _assert_parity(got, ref, T, 3, label="48^3 whole mesh")


def test_rk_step_parity_vortex_p2_10_steps():
    """Ten LSRK(5,4) steps at CFL 0.2 on the small workload."""
    dev = _dev()
    c = _case(2, (4, 4, 4), seed=1001)
    mesh = dg.Mesh(2, c["xyz"], c["vid"])
    dt = oe.cfl_dt(c["ops"], c["geo"], c["q"], 0.2)
    f = lambda qq, tt: oe.rhs(c["ops"], c["geo"], c["conn"], qq)
    qo = c["q"].copy()
    for s in range(10):
        qo, _ = olsrk.lsrk_step(f, qo, s * dt, dt)
    q = torch.from_numpy(c["q"]).to(dev)
    work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
    for s in range(10):
        dg.rk_step(mesh, q, work, s * dt, dt)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    # momentum components are scaled by the momentum vector's magnitude (the
    # z-momentum of the z-independent vortex stays near zero)
    scale = np.abs(qo).max(axis=(1, 2))
    scale[1:4] = scale[1:4].max()
    err = np.abs(got - qo).max(axis=(1, 2)) / scale
    print("10-step per-field rel err", err)
    assert np.all(err <= TOL)


def test_rk_step_parity_p3_6cubed_100_steps():
    """100 LSRK(5,4) steps at CFL 0.2 of the 48^3 workload's setup on a
    reduced mesh (6^3 x 6 = 1,296 tets, p = 3, 3 % jitter, mesh seed 1002,
    perturbation seed 2002), FP64 against the oracle's 100 steps: per field
    max|dq| <= 1e-12 max|q_f|."""
    dev = _dev()
    c = _case(3, (6, 6, 6), jitter=0.03, seed=1002, pert_seed=2002)
    mesh = dg.Mesh(3, c["xyz"], c["vid"])
    dt = oe.cfl_dt(c["ops"], c["geo"], c["q"], 0.2)
    f = lambda qq, tt: oe.rhs(c["ops"], c["geo"], c["conn"], qq)
    qo = c["q"].copy()
    for s in range(100):
        qo, _ = olsrk.lsrk_step(f, qo, s * dt, dt)
    q = torch.from_numpy(c["q"]).to(dev)
    work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
    for s in range(100):
        dg.rk_step(mesh, q, work, s * dt, dt)
    dg.synchronize()
    got = q.cpu().numpy()
    scale = np.abs(qo).max(axis=(1, 2))
    scale[1:4] = scale[1:4].max()
    err = np.abs(got - qo).max(axis=(1, 2)) / scale
    change = np.abs(qo - c["q"]).max(axis=(1, 2)) / scale
    print(f"100 steps (t = {100 * dt:.3f}): per-field rel err {err}, relative change {change}")
    assert np.all(change[[0, 1, 2, 4]] > 1e-4)  # the vortex moved
    assert np.all(err <= TOL)


def test_lsrk_update_matches_definition():
    dev = _dev()
    rng = np.random.default_rng(3)
    n = 100003
    rhs_, res, q = (rng.standard_normal(n) for _ in range(3))
    a, b, dt = float(olsrk.A[2]), float(olsrk.B[2]), 0.0123
    r_exp = a * res + dt * rhs_
    q_exp = q + b * r_exp
    t_rhs, t_res, t_q = (torch.from_numpy(x.copy()).to(dev) for x in (rhs_, res, q))
    dg.lsrk_update(a, b, dt, t_rhs, t_res, t_q)
    torch.cuda.synchronize()
    np.testing.assert_allclose(t_res.cpu().numpy(), r_exp, rtol=0, atol=1e-15 * np.abs(r_exp).max())
    np.testing.assert_allclose(t_q.cpu().numpy(), q_exp, rtol=0, atol=1e-15 * np.abs(q_exp).max())
    # a = 0 ignores whatever res holds
    t_res.fill_(float("nan"))
    dg.lsrk_update(0.0, b, dt, t_rhs, t_res, t_q)
    torch.cuda.synchronize()
    assert torch.isfinite(t_res).all()


def test_rhs_is_deterministic():
    dev = _dev()
    c = _case(3, (4, 4, 4), pert_seed=9)
    mesh = dg.Mesh(3, c["xyz"], c["vid"])
    q = torch.from_numpy(c["q"]).to(dev)
    o1, o2 = torch.empty_like(q), torch.empty_like(q)
    dg.rhs(mesh, q, o1)
    dg.rhs(mesh, q, o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


def test_error_paths():
    dev = _dev()
    c = _case(2, (3, 3, 3))
    mesh = dg.Mesh(2, c["xyz"], c["vid"])
    q = torch.from_numpy(c["q"]).to(dev)
    with pytest.raises(dg.DGError) as ei:
        dg.rhs(mesh, q, q)
    assert ei.value.status == 1
    bad = c["xyz"].copy()
    bad[4, [2, 3]] = bad[4, [3, 2]]
    with pytest.raises(dg.DGError) as ei:
        dg.Mesh(2, bad, c["vid"])
    assert ei.value.status == 2
    xyz1, vid1 = wl.kuhn_mesh((1, 1, 1), (1.0, 1.0, 1.0), 0.0, 0)
    with pytest.raises(dg.DGError) as ei:
        dg.Mesh(2, xyz1, vid1)  # a single periodic cube shares faces more than twice
    assert ei.value.status == 2
    with pytest.raises(dg.DGError) as ei:
        dg.Mesh(5, c["xyz"], c["vid"])
    assert ei.value.status == 1


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_launch_configurations_give_the_same_bits(p):
    """Every launch configuration (2 or 4 tiles per block; fused or unfused
    Runge-Kutta stages; LDS DMA or register staging of the state tile) of
    every contraction precision gives bitwise the
    right-hand side and the steps of the initial one, on a ragged mesh with
    jumping traces."""
    dev = _dev()
    c = _case(p, (3, 4, 5), pert_seed=2003)
    q_np = c["q"] * (1.0 + 1e-3 * np.random.default_rng(77).standard_normal(c["q"].shape))
    mesh = dg.Mesh(p, c["xyz"], c["vid"])
    q0 = torch.from_numpy(np.ascontiguousarray(q_np)).to(dev)
    dt = 0.2 * oe.cfl_dt(c["ops"], c["geo"], q_np, 1.0)
    for mode in ("fp64", "fp32", "split_bf16"):
        assert mesh.get_launch(mode) == dict(waves_per_block=4, rk_fused=1, lds_stage=1, xcd_run=1)
        ref_rhs, ref_q = None, None
        for w, fused, lds in itertools.product((4, 2), (1, 0), (1, 0)):
            mesh.set_launch(mode, w, fused, lds)
            out = torch.empty_like(q0)
            dg.rhs(mesh, q0, out, mode)
            q = q0.clone()
            work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
            for s in range(2):
                dg.rk_step(mesh, q, work, s * dt, dt, mode)
            torch.cuda.synchronize()
            if ref_rhs is None:
                ref_rhs, ref_q = out.clone(), q.clone()
            assert torch.equal(out, ref_rhs), f"{mode} rhs waves={w} lds={lds}"
            assert torch.equal(q, ref_q), f"{mode} rk waves={w} fused={fused} lds={lds}"
        mesh.set_launch(mode, 4, 1)


@pytest.mark.parametrize("p", [1, 3, 4])
def test_xcd_runs_permute_tiles_only(p):
    """A run length of k blocks per XCD only renumbers the tiles: on a mesh
    with whole runs and a ragged tail (k = 2 and 5, both block widths, every
    contraction precision), the right-hand side and the fused steps are
    bitwise those of the plain order, and every entry is written (outputs
    start as NaN)."""
    dev = _dev()
    c = _case(p, (8, 8, 8), pert_seed=2011)
    mesh = dg.Mesh(p, c["xyz"], c["vid"])
    q0 = torch.from_numpy(np.ascontiguousarray(c["q"])).to(dev)
    dt = 0.2 * oe.cfl_dt(c["ops"], c["geo"], c["q"], 1.0)
    for mode in ("fp64", "fp32", "split_bf16"):
        ref = None
        for w, x in itertools.product((4, 2), (1, 2, 5)):
            mesh.set_launch(mode, w, 1, 1, x)
            out = torch.full_like(q0, float("nan"))
            dg.rhs(mesh, q0, out, mode)
            q = q0.clone()
            work = torch.full((2,) + tuple(q.shape), float("nan"), dtype=torch.float64, device=dev)
            for s in range(2):
                dg.rk_step(mesh, q, work, s * dt, dt, mode)
            torch.cuda.synchronize()
            label = f"{mode} waves={w} xcd_run={x}"
            assert not torch.isnan(out).any() and not torch.isnan(q).any(), label
            if ref is None:
                ref = (out.clone(), q.clone())
            assert torch.equal(out, ref[0]) and torch.equal(q, ref[1]), label
        mesh.set_launch(mode)


def test_autotune_chooses_sets_and_caches(tmp_path):
    dev = _dev()
    c = _case(3, (4, 4, 4))
    mesh = dg.Mesh(3, c["xyz"], c["vid"])
    cache = tmp_path / "tune.json"
    cfg, ms = mesh.autotune("split_bf16", cache_path=cache, trials=2)
    assert ms > 0 and cfg == mesh.get_launch("split_bf16")
    assert cfg["waves_per_block"] in (2, 4) and cfg["rk_fused"] in (0, 1) and cfg["lds_stage"] in (0, 1)
    assert cfg["xcd_run"] in (1, 9, 27)
    assert mesh.get_launch("fp64") == dict(waves_per_block=4, rk_fused=1, lds_stage=1, xcd_run=1)  # untouched
    import json
    (key, entry), = json.loads(cache.read_text())["entries"].items()
    assert "split_bf16" in key and ":p3:" in key and f":E{mesh.E}" in key
    assert {k: entry[k] for k in cfg} == cfg
    mesh2 = dg.Mesh(3, c["xyz"], c["vid"])
    cfg2, ms2 = mesh2.autotune("split_bf16", cache_path=cache, trials=2)
    assert cfg2 == cfg and ms2 < 0
    with pytest.raises(dg.DGError, match="waves_per_block"):
        mesh.set_launch("fp64", 3, 1)
    for x in (0, 65):
        with pytest.raises(dg.DGError, match="xcd_run"):
            mesh.set_launch("fp64", 4, 1, 1, x)
    with pytest.raises(dg.DGError, match="trials"):
        mesh.autotune("fp64", trials=0)
    # tuned mesh still matches the oracle
    q = torch.from_numpy(c["q"]).to(dev)
    out = torch.empty_like(q)
    mesh.set_launch("fp64", 2, 0)
    dg.rhs(mesh, q, out)
    torch.cuda.synchronize()
    _check(c, out.cpu().numpy(), label="p=3 waves=2")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_state_staging_paths_agree_bitwise(order, precision):
    """A state that is 16-byte aligned is staged into LDS by the DMA path (Np a
    multiple of 4: p = 1, 3), one that is only 8-byte aligned by register
    loads; both paths feed the same arithmetic, so the right-hand sides and a
    Runge-Kutta step agree bit for bit (p = 2 takes the register path either
    way).  The 3 x 4 x 5 box gives 360 elements: a ragged last tile."""
    c = _case(order, (3, 4, 5), seed=1207)
    mesh = dg.Mesh(order, c["xyz"], c["vid"], 0)
    dev = _dev()
    n = c["q"].size
    q_al = torch.from_numpy(c["q"]).to(dev)
    buf = torch.empty(n + 1, dtype=torch.float64, device=dev)
    q_un = buf[1:].view(c["q"].shape)
    q_un.copy_(q_al)
    assert q_al.data_ptr() % 16 == 0 and q_un.data_ptr() % 16 == 8
    outs = []
    for q in (q_al, q_un):
        out = torch.empty_like(q_al)
        dg.rhs(mesh, q, out, precision=precision)
        outs.append(out)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    dt = 1e-3
    work = torch.empty((2,) + tuple(q_al.shape), dtype=torch.float64, device=dev)
    dg.rk_step(mesh, q_al, work, 0.0, dt, precision=precision)
    dg.rk_step(mesh, q_un, work, 0.0, dt, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(q_al, q_un)
