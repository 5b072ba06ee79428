"""GPU reduced-precision contractions (FP32, split BF16) against the FP64
oracle, through the C ABI.  Bar: every RHS entry within the mode's stated
error bound (operand representation + FP32 accumulation, times the magnitude
of the summed terms), and the per-field errors reported."""
import numpy as np
import pytest

from oracle import euler as oe, lsrk as olsrk, mesh as om, precision as opr, reference_element as ore
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(p, dims, seed=1001, jitter=0.05, pert_seed=7):
    xyz, vid = wl.kuhn_mesh(dims, (10.0, 10.0, 10.0), jitter, seed)
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    q = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]), pert=wl.density_perturbation(pert_seed))
    return xyz, vid, ops, geo, conn, q


def _gpu(mesh, q_np, mode):
    q = torch.from_numpy(q_np).to(_dev())
    out = torch.empty_like(q)
    dg.rhs(mesh, q, out, mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_reduced_precision_rhs_within_bound(p, mode):
    xyz, vid, ops, geo, conn, q = _case(p, (3, 4, 5))
    mesh = dg.Mesh(p, xyz, vid)
    got = _gpu(mesh, q, mode)
    r64 = oe.rhs(ops, geo, conn, q)
    _, bound = opr.rhs(ops, geo, conn, q, mode)
    err = np.abs(got - r64)
    rel = err.max(axis=(1, 2)) / np.abs(r64).max(axis=(1, 2))
    print(f"p={p} {mode}: max err/bound {np.max(err / bound):.3f}  per-field Linf rel {rel}")
    assert np.all(np.isfinite(got))
    assert np.all(err <= bound)


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_reduced_precision_rhs_within_bound_discontinuous(p, mode):
    """Same bound with 1 % per-node noise, so every face jump is nonzero."""
    xyz, vid, ops, geo, conn, q = _case(p, (3, 4, 5))
    q = np.ascontiguousarray(q * (1.0 + 0.01 * np.random.default_rng(10 + p).standard_normal(q.shape)))
    mesh = dg.Mesh(p, xyz, vid)
    got = _gpu(mesh, q, mode)
    r64 = oe.rhs(ops, geo, conn, q)
    _, bound = opr.rhs(ops, geo, conn, q, mode)
    print(f"p={p} {mode} noisy: max err/bound {np.max(np.abs(got - r64) / bound):.3f}")
    assert np.all(np.abs(got - r64) <= bound)


def test_split_bf16_far_better_than_its_bf16_part():
    """The lo terms are really used: the split result is >30x closer to FP64
    than BF16-only operands would be (emulated on the same inputs)."""
    xyz, vid, ops, geo, conn, q = _case(3, (4, 4, 4))
    mesh = dg.Mesh(3, xyz, vid)
    got = _gpu(mesh, q, "split_bf16")
    r64 = oe.rhs(ops, geo, conn, q)
    Op, X = opr.contraction_inputs(ops, geo, conn, q)
    plain = (opr.round_bf16(X).astype(np.float32) @ opr.round_bf16(Op).astype(np.float32).T).astype(np.float64)
    assert np.abs(plain - r64).max() > 30 * np.abs(got - r64).max()


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
def test_reduced_precision_multi_tile_and_deterministic(mode):
    xyz, vid, ops, geo, conn, q = _case(3, (8, 8, 8), seed=5, jitter=0.03, pert_seed=2002)
    mesh = dg.Mesh(3, xyz, vid)
    a = _gpu(mesh, q, mode)
    b = _gpu(mesh, q, mode)
    assert np.array_equal(a, b)
    idx = np.random.default_rng(4).choice(xyz.shape[0], 512, replace=False)
    r64 = oe.rhs(ops, geo, conn, q, elems=idx)
    _, bound = opr.rhs(ops, geo, conn, q, mode, elems=idx)
    assert np.all(np.abs(a[:, idx] - r64) <= bound)


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
def test_reduced_precision_rk_steps_track_emulation(mode):
    """Ten LSRK steps with reduced contractions stay within 1e-5 (relative, per
    field) of the same steps with the oracle's emulated contraction."""
    dev = _dev()
    xyz, vid, ops, geo, conn, q0 = _case(2, (4, 4, 4), pert_seed=3)
    mesh = dg.Mesh(2, xyz, vid)
    dt = oe.cfl_dt(ops, geo, q0, 0.2)
    f = lambda qq, tt: opr.rhs(ops, geo, conn, qq, mode)[0]
    qe = q0.copy()
    for s in range(10):
        qe, _ = olsrk.lsrk_step(f, qe, s * dt, dt)
    q = torch.from_numpy(q0).to(dev)
    work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
    for s in range(10):
        dg.rk_step(mesh, q, work, s * dt, dt, mode)
    torch.cuda.synchronize()
    scale = np.abs(qe).max(axis=(1, 2))
    scale[1:4] = scale[1:4].max()
    err = np.abs(q.cpu().numpy() - qe).max(axis=(1, 2)) / scale
    print(f"{mode} 10 steps: per-field rel diff vs emulation {err}")
    assert np.all(err <= 1e-5)
