"""The no-allocation LSRK step (dg_rk_step_noalloc) against dg_rk_step,
through the C ABI: same kernels, so the same bits, on two calls in a row (the
second on a smaller mesh, so stale contents of the shared scratch array from
the first call are present), in every contraction precision and in both the
fused and split stage forms; and the size limit."""
import numpy as np
import pytest

from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _clear_flags():
    """Failure flags are sticky per device until a synchronising call reads
    them; earlier work in the process (a forced non-convergence, say) may
    have left one set."""
    try:
        dg.synchronize()
    except dg.DGError:
        pass


def _case(n, p, seed):
    xyz, vid = wl.kuhn_box_mesh(n, 10.0, 0.05, seed)
    mesh = dg.Mesh(p, xyz, vid)
    q = torch.from_numpy(wl.vortex_state(mesh.nodes())).to(_dev())
    return mesh, q


@pytest.mark.parametrize("fused", [1, 0])
def test_noalloc_step_matches_rk_step_twice(fused):
    dev = _dev()
    _clear_flags()
    # first a large state (24^3 x 6 = 82,944 tets at p = 3: 8,294,400 doubles,
    # just under the limit), then a small one
    for n, p, seed in ((24, 3, 1002), (5, 2, 1001)):
        mesh, q0 = _case(n, p, seed)
        assert q0.numel() <= dg.NOALLOC_MAX_STATE
        work = torch.empty((2,) + tuple(q0.shape), dtype=torch.float64, device=dev)
        for mode in ("fp64", "fp32", "split_bf16"):
            mesh.set_launch(mode, 4, fused)
            qa, qb = q0.clone(), q0.clone()
            for _ in range(2):
                dg.rk_step(mesh, qa, work, 0.0, 1e-3, mode)
                dg.rk_step_noalloc(mesh, qb, 0.0, 1e-3, mode)
            dg.synchronize()
            print(f"n={n} p={p} {mode} fused={fused}: max |noalloc - rk_step| = "
                  f"{(qa - qb).abs().max().item():.3e}", flush=True)
            assert torch.equal(qa, qb), (n, p, mode, fused)
            assert not torch.equal(qa, q0)


def test_noalloc_step_rejects_state_above_limit():
    _dev()
    xyz, vid = wl.kuhn_box_mesh(25, 10.0, 0.05, 1002)  # 93,750 tets at p = 3: 9,375,000 doubles
    mesh = dg.Mesh(3, xyz, vid)
    q = torch.zeros((5, mesh.E, mesh.Np), dtype=torch.float64, device=_dev())
    with pytest.raises(dg.DGError) as ei:
        dg.rk_step_noalloc(mesh, q, 0.0, 1e-3)
    assert ei.value.status == 1 and "limit" in str(ei.value)
    assert torch.count_nonzero(q).item() == 0  # nothing ran
