"""GPU tests of device-side failure reporting, checkpoint/resume, the
reacting model through dg_rhs / dg_rk_step, and the temperature call with a
learned guess, all through the C ABI.

Failures a kernel cannot return (a Newton solve without convergence, a
non-finite state) raise a per-device flag that dg_synchronize turns into
DG_ERR_NOCONV / DG_ERR_NONFINITE and clears."""
import numpy as np
import pytest

from oracle import mesh as om, ns, reference_element as ore, thermo as ot
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TH = wl.synthetic_thermo(3003)
MECH = wl.synthetic_mechanism(3004)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _clear_flags():
    try:
        dg.synchronize()
    except dg.DGError:
        pass


def _euler_case(n=4, p=2):
    xyz, vid = wl.kuhn_box_mesh(n, 10.0, 0.05, 1001)
    mesh = dg.Mesh(p, xyz, vid)
    q = torch.from_numpy(wl.vortex_state(mesh.nodes())).to(_dev())
    return mesh, q


def test_clean_step_reports_ok_and_nan_reports_nonfinite():
    dev = _dev()
    _clear_flags()
    mesh, q = _euler_case()
    work = torch.empty((2,) + tuple(q.shape), dtype=torch.float64, device=dev)
    for mode in ("fp64", "fp32", "split_bf16"):
        qq = q.clone()
        dg.rk_step(mesh, qq, work, 0.0, 1e-3, mode)
        dg.synchronize()  # no failure: returns normally
        qq[0, 7, 3] = float("nan")
        dg.rk_step(mesh, qq, work, 0.0, 1e-3, mode)
        with pytest.raises(dg.DGError) as ei:
            dg.synchronize()
        assert ei.value.status == 6, mode  # DG_ERR_NONFINITE
        dg.synchronize()  # the flag was cleared by the previous call
    # the plain right-hand side and the unfused stage update report it too
    qq = q.clone()
    qq[4, 100, 0] = float("inf")
    out = torch.empty_like(q)
    dg.rhs(mesh, qq, out)
    with pytest.raises(dg.DGError) as ei:
        dg.synchronize()
    assert ei.value.status == 6
    mesh.set_launch("fp64", 4, 0)
    dg.rk_step(mesh, qq, work, 0.0, 1e-3)
    with pytest.raises(dg.DGError):
        dg.synchronize()
    mesh.set_launch("fp64", 4, 1)


def _reacting_state(n_cells=4, order=3):
    xyz, vid = wl.kuhn_box_mesh(n_cells, 0.01, 0.03, 1003)
    X = om.node_coordinates(xyz, ore.nodes(order))
    return xyz, vid, wl.reacting_state(X, n_cells=n_cells)


def test_newton_failures_report_noconv_and_match_oracle():
    dev = _dev()
    _clear_flags()
    th = dg.Thermo(TH["W"], TH["a"])
    _, _, q_np = _reacting_state()
    q_np = q_np.reshape(12, -1).copy()
    n = q_np.shape[1]
    # points 0..9: internal energies whose roots lie beyond the clamp interval
    rho, u, v, w, e, Y = ot.primitives(q_np)
    e_hot = ot.mixture_e(np.full(5, 9000.0), Y[:, :5], TH)
    e_cold = ot.mixture_e(np.full(5, 40.0), Y[:, 5:10], TH)
    kin = 0.5 * (u[:10] ** 2 + v[:10] ** 2 + w[:10] ** 2)
    q_np[4, :10] = rho[:10] * (np.concatenate([e_hot, e_cold]) + kin)
    rho, u, v, w, e, Y = ot.primitives(q_np)
    T_ref, it_ref = ot.newton_temperature(e, Y, TH, 1000.0)
    assert np.all(it_ref[:10] == -1) and np.all(it_ref[10:] > 0)
    q = torch.from_numpy(q_np).to(dev)
    T = torch.empty(n, dtype=torch.float64, device=dev)
    it = torch.empty(n, dtype=torch.int32, device=dev)
    dg.temperature(th, q, T, it)
    with pytest.raises(dg.DGError) as ei:
        dg.synchronize()
    assert ei.value.status == 5  # DG_ERR_NOCONV
    Tc, itc = T.cpu().numpy(), it.cpu().numpy()
    assert np.array_equal(itc[:10], it_ref[:10])
    np.testing.assert_array_equal(Tc[:10], T_ref[:10])  # the clamp bounds
    assert np.abs(Tc[10:] - T_ref[10:]).max() <= 1e-9
    # max_iter = 1 fails everywhere
    dg.temperature(th, q[:, 10:].contiguous(), T[10:], it[10:], max_iter=1)
    with pytest.raises(dg.DGError) as ei:
        dg.synchronize()
    assert ei.value.status == 5
    # a non-finite state: -1 and the non-finite flag
    q[0, 20] = float("nan")
    dg.temperature(th, q, T, it)
    with pytest.raises(dg.DGError) as ei:
        dg.synchronize()
    assert ei.value.status == 6
    assert it[20].item() == -1 and not np.isfinite(T[20].item())


def test_checkpoint_resume_is_bitwise():
    """Ten steps in a row equal five steps, a round trip of the state through
    host memory (a checkpoint file's contents), and five more steps."""
    dev = _dev()
    _clear_flags()
    mesh, q0 = _euler_case(4, 3)
    work = torch.empty((2,) + tuple(q0.shape), dtype=torch.float64, device=dev)
    for mode in ("fp64", "fp32", "split_bf16"):
        a = q0.clone()
        for _ in range(10):
            dg.rk_step(mesh, a, work, 0.0, 2e-3, mode)
        b = q0.clone()
        for _ in range(5):
            dg.rk_step(mesh, b, work, 0.0, 2e-3, mode)
        saved = b.cpu().numpy().tobytes()
        work.fill_(float("nan"))  # the scratch carries nothing between steps
        b = torch.from_numpy(np.frombuffer(saved, dtype=np.float64).reshape(q0.shape).copy()).to(dev)
        for _ in range(5):
            dg.rk_step(mesh, b, work, 0.0, 2e-3, mode)
        dg.synchronize()
        assert torch.equal(a, b), mode


def test_reacting_model_through_rhs_and_rk_step():
    """dg_rhs / dg_rk_step with model 1 are the reacting path: bitwise the
    result of dg_temperature (from 1000 K) + dg_ns_rhs, and of dg_ns_rk_step
    started from a uniform 1000 K temperature field."""
    dev = _dev()
    _clear_flags()
    th = dg.Thermo(TH["W"], TH["a"])
    mk = dg.Mechanism(th, MECH["A"], MECH["Ea"], MECH["nu_r"], MECH["nu_p"])
    xyz, vid, q_np = _reacting_state(3)
    mesh = dg.Mesh(3, xyz, vid)
    q = torch.from_numpy(np.ascontiguousarray(q_np.reshape(12, mesh.E, mesh.Np))).to(dev)
    nn = mesh.E * mesh.Np
    out1 = torch.empty_like(q)
    work = torch.empty(dg.NS_STEP_WORK * nn, dtype=torch.float64, device=dev)
    dg.reacting_rhs(mesh, th, q, out1, work, mech=mk)
    T = torch.empty((mesh.E, mesh.Np), dtype=torch.float64, device=dev)
    it = torch.empty((mesh.E, mesh.Np), dtype=torch.int32, device=dev)
    dg.temperature(th, q, T, it)
    sig = torch.empty((mesh.E, mesh.Np, 33), dtype=torch.float64, device=dev)
    out2 = torch.empty_like(q)
    dg.ns_rhs(mesh, th, q, T, sig, out2, mech=mk)
    dg.synchronize()
    assert torch.equal(out1, out2)
    assert torch.equal(work[:nn].view(mesh.E, mesh.Np), T)
    # with sources the seeded rates (A up to 1e12 SI) are stiff: an explicit
    # step of 1e-14 s; without them an acoustic-scale step of 1e-9 s
    for mech, dt in ((mk, 1e-14), (None, 1e-9)):
        qa, qb = q.clone(), q.clone()
        dg.reacting_rk_step(mesh, th, qa, work, dt, mech=mech)
        Tb = torch.full((mesh.E, mesh.Np), 1000.0, dtype=torch.float64, device=dev)
        wb = torch.empty(dg.NS_WORK_PER_NODE * nn, dtype=torch.float64, device=dev)
        dg.ns_rk_step(mesh, th, qb, Tb, wb, dt, mech=mech)
        dg.synchronize()
        assert torch.equal(qa, qb)
        assert not torch.equal(qa, q)
    # reduced-precision contractions are not offered for the reacting model
    with pytest.raises(dg.DGError) as ei:
        prm = dg._ns_params(th, mk, dg.MU, dg.PR, dg.SC, work)
        import ctypes
        dg._check(dg.lib().dg_rhs(mesh.handle, ctypes.byref(prm), dg.DG_FP32, dg._dev_ptr(q), dg._dev_ptr(out1),
                                  dg._stream(None)))
    assert ei.value.status == 7


def test_learned_guess_forced_fallback_and_temperature_call():
    """learned_max_iter = 1 leaves nearly every point unconverged: each falls
    back to the plain start and ends on the plain answer; dg_temperature with
    the network as its guess is the learned solve with at most 8 steps."""
    dev = _dev()
    _clear_flags()
    th = dg.Thermo(TH["W"], TH["a"])
    _, _, q_np = _reacting_state(3)
    q = torch.from_numpy(np.ascontiguousarray(q_np.reshape(12, -1))).to(dev)
    n = q.shape[1]
    net = dg.MLP(seed=4002)
    idx = torch.arange(n, device=dev)
    Tp = torch.empty(n, dtype=torch.float64, device=dev)
    ip = torch.empty(n, dtype=torch.int32, device=dev)
    dg.temperature(th, q, Tp, ip)
    net.fit_normalization(q, idx, Tp)
    Tl, il = torch.empty_like(Tp), torch.empty_like(ip)
    fb = torch.zeros(1, dtype=torch.int32, device=dev)
    dg.temperature_learned(th, net, q, Tl, il, learned_max_iter=1, fallback_count=fb)
    dg.synchronize()
    nfb = fb.item()
    print("fallbacks", nfb, "of", n)
    assert nfb > 0
    assert torch.all(il > 0)
    failed = il > 1  # a fallback point took 1 learned step + the plain restart
    assert int(failed.sum()) == nfb
    assert torch.equal(Tl[failed], Tp[failed])  # the restart is the plain solve
    assert (Tl - Tp).abs().max().item() <= 1e-9
    # the network as dg_temperature's guess: learned_max_iter = 8
    Tg, ig = torch.empty_like(Tp), torch.empty_like(ip)
    dg.temperature(th, q, Tg, ig, guess=net)
    dg.temperature_learned(th, net, q, Tl, il, learned_max_iter=8)
    dg.synchronize()
    assert torch.equal(Tg, Tl) and torch.equal(ig, il)
    with pytest.raises(dg.DGError):
        dg.temperature(th, q, Tg, ig, T_guess=Tp, guess=net)
