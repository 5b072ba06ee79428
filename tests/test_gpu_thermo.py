"""GPU temperature Newton solve and Arrhenius sources against the oracle,
through the C ABI: temperatures within 1e-9 K with identical iteration counts
(both take the same steps from the same start), sources within 1e-12 of each
species' largest magnitude, forced non-convergence and error paths."""
import numpy as np
import pytest

from oracle import mesh as om, reference_element as ore, thermo as ot
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TH = wl.synthetic_thermo(3003)
MECH = wl.synthetic_mechanism(3004)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _handles():
    th = dg.Thermo(TH["W"], TH["a"])
    mk = dg.Mechanism(th, MECH["A"], MECH["Ea"], MECH["nu_r"].astype(np.int32), MECH["nu_p"].astype(np.int32))
    return th, mk


def _state(n_cells=8, order=3):
    xyz, _ = wl.kuhn_box_mesh(n_cells, 0.01, 0.03, 1003)
    X = om.node_coordinates(xyz, ore.nodes(order))
    return wl.reacting_state(X, n_cells=n_cells)


def test_temperature_matches_oracle():
    dev = _dev()
    th, _ = _handles()
    q_np = _state()
    rho, u, v, w, e, Y = ot.primitives(q_np)
    T_ref, it_ref = ot.newton_temperature(e, Y, TH, 1000.0, tol=1e-10, max_iter=50)
    q = torch.from_numpy(q_np).to(dev)
    T = torch.empty(q.shape[1:], dtype=torch.float64, device=dev)
    it = torch.empty(q.shape[1:], dtype=torch.int32, device=dev)
    dg.temperature(th, q, T, it)
    torch.cuda.synchronize()
    T, it = T.cpu().numpy(), it.cpu().numpy()
    print("max |T - T_oracle| =", np.abs(T - T_ref).max(), "iteration histogram", np.bincount(it.ravel() + 1))
    assert np.abs(T - T_ref).max() <= 1e-9
    assert np.all(it > 0)
    assert np.abs(it - it_ref).max() <= 1  # last step can land either side of tol


def test_temperature_with_guess_array_and_forced_failure():
    dev = _dev()
    th, _ = _handles()
    q_np = _state(4)
    rho, u, v, w, e, Y = ot.primitives(q_np)
    T_ref, _ = ot.newton_temperature(e, Y, TH, 1000.0)
    q = torch.from_numpy(q_np).to(dev)
    guess = torch.from_numpy(T_ref + 5.0).to(dev)
    T = torch.empty_like(guess)
    it = torch.empty(guess.shape, dtype=torch.int32, device=dev)
    dg.temperature(th, q, T, it, T_guess=guess)
    torch.cuda.synchronize()
    assert np.abs(T.cpu().numpy() - T_ref).max() <= 1e-9
    dg.temperature(th, q, T, it, max_iter=1)
    torch.cuda.synchronize()
    assert torch.all(it == -1)


def test_sources_match_oracle_and_conserve_mass():
    dev = _dev()
    th, mk = _handles()
    q_np = _state()
    rho, u, v, w, e, Y = ot.primitives(q_np)
    T_ref, _ = ot.newton_temperature(e, Y, TH, 1000.0)
    w_ref = ot.sources(rho, T_ref, Y, TH, MECH)
    q = torch.from_numpy(q_np).to(dev)
    T = torch.from_numpy(T_ref).to(dev)
    om_ = torch.empty((7,) + tuple(T.shape), dtype=torch.float64, device=dev)
    dg.sources(mk, q, T, om_)
    torch.cuda.synchronize()
    got = om_.cpu().numpy()
    axes = tuple(range(1, w_ref.ndim))
    scale = np.abs(w_ref).max(axis=axes)
    inert = scale == 0.0  # species in no reaction: exactly zero on both sides
    assert np.all(got[inert] == 0.0)
    err = np.abs(got[~inert] - w_ref[~inert]).max(axis=axes) / scale[~inert]
    print("per-species rel err (reacting species)", err)
    assert np.all(err <= 1e-12)
    assert np.all(np.abs(got.sum(axis=0)) <= 1e-13 * np.abs(got).sum(axis=0).max())


def test_thermo_error_paths():
    _dev()
    with pytest.raises(dg.DGError):
        dg.Thermo(np.ones(9), np.ones((9, 6)))
    with pytest.raises(dg.DGError):
        dg.Thermo(-np.ones(7), np.ones((7, 6)))
    th = dg.Thermo(TH["W"], TH["a"])
    bad = MECH["nu_r"].astype(np.int32).copy()
    bad[0, 0] = -1
    with pytest.raises(dg.DGError):
        dg.Mechanism(th, MECH["A"], MECH["Ea"], bad, MECH["nu_p"].astype(np.int32))


def test_temperature_and_sources_full_size_sampled():
    """The learned-guess evaluation size: the 48^3 x 6 p = 3 mesh's 13.27M
    nodes (1 cm box) with reacting fields, one launch each; the oracle solves
    and evaluates a random sample of 20,000 nodes (first and last included)
    to the same bars.  The sources take a seeded temperature field in
    [300, 2200] K as input on both sides."""
    dev = _dev()
    th, mk = _handles()
    xyz, _ = wl.kuhn_box_mesh(48, 0.01, 0.03, 1002)
    X = om.node_coordinates(xyz, ore.nodes(3))
    q_np = wl.reacting_state(X.reshape(-1, 3), seed=3005, L=0.01, n_cells=48)
    n = q_np.shape[1]
    T_in = np.random.default_rng(15).uniform(300.0, 2200.0, n)
    q = torch.from_numpy(q_np).to(dev)
    T = torch.empty(n, dtype=torch.float64, device=dev)
    it = torch.empty(n, dtype=torch.int32, device=dev)
    om_ = torch.empty((7, n), dtype=torch.float64, device=dev)
    dg.temperature(th, q, T, it)
    dg.sources(mk, q, torch.from_numpy(T_in).to(dev), om_)
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(14).choice(n, 20000, replace=False)]))
    Tg, itg, wg = T.cpu().numpy()[idx], it.cpu().numpy()[idx], om_.cpu().numpy()[:, idx]
    qs = np.ascontiguousarray(q_np[:, idx])
    rho, u, v, w, e, Y = ot.primitives(qs)
    T_ref, it_ref = ot.newton_temperature(e, Y, TH, 1000.0, tol=1e-10, max_iter=50)
    print(f"{n} nodes, sample {len(idx)}: max |T - T_oracle| = {np.abs(Tg - T_ref).max():.2e}")
    assert np.all(itg > 0) and np.abs(Tg - T_ref).max() <= 1e-9
    assert np.abs(itg - it_ref).max() <= 1
    w_ref = ot.sources(rho, T_in[idx], Y, TH, MECH)
    scale = np.abs(w_ref).max(axis=1)
    inert = scale == 0.0
    assert np.all(wg[inert] == 0.0)
    err = np.abs(wg[~inert] - w_ref[~inert]).max(axis=1) / scale[~inert]
    print("sources err / per-species max (reacting species)", err)
    assert np.all(err <= 1e-12)
