"""GPU reacting Navier-Stokes right-hand side (BR1 viscous terms) against the
oracle, through the C ABI.

Bar (FP64), per entry i: |gpu_i - oracle_i| <= K u M_i for every lifted
gradient and every right-hand-side entry, with u = 2^-53, K = 3 Np + 4 Nfp
(products summed into an entry) and M_i the sum of their absolute values
before any cancellation (oracle ns.gradient_term_magnitude /
ns.rhs_term_magnitude: Higham's error scale of a computed sum of products;
the oracle's own error against long double is about 2 u M_i).  On ragged
meshes of every order; Runge-Kutta steps with the GPU's own temperature
Newton track the oracle's steps to 1e-12 of each field's largest value."""
import numpy as np
import pytest

from oracle import lsrk as olsrk, mesh as om, ns, reference_element as ore, thermo as ot
from paper_2512_17101_amd import dg, workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TH = wl.synthetic_thermo(3003)
MECH = wl.synthetic_mechanism(3004)
L = 0.01


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(p, dims, seed=1003, state_seed=3005, jitter=0.03, noise=1e-3):
    xyz, vid = wl.kuhn_mesh(dims, (L * dims[0] / max(dims), L * dims[1] / max(dims), L * dims[2] / max(dims)),
                            jitter, seed)
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    X = om.node_coordinates(xyz, ops["rst"])
    q = wl.reacting_state(X.reshape(-1, 3), seed=state_seed, L=L, n_cells=max(dims)).reshape((12,) + X.shape[:2])
    # per-node noise: every face trace of q (and so of T and the gradients) jumps
    q = q * (1.0 + noise * np.random.default_rng(state_seed).standard_normal(q.shape))
    T, it = ns.temperature(q, TH)
    assert np.all(it > 0)
    return xyz, vid, ops, geo, conn, np.ascontiguousarray(q), T


def _run(mesh, q_np, T_np, mech, mu):
    dev = _dev()
    q = torch.from_numpy(q_np).to(dev)
    T = torch.from_numpy(np.ascontiguousarray(T_np)).to(dev)
    sig = torch.empty(tuple(T.shape) + (33,), dtype=torch.float64, device=dev)
    out = torch.empty_like(q)
    th = dg.Thermo(TH["W"], TH["a"])
    mk = dg.Mechanism(th, MECH["A"], MECH["Ea"], MECH["nu_r"], MECH["nu_p"]) if mech else None
    dg.ns_rhs(mesh, th, q, T, sig, out, mech=mk, mu=mu)
    torch.cuda.synchronize()
    return sig.cpu().numpy(), out.cpu().numpy()


def _ratios(ops, geo, conn, q, T, sig_gpu, rhs_gpu, mech, mu, elems=None):
    """max_i err_i / M_i (in units of u) of the gradients and, per field, of
    the right-hand side; the oracle evaluates at `elems` (all by default)."""
    u = 2.0 ** -53
    ix = np.arange(q.shape[1]) if elems is None else np.asarray(elems)
    v = ns.primitive_fields(q, T)
    S = np.unique(np.concatenate([ix, conn["mapP_elem"][ix].ravel()]))
    sig_S = ns.gradients(ops, geo, conn, v, elems=S)
    sig_ref = sig_S[:, :, np.searchsorted(S, ix)]
    smag = ns.gradient_term_magnitude(ops, geo, conn, v, elems=ix)
    # device layout [E][Np][3 c + d]  ->  reference layout [d][c][E][Np]
    sg = np.moveaxis(sig_gpu[ix].reshape((len(ix), ops["Np"], 11, 3)), (2, 3), (1, 0))
    es = (np.abs(sg - sig_ref) / smag).max() / u
    r_ref = ns.rhs(ops, geo, conn, q, T, TH, MECH if mech else None, mu=mu, elems=ix)
    mag = ns.rhs_term_magnitude(ops, geo, conn, q, T, TH, MECH if mech else None, mu=mu, elems=ix)
    er = (np.abs(rhs_gpu[:, ix] - r_ref) / mag).max(axis=(1, 2)) / u
    return es, er


def _check(ops, geo, conn, q, T, sig_gpu, rhs_gpu, mech, mu, label, elems=None):
    K = 3 * ops["Np"] + 4 * ops["Nfp"]
    es, er = _ratios(ops, geo, conn, q, T, sig_gpu, rhs_gpu, mech, mu, elems)
    print(f"{label}: max sigma err/M {es:.2f} u, rhs err/M per field {np.array2string(er, precision=2)} u (K = {K})")
    assert np.all(np.isfinite(rhs_gpu)) and np.all(np.isfinite(sig_gpu))
    assert es <= K
    assert np.all(er <= K)


@pytest.mark.parametrize("p,dims", [(1, (3, 3, 4)), (2, (3, 4, 3)), (3, (3, 3, 5)), (4, (3, 3, 3))])
def test_ns_rhs_matches_oracle(p, dims):
    xyz, vid, ops, geo, conn, q, T = _case(p, dims)
    mesh = dg.Mesh(p, xyz, vid)
    for mech, mu in ((True, ns.MU), (False, 50.0 * ns.MU)):
        sig, rhs = _run(mesh, q, T, mech, mu)
        _check(ops, geo, conn, q, T, sig, rhs, mech, mu, f"p={p} E={mesh.E} mech={mech} mu={mu:.1e}")


def test_ns_rhs_multi_block_p3():
    xyz, vid, ops, geo, conn, q, T = _case(3, (6, 6, 6), seed=1004, state_seed=3007)
    mesh = dg.Mesh(3, xyz, vid)
    sig, rhs = _run(mesh, q, T, True, ns.MU)
    _check(ops, geo, conn, q, T, sig, rhs, True, ns.MU, f"p=3 E={mesh.E}")
    sig2, rhs2 = _run(mesh, q, T, True, ns.MU)
    assert np.array_equal(rhs, rhs2) and np.array_equal(sig, sig2)


def test_ns_uniform_state_gives_zero():
    xyz, vid, ops, geo, conn, q, T = _case(2, (3, 3, 3))
    qu = np.ascontiguousarray(np.broadcast_to(q[:, :1, :1], q.shape))
    Tu, _ = ns.temperature(qu, TH)
    mesh = dg.Mesh(2, xyz, vid)
    sig, rhs = _run(mesh, qu, Tu, False, 1.0)
    # a uniform state's exact right-hand side and gradients are zero: what is
    # left is rounding, within the per-entry bar
    K = 3 * ops["Np"] + 4 * ops["Nfp"]
    u = 2.0 ** -53
    mag = ns.rhs_term_magnitude(ops, geo, conn, qu, Tu, TH, None, mu=1.0)
    assert np.all(np.abs(rhs) <= K * u * mag)
    v = ns.primitive_fields(qu, Tu)
    smag = ns.gradient_term_magnitude(ops, geo, conn, v)
    sg = np.moveaxis(sig.reshape(Tu.shape + (11, 3)), (2, 3), (1, 0))
    assert np.all(np.abs(sg) <= K * u * smag)


def test_ns_rk_steps_track_oracle():
    """Three fused LSRK steps (temperature Newton, gradient and right-hand-side
    passes per stage) track the oracle's steps.  Without sources: the seeded
    mechanism's rates (A up to 1e12 in SI units) are far too stiff for an
    explicit step at the acoustic limit; the sources' parity is checked on
    the right-hand side itself."""
    dev = _dev()
    p = 2
    xyz, vid, ops, geo, conn, q0, T0 = _case(p, (3, 3, 3), state_seed=3006)
    mesh = dg.Mesh(p, xyz, vid)
    dt = 2e-8
    mu = 10.0 * ns.MU

    def f(qq, tt):
        T, it = ns.temperature(qq, TH)
        assert np.all(it > 0)
        return ns.rhs(ops, geo, conn, qq, T, TH, None, mu=mu)

    qe = q0.copy()
    for s in range(3):
        qe, _ = olsrk.lsrk_step(f, qe, s * dt, dt)
    th = dg.Thermo(TH["W"], TH["a"])
    q = torch.from_numpy(q0).to(dev)
    T = torch.full(T0.shape, 1000.0, dtype=torch.float64, device=dev)
    work = torch.empty(dg.NS_WORK_PER_NODE * mesh.E * mesh.Np, dtype=torch.float64, device=dev)
    for s in range(3):
        dg.ns_rk_step(mesh, th, q, T, work, dt, mech=None, mu=mu)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    n = mesh.E * mesh.Np
    iters = work[57 * n:58 * n].view(torch.int32)[:n].cpu().numpy()
    assert np.all(iters >= 1)  # last stage's Newton converged everywhere
    scale = np.abs(qe).max(axis=(1, 2))
    scale[1:4] = scale[1:4].max()
    err = np.abs(got - qe).max(axis=(1, 2)) / scale
    change = np.abs(qe - q0).max(axis=(1, 2)) / scale
    print("3 NS steps: per-field rel diff vs oracle", err, "relative change", change)
    assert np.all(change[1:] > 1e-9)  # the steps moved the state
    assert np.all(err <= 1e-12)


def test_ns_error_paths():
    dev = _dev()
    xyz, vid, ops, geo, conn, q, T = _case(1, (3, 3, 3))
    mesh = dg.Mesh(1, xyz, vid)
    th = dg.Thermo(TH["W"], TH["a"])
    qt = torch.from_numpy(q).to(dev)
    Tt = torch.from_numpy(np.ascontiguousarray(T)).to(dev)
    sig = torch.empty(T.shape + (33,), dtype=torch.float64, device=dev)
    out = torch.empty_like(qt)
    with pytest.raises(dg.DGError, match="mu >= 0"):
        dg.ns_rhs(mesh, th, qt, Tt, sig, out, mu=-1.0)
    with pytest.raises(dg.DGError, match="overlap"):
        dg.ns_rhs(mesh, th, qt, Tt, sig, qt)
    prm = dg._Params(0, 1.4, 0.0, 0.0, 0.0, None, None)
    import ctypes
    st = dg.lib().dg_ns_rhs(mesh.handle, ctypes.byref(prm), dg._dev_ptr(qt), dg._dev_ptr(Tt), dg._dev_ptr(sig),
                            dg._dev_ptr(out), dg._stream(None))
    assert st == 1 and b"model must be 1" in dg.lib().dg_last_error()


def test_ns_rhs_full_size_sampled_p3_32cubed():
    """The reacting workload the benchmark times: 32^3 x 6 = 196,608 tets,
    p = 3, 1 cm box, 3 % jitter, seeded fronts, sources on, in the launch
    configuration the benchmark uses.  Gradients and right-hand side of a
    sample of elements (first and last tiles, 1024 random) against the
    oracle, which evaluates the gradients only at the sample and its face
    neighbours; same bar as the small meshes."""
    n, p = 32, 3
    xyz, vid = wl.kuhn_box_mesh(n, 0.01, 0.03, 1003)
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    X = om.node_coordinates(xyz, ops["rst"])
    q = wl.reacting_state(X.reshape(-1, 3), seed=3005, L=0.01, n_cells=n).reshape((12,) + X.shape[:2])
    T, it = ns.temperature(q, TH)
    assert np.all(it > 0)
    mesh = dg.Mesh(p, xyz, vid)
    sig_gpu, rhs_gpu = _run(mesh, q, T, True, ns.MU)
    E = xyz.shape[0]
    ix = np.unique(np.concatenate([np.arange(16), np.arange(E - 16, E),
                                   np.random.default_rng(13).choice(E, 1024, replace=False)]))
    _check(ops, geo, conn, q, T, sig_gpu, rhs_gpu, True, ns.MU, f"32^3 sampled ({len(ix)} elements)", elems=ix)
