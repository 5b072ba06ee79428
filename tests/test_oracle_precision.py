"""Pins of the oracle's reduced-precision emulation: BF16 round-to-nearest-even
agrees with torch's CPU conversion (a library routine) and with hand-checked
tie cases, the hi/lo split leaves a 2^-16 residual, and the emulated
contractions respect the stated error bound against FP64."""
import numpy as np
import pytest
import torch

from oracle import euler as oe, mesh as om, precision as op, reference_element as ore
from paper_2512_17101_amd import workload as wl


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(op.round_bf16(x.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    assert op.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0           # tie -> even (1.0)
    assert op.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even (up)
    assert op.round_bf16(np.array([1 + 3 * 2.0 ** -9]))[0] == 1 + 2.0 ** -7  # above half -> up
    assert op.round_bf16(np.array([-(1 + 2.0 ** -8)]))[0] == -1.0


def test_split_residual():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100000) * 10.0 ** rng.uniform(-3, 3, 100000)
    hi, lo = op.split_bf16(x)
    assert np.all(np.abs(x - hi) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= (2.0 ** -16 + 2.0 ** -24) * np.abs(x))


@pytest.mark.parametrize("mode", ["fp32", "split_bf16"])
def test_emulated_contraction_within_bound(mode):
    rng = np.random.default_rng(2)
    Op = rng.standard_normal((20, 100))
    X = rng.standard_normal((5, 64, 100)) * 10.0 ** rng.uniform(-1, 1, (5, 64, 100))
    y = op.contract(Op, X, "fp64")
    ym = op.contract(Op, X, mode)
    T = np.abs(X) @ np.abs(Op).T
    assert np.all(np.abs(ym - y) <= op.error_bound_factor(mode, 100) * T)
    # and the mode is genuinely reduced: plain BF16 (no lo terms) is far worse
    if mode == "split_bf16":
        plain = (op.round_bf16(X).astype(np.float32) @ op.round_bf16(Op).astype(np.float32).T).astype(np.float64)
        assert np.abs(plain - y).max() > 30 * np.abs(ym - y).max()


def test_exactly_representable_operands_reduce_to_fp32_sum():
    rng = np.random.default_rng(3)
    Op = op.round_bf16(rng.standard_normal((20, 100)))
    X = op.round_bf16(rng.standard_normal((5, 8, 100)))
    exact_products_fp32 = (X.astype(np.float32) @ Op.astype(np.float32).T).astype(np.float64)
    np.testing.assert_allclose(op.contract(Op, X, "split_bf16"), exact_products_fp32,
                               atol=100 * 2.0 ** -24 * (np.abs(X) @ np.abs(Op).T).max())


@pytest.mark.parametrize("p", [2, 3])
def test_reduced_rhs_within_bound_of_fp64(p):
    xyz, vid = wl.kuhn_box_mesh(4, 10.0, 0.05, 1001)
    ops = ore.operators(p)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, p)
    q = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]), pert=wl.density_perturbation(5))
    r64 = oe.rhs(ops, geo, conn, q)
    Op, X = op.contraction_inputs(ops, geo, conn, q)
    np.testing.assert_allclose(X @ Op.T, r64, atol=1e-13 * np.abs(r64).max())
    for mode in ("fp32", "split_bf16"):
        y, bound = op.rhs(ops, geo, conn, q, mode)
        assert np.all(np.abs(y - r64) <= bound)


def test_delta_form_is_exact_and_shrinks_reduced_errors():
    """Subtracting each element's node-0 flux leaves the FP64 contraction
    unchanged to rounding (rows of D sum to zero) and cuts the emulated
    split-BF16 and FP32 errors (rms by more than 3x on a 12^3 mesh, where the
    vortex core still varies strongly inside an element) on the perturbed
    vortex, whose fluxes carry a large constant part (pressure)."""
    xyz, vid = wl.kuhn_box_mesh(12, 10.0, 0.03, 1001)
    ops = ore.operators(3)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, 3)
    q = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]), pert=wl.density_perturbation(5))
    r64 = oe.rhs(ops, geo, conn, q)
    Op, X = op.contraction_inputs(ops, geo, conn, q)
    _, Xd = op.contraction_inputs(ops, geo, conn, q, delta=True)
    T = np.abs(X) @ np.abs(Op).T
    np.testing.assert_allclose(Xd @ Op.T, r64, atol=1e-13 * T.max())
    V = slice(0, 3 * ops["Np"])
    print("volume operand rms: plain", np.sqrt((X[..., V] ** 2).mean()), "delta", np.sqrt((Xd[..., V] ** 2).mean()))
    for mode in ("fp32", "split_bf16"):
        d_plain = op.contract(Op, X, mode) - r64
        d_delta = op.contract(Op, Xd, mode) - r64
        print(mode, "max", np.abs(d_plain).max(), np.abs(d_delta).max(),
              "rms", np.sqrt((d_plain ** 2).mean()), np.sqrt((d_delta ** 2).mean()))
        assert np.sqrt((d_delta ** 2).mean()) < 0.35 * np.sqrt((d_plain ** 2).mean())
        assert np.abs(d_delta).max() < np.abs(d_plain).max()
