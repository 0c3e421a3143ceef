"""Host logic of the benchmark (no GPU): the algorithmic byte counts behind
the roofline figure, the permittivity-table rule they follow, the oracle
timing helper and the field-error summary."""
import numpy as np

import bench
from sbp_inputs import make_config


def _nodes(n):
    nx, ny, nz = n
    e = (nx + 2) * (ny + 1) * (nz + 1) + (nx + 1) * (ny + 2) * (nz + 1) + (nx + 1) * (ny + 1) * (nz + 2)
    h = (nx + 1) * (ny + 2) * (nz + 2) + (nx + 2) * (ny + 1) * (nz + 2) + (nx + 2) * (ny + 2) * (nz + 1)
    return e, h


def test_node_counts_are_the_component_shapes():
    # Ex (Nx+2, Ny+1, Nz+1) ... Hz (Nx+2, Ny+2, Nz+1), written out per component
    for n in ((4, 4, 4), (5, 7, 9), (256, 256, 256)):
        assert bench.node_counts(n) == _nodes(n)


def _block(n, eps):
    return {"n": n, "h": (1e-3,) * 3, "eps_r": eps, "mu_r": None, "sigma": None, "faces": ["pec"] * 6}


def test_algorithmic_bytes_two_pass_and_tables():
    n = (6, 5, 4)
    cells = 6 * 5 * 4
    ne, nh = _nodes(n)
    few = np.resize(np.array([1.0, 2.0, 3.5]), (4, 5, 6))           # 3 values: tabled
    many = 1.0 + np.arange(cells, dtype=float).reshape(4, 5, 6) / cells  # 120 values: cells
    for eps, cell_bytes in ((None, 0), (few, 1), (many, 4)):
        prob = {"blocks": [_block(n, eps)], "interfaces": []}
        hb, eb, fb = bench.algorithmic_bytes(prob, 4)
        assert hb == 4 * (2 * nh + ne)
        assert eb == 4 * (2 * ne + nh) + cell_bytes * cells
        assert fb == 0
    # fp64: 8 bytes per value, still one byte per tabled cell
    hb, eb, _ = bench.algorithmic_bytes({"blocks": [_block(n, few)], "interfaces": []}, 8)
    assert (hb, eb) == (8 * (2 * nh + ne), 8 * (2 * ne + nh) + cells)
    # an interface block takes the general kernels: the cell array
    prob = {"blocks": [_block(n, few), _block(n, None)], "interfaces": [(0, 1, 1, 0, 1)]}
    assert bench.algorithmic_bytes(prob, 4)[1] == 2 * 4 * (2 * ne + nh) + 4 * cells
    # one pass: both fields read and written once
    _, _, fb = bench.algorithmic_bytes({"blocks": [_block(n, many)], "interfaces": []}, 4, fused=True)
    assert fb == 4 * (2 * ne + 2 * nh + cells)


def test_table_rule_counts_values_in_the_field_precision():
    n = (4, 4, 4)
    v64 = 1.0 + np.arange(64) / 64.0  # 64 distinct values: tabled
    assert bench.tabled(_block(n, v64.reshape(4, 4, 4)), 4)
    over = np.resize(1.0 + np.arange(65) / 65.0, (5, 4, 4))  # 65: the cell array
    assert not bench.tabled(_block((4, 4, 5), over), 4)
    # values equal in fp32 but not in fp64
    close = np.resize(np.array([1.0 + k / 64.0 + d for k in range(40) for d in (0.0, 1e-12)]), (5, 4, 4))
    assert bench.tabled(_block((4, 4, 5), close), 4)
    assert not bench.tabled(_block((4, 4, 5), close), 8)
    # the 256^3 dielectric-boxes workload has 33 values
    assert bench.tabled(make_config(2, scale=8)["blocks"][0], 4)


def test_grow_rate_excludes_setup_and_stays_bounded():
    calls = []

    def timed(steps):  # 2 s of set-up per call, 0.01 s per step
        calls.append(steps)
        return 2.0 + 0.01 * steps
    rate, k = bench.grow_rate(timed, 1000, 1.0)
    assert abs(rate - 1000 / 0.01) / (1000 / 0.01) < 1e-9
    assert 0.01 * k >= 0.8          # the timed steps fill most of the target
    assert max(calls) == k + 1 and len(calls) <= 5


def test_field_accuracy_per_field_and_component():
    rng = np.random.default_rng(5)
    ref = {(b, c): rng.standard_normal(50) * (1e-4 if c == "Hz" else 1.0)
           for b in range(2) for c in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")}
    got = {k: v * (1 + 1e-6) for k, v in ref.items()}
    acc = bench.field_accuracy(got, ref)
    assert abs(acc["E_rel_l2"] - 1e-6) < 1e-12 and abs(acc["H_rel_l2"] - 1e-6) < 1e-12
    assert all(abs(v - 1e-6) < 1e-12 for v in acc["components_rel_l2"].values())
    assert acc["components_norm_over_field_norm"]["Hz"] < 1e-3


def test_field_error_report_energy_norm_weighs_both_fields():
    # E exact, H 1e-3 off, with eta0 |H| = 0.02 |E|: the energy-norm error is
    # H's error scaled by the fields' energy ratio
    eta0 = (1.25663706212e-6 / 8.8541878128e-12) ** 0.5
    ref = {(0, "Ex"): np.ones(10), (0, "Hx"): np.full(10, 0.02 / eta0)}
    got = {(0, "Ex"): ref[(0, "Ex")].copy(), (0, "Hx"): ref[(0, "Hx")] * (1 + 1e-3)}
    rep = bench.field_error_report(got, ref)
    assert rep["E_rel_l2"] == 0.0 and abs(rep["H_rel_l2"] - 1e-3) < 1e-12
    expect = 1e-3 * 0.02 / (1 + 0.02 ** 2) ** 0.5
    assert abs(rep["energy_norm_rel"] - expect) < 1e-9 * expect + 1e-15


def test_field_accuracy_zero_component_against_field_norm():
    ref = {(0, "Ex"): np.ones(8), (0, "Ey"): np.ones(8), (0, "Ez"): np.ones(8),
           (0, "Hx"): np.ones(8), (0, "Hy"): np.ones(8), (0, "Hz"): np.full(8, 1e-17)}
    got = dict(ref)
    got[(0, "Hz")] = np.full(8, 1e-9)
    acc = bench.field_accuracy(got, ref)
    assert acc["components_zero_in_exact_arithmetic"] == ["Hz"]
    assert abs(acc["components_rel_l2"]["Hz"] - 1e-9 / 2 ** 0.5) < 1e-15
