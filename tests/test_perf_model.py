"""The benchmark's byte model against the numbers the paper prints for its
own performance model (tests/golden/paper_performance_model.json)."""
import json
import os

import pytest

from paper_2012_06144_amd import perf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_performance_model.json")


@pytest.fixture(scope="module")
def paper():
    return json.load(open(GOLDEN))


def test_fp64_bytes_per_cell_match_paper(paper):
    b = perf.bytes_per_cell("f64")
    assert b["phase_read"] == 8 * paper["phase_counts"]["double_loads"]
    assert b["phase_write"] == 8 * paper["phase_counts"]["double_stores"]
    assert b["hydro_read"] == 8 * paper["hydro_counts"]["double_loads"]
    assert b["hydro_write"] == 8 * paper["hydro_counts"]["double_stores"]
    for row in paper["rows"]:
        assert b[row["kernel"]] == row["n_b"]
    assert b["total"] == 768


def test_paper_roofline_estimates(paper):
    """P_max = b_s / n_b and the balance model reproduce the printed table."""
    for row in paper["rows"]:
        est = perf.p_max_glups(row["b_s"], row["n_b"])
        assert abs(est - row["estimate_glups"]) < 0.006, row
        bal = perf.balance(row["n_b"], row["n_f"], row["b_s"], row["p_peak"])
        assert abs(bal["B_c"] - row["B_c"]) < 0.006
        assert abs(bal["B_m"] - row["B_m"]) < 0.006
        # the printed l is min(1, B_m/B_c) of the printed (2-digit) balances,
        # cut to two digits
        assert 0 <= row["B_m"] / row["B_c"] - row["l"] < 0.01


def test_reduced_precision_bytes():
    assert perf.bytes_per_cell("f32")["total"] == 384
    assert perf.bytes_per_cell("f16s")["total"] == 216
    assert perf.bytes_per_cell("bf16s") == perf.bytes_per_cell("f16s")


@pytest.mark.parametrize("storage,expect", [("f64", 736), ("f32", 368)])
def test_fused_kernel_bytes(storage, expect):
    """The fused kernel (hydrodynamic sweep of one step with the phase sweep
    of the next) reads u and the phase field once instead of twice: the
    coupled count less one u read (3 values) and one phi read."""
    b = perf.bytes_per_cell(storage)
    r = 8 if storage == "f64" else 4
    assert b["fused"] == b["total"] - 4 * r == expect


@pytest.mark.parametrize("storage,expect", [("f64", 1808), ("f32", 904)])
def test_straightforward_bytes(storage, expect):
    """The six passes of the straightforward algorithm read every population
    set three times and write it twice: 3 x 42 + 2 x 42 populations, phi
    written once and read three times, u read three times and written once."""
    b = perf.bytes_per_cell(storage)
    p = 8 if storage == "f64" else 4
    assert b["straightforward"] == (5 * 42) * p + (1 + 3 + 9 + 3) * p == expect


@pytest.mark.parametrize("qp,qh,expect", [(19, 19, 8 * (4 * 19 + 8)), (27, 27, 8 * (4 * 27 + 8)),
                                          (15, 15, 8 * (4 * 15 + 8))])
def test_fused_bytes_other_lattices(qp, qh, expect):
    """Every population of both sets read and written once, u and phi read once
    and written once (FP64)."""
    assert perf.bytes_per_cell("f64", qp, qh)["fused"] == expect
