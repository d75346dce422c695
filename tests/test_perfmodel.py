"""Eq. (1) / eq. (2) code-balance model against the numbers the paper prints
(Sect. 2 worked example on one Nehalem EP socket; Sect. 3.1 split penalty)."""
import json
import os

import pytest

from paper_1101_0091_amd import perfmodel as pm

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_worked_numbers.json")))
NODE = G["node_nehalem"]


def test_eq1_balance_at_15():
    # 6 + 12/15 = 6.8 bytes/flop
    assert pm.code_balance_crs(15, 0) == pytest.approx(6.8, abs=1e-12)


def test_max_performance_from_bandwidth():
    assert pm.perf_bound_gflops(NODE["spmv_bw_gbs"], NODE["nnzr"]) == pytest.approx(
        NODE["max_perf_at_spmv_bw_gflops"], abs=0.005)
    assert pm.perf_bound_gflops(NODE["stream_triad_gbs"], NODE["nnzr"]) == pytest.approx(
        NODE["max_perf_at_stream_gflops"], abs=0.005)


def test_kappa_extraction():
    k = pm.kappa_from_measurement(NODE["measured_gflops"], NODE["spmv_bw_gbs"], NODE["nnzr"])
    assert k == pytest.approx(NODE["kappa"], abs=0.05)
    assert k * NODE["nnzr"] == pytest.approx(NODE["extra_bytes_per_row"], abs=0.1)
    assert round(pm.extra_b_loads(k, NODE["nnzr"])) == NODE["b_loads"]


def test_wider_bandwidth_numbering():
    k1 = pm.kappa_from_measurement(NODE["measured_gflops"], NODE["spmv_bw_gbs"], NODE["nnzr"])
    k2 = NODE["kappa_hmep_wide"]
    assert k2 / k1 - 1 == pytest.approx(NODE["extra_b_traffic_increase"], abs=0.05)
    drop = 1 - pm.code_balance_crs(15, k1) / pm.code_balance_crs(15, k2)
    # the model gives ~7.5%; the text reports "about 10%" measured
    assert 0.05 < drop < NODE["perf_drop_about"] + 0.01


def test_eq2_split_penalty():
    e = G["eq2"]
    assert pm.split_penalty(e["nnzr_lo"]) == pytest.approx(e["penalty_at_lo"], abs=0.005)
    assert pm.split_penalty(e["nnzr_hi"]) == pytest.approx(e["penalty_at_hi"], abs=0.005)
    # and less when kappa > 0
    assert pm.split_penalty(15, 2.5) < pm.split_penalty(15, 0)


def test_gpu_form():
    # 2D Laplacian 256^2: 326,656 nnz -> 5.23 MB compulsory (FP64)
    b = pm.compulsory_bytes(65536, 65536, 326656)
    assert b == 12 * 326656 + 4 * 65537 + 8 * 65536 * 2
    assert pm.compulsory_bytes(65536, 65536, 326656, val_bytes=4, b_bytes=4) == \
        8 * 326656 + 4 * 65537 + 4 * 65536 + 8 * 65536
    # kappa from bytes inverts compulsory
    assert pm.kappa_from_bytes(b + 2.5 * 326656, 65536, 65536, 326656) == pytest.approx(2.5)
    assert pm.gflops(10**9, 1.0) == 2.0
