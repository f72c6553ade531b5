"""Host-side helpers of bench.py (no GPU): the name of the chain-step
instance the library launches, which keys the measured HBM traffic, and the
structure of the committed traffic files."""
import json
import os

import bench
from paper_2003_12759_amd.workloads import make_workload


def test_chain_kernel_labels():
    w1 = make_workload(1, N=8)  # 7-point: every row of S and S^T has at most 8 entries
    name = bench.chain_kernel_name
    assert name(w1.A, "float", "double", 10, 2, True) == "k_chain_halo<float, double, 2>"
    assert name(w1.A, "float", "double", 10, 2, False) == "k_chain_narrow<float, double, 2>"
    # 10 columns balanced into chunks of at most 8 (two of 5) or 16 (one of 10)
    assert name(w1.A, "float", "double", 10, 8, True) == "k_chain_halo<float, double, 5>"
    assert name(w1.A, "float", "double", 10, 16, True) == "k_chain_halo<float, double, 10>"
    w4 = make_workload(4, N=6)  # 27-point
    assert (name(w4.A, "unsigned short", "double", 12, 16, False)
            == "k_chain_step<unsigned short, double, 12>")
    assert (name(w4.A, "unsigned short", "double", 12, 16, True)
            == "k_chain_halo<unsigned short, double, 12>")


def test_traffic_files_describe_their_workload():
    for workload in ("convdiff3d_n262144", "varcoef27_n2097152"):
        with open(bench.traffic_file(workload)) as f:
            d = json.load(f)
        assert workload in d["workload"] and len(d["source_sha256"]) == 64
        assert d["kernels"]
        for label, e in d["kernels"].items():
            assert label.startswith("k_chain_")
            assert e["bytes_per_launch"] > 0 and 0.5 < e["traffic_over_alg"] < 2.0
            cal = e["calibration"]
            # a 1 GiB copy reads FETCH_SIZE in half units and WRITE_SIZE in whole ones
            assert abs(cal["fetch_scale"] - 2.0) < 0.05 and abs(cal["write_scale"] - 1.0) < 0.05
            assert len(e["commands"]) == 2
