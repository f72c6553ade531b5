"""Host-side parts of bench.py (no GPU): the CPU baseline's job-time model
and the structure of the committed traffic files."""
import json

import bench


class _W:
    n = 1000


def test_cpu_baseline_job_model():
    """Factor builds at the pool's column rate, then the shifts' solves spread
    over the workers longest first (the makespan), value = solves / time."""
    sample = {"model": "x", "cores": 2, "cols_per_s": 1000.0, "iter_s_base": 0.01,
              "iter_s_per_factor": 0.002, "wall_s": 1.0}
    # 3 factors of 1000 columns: 3 s; solves of 100 iterations with chains of
    # 1, 2, 3: 1.2, 1.4, 1.6 s; on 2 workers: {1.6}, {1.4, 1.2} -> 2.6 s
    out = bench.cpu_baseline(_W(), sample, [1, 2, 3], [100, 100, 100], 3)
    assert abs(out["projected_job_s"] - 5.6) < 1e-9
    assert abs(out["value"] - round(3 / 5.6, 6)) < 1e-12
    assert out["cores"] == 2 and out["kind"] == "oracle" and out["unit"] == "solves/s"


def test_host_cpu_description():
    model, cores = bench._host_cpu()
    assert isinstance(model, str) and cores >= 1


def test_traffic_files_describe_their_workload():
    import glob
    import os

    files = glob.glob(os.path.join(bench.ROOT, "profiles", "traffic_chain_step_*.json"))
    assert files
    for path in files:
        with open(path) as f:
            d = json.load(f)
        workload = os.path.basename(path)[len("traffic_chain_step_"):-len(".json")]
        assert workload in d["workload"] and len(d["source_sha256"]) == 64
        assert d["kernels"]
        for label, e in d["kernels"].items():
            assert label.startswith("k_chain_")
            assert e["bytes_per_launch"] > 0 and 0.5 < e["traffic_over_alg"] < 3.0
            cal = e["calibration"]
            # a 1 GiB copy reads FETCH_SIZE in half units and WRITE_SIZE in whole ones
            assert abs(cal["fetch_scale"] - 2.0) < 0.05 and abs(cal["write_scale"] - 1.0) < 0.05
            assert len(e["commands"]) == 2
