"""Host logic of bench.py that needs no GPU: the oracle-agreement figures of
the benchmark line."""
import numpy as np

import bench


def test_oracle_agreement_counts_set_difference_and_value_error():
    refs = [dict(locs=np.array([3, 7, 9]), vals=np.array([1.0 + 0j, 0.5j, 2.0])),
            dict(locs=np.array([1]), vals=np.array([1.0 + 1.0j]))]
    res = [dict(locs=np.array([3, 9, 11]), vals=np.array([1.0 + 1e-5j, 2.0 + 4e-5, 0.1])),
           dict(locs=np.array([1]), vals=np.array([1.0 + 1.0j]))]
    a = bench.oracle_agreement(res, refs)
    assert a["oracle_signals"] == 2
    assert a["oracle_set_diff"] == 2 and a["oracle_set_diff_per_signal"] == [2, 0]
    # on the common frequencies 3 and 9: 1e-5 / 1 and 4e-5 / 2
    assert abs(a["oracle_max_rel_err"] - 2e-5) < 1e-12
    assert abs(a["oracle_mean_rel_err"] - 1e-5) < 1e-12


def test_oracle_agreement_uses_the_floor_denominator():
    # a near-zero oracle value is measured against 1e-3 of the largest one
    refs = [dict(locs=np.array([0, 1]), vals=np.array([1e-9 + 0j, 10.0 + 0j]))]
    res = [dict(locs=np.array([0, 1]), vals=np.array([1e-3 + 0j, 10.0 + 0j]))]
    a = bench.oracle_agreement(res, refs, floor=1e-3)
    assert abs(a["oracle_max_rel_err"] - (1e-3 - 1e-9) / 1e-2) < 1e-9
    a = bench.oracle_agreement(res, refs)  # FP32 floor: 1e-2 of the largest
    assert abs(a["oracle_max_rel_err"] - (1e-3 - 1e-9) / 1e-1) < 1e-9


def test_cpu_model_is_named():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_traffic_summary_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    """The committed HBM-traffic summary is reported only while the k_hash
    source section, the lines that size its grid and the batch are the ones
    the counters were taken on."""
    p = tmp_path / "traffic.txt"

    def write(src_sha, launch_sha, batch=32):
        p.write_text("# counters\nkernel = k_hash main loops\n"
                     f"batch = {batch}\nhbm_bytes_per_launch = 123456\n"
                     f"k_hash_source_sha256 = {src_sha}\nk_hash_launch_sha256 = {launch_sha}\n")

    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    src, launch = bench.hash_kernel_sha256(), bench.hash_launch_sha256()
    assert len(src) == 64 and len(launch) == 64 and src != launch
    write(src, launch)
    assert bench.measured_traffic(32) == 123456.0
    assert bench.measured_traffic(64) is None  # another batch
    write("0" * 64, launch)
    assert bench.measured_traffic(32) is None  # the k_hash section changed
    write(src, "0" * 64)
    assert bench.measured_traffic(32) is None  # the grid sizing changed
