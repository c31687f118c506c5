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
