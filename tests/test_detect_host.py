"""Super-point selection: the oracle's definition on hand-made cases (CPU)."""
import numpy as np

from oracle import oracle


def test_select_hosts_definition():
    est = np.array([0.0, 5.0, 4.999999, 5.0000005, np.nan, np.inf, -1.0, 7.5], np.float32)
    hosts = np.array([10, 11, 12, 13, 14, 15, 16, 17], np.uint32)
    rows = oracle.select_hosts(est, hosts, 5.0)
    assert [h for h, _ in rows] == [11, 13, 15, 17]  # ties at the threshold are kept, NaN never
    assert oracle.select_hosts(est, hosts, np.inf) == [(15, float("inf"))]
    assert oracle.select_hosts(est[:0], hosts[:0], 1.0) == []
