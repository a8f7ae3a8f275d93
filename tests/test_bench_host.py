"""Host-side helpers of bench.py that need no GPU: the oracle's bounded run
per serving request, which the serving leg's CPU baseline is built from."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
import oracle  # noqa: E402
from inputs import layered_circuit  # noqa: E402


def test_request_runs_in_full_within_budget():
    oracle.build(force=False)
    c = layered_circuit(16, 32, 3, gen_seed=[90])
    secs, layers, measured = bench._oracle_request_seconds(c, gate_s=30.0, meas_s=30.0)
    assert layers == 32 and measured == 16 and secs > 0


def test_zero_budget_still_samples_and_scales():
    """With no time budget one block of layers and one measurement still run,
    and the estimate is scaled to the full depth and to n x shots."""
    oracle.build(force=False)
    c = layered_circuit(24, 40, 5, gen_seed=[91])
    secs, layers, measured = bench._oracle_request_seconds(c, gate_s=0.0, meas_s=0.0)
    assert layers == 4 and measured == 1 and np.isfinite(secs) and secs > 0
