"""The precision policy's escalation decision (did FP32 sweeps miss eps?) is
taken on a 4096-sample check.  Against the same check on 1e6 samples (the
4096 being their prefix), on the FP32 results of the mixed batch's first
problems: the same decision for every problem, and near eps the two errors
agree closely (bench.py --workload escalation measures all 512)."""
import numpy as np
import pytest

from paper_2407_11290_amd import PREC_FP32
from paper_2407_11290_amd.api import TTCross, batch_run
from paper_2407_11290_amd.workloads import batch_mix

pytestmark = pytest.mark.gpu


def test_4096_sample_check_decides_as_1e6_samples():
    specs = batch_mix()[:64]
    hs = [TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, grid=p.grid, precision=PREC_FP32, verify=0)
          for p in specs]
    batch_run(hs)
    near = 0
    for p, h in zip(specs, hs):
        e4 = h.sampled_error(4096, seed=p.seed + 1)
        e6 = h.sampled_error(1_000_000, seed=p.seed + 1)
        print("[case]", p.n, p.fn_id, p.seed, e4 / p.eps, e6 / p.eps, flush=True)
        assert (e4 > p.eps) == (e6 > p.eps), (p.n, p.seed, e4, e6)
        if 0.3 * p.eps < e6 < 3 * p.eps:
            near += 1
            assert 0.8 < e4 / e6 < 1.25, (p.n, p.seed, e4, e6)
        h.close()
    assert near >= 1
