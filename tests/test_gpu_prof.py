"""Kernel timing support: events around every launch or around a sample of them."""
import pytest

import workloads as W
from tests.gpu_common import gpu_space, say, torch

pytestmark = pytest.mark.gpu


def test_prof_sample_and_seen():
    """ct_prof_sample(k) records events around every k-th launch of a kernel name; ct_prof_seen
    counts them all; the timings are positive; 0 is refused."""
    import paper_2606_28372_amd as ct
    t = torch()
    sp = gpu_space(W.gemm10())
    obj = t.tensor(W.objective(sp.n_valid, 11), device="cuda")
    pop = ct.Pop.from_opt(sp, W.OptParams(W.ALGO_PSO, 200, 2), obj)
    say("[gpu_prof] every launch")
    ct.prof_select("k_propose")
    ct.prof_sample(1)
    ct.prof_enable(True)
    pop.step(9)
    ms, n = ct.prof_read("k_propose")
    seen = ct.prof_seen("k_propose")
    ct.prof_enable(False)
    assert n == seen == 9 and ms > 0
    say("[gpu_prof] every 4th launch")
    ct.prof_sample(4)
    ct.prof_enable(True)
    pop.step(9)
    ms, n = ct.prof_read("k_propose")
    seen = ct.prof_seen("k_propose")
    ct.prof_enable(False)
    assert seen == 9 and n == 3 and ms > 0          # launches 0, 4 and 8
    assert ct.prof_seen("k_select") == 0            # not selected: not counted
    ct.prof_sample(1)
    ct.prof_select(None)
    with pytest.raises(ct.CtError):
        ct.prof_sample(0)
    pop.close()
    t.cuda.synchronize()
