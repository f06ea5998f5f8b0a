"""ct_repair_noalloc (static device scratch, no allocation) against ct_repair, bit-exact.

Two calls in a row share the GPU's static scratch array, the second with a
smaller input and another space, so anything the first call leaves behind in
the scratch (list counters, per-part winners, the plan) would show up as a
difference.  Row counts at and above CT_NOALLOC_MAX_ROWS check the size limit.
"""
import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from tests.gpu_common import gpu_space, oracle_space, say, torch

pytestmark = pytest.mark.gpu

METRICS = [ocore.HAMMING, ocore.INDEX_L1, ocore.TIER_EUCLID, ocore.TIER_RANDOM, ocore.HAM1_RANDOM]
MAX_ROWS = 16384   # CT_NOALLOC_MAX_ROWS


def candidates(sp, osp, n, seed):
    t = torch()
    rng = np.random.default_rng(seed)
    dig = np.stack([rng.integers(0, r, n) for r in osp.radices], 1).astype(np.int32)
    nv = n // 5
    dig[:nv] = osp.vrows[rng.integers(0, osp.n_valid, nv)]
    rows = sp.pack_rows(dig)
    X = (dig.astype(np.int64) << 16) + rng.integers(0, 65536, size=dig.shape)
    Xt = t.tensor(X.astype(np.int32), device="cuda")
    who = t.tensor(rng.integers(0, 2 ** 31, n), device="cuda").to(t.int32)
    return rows, Xt, who


def compare(sp, rows, Xt, who, metric, tag):
    t = torch()
    n = rows.shape[0]
    say(f"[no_alloc] {tag} metric={metric} n={n}")
    kw = dict(seed=0xC0FFEE, generation=9, who=who, pos_q16=Xt if metric == ocore.TIER_EUCLID else None)
    ref_rows, ref_pos = sp.repair(rows, metric, **kw)
    out_rows = t.full_like(rows, 0xAB)
    out_pos = t.full((n,), -7, dtype=t.int32, device="cuda")
    sp.repair_noalloc(rows, metric, out_rows=out_rows, out_pos=out_pos, **kw)
    t.cuda.synchronize()
    assert t.equal(out_rows, ref_rows), f"{tag} metric {metric}: rows differ"
    assert t.equal(out_pos, ref_pos), f"{tag} metric {metric}: positions differ"


def test_noalloc_matches_repair_two_calls():
    big = gpu_space(W.gemm10())
    small = gpu_space(W.gemm13())
    rb = candidates(big, oracle_space("gemm10"), 12000, 11)
    rs = candidates(small, oracle_space("gemm13"), 600, 12)
    for metric in METRICS:
        compare(big, *rb, metric, "gemm10 first call")
        compare(small, *rs, metric, "gemm13 second, smaller call")


def test_noalloc_size_limit_and_empty():
    from paper_2606_28372_amd import CtError
    t = torch()
    sp = gpu_space(W.tiny())
    rows, Xt, who = candidates(sp, oracle_space("tiny"), MAX_ROWS, 13)
    compare(sp, rows, Xt, who, ocore.INDEX_L1, "tiny at the row limit")
    over = t.zeros((MAX_ROWS + 1, sp.row_bytes), dtype=t.uint8, device="cuda")
    out = t.zeros_like(over)
    pos = t.zeros(MAX_ROWS + 1, dtype=t.int32, device="cuda")
    with pytest.raises(CtError):
        sp.repair_noalloc(over, ocore.HAMMING, out_rows=out, out_pos=pos)
    r0 = sp.pack_rows(np.zeros((0, 3), dtype=np.int64))
    sp.repair_noalloc(r0, ocore.HAMMING, out_rows=r0.clone(), out_pos=t.zeros(0, dtype=t.int32, device="cuda"))
    compare(sp, rows[:5], Xt[:5], who[:5], ocore.TIER_EUCLID, "tiny, 5 rows after the limit")
