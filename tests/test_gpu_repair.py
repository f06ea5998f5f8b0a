"""GPU parity of ct_repair against the oracle's argmin scans, every metric (bit-exact).

Candidates: random rows (mostly invalid) on the tiny, GEMM-like and
absent-value spaces, a few hundred on the 206,786-row GEMM space (several LDS
tiles and valid-list parts), and a sample on the 4.66M-row sparse space.
"""
import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from tests.gpu_common import gpu_space, oracle_space, say, torch
from tests.test_oracle_repair import gap_space

pytestmark = pytest.mark.gpu

METRICS = [ocore.HAMMING, ocore.INDEX_L1, ocore.TIER_EUCLID, ocore.TIER_RANDOM, ocore.HAM1_RANDOM]


def gap_spec():
    return W.SpaceSpec("gap", {"p0": list(range(6)), "p1": list(range(5)), "p2": [0, 1, 2]},
                       ["p0 != 2 and p0 != 3", "p0 + p1 + p2 <= 6", "(p0 * p1) % 4 != 3"])


def run_parity(spec, osp, n, seed, metrics=METRICS, valid_share=0.2):
    t = torch()
    sp = gpu_space(spec)
    rng = np.random.default_rng(seed)
    dig = np.stack([rng.integers(0, r, n) for r in osp.radices], 1).astype(np.int32)
    nv = int(n * valid_share)
    dig[:nv] = osp.vrows[rng.integers(0, osp.n_valid, nv)]
    rows = sp.pack_rows(dig)
    X = (dig.astype(np.int64) << 16) + rng.integers(0, 65536, size=dig.shape)
    Xt = t.tensor(X.astype(np.int32), device="cuda")
    who = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    who_t = t.tensor(who.astype(np.int64), device="cuda").to(t.int32)
    for metric in metrics:
        say(f"[gpu_repair] {spec.name} metric={metric} n={n}")
        seed_k, gen = 0x1234_5678_9ABC, 17
        out_rows, out_pos = sp.repair(rows, metric, seed=seed_k, generation=gen, who=who_t,
                                      pos_q16=Xt if metric == ocore.TIER_EUCLID else None)
        got = out_rows.cpu().numpy()[:, : osp.D].astype(np.int32)
        gpos = out_pos.cpu().numpy().view(np.uint32)
        expect = osp.repair(dig, metric, who=who, key=seed_k, gen=gen, pos_q16=X)
        bad = np.flatnonzero(np.any(got != expect, axis=1))
        assert len(bad) == 0, f"metric {metric}: {len(bad)} rows differ, first {bad[:5]}"
        ok = osp.valid_rows(expect)
        lin = osp.encode(expect)
        exp_pos = np.where(ok, np.searchsorted(osp.vlin, lin), 0xFFFFFFFF).astype(np.uint32)
        assert np.array_equal(gpos, exp_pos)


@pytest.mark.parametrize("name", ["tiny", "gemm10"])
def test_repair_small(name):
    run_parity(W.space(name), oracle_space(name), 3000, 1)


def test_repair_gap_space():
    run_parity(gap_spec(), gap_space(), 2000, 2)


def test_repair_gemm13():
    run_parity(W.gemm13(), oracle_space("gemm13"), 700, 3)


def test_repair_wide20():
    """20 parameters: 32-byte rows, the widest scan kernels."""
    run_parity(W.space("wide20"), oracle_space("wide20"), 400, 5)


def test_repair_sparse16_sample():
    osp = oracle_space("sparse16")
    run_parity(W.sparse16(), osp, 40, 4,
               metrics=[ocore.HAMMING, ocore.INDEX_L1, ocore.TIER_RANDOM, ocore.TIER_EUCLID, ocore.HAM1_RANDOM])


def test_repair_empty_space_and_empty_batch():
    from paper_2606_28372_amd import CtError
    t = torch()
    sp = gpu_space(W.SpaceSpec("none", {"a": [1, 2]}, ["a > 5"]))
    rows = sp.pack_rows(np.zeros((4, 1), dtype=np.int64))
    with pytest.raises(CtError):
        sp.repair(rows, ocore.HAMMING)
    sp2 = gpu_space(W.tiny())
    r0 = sp2.pack_rows(np.zeros((0, 3), dtype=np.int64))
    out, pos = sp2.repair(r0, ocore.HAMMING)
    t.cuda.synchronize()
    assert out.shape[0] == 0


def test_repair_large_batch():
    """More candidates than the scan launches items for: one part per candidate."""
    run_parity(W.gemm10(), oracle_space("gemm10"), 20000, 5, metrics=[ocore.HAMMING, ocore.INDEX_L1,
                                                                          ocore.TIER_RANDOM, ocore.HAM1_RANDOM])


@pytest.mark.parametrize("n", [1480, 2070, 3450])
def test_repair_gemm13_part_counts(n):
    """Candidate counts for which the plan gives each candidate 7, 5 or 3 parts of the list (about
    8,192 items over ~0.79 n candidates to repair): the parts then share each chunk's boxes two or
    one ways instead of eight, and the result must not change."""
    run_parity(W.gemm13(), oracle_space("gemm13"), n, 6, metrics=[ocore.INDEX_L1, ocore.TIER_EUCLID])
