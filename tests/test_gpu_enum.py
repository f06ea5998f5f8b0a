"""ct_repair_enum: repair by enumerating neighbour shells through the validity bitmask.

Bit-exact against the oracle's argmin scans and against ct_repair (the branch-and-bound scan),
every metric, on the tiny, GEMM-like, absent-value, 20-parameter and Table III stand-in spaces:
with an unlimited lookup budget, with
small budgets (rows split between enumeration and the scans), with out-of-domain rows and with
the GA mutation metric (both always scanned).  With an unlimited budget, exactly the rows whose
winner lies within the enumerated radius are settled by enumeration.  On the 4.66M-row sparse space the enumeration is
checked against the scan alone.
"""
import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from tests.gpu_common import gpu_space, oracle_space, say, torch
from tests.test_gpu_repair import gap_spec
from tests.test_oracle_repair import gap_space

pytestmark = pytest.mark.gpu

SCANNED = [ocore.HAMMING, ocore.INDEX_L1, ocore.TIER_EUCLID, ocore.TIER_RANDOM]
UNLIMITED = 1 << 40


def candidates(osp, n, seed, valid_share=0.2, out_of_domain=0):
    rng = np.random.default_rng(seed)
    dig = np.stack([rng.integers(0, r, n) for r in osp.radices], 1).astype(np.int32)
    nv = int(n * valid_share)
    dig[:nv] = osp.vrows[rng.integers(0, osp.n_valid, nv)]
    for k in range(out_of_domain):                       # a digit at its radix: outside the domain
        j = k % osp.D
        dig[nv + k, j] = osp.radices[j]
    X = (np.minimum(dig, osp.radices - 1).astype(np.int64) << 16) + rng.integers(0, 65536, size=dig.shape)
    who = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    return dig, X, who


def run(spec, osp, n, seed, budgets=(UNLIMITED,), metrics=SCANNED, oracle=True, out_of_domain=0):
    t = torch()
    sp = gpu_space(spec)
    dig, X, who = candidates(osp, n, seed, out_of_domain=out_of_domain)
    rows = sp.pack_rows(dig)
    Xt = t.tensor(X.astype(np.int32), device="cuda")
    who_t = t.tensor(who.astype(np.int64), device="cuda").to(t.int32)
    in_dom = np.all(dig < osp.radices, axis=1)
    invalid = in_dom.copy()
    invalid[in_dom] = ~osp.valid_rows(dig[in_dom])
    stats = {}
    reach = {}
    for metric in metrics:
        kw = dict(seed=0x1234_5678_9ABC, generation=17, who=who_t, pos_q16=Xt if metric == ocore.TIER_EUCLID else None)
        ref_rows, ref_pos = sp.repair(rows, metric, **kw)
        ref = ref_rows.cpu().numpy()[:, : osp.D].astype(np.int32)
        if oracle:
            expect = osp.repair(dig, metric, who=who, key=kw["seed"], gen=17, pos_q16=X)
            assert np.array_equal(ref, expect), f"{spec.name} metric {metric}: the scan differs from the oracle"
        # invalid in-domain rows whose winner lies within the enumerated radius (8): the index
        # distance for INDEX_L1, the Hamming distance otherwise (tier boxes have no radius, so for
        # the tiered metrics this is a lower bound)
        d = np.abs(ref - dig).sum(1) if metric == ocore.INDEX_L1 else (ref != dig).sum(1)
        reach[metric] = int((invalid & (d <= 8)).sum())
        for budget in budgets:
            say(f"[gpu_enum] {spec.name} metric={metric} n={n} max_lookups={budget}")
            out_rows, out_pos, st = sp.repair_enum(rows, metric, max_lookups=budget, **kw)
            got = out_rows.cpu().numpy()[:, : osp.D].astype(np.int32)
            bad = np.flatnonzero(np.any(got != ref, axis=1))
            assert len(bad) == 0, f"{spec.name} metric {metric} budget {budget}: {len(bad)} rows differ, first {bad[:5]}"
            assert np.array_equal(out_pos.cpu().numpy(), ref_pos.cpu().numpy())
            assert st["settled"] <= int(invalid.sum())
            if budget == UNLIMITED and metric in SCANNED:
                if metric in (ocore.HAMMING, ocore.INDEX_L1):
                    assert st["settled"] == reach[metric], (spec.name, metric)
                else:
                    assert st["settled"] >= reach[metric], (spec.name, metric)
            stats[(metric, budget)] = st
    return stats, int(invalid.sum())


@pytest.mark.parametrize("name", ["tiny", "gemm10"])
def test_enum_small_spaces_settle_everything(name):
    stats, n_inv = run(W.space(name), oracle_space(name), 2000, 11, budgets=(UNLIMITED, 64, 0))
    for m in SCANNED:
        if m != ocore.INDEX_L1:                  # (a few gemm10 rows lie beyond index distance 8)
            assert stats[(m, UNLIMITED)]["settled"] == n_inv, (name, m)
        assert stats[(m, 0)]["settled"] == 0 and stats[(m, 0)]["lookups"] == 0
        assert stats[(m, 64)]["lookups"] <= 64 * n_inv


def test_enum_absent_values():
    """Values that occur in no solution: the adjacent box differs from the strictly-adjacent one."""
    run(gap_spec(), gap_space(), 1500, 12, budgets=(UNLIMITED, 16))


def test_enum_gemm13_and_wide20():
    run(W.gemm13(), oracle_space("gemm13"), 400, 13, budgets=(UNLIMITED, 256))
    run(W.space("wide20"), oracle_space("wide20"), 300, 14, budgets=(UNLIMITED, 256))


@pytest.mark.parametrize("name", list(W.BAT_SPACES))
def test_enum_table_iii_stand_ins(name):
    run(W.space(name), oracle_space(name), 400, 15, budgets=(UNLIMITED, 512))


def test_enum_out_of_domain_and_mutation_rows_go_to_the_scan():
    stats, n_inv = run(W.gemm10(), oracle_space("gemm10"), 600, 16, out_of_domain=50,
                       metrics=SCANNED + [ocore.HAM1_RANDOM], oracle=False)
    assert stats[(ocore.HAM1_RANDOM, UNLIMITED)]["settled"] == 0
    for m in (ocore.HAMMING, ocore.TIER_EUCLID, ocore.TIER_RANDOM):
        assert stats[(m, UNLIMITED)]["settled"] == n_inv          # in-domain invalid rows only


def test_enum_sparse16_against_the_scan():
    """4.35e9 configurations, 4.66M valid: enumeration against the scan (no oracle scans)."""
    stats, _ = run(W.sparse16(), oracle_space("sparse16"), 200, 17, budgets=(1 << 20, 4096), oracle=False)
    assert stats[(ocore.INDEX_L1, 1 << 20)]["settled"] > 0


def test_enum_empty_batch_and_errors():
    from paper_2606_28372_amd import CtError
    t = torch()
    sp = gpu_space(W.tiny())
    rows = t.zeros((0, sp.row_bytes), dtype=t.uint8, device="cuda")
    _, _, st = sp.repair_enum(rows, ocore.HAMMING)
    assert st == {"settled": 0, "lookups": 0}
    one = sp.pack_rows(np.zeros((1, 3), dtype=np.int32))
    with pytest.raises(CtError):
        sp.repair_enum(one, 9)
    with pytest.raises(CtError):
        sp.repair_enum(one, ocore.TIER_EUCLID)                  # needs particle positions
