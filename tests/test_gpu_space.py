"""GPU parity of space resolution, validity and rank against the oracle (bit-exact).

Spaces: the tiny, 10- and 13-parameter GEMM-like spaces in full; a 67M-
configuration space whose prefix table does not cover every parameter; edge
cases (empty and full valid sets, a single configuration, one parameter,
32 parameters, radix 255, ragged tails); and the 4.35e9-configuration sparse
space through its golden count and digests plus sampled bitmask words.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from tests.gpu_common import gpu_space, oracle_space, say, torch

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

EDGE = {
    "empty": W.SpaceSpec("empty", {"a": [1, 2, 3], "b": [4, 5]}, ["a > 10"]),
    "full": W.SpaceSpec("full", {"a": list(range(7)), "b": list(range(9)), "c": [0, 1]}, []),
    "single": W.SpaceSpec("single", {"a": [5]}, ["a == 5"]),
    "one_param": W.SpaceSpec("one_param", {"a": list(range(255))}, ["a % 7 == 3 or a > 250"]),
    "wide32": W.SpaceSpec("wide32", {f"p{j}": ([0, 1] if j % 4 == 0 else [j]) for j in range(32)},
                          ["p0 + p4 + p8 + p12 <= 2", "p16 * p20 == p24 * p28 or p0 == 1"]),
    "ragged": W.SpaceSpec("ragged", {"a": list(range(13)), "b": list(range(11)), "c": list(range(7)),
                                     "d": [-3, -1, 0, 2, 9]}, ["(a*b - c) % 5 != 0", "a // (d + 1) >= -2"]),
    "bigsplit": W.SpaceSpec("bigsplit", {f"q{j}": list(range(1, 17)) for j in range(6)} | {"z": [1, 2, 3, 4]},
                            ["q0 + q1 + q2 <= 20", "q3 * q4 % 6 != 1", "(q5 + z) % 3 == 0 and q0 <= q5 + 8"]),
}


def check_space(spec, osp=None):
    t = torch()
    say(f"[gpu_space] {spec.name}: N={spec.n_cartesian}")
    if osp is None:
        osp = ocore.Space.from_spec(spec).enumerate()
    sp = gpu_space(spec)
    assert sp.n_cartesian == osp.n_cartesian
    assert sp.n_valid == osp.n_valid
    words = sp.bitmask().cpu().numpy().view(np.uint64)
    assert np.array_equal(words, osp.words), "bitmask differs"
    lin, rows = sp.valid_list()
    t.cuda.synchronize()
    assert np.array_equal(lin.cpu().numpy().astype(np.uint64), osp.vlin)
    r = rows.cpu().numpy()
    assert np.array_equal(r[:, : len(spec.params)].astype(np.int32), osp.vrows)
    assert not r[:, len(spec.params):].any(), "row padding must be zero"
    return sp, osp


@pytest.mark.parametrize("name", ["tiny", "gemm10", "gemm13"] + list(W.BAT_SPACES))
def test_space_build_parity(name):
    """The GEMM-like spaces and the four Table III stand-ins (hotspot: 22.2M configurations)."""
    check_space(W.space(name), oracle_space(name))


@pytest.mark.parametrize("name", sorted(EDGE))
def test_space_build_edge_cases(name):
    check_space(EDGE[name])


def test_random_small_spaces():
    rng = np.random.default_rng(7)
    pool = ["p0 + p1 <= 7", "p0 * p1 % 3 != 0", "max(p0, p1) - min(p0, p1) >= 2", "p0 // (p1 - 2) > 0",
            "p0 < p1 <= 9", "abs(p0 - 3) != 1 or p1 == 0", "not (p0 % 2 == 0 and p1 % 2 == 0)", "p1 - p0 and p0"]
    for k in range(12):
        D = int(rng.integers(2, 6))
        vals = {f"p{j}": sorted(set(rng.integers(-5, 40, size=int(rng.integers(1, 30))).tolist())) for j in range(D)}
        cons = list(rng.choice(pool, size=int(rng.integers(0, 4)), replace=False))
        check_space(W.SpaceSpec(f"rand{k}", vals, cons))


def test_sparse16_golden_and_sampled_words():
    g = json.load(open(os.path.join(HERE, "golden", "sparse16_space.json")))
    spec = W.sparse16()
    say("[gpu_space] sparse16 build")
    sp = gpu_space(spec)
    assert sp.n_cartesian == g["n_cartesian"]
    assert sp.n_valid == g["n_valid"] == 4657116
    lin, rows = sp.valid_list()
    l = lin.cpu().numpy().astype(np.uint64)
    assert np.all(np.diff(l.astype(np.int64)) > 0)
    assert int(np.sum(l, dtype=np.uint64)) == g["sum_lin_mod64"]
    assert int(np.sum(l * l, dtype=np.uint64)) == g["sumsq_lin_mod64"]
    assert np.array_equal(l[g["sample_pos"]], np.array(g["sample_lin"], dtype=np.uint64))
    osp = ocore.Space.from_spec(spec)
    # rows at the golden sample positions are the oracle's decoding of the golden indices
    sp_pos = np.array(g["sample_pos"])
    assert np.array_equal(rows.cpu().numpy()[sp_pos, :16].astype(np.int32),
                          osp.decode(np.array(g["sample_lin"], dtype=np.uint64)))
    # and every sampled list entry is a solution (a property checked by the oracle)
    pick = np.random.default_rng(1).integers(0, len(l), 2000)
    assert osp.valid_lin(l[pick]).all()
    words = sp.bitmask()
    n_words = words.shape[0]
    w = words.cpu().numpy().view(np.uint64)
    chunk = (1 << 28) // 64
    assert [int(np.unpackbits(w[s:s + chunk].view(np.uint8)).sum()) for s in range(0, n_words, chunk)] == \
        g["chunk_counts"]
    sample = sorted(set(np.random.default_rng(2).integers(0, n_words, 300).tolist() +
                        [int(x) // 64 for x in g["sample_lin"][::10]] + [n_words - 1]))
    for s in sample:
        assert w[s] == osp.mask_words(s, s + 1)[0], f"word {s}"


@pytest.mark.parametrize("name", ["tiny", "gemm10", "gemm13"])
def test_valid_mask_and_rank(name):
    t = torch()
    osp = oracle_space(name)
    sp = gpu_space(W.space(name))
    rng = np.random.default_rng(3)
    n = 5000
    dig = np.stack([rng.integers(0, r, n) for r in osp.radices], 1).astype(np.int32)
    dig[:300] = osp.vrows[rng.integers(0, osp.n_valid, 300)]
    dig[300:320, 0] = osp.radices[0] + rng.integers(0, 3, 20)         # out of the domain
    rows = sp.pack_rows(dig)
    got = sp.valid_mask(rows).cpu().numpy().astype(bool)
    inb = np.all(dig < osp.radices[None, :], axis=1)
    expect = np.zeros(n, dtype=bool)
    expect[inb] = osp.valid_rows(dig[inb])
    assert np.array_equal(got, expect)
    rk = sp.rank(rows).cpu().numpy()
    lin = osp.encode(np.where(inb[:, None], dig, 0))
    exp_rank = np.where(expect, np.searchsorted(osp.vlin, lin), -1)
    assert np.array_equal(rk, exp_rank)
    t.cuda.synchronize()


def test_valid_mask_empty_batch():
    sp = gpu_space(W.tiny())
    rows = sp.pack_rows(np.zeros((0, 3), dtype=np.int64))
    assert sp.valid_mask(rows).shape[0] == 0


def _hip_runtime():
    """The HIP runtime this process already loaded (torch's), for raw device-to-host copies."""
    import ctypes
    with open("/proc/self/maps") as f:
        paths = sorted({ln.split()[-1] for ln in f if "libamdhip64.so" in ln})
    assert paths, "no HIP runtime loaded"
    return ctypes.CDLL(paths[0])


def test_borrowed_list_and_bitmask_pointers():
    """ct_space_valid_list and ct_space_bitmask hand out the space's own buffers: read through them
    they hold the oracle's valid list, rows and bitmask."""
    import ctypes
    t = torch()
    osp = oracle_space("gemm10")
    sp = gpu_space(W.gemm10())
    t.cuda.synchronize()
    plin, prows, pw, nw = sp.borrowed()
    assert plin and prows and pw and nw == (osp.n_cartesian + 63) // 64
    hip = _hip_runtime()
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lin = np.empty(osp.n_valid, dtype=np.uint64)
    rows = np.empty((osp.n_valid, sp.row_bytes), dtype=np.uint8)
    words = np.empty(nw, dtype=np.uint64)
    for host, dev in ((lin, plin), (rows, prows), (words, pw)):
        assert hip.hipMemcpy(host.ctypes.data, dev, host.nbytes, 2) == 0     # device to host
    assert np.array_equal(lin, osp.vlin)
    assert np.array_equal(rows[:, :osp.D].astype(np.int32), osp.vrows)
    assert np.all(rows[:, osp.D:] == 0)
    bits = np.zeros(nw * 64, dtype=bool)
    bits[osp.vlin.astype(np.int64)] = True
    assert np.array_equal(words, np.packbits(bits.reshape(-1, 64)[:, ::-1], axis=1).view(">u8").ravel().astype(np.uint64))


def test_many_problem_counts_match_dynamic_programming():
    """ct_space_count on the first 64 problems of the 256-problem batch (up to ~1e9 configurations
    each) equals the exact DP count of their linear and modulo constraints."""
    from tests.helpers import dpcount
    for pr in W.batched(64, seed=3):
        sp = gpu_space(pr.spec)
        assert sp.n_valid == dpcount.count(pr.spec), pr.spec.name
        assert sp.n_cartesian == pr.spec.n_cartesian
        sp.close()


@pytest.mark.parametrize("name,log2n", [("gemm13", 22), ("sparse16", 23)])
def test_valid_mask_at_scale_matches_the_bitmask(name, log2n):
    """Millions of rows (every round of the persistent kernel, every row slot of a thread): half
    valid, half uniform over the Cartesian space, against the bitmask (checked against the oracle
    by the build tests) looked up with torch."""
    t = torch()
    spec = W.space(name)
    sp = gpu_space(spec)
    n = 1 << log2n
    g = t.Generator(device="cuda")
    g.manual_seed(7)
    D = len(spec.params)
    dig = t.stack([t.randint(0, r, (n,), generator=g, device="cuda") for r in spec.radices], 1)
    _, vrows = sp.valid_list()
    half = n // 2
    dig[:half] = vrows[t.randint(0, sp.n_valid, (half,), generator=g, device="cuda")][:, :D].long()
    say(f"[gpu_space] valid_mask {name} n=2^{log2n}")
    got = sp.valid_mask(sp.pack_rows(dig)).bool()
    strides = np.cumprod([1] + spec.radices[::-1][:-1])[::-1].copy()
    L = (dig * t.tensor(strides, device="cuda", dtype=t.int64)).sum(1)
    words = sp.bitmask().view(t.int64)
    expect = ((words[L >> 6] >> (L & 63)) & 1).bool()
    bad = t.nonzero(got != expect).flatten()
    assert bad.numel() == 0, f"{bad.numel()} rows differ, first {bad[:5].tolist()}"
    assert bool(expect[:half].all())
