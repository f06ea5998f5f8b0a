"""GPU parity of the DE / PSO / GA generation steps against the oracle (bit-exact).

Every generation's full state is compared: DE/GA population positions and
objective values, best, generation and reinitialisation counters; PSO
positions, velocities, personal bests and the global-best index.  Configs:
the tiny space's 100-generation DE run in full, DE/PSO/GA with population 1024
on the 10- and 13-parameter GEMM spaces, and GA with population 4096 on the
sparse space through sampled children.
"""
import struct

import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from oracle import steps as ost
from tests.gpu_common import gpu_space, oracle_space, parse_snapshot, say, torch

pytestmark = pytest.mark.gpu


def ord_to_f32(o):
    bits = (o & 0x7FFFFFFF) if (o & 0x80000000) else (~o & 0xFFFFFFFF)
    return struct.unpack("<f", struct.pack("<I", bits))[0]


def make_pop(sp, opt, obj_t):
    from paper_2606_28372_amd import Pop
    return Pop.from_opt(sp, opt, obj_t)


def oracle_init(osp, obj, opt):
    return ost.init_run(osp, obj, opt)


def oracle_step(osp, obj, st, opt):
    return ost.step_run(osp, obj, st, opt)


def compare(pop, st, opt, D, where):
    g = parse_snapshot(pop.snapshot(), opt.algo, opt.pop_size, D)
    assert g["gen"] == st.gen, where
    if getattr(st, "evaluated", None) is not None:
        # the configurations the last step evaluated (ct_pop_evaluated)
        bad = np.flatnonzero(pop.evaluated() != st.evaluated)
        assert len(bad) == 0, f"{where}: evaluated positions differ at {bad[:5].tolist()}"
    if opt.algo == W.ALGO_PSO:
        for k in ("X", "V", "PB"):
            bad = np.argwhere(g[k] != getattr(st, k))
            assert len(bad) == 0, f"{where}: PSO {k} differs at {bad[:3].tolist()}"
        assert np.array_equal(g["f_pb"], st.f_pb), where
        assert np.array_equal(g["pb_pos"], st.pb_pos), where
        assert g["g_idx"] == st.g_idx, where
        assert g["best_pos"] == st.best_pos
    else:
        if opt.algo == W.ALGO_FF:
            bad = np.argwhere(g["X"] != st.X)
            assert len(bad) == 0, (f"{where}: Firefly X differs at {bad[:3].tolist()}: GPU "
                                   f"{g['X'][bad[0][0]].tolist()} oracle {st.X[bad[0][0]].tolist()}")
        bad = np.flatnonzero(g["pos"] != st.pos)
        assert len(bad) == 0, (f"{where}: population differs at {bad[:5].tolist()}: GPU {g['pos'][bad[:5]].tolist()} "
                               f"oracle {st.pos[bad[:5]].tolist()}")
        assert np.array_equal(g["f"], st.f.astype(np.float32)), where
        assert g["best_pos"] == st.best_pos, where
        assert np.float32(ord_to_f32(g["best_ord"])) == np.float32(st.best_f), where
        if opt.algo == W.ALGO_DE:
            assert g["reinits"] == st.reinits, where



def run(space_name, opt, gens, obj_seed):
    t = torch()
    osp = oracle_space(space_name)
    obj = W.objective(osp.n_valid, obj_seed)
    sp = gpu_space(W.space(space_name))
    obj_t = t.tensor(obj, device="cuda")
    pop = make_pop(sp, opt, obj_t)
    st = oracle_init(osp, obj, opt)
    name = f"{space_name}/{W.ALGO_NAMES[opt.algo]}/P{opt.pop_size}"
    compare(pop, st, opt, osp.D, f"{name} init")
    for gnum in range(gens):
        say(f"[gpu_steps] {name} generation {gnum}")
        pop.step(1)
        st = oracle_step(osp, obj, st, opt)
        compare(pop, st, opt, osp.D, f"{name} gen {gnum + 1}")
    return pop, st


def test_tiny_de_full_run():
    run("tiny", W.OptParams(W.ALGO_DE, 20, 0), 100, 0)


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA])
def test_gemm10_steps(algo):
    run("gemm10", W.OptParams(algo, 1024, 1), 4, 1)


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA])
def test_gemm13_steps(algo):
    run("gemm13", W.OptParams(algo, 1024, 1), 2, 1)


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA])
def test_wide20_steps(algo):
    """20 parameters: two digits per proposal lane, 32-byte rows in the scans and the mutation."""
    run("wide20", W.OptParams(algo, 256, 12), 3, 2)


def test_small_populations_and_odd_sizes():
    run("tiny", W.OptParams(W.ALGO_GA, 33, 5), 6, 0)
    run("tiny", W.OptParams(W.ALGO_PSO, 100, 6), 5, 0)             # P == |V|: one member per stratum
    run("gemm10", W.OptParams(W.ALGO_DE, 4, 7), 8, 1)               # smallest DE population
    run("tiny", W.OptParams(W.ALGO_DE, 20, 8, F_q16=0, CR_q32=1 << 32), 3, 0)   # forced reinitialisation


@pytest.mark.parametrize("P", [1500, 3000])
def test_ga_populations_past_the_block_size(P):
    """GA populations larger than the selection block (1,024 threads) rank-sort with several keys
    per thread (2 and 4 here): generation by generation equal to the oracle."""
    run("gemm10", W.OptParams(W.ALGO_GA, P, 9), 3, 1)


def test_ga_largest_population():
    """GA at its largest population (8,192: eight keys per thread in the rank sort)."""
    run("gemm13", W.OptParams(W.ALGO_GA, 8192, 10), 2, 1)


def test_rand1bin_and_other_coefficients():
    run("gemm10", W.OptParams(W.ALGO_DE, 64, 9, de_method=0, F_q16=65536, CR_q32=1 << 31), 4, 1)
    run("gemm10", W.OptParams(W.ALGO_PSO, 64, 10, w_q16=50000, c1_q16=70000, c2_q16=150000), 4, 1)
    run("gemm10", W.OptParams(W.ALGO_GA, 64, 11, mutation_chance=2, beta_b=1), 4, 1)


def test_sparse16_ga_sampled_children():
    """Generation 0 -> 1 at population 4096: 24 sampled children against the oracle's own state;
    later generations through properties the oracle checks (population valid, best monotone)."""
    t = torch()
    osp = oracle_space("sparse16")
    opt = W.OptParams(W.ALGO_GA, 4096, 2)
    obj = W.objective(osp.n_valid, 2)
    sp = gpu_space(W.sparse16())
    pop = make_pop(sp, opt, t.tensor(obj, device="cuda"))
    st = ost.ga_init(osp, obj, opt.pop_size, opt.seed)
    compare(pop, st, opt, osp.D, "sparse16 init")
    sample = np.random.default_rng(12).choice(opt.pop_size, 24, replace=False)
    say("[gpu_steps] sparse16 GA generation 0")
    pop.step(1)
    after = parse_snapshot(pop.snapshot(), opt.algo, opt.pop_size, osp.D)
    kids = ost.ga_children(osp, obj, st, opt.seed, opt.mutation_chance, opt.beta_b, sample)
    assert np.array_equal(after["pos"][sample], osp.pos(osp.encode(kids)))
    best = ord_to_f32(after["best_ord"])
    for gnum in range(1, 4):
        say(f"[gpu_steps] sparse16 GA generation {gnum}")
        pop.step(1)
        g = parse_snapshot(pop.snapshot(), opt.algo, opt.pop_size, osp.D)
        assert g["gen"] == gnum + 1
        assert np.all(g["pos"] < osp.n_valid) and osp.valid_rows(osp.vrows[g["pos"]]).all()
        assert np.array_equal(g["f"], obj[g["pos"]])
        b = ord_to_f32(g["best_ord"])
        assert b <= best and np.float32(obj[g["best_pos"]]) == np.float32(b)
        best = b


def test_snapshot_restore_replays_bit_identically():
    t = torch()
    osp = oracle_space("gemm10")
    obj_t = t.tensor(W.objective(osp.n_valid, 1), device="cuda")
    sp = gpu_space(W.gemm10())
    for algo in (W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA):
        pop = make_pop(sp, W.OptParams(algo, 128, 3), obj_t)
        pop.step(3)
        snap = pop.snapshot()
        pop.step(4)
        a = pop.snapshot()
        pop.restore(snap)
        pop.step(4)
        assert pop.snapshot() == a


def test_population_errors():
    from paper_2606_28372_amd import CtError, Pop
    t = torch()
    sp = gpu_space(W.tiny())
    obj_t = t.ones(sp.n_valid, device="cuda")
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 101, 0, obj_t)     # more members than valid configurations
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 3, 0, obj_t)       # DE needs four distinct members
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_GA, 10, 0, obj_t, beta_b=9)
