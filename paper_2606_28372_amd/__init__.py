"""MI355X-native constraint-aware evolutionary auto-tuning (Python binding of libct).

Thin marshalling over the C ABI of include/ct.h: torch tensors provide device
memory and the current HIP stream; every step of the method runs in the
library's HIP kernels.  Importing this package loads nothing; the first call
loads lib/libct.so and raises if it was not built.

    sp = Space(names, values, constraints)          # ct_compile + ct_space_build
    sp.n_valid, sp.valid_list(), sp.bitmask()
    sp.valid_mask(rows), sp.rank(rows), sp.repair(rows, CT_HAMMING)
    run = Pop(sp, algo=CT_DE, pop_size=20, seed=0, objective=obj)   # ct_pop_create
    run.step(100); run.read()                                        # ct_step, ct_pop_read
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import (CT_DE, CT_FIREFLY, CT_GA, CT_HAM1_RANDOM, CT_HAMMING, CT_INDEX_L1, CT_PSO, CT_SCAN_FUSED,  # noqa: F401
                   CT_SCAN_SERIAL, CT_SCAN_STREAMS, CT_STEP_BATCHED, CT_STEP_GRAPH, CT_STEP_PLAIN, CT_TIER_EUCLID,
                   CT_TIER_RANDOM, CtError, ct_pop_params)

__all__ = ["Space", "Pop", "Batch", "Server", "compile_constraints", "step_many", "CtError", "CT_HAMMING", "CT_INDEX_L1",
           "CT_TIER_EUCLID", "CT_TIER_RANDOM", "CT_HAM1_RANDOM", "CT_DE", "CT_PSO", "CT_GA", "CT_FIREFLY",
           "CT_STEP_PLAIN", "CT_STEP_BATCHED", "CT_STEP_GRAPH", "CT_SCAN_SERIAL", "CT_SCAN_STREAMS", "CT_SCAN_FUSED"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _device_arg(t, name: str, dtypes, shape=None):
    """Check a tensor handed to the library by pointer: device memory, dtype, dense layout, shape."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU, got {type(t).__name__}")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be in GPU memory")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def compile_constraints(names: Sequence[str], values: Sequence[Sequence[int]],
                        constraints: Sequence[str]) -> Tuple[np.ndarray, np.ndarray]:
    """ct_compile: constraint strings -> (bytecode words, program offsets)."""
    L = _lib.load()
    n = len(names)
    flat = np.ascontiguousarray([int(x) for v in values for x in v], dtype=np.int64)
    rad = np.ascontiguousarray([len(v) for v in values], dtype=np.uint32)
    cnames = (ctypes.c_char_p * n)(*[s.encode() for s in names])
    ccons = (ctypes.c_char_p * max(1, len(constraints)))(*[c.encode() for c in constraints])
    cap = 64 + 64 * sum(len(c) for c in constraints)
    code = np.zeros(cap, dtype=np.uint32)
    offs = np.zeros(len(constraints) + 1, dtype=np.uint32)
    used = ctypes.c_uint32(0)
    _lib.check(L.ct_compile(cnames, n, flat.ctypes.data, rad.ctypes.data, ccons, len(constraints),
                            code.ctypes.data, cap, offs.ctypes.data, ctypes.byref(used)))
    return code[: used.value].copy(), offs


class Space:
    """A resolved search space on the current GPU (ct_space)."""

    def __init__(self, names: Sequence[str], values: Sequence[Sequence[int]], constraints: Sequence[str]):
        L = _lib.load()
        self.names = list(names)
        self.values = [list(map(int, v)) for v in values]
        self.constraints = list(constraints)
        self.code, self.offsets = compile_constraints(self.names, self.values, self.constraints)
        flat = np.ascontiguousarray([x for v in self.values for x in v], dtype=np.int64)
        rad = np.ascontiguousarray([len(v) for v in self.values], dtype=np.uint32)
        self._h = ctypes.c_void_p()
        code = self.code if len(self.code) else np.zeros(1, dtype=np.uint32)
        _lib.check(L.ct_space_build(flat.ctypes.data, rad.ctypes.data, len(self.names), code.ctypes.data,
                                    self.offsets.ctypes.data, len(self.constraints), _stream(),
                                    ctypes.byref(self._h)))
        nv, nc = ctypes.c_uint64(), ctypes.c_uint64()
        _lib.check(L.ct_space_count(self._h, ctypes.byref(nv), ctypes.byref(nc)))
        d, r = ctypes.c_uint32(), ctypes.c_uint32()
        _lib.check(L.ct_space_info(self._h, ctypes.byref(d), ctypes.byref(r)))
        self.n_valid, self.n_cartesian = int(nv.value), int(nc.value)
        self.D, self.row_bytes = int(d.value), int(r.value)

    @classmethod
    def from_spec(cls, spec) -> "Space":
        return cls(spec.names, list(spec.params.values()), spec.constraints)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def footprint(self) -> int:
        """Device bytes the built space holds (ct_space_footprint)."""
        b = ctypes.c_uint64()
        _lib.check(_lib.load().ct_space_footprint(self._h, ctypes.byref(b)))
        return int(b.value)

    def valid_list(self):
        """(linear indices int64 [n_valid], digit rows uint8 [n_valid, row_bytes]) as new device tensors."""
        torch = _torch()
        lin = torch.empty(self.n_valid, dtype=torch.int64, device="cuda")
        rows = torch.empty((self.n_valid, self.row_bytes), dtype=torch.uint8, device="cuda")
        _lib.check(_lib.load().ct_space_copy_list(self._h, _ptr(lin), _ptr(rows), _stream()))
        return lin, rows

    def bitmask(self):
        torch = _torch()
        w = torch.empty((self.n_cartesian + 63) // 64, dtype=torch.int64, device="cuda")
        _lib.check(_lib.load().ct_space_copy_bitmask(self._h, _ptr(w), _stream()))
        return w

    def borrowed(self):
        """ct_space_valid_list / ct_space_bitmask: the space's own device pointers (borrowed, valid until
        close) as integers: (linear indices, digit rows, bitmask words, number of words)."""
        lib = _lib.load()
        lin, rows, words = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        nw = ctypes.c_uint64()
        _lib.check(lib.ct_space_valid_list(self._h, ctypes.byref(lin), ctypes.byref(rows)))
        _lib.check(lib.ct_space_bitmask(self._h, ctypes.byref(words), ctypes.byref(nw)))
        return lin.value or 0, rows.value or 0, words.value or 0, nw.value

    def pack_rows(self, digits) -> "object":
        """Digit matrix [n, D] (any integer tensor/array) -> uint8 rows [n, row_bytes] on the GPU."""
        torch = _torch()
        d = torch.as_tensor(np.asarray(digits) if not isinstance(digits, torch.Tensor) else digits)
        out = torch.zeros((d.shape[0], self.row_bytes), dtype=torch.uint8, device="cuda")
        out[:, : self.D] = d.to(device="cuda", dtype=torch.uint8)
        return out

    def _rows_arg(self, rows, name="rows"):
        torch = _torch()
        n = rows.shape[0] if isinstance(rows, torch.Tensor) and rows.dim() == 2 else -1
        return _device_arg(rows, name, (torch.uint8,), (n, self.row_bytes))

    def valid_mask(self, rows):
        torch = _torch()
        self._rows_arg(rows)
        out = torch.empty(rows.shape[0], dtype=torch.uint8, device="cuda")
        _lib.check(_lib.load().ct_valid_mask(self._h, _ptr(rows), rows.shape[0], _ptr(out), _stream()))
        return out

    def rank(self, rows):
        torch = _torch()
        self._rows_arg(rows)
        out = torch.empty(rows.shape[0], dtype=torch.int64, device="cuda")
        _lib.check(_lib.load().ct_rank(self._h, _ptr(rows), rows.shape[0], _ptr(out), _stream()))
        return out

    def repair(self, rows, metric: int, seed: int = 0, generation: int = 0, who=None, pos_q16=None,
               out_rows=None, out_pos=None):
        """ct_repair: returns (rows uint8 [n, row_bytes], positions int32 [n] (0xFFFFFFFF = none))."""
        torch = _torch()
        self._rows_arg(rows)
        n = rows.shape[0]
        if who is not None:
            _device_arg(who, "who", (torch.int32,), (n,))
        if pos_q16 is not None:
            _device_arg(pos_q16, "pos_q16", (torch.int32,), (n, self.D))
        if out_rows is None:
            out_rows = torch.empty_like(rows)
        if out_pos is None:
            out_pos = torch.empty(n, dtype=torch.int32, device="cuda")
        self._rows_arg(out_rows, "out_rows")
        _device_arg(out_pos, "out_pos", (torch.int32,), (n,))
        _lib.check(_lib.load().ct_repair(self._h, _ptr(rows), n, metric, seed, generation, _ptr(who),
                                         _ptr(pos_q16), _ptr(out_rows), _ptr(out_pos), _stream()))
        return out_rows, out_pos

    def repair_enum(self, rows, metric: int, seed: int = 0, generation: int = 0, who=None, pos_q16=None,
                    max_lookups: int = 1 << 16, out_rows=None, out_pos=None):
        """ct_repair_enum: ct_repair's results, by enumeration of neighbour shells through the bitmask
        where a row needs at most max_lookups lookups, by the scans otherwise.
        Returns (rows, positions, {"settled": rows enumeration settled, "lookups": lookups spent})."""
        torch = _torch()
        self._rows_arg(rows)
        n = rows.shape[0]
        if who is not None:
            _device_arg(who, "who", (torch.int32,), (n,))
        if pos_q16 is not None:
            _device_arg(pos_q16, "pos_q16", (torch.int32,), (n, self.D))
        if out_rows is None:
            out_rows = torch.empty_like(rows)
        if out_pos is None:
            out_pos = torch.empty(n, dtype=torch.int32, device="cuda")
        self._rows_arg(out_rows, "out_rows")
        _device_arg(out_pos, "out_pos", (torch.int32,), (n,))
        st = (ctypes.c_uint64 * 2)()
        _lib.check(_lib.load().ct_repair_enum(self._h, _ptr(rows), n, metric, seed, generation, _ptr(who),
                                              _ptr(pos_q16), max_lookups, _ptr(out_rows), _ptr(out_pos),
                                              ctypes.cast(st, ctypes.c_void_p), _stream()))
        return out_rows, out_pos, {"settled": int(st[0]), "lookups": int(st[1])}

    def repair_noalloc(self, rows, metric: int, seed: int = 0, generation: int = 0, who=None, pos_q16=None,
                       out_rows=None, out_pos=None):
        """ct_repair_noalloc: ct_repair on the library's static scratch (at most CT_NOALLOC_MAX_ROWS rows);
        out_rows / out_pos must be given (this call allocates nothing)."""
        torch = _torch()
        self._rows_arg(rows)
        n = rows.shape[0]
        if who is not None:
            _device_arg(who, "who", (torch.int32,), (n,))
        if pos_q16 is not None:
            _device_arg(pos_q16, "pos_q16", (torch.int32,), (n, self.D))
        self._rows_arg(out_rows, "out_rows")
        _device_arg(out_pos, "out_pos", (torch.int32,), (n,))
        _lib.check(_lib.load().ct_repair_noalloc(self._h, _ptr(rows), n, metric, seed, generation, _ptr(who),
                                                 _ptr(pos_q16), _ptr(out_rows), _ptr(out_pos), _stream()))
        return out_rows, out_pos

    def close(self):
        if self._h:
            _lib.load().ct_space_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(algo: int, pop_size: int, seed: int, **kw) -> ct_pop_params:
    p = ct_pop_params()
    p.algo, p.pop_size, p.seed = algo, pop_size, seed
    p.F_q16, p.CR_q32, p.de_method = kw.get("F_q16", 45875), kw.get("CR_q32", 2576980378), kw.get("de_method", 1)
    p.w_q16, p.c1_q16, p.c2_q16 = kw.get("w_q16", 32768), kw.get("c1_q16", 196608), kw.get("c2_q16", 32768)
    p.mutation_chance, p.beta_b = kw.get("mutation_chance", 5), kw.get("beta_b", 3)
    p.ff_B0_q16, p.ff_gamma_q16 = kw.get("ff_B0_q16", 65536), kw.get("ff_gamma_q16", 65536)
    p.ff_alpha_q16 = kw.get("ff_alpha_q16", 13107)
    p.de_crossover, p.ga_crossover = kw.get("de_crossover", 0), kw.get("ga_crossover", 0)
    p.unaware = kw.get("unaware", 0)
    return p


def opt_kwargs(opt) -> Dict[str, int]:
    """The hyperparameters of a workloads.OptParams as make_params keywords."""
    return dict(F_q16=opt.F_q16, CR_q32=opt.CR_q32, de_method=opt.de_method, w_q16=opt.w_q16, c1_q16=opt.c1_q16,
                c2_q16=opt.c2_q16, mutation_chance=opt.mutation_chance, beta_b=opt.beta_b,
                ff_B0_q16=opt.ff_B0_q16, ff_gamma_q16=opt.ff_gamma_q16, ff_alpha_q16=opt.ff_alpha_q16,
                de_crossover=opt.de_crossover, ga_crossover=opt.ga_crossover, unaware=opt.unaware)


class Pop:
    """One optimiser run (ct_pop) over a Space; the objective tensor must outlive it."""

    def __init__(self, space: Space, algo: int, pop_size: int, seed: int, objective, **kw):
        torch = _torch()
        _device_arg(objective, "objective", (torch.float32,), (space.n_valid,))
        self.space = space
        self.objective = objective
        self.algo, self.pop_size = algo, pop_size
        self.params = make_params(algo, pop_size, seed, **kw)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().ct_pop_create(space.handle, ctypes.byref(self.params), _ptr(objective), _stream(),
                                             ctypes.byref(self._h)))

    @classmethod
    def from_opt(cls, space: Space, opt, objective) -> "Pop":
        """From a workloads.OptParams."""
        return cls(space, opt.algo, opt.pop_size, opt.seed, objective, **opt_kwargs(opt))

    @property
    def handle(self):
        return self._h

    def step(self, n_generations: int = 1, flags: int = CT_STEP_PLAIN):
        step_many([self], n_generations, flags)

    def read(self) -> Dict[str, object]:
        pos = np.zeros(self.pop_size, dtype=np.uint32)
        f = np.zeros(self.pop_size, dtype=np.float32)
        bp, bf, g, r = ctypes.c_uint32(), ctypes.c_float(), ctypes.c_uint32(), ctypes.c_uint32()
        _lib.check(_lib.load().ct_pop_read(self._h, pos.ctypes.data, f.ctypes.data, ctypes.byref(bp),
                                           ctypes.byref(bf), ctypes.byref(g), ctypes.byref(r)))
        return {"pos": pos, "f": f, "best_pos": int(bp.value), "best_f": np.float32(bf.value),
                "generation": int(g.value), "reinits": int(r.value)}

    def evaluated(self) -> np.ndarray:
        """Valid-list positions the last generation evaluated (0xFFFFFFFF: invalid, non-aware)."""
        pos = np.zeros(self.pop_size, dtype=np.uint32)
        _lib.check(_lib.load().ct_pop_evaluated(self._h, pos.ctypes.data))
        return pos

    def best(self):
        """(position, objective) of the best configuration evaluated so far (synchronises)."""
        bp, bf = ctypes.c_uint32(), ctypes.c_float()
        _lib.check(_lib.load().ct_pop_read(self._h, None, None, ctypes.byref(bp), ctypes.byref(bf), None, None))
        return int(bp.value), float(np.float32(bf.value))

    def counters(self) -> Dict[str, int]:
        r, m = ctypes.c_uint64(), ctypes.c_uint64()
        _lib.check(_lib.load().ct_pop_counters(self._h, ctypes.byref(r), ctypes.byref(m)))
        return {"repairs": int(r.value), "mutations": int(m.value)}

    def footprint(self) -> int:
        """Device bytes the run holds (ct_pop_footprint)."""
        b = ctypes.c_uint64()
        _lib.check(_lib.load().ct_pop_footprint(self._h, ctypes.byref(b)))
        return int(b.value)

    def snapshot(self) -> bytes:
        L = _lib.load()
        n = ctypes.c_size_t(0)
        _lib.check(L.ct_pop_snapshot(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _lib.check(L.ct_pop_snapshot(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def restore(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _lib.check(_lib.load().ct_pop_restore(self._h, buf, len(blob)))

    def close(self):
        if self._h:
            _lib.load().ct_pop_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A fixed group of runs advanced together (ct_batch): one launch per phase for all of them;
    with CT_STEP_GRAPH one generation is captured into a hipGraph once and replayed."""

    def __init__(self, pops: List[Pop], lanes: Optional[int] = None):
        """lanes: sub-batches stepped on streams of their own (None: the library's choice,
        ct_batch_create; else ct_batch_create_lanes)."""
        self.pops = list(pops)
        arr = (ctypes.c_void_p * max(1, len(self.pops)))(*[p.handle for p in self.pops])
        self._h = ctypes.c_void_p()
        if lanes is None:
            _lib.check(_lib.load().ct_batch_create(arr, len(self.pops), ctypes.byref(self._h)))
        else:
            _lib.check(_lib.load().ct_batch_create_lanes(arr, len(self.pops), int(lanes), ctypes.byref(self._h)))

    def step(self, n_generations: int = 1, flags: int = CT_STEP_GRAPH):
        _lib.check(_lib.load().ct_batch_step(self._h, n_generations, flags, _stream()))

    def autotune(self, n_generations: int = 1, sample_every: int = 1, force: bool = False):
        """n_generations generations, every sample_every-th of which also times the repair scans'
        candidate work partitionings; the best total is kept (ct_batch_autotune)."""
        _lib.check(_lib.load().ct_batch_autotune(self._h, n_generations, sample_every, 1 if force else 0,
                                                 _stream()))

    def set_tuning(self, items: int, min_boxes: int, grid_waves: int, mode: int = 0):
        """Install a scan partitioning; mode is one of CT_SCAN_* (ct_batch_set_tuning)."""
        _lib.check(_lib.load().ct_batch_set_tuning(self._h, items, min_boxes, grid_waves, mode))

    def tuning(self) -> Dict[str, int]:
        v = [ctypes.c_uint32() for _ in range(5)]
        _lib.check(_lib.load().ct_batch_tuning(self._h, *[ctypes.byref(x) for x in v]))
        return {"items": v[0].value, "min_boxes": v[1].value, "grid_waves": v[2].value,
                "mode": v[3].value, "tuned": bool(v[4].value)}

    def close(self):
        if self._h:
            _lib.load().ct_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """ct_server: runs arriving over time, admitted by device footprint into one continuously
    re-formed batch.  `objective(run_id, n_valid)` returns the float32 objective table of an
    admitted run (called from inside step())."""

    def __init__(self, objective, hbm_budget: int, max_active: int = 1024, max_admit_per_step: int = 0,
                 keep_snapshots: bool = False):
        self._objective = objective
        self._errors: List[BaseException] = []

        def fill(ctx, run_id, n_valid, h_out):
            try:
                v = np.ascontiguousarray(self._objective(int(run_id), int(n_valid)), dtype=np.float32)
                if v.shape != (int(n_valid),):
                    raise ValueError(f"objective table of run {run_id} has shape {v.shape}, expected ({n_valid},)")
                ctypes.memmove(h_out, v.ctypes.data, v.nbytes)
                return 0
            except BaseException as e:  # reported by step()
                self._errors.append(e)
                return 1

        self._cb = _lib.ct_objective_fn(fill)
        cfg = _lib.ct_server_config(hbm_budget=int(hbm_budget), max_active=int(max_active),
                                    max_admit_per_step=int(max_admit_per_step),
                                    keep_snapshots=1 if keep_snapshots else 0, objective=self._cb)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().ct_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def submit(self, spec, opt, n_generations: int, arrival_s: float = -1.0) -> int:
        values = list(spec.params.values())
        code, offs = compile_constraints(spec.names, values, spec.constraints)
        flat = np.ascontiguousarray([int(x) for v in values for x in v], dtype=np.int64)
        rad = np.ascontiguousarray([len(v) for v in values], dtype=np.uint32)
        code = code if len(code) else np.zeros(1, dtype=np.uint32)
        prm = make_params(opt.algo, opt.pop_size, opt.seed, **opt_kwargs(opt))
        rid = ctypes.c_uint64()
        _lib.check(_lib.load().ct_server_submit(self._h, flat.ctypes.data, rad.ctypes.data, len(values),
                                                code.ctypes.data, offs.ctypes.data, len(spec.constraints),
                                                ctypes.byref(prm), int(n_generations), float(arrival_s),
                                                ctypes.byref(rid)))
        return int(rid.value)

    def step(self) -> int:
        """One server step; returns the number of active + queued runs."""
        busy = ctypes.c_uint32()
        _lib.check(_lib.load().ct_server_step(self._h, ctypes.byref(busy)))
        if self._errors:
            raise self._errors.pop(0)
        return int(busy.value)

    def now(self) -> float:
        return float(_lib.load().ct_server_now(self._h))

    def poll(self) -> List[Dict[str, object]]:
        out = []
        buf = (_lib.ct_run_result * 256)()
        while True:
            n = ctypes.c_uint32()
            _lib.check(_lib.load().ct_server_poll(self._h, buf, 256, ctypes.byref(n)))
            for k in range(n.value):
                r = buf[k]
                out.append({f: getattr(r, f) for f, _ in _lib.ct_run_result._fields_})
            if n.value < 256:
                return out

    def snapshot(self, run_id: int) -> bytes:
        L = _lib.load()
        n = ctypes.c_size_t(0)
        _lib.check(L.ct_server_snapshot(self._h, run_id, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _lib.check(L.ct_server_snapshot(self._h, run_id, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def release(self, run_id: int):
        _lib.check(_lib.load().ct_server_release(self._h, run_id))

    def stats(self) -> Dict[str, int]:
        c = _lib.ct_server_counters()
        _lib.check(_lib.load().ct_server_stats(self._h, ctypes.byref(c)))
        return {f: int(getattr(c, f)) for f, _ in _lib.ct_server_counters._fields_}

    def step_times(self):
        """(interval ms float32 [n], runs advanced uint32 [n]) of every step that followed another."""
        L = _lib.load()
        n = ctypes.c_uint64()
        _lib.check(L.ct_server_step_times(self._h, None, None, 0, ctypes.byref(n)))
        ms = np.zeros(n.value, dtype=np.float32)
        act = np.zeros(n.value, dtype=np.uint32)
        _lib.check(L.ct_server_step_times(self._h, ms.ctypes.data, act.ctypes.data, n.value, ctypes.byref(n)))
        return ms[: n.value], act[: n.value]

    def close(self):
        if self._h:
            _lib.load().ct_server_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prof_enable(on: bool = True):
    """Kernel timing with HIP events (measurement support)."""
    _lib.check(_lib.load().ct_prof_enable(1 if on else 0))


def prof_select(kernel: Optional[str]):
    """Record events only around the named kernel's launches (None: all kernels)."""
    _lib.check(_lib.load().ct_prof_select(kernel.encode() if kernel else None))


def prof_sample(every: int = 1):
    """Record events only around every `every`-th launch of each kernel (ct_prof_sample)."""
    _lib.check(_lib.load().ct_prof_sample(int(every)))


def prof_read(kernel: str):
    """(total milliseconds, launches) of a kernel's base name since prof_enable."""
    t, n = ctypes.c_double(), ctypes.c_uint64()
    _lib.check(_lib.load().ct_prof_read(kernel.encode(), ctypes.byref(t), ctypes.byref(n)))
    return float(t.value), int(n.value)


def prof_seen(kernel: str) -> int:
    """Launches of a kernel's base name since prof_enable, recorded or not (ct_prof_seen)."""
    n = ctypes.c_uint64()
    _lib.check(_lib.load().ct_prof_seen(kernel.encode(), ctypes.byref(n)))
    return int(n.value)


def prof_count_boxes(on: bool = True):
    """Count the boxes and chunks the repair scans open (measurement support; clears the counters)."""
    _lib.check(_lib.load().ct_prof_count_boxes(1 if on else 0))


def prof_boxes() -> List[int]:
    """[main-pass boxes, main-pass chunks, fallback boxes, fallback chunks] since prof_count_boxes(True)."""
    out = np.zeros(4, dtype=np.uint64)
    _lib.check(_lib.load().ct_prof_boxes(out.ctypes.data))
    return [int(x) for x in out]


def step_many(pops: List[Pop], n_generations: int = 1, flags: int = CT_STEP_PLAIN):
    """ct_step over several runs (possibly of different spaces)."""
    arr = (ctypes.c_void_p * max(1, len(pops)))(*[p.handle for p in pops])
    _lib.check(_lib.load().ct_step(arr, len(pops), n_generations, flags, _stream()))
