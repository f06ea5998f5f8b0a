"""Shared helpers of the GPU parity tests (loaded only by tests marked gpu)."""
import functools
import struct
import sys

import numpy as np

import workloads as W
from oracle import core as ocore


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@functools.lru_cache(maxsize=None)
def oracle_space(name):
    """The oracle's own enumeration (sparse16 takes about a minute on 16 cores; it prints progress)."""
    return ocore.Space.from_spec(W.space(name)).enumerate(progress=say if name == "sparse16" else None)


def gpu_space(spec):
    from paper_2606_28372_amd import Space
    return Space(spec.names, list(spec.params.values()), spec.constraints)


def rows_to_digits(rows_u8, D):
    return rows_u8[:, :D].astype(np.int32)


def digits_to_rows(sp_gpu, digits):
    return sp_gpu.pack_rows(np.asarray(digits, dtype=np.int64))


def parse_snapshot(blob, algo, P, D):
    h = struct.unpack_from("<8I", blob, 0)
    assert h[0] in (0x43545031, 0x43545531) and h[1] == algo and h[2] == P and h[3] == D
    unaware = h[0] == 0x43545531
    o = 32
    out = {"gen": h[4], "reinits": h[5], "best_pos": h[6], "best_ord": h[7], "unaware": unaware}
    if algo == 1:
        PD = P * D
        out["X"] = np.frombuffer(blob, dtype=np.int32, count=PD, offset=o).reshape(P, D).astype(np.int64); o += PD * 4
        out["V"] = np.frombuffer(blob, dtype=np.int64, count=PD, offset=o).reshape(P, D).copy(); o += PD * 8
        out["PB"] = np.frombuffer(blob, dtype=np.int32, count=PD, offset=o).reshape(P, D).astype(np.int64); o += PD * 4
        out["f_pb"] = np.frombuffer(blob, dtype=np.float32, count=P, offset=o).copy(); o += P * 4
        out["pb_pos"] = np.frombuffer(blob, dtype=np.uint32, count=P, offset=o).astype(np.int64); o += P * 4
        out["g_idx"] = struct.unpack_from("<I", blob, o)[0]
    else:
        out["pos"] = np.frombuffer(blob, dtype=np.uint32, count=P, offset=o).astype(np.int64); o += P * 4
        out["f"] = np.frombuffer(blob, dtype=np.float32, count=P, offset=o).copy(); o += P * 4
        if algo == 3:
            out["X"] = np.frombuffer(blob, dtype=np.int32, count=P * D, offset=o).reshape(P, D).astype(np.int64)
        elif unaware:
            out["rows"] = np.frombuffer(blob, dtype=np.uint8, count=P * D, offset=o).reshape(P, D).astype(np.int32)
    return out
