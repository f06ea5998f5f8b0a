"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_goldens.py [sparse16]

sparse16_space.json: the full oracle enumeration of the 4,353,564,672-configuration
sparse space (about 90 s on 8 cores): |V|, digests of the ascending valid list
(sum and sum of squares of the linear indices mod 2^64, popcount of every 2^28-index
chunk of the bitmask) and every 9973rd list entry with its position.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import core  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


def digests(vlin: np.ndarray):
    s = int(np.sum(vlin, dtype=np.uint64))                      # wraps mod 2^64
    s2 = int(np.sum(vlin * vlin, dtype=np.uint64))
    return s & M64, s2 & M64


def sparse16():
    sp = core.Space.from_spec(W.sparse16())
    n_words = (sp.n_cartesian + 63) // 64
    chunk_words = (1 << 28) // 64
    parts, chunk_counts = [], []
    for w0 in range(0, n_words, chunk_words):
        w1 = min(n_words, w0 + chunk_words)
        words = sp.mask_words(w0, w1)
        chunk_counts.append(int(np.unpackbits(words.view(np.uint8)).sum()))
        parts.append(core.words_to_lin(words, w0))
        print(f"words {w0}..{w1}: {chunk_counts[-1]}", flush=True)
    vlin = np.concatenate(parts)
    s, s2 = digests(vlin)
    step = 9973
    out = {
        "space": "sparse16",
        "n_cartesian": sp.n_cartesian,
        "n_valid": int(len(vlin)),
        "sum_lin_mod64": s,
        "sumsq_lin_mod64": s2,
        "chunk_log2": 28,
        "chunk_counts": chunk_counts,
        "sample_stride": step,
        "sample_pos": list(range(0, len(vlin), step)),
        "sample_lin": [int(x) for x in vlin[::step]],
        "first_lin": int(vlin[0]),
        "last_lin": int(vlin[-1]),
    }
    with open(os.path.join(HERE, "sparse16_space.json"), "w") as f:
        json.dump(out, f)
    print("sparse16", out["n_valid"])


if __name__ == "__main__":
    which = sys.argv[1:] or ["sparse16"]
    if "sparse16" in which:
        sparse16()
