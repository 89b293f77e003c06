"""Helpers for the GPU parity tests: device upload and result normalisation."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dev(a):
    """numpy uint32 -> device int32 tensor with the same bits."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to("cuda")


def sort_rows(t: np.ndarray) -> np.ndarray:
    t = np.asarray(t, dtype=np.uint32).reshape(-1, 3)
    if len(t) == 0:
        return t
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


def packed_sorted(t: np.ndarray, bits: int = 21) -> np.ndarray:
    """Sorted uint64 keys a<<2b | b<<b | c of canonical triangles (ids < 2^bits)."""
    t = np.asarray(t, dtype=np.uint64).reshape(-1, 3)
    k = (t[:, 0] << np.uint64(2 * bits)) | (t[:, 1] << np.uint64(bits)) | t[:, 2]
    k.sort()
    return k


def edge_fingerprint(src, dst) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(src, np.uint32).tobytes())
    h.update(np.ascontiguousarray(dst, np.uint32).tobytes())
    return h.hexdigest()[:32]


def load_expected():
    with open(os.path.join(GOLDEN, "oracle_expected.json")) as f:
        return json.load(f)
