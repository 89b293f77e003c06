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


# ------------------------------------------------ on-device result checks

MASK64 = (1 << 64) - 1
# splitmix64's output-function constants as signed 64-bit values (torch has
# no unsigned 64-bit arithmetic; multiplication and addition wrap modulo 2^64)
_SM_C1 = 0xBF58476D1CE4E5B9 - (1 << 64)
_SM_C2 = 0x94D049BB133111EB - (1 << 64)


def _srl(z, k):
    """Logical right shift of int64 tensors holding uint64 bits."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix(z):
    z = (z ^ _srl(z, 30)) * _SM_C1
    z = (z ^ _srl(z, 27)) * _SM_C2
    return z ^ _srl(z, 31)


def digest_sum_torch(tri) -> int:
    """Wrapping 64-bit sum over the rows (a, b, c) of an int32 tensor (k, 3)
    of canonical triangles of h(a,b,c) = f(f((a << 32) | b) + c), f the
    splitmix64 output function (the library's digest convention), computed
    with torch integer ops on the tensor's device."""
    import torch
    if tri.shape[0] == 0:
        return 0
    t = tri.to(torch.int64) & 0xFFFFFFFF
    h = _mix(_mix((t[:, 0] << 32) | t[:, 1]) + t[:, 2])
    return int(h.sum().item()) & MASK64


def sorted_rows_device(tri, bits: int):
    """The rows (a, b, c) of an int32 tensor (k, 3) of ids below 2^bits in
    ascending lexicographic order, sorted on the tensor's device."""
    import torch
    t = tri.to(torch.int64) & 0xFFFFFFFF
    if 3 * bits <= 63:
        key = (t[:, 0] << (2 * bits)) | (t[:, 1] << bits) | t[:, 2]
        key, _ = torch.sort(key)
        m = (1 << bits) - 1
        return torch.stack([key >> (2 * bits), (key >> bits) & m, key & m], 1).to(torch.int32)
    # stable passes from the last column to the first
    for col in (2, 1, 0):
        _, o = torch.sort(t[:, col], stable=True)
        t = t[o]
    return t.to(torch.int32)


def sorted_sha256_device(tri, bits: int) -> str:
    """SHA-256 of the rows sorted as sorted_rows_device, as little-endian
    uint32 triples (the stored oracle digests' layout)."""
    s = sorted_rows_device(tri, bits).cpu().numpy().view(np.uint32)
    return hashlib.sha256(np.ascontiguousarray(s).astype("<u4").tobytes()).hexdigest()
