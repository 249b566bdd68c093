"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle.  Only tests/, the smoke check
and the bench's cpu_baseline leg may import it.

Published definition restated: a 256-bit counter (c0, c1, c2, c3) and a 128-bit
key (k0, k1) go through ten rounds.  One round multiplies c0 and c2 by the
two Philox multipliers, keeping both halves of each 128-bit product, and
outputs (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
Between rounds the key is advanced by the two Weyl constants.

Draw map used by the trajectory algorithm (identical on the GPU):
    key     = (seed, instance_id)
    counter = (trajectory_id, draw >> 2, 0, 0); the draw uses word draw & 3
    u       = ((x >> 12) + 0.5) * 2^-52, exact in binary64 and strictly inside (0, 1)
Pinned against numpy's independent Philox implementation in tests.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1

_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """(hi, lo) 64-bit halves of the 128-bit product a*b, vectorised over b (uint64)."""
    b = b.astype(np.uint64)
    a_lo = np.uint64(a & 0xFFFFFFFF)
    a_hi = np.uint64(a >> 32)
    b_lo = b & _U32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _U32) + (hl & _U32)
    lo = (ll & _U32) | ((mid & _U32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply Philox4x64-10.  ctr: 4 uint64 arrays (broadcastable), key: 2 python ints.

    Returns a list of four uint64 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return [c0, c1, c2, c3]


def uniform_from_word(x: np.ndarray) -> np.ndarray:
    """Map a raw 64-bit word to a double strictly inside (0, 1)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def draw(seed: int, instance_id: int, traj, idx) -> np.ndarray:
    """Uniform draw number `idx` of trajectory `traj` (both broadcastable integer arrays)."""
    traj = np.asarray(traj, dtype=np.uint64)
    idx = np.asarray(idx, dtype=np.uint64)
    traj, idx = np.broadcast_arrays(traj, idx)
    zero = np.zeros_like(traj)
    words = philox4x64_10((traj, idx >> np.uint64(2), zero, zero), (seed, instance_id))
    sel = (idx & np.uint64(3)).astype(np.int64)
    out = np.choose(sel, words)
    return uniform_from_word(out)


def draw_scalar(seed: int, instance_id: int, traj: int, idx: int) -> float:
    """Same as draw() for one (trajectory, draw) pair, with Python integers."""
    c0, c1, c2, c3 = int(traj) & MASK64, (int(idx) >> 2) & MASK64, 0, 0
    k0, k1 = int(seed) & MASK64, int(instance_id) & MASK64
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & MASK64, (p0 >> 64) ^ c3 ^ k1, p0 & MASK64
    x = (c0, c1, c2, c3)[int(idx) & 3]
    return ((x >> 12) + 0.5) * 2.0 ** -52
