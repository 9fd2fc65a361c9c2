"""Order-sensitive 64-bit digest of a (position, id) match list.

Test infrastructure: the golden-value script computes it from the oracle's
lists (numpy), the GPU tests from the library's device lists (torch); neither
side's matching code is involved in it.

For the k-th pair (0-based) of a list, key_k = pos_k * 2^32 + id_k and

    h_k = mix(key_k XOR (k * 0x9E3779B97F4A7C15)),
    digest = sum_k h_k  (mod 2^64),

where mix is the SplitMix64 output function (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014; the multipliers of
Stafford's variant 13). Including k makes the digest depend on the order; the
sum lets a list be digested in consecutive pieces (each piece passes the index
of its first pair) and per text in one segmented sum.
"""

from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1


def mix_int(z: int) -> int:
    """Reference mix on Python integers (for tests of the array versions)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def digest_int(pos, ids) -> int:
    """Plain-Python digest (small lists)."""
    s = 0
    for k, (p, i) in enumerate(zip(pos, ids)):
        s = (s + mix_int(((int(p) << 32) | int(i)) ^ ((k * GOLDEN) & MASK64))) & MASK64
    return s


# ---------------------------------------------------------------------------
# numpy (uint64 arithmetic wraps modulo 2^64)
# ---------------------------------------------------------------------------
def _mix_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def hashes_np(pos: np.ndarray, ids: np.ndarray, first_index: int = 0) -> np.ndarray:
    """h_k of the pairs, the first being pair number first_index of its list."""
    with np.errstate(over="ignore"):
        key = (pos.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)
        k = np.arange(first_index, first_index + len(pos), dtype=np.uint64)
        return _mix_np(key ^ (k * np.uint64(GOLDEN)))


def digest_np(pos: np.ndarray, ids: np.ndarray, first_index: int = 0) -> int:
    """Digest (mod 2^64) of a list piece starting at pair first_index."""
    if len(pos) == 0:
        return 0
    return int(hashes_np(pos, ids, first_index).sum(dtype=np.uint64))


# ---------------------------------------------------------------------------
# torch int64 (two's complement: additions and products wrap modulo 2^64;
# right shifts are arithmetic, so a logical shift masks the sign copies off)
# ---------------------------------------------------------------------------
def _s64(x: int) -> int:
    x &= MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def hashes_torch(pairs, first_index: int = 0):
    """h_k (int64 bit patterns) of an int32 [M, 2] (pos, id) tensor."""
    import torch
    p = pairs[:, 0].to(torch.int64) & 0xFFFFFFFF
    i = pairs[:, 1].to(torch.int64) & 0xFFFFFFFF
    k = torch.arange(first_index, first_index + pairs.shape[0], dtype=torch.int64,
                     device=pairs.device)
    z = ((p << 32) | i) ^ (k * _s64(GOLDEN))
    z = (z ^ _lsr(z, 30)) * _s64(M1)
    z = (z ^ _lsr(z, 27)) * _s64(M2)
    return z ^ _lsr(z, 31)


def digest_torch(pairs, piece: int = 1 << 27) -> int:
    """Digest of a whole int32 [M, 2] list (processed in pieces of `piece`
    pairs to bound temporary memory)."""
    import torch
    M = pairs.shape[0]
    s = torch.zeros((), dtype=torch.int64, device=pairs.device)
    for a in range(0, M, piece):
        s = s + hashes_torch(pairs[a:a + piece], a).sum()
    return int(s.item()) & MASK64


def segment_digests_torch(pairs, starts, counts):
    """Per-segment digests: segment j is pairs[starts[j] : starts[j] + counts[j]]
    (int64 tensors on the pairs' device), each digested as a list of its own."""
    import torch
    R = starts.numel()
    out = torch.zeros(R, dtype=torch.int64, device=pairs.device)
    total = int(counts.sum().item())
    if total == 0:
        return [0] * R
    seg = torch.repeat_interleave(torch.arange(R, device=pairs.device), counts)
    first = torch.repeat_interleave(starts, counts)
    rows = first + (torch.arange(total, device=pairs.device) -
                    torch.repeat_interleave(torch.cumsum(counts, 0) - counts, counts))
    sub = pairs[rows]
    # index within the segment
    k = rows - first
    p = sub[:, 0].to(torch.int64) & 0xFFFFFFFF
    i = sub[:, 1].to(torch.int64) & 0xFFFFFFFF
    z = ((p << 32) | i) ^ (k * _s64(GOLDEN))
    z = (z ^ _lsr(z, 30)) * _s64(M1)
    z = (z ^ _lsr(z, 27)) * _s64(M2)
    z = z ^ _lsr(z, 31)
    out.index_add_(0, seg, z)
    return [int(x) & MASK64 for x in out.cpu().tolist()]
