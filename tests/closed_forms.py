"""Closed forms of the D/N-ratio workload, derived from its construction.

String i of ``synth.dn_strings`` is 'A'*F + code_k(pi(i)) + tail, where code_k
writes pi(i) in k base-26 digits ('A'+digit, most significant first).  The codes
are distinct, so the sorted order is the order of pi(i) and the random tail
never matters:

* sorted position c holds the string with pi(i) = c, i.e. perm = pi^{-1};
* lcp at sorted position c >= 1 is F + (number of equal leading base-26
  digits of c-1 and c);
* dist (Section 2 of the paper, reading R5) at sorted position c is
  min(len, 1 + max(lcp[c], lcp[c+1])) with lcp[n] = 0 -- here computed from
  the digit counts only;
* without hash collisions the prefix-doubling result is
  min(len, l0 * 2^t) for the smallest t with l0 * 2^t >= dist.

Everything here is integer arithmetic on pi; no string is compared.
"""
from __future__ import annotations

import numpy as np


def common_digits(a: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """Equal leading digits of the k-digit base-26 codes of a and b."""
    a = a.astype(np.int64)
    b = b.astype(np.int64)
    out = np.zeros(a.shape, dtype=np.int64)
    alive = np.ones(a.shape, dtype=bool)
    for d in range(k):
        p = 26 ** (k - 1 - d)
        eq = (a // p) % 26 == (b // p) % 26
        alive &= eq
        out += alive
    return out


def dn_perm(pi: np.ndarray) -> np.ndarray:
    n = pi.size
    perm = np.empty(n, dtype=np.uint32)
    perm[pi] = np.arange(n, dtype=np.uint32)
    return perm


def dn_lcp(n: int, k: int, F: int) -> np.ndarray:
    lcp = np.zeros(n, dtype=np.uint32)
    if n > 1:
        c = np.arange(1, n, dtype=np.int64)
        lcp[1:] = F + common_digits(c - 1, c, k)
    return lcp


def dn_dist_sorted(n: int, k: int, F: int, length: int) -> np.ndarray:
    """dist by sorted position."""
    lcp = dn_lcp(n, k, F).astype(np.int64)
    nxt = np.zeros(n, dtype=np.int64)
    nxt[:-1] = lcp[1:]
    return np.minimum(length, 1 + np.maximum(lcp, nxt)).astype(np.uint32)


def doubling_closed_form(dist: np.ndarray, lengths: np.ndarray, l0: int) -> np.ndarray:
    """min(len, l0 * 2^t) for the smallest t >= 0 with l0 * 2^t >= dist."""
    d = dist.astype(np.int64)
    L = np.full(d.shape, l0, dtype=np.int64)
    while True:
        m = L < d
        if not m.any():
            break
        L[m] *= 2
    return np.minimum(L, lengths.astype(np.int64)).astype(np.uint32)


def doubling_rounds_closed_form(dist: np.ndarray, lengths: np.ndarray, l0: int) -> int:
    """Rounds of collision-free prefix doubling (Section 4): a string leaves in
    the first round t (1-based, tested length l0 * 2^(t-1)) whose length covers
    min(len, dist) -- its prefix of that length is then unique among the
    strings still active, or the string is exhausted.  The process runs until
    the last string leaves (0 rounds for no strings)."""
    if dist.size == 0:
        return 0
    need = np.minimum(dist.astype(np.int64), lengths.astype(np.int64))
    t, L = 1, l0
    while (need > L).any():
        t += 1
        L *= 2
    return t
