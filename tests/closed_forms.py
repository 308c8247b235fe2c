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


def dn_front_coded_runs(s, run, k: int, pdms: bool):
    """k sorted front-coded runs of the D/N strings ``s`` (torch, on their
    device), string i going to run ``run[i]``: order within a run by pi, the
    LCP entry from the common base-26 digits above, 0 at each run's start;
    d = the string length, or in the PDMS variant the smallest 8 * 2^t >= F + k
    for every string (F + k is the distinguishing prefix wherever a neighbour
    shares k - 1 digits, i.e. everywhere but possibly at the last position;
    any d at least the distinguishing prefix gives the same merge).
    Returns run_off (int64[k+1]), e, d, ids (int32[n]), suf_off (int64[n+1])
    and suf (uint8), the arrays of the merge's input."""
    import torch
    dev = s.bytes.device
    n, length = s.n, s.meta["length"]
    K, F = s.meta["k"], s.meta["filler"]
    pi = s.meta["pi"].to(dev)
    ids = torch.sort(run.to(torch.int64) * (1 << 32) + pi).indices   # runs in order, each sorted by pi
    run_off = torch.zeros(k + 1, dtype=torch.int64, device=dev)
    run_off[1:] = torch.cumsum(torch.bincount(run.to(torch.int64), minlength=k), 0)
    pv = pi[ids]
    a, c = pv[:-1], pv[1:]
    common = torch.zeros(max(n - 1, 0), dtype=torch.int64, device=dev)
    alive = torch.ones(max(n - 1, 0), dtype=torch.bool, device=dev)
    for dgt in range(K):
        p = 26 ** (K - 1 - dgt)
        alive &= (a // p) % 26 == (c // p) % 26
        common += alive
    del a, c, alive
    e = torch.zeros(n, dtype=torch.int64, device=dev)
    e[1:] = F + common
    del common
    e[run_off[:-1][run_off[:-1] < n]] = 0
    dist = F + K
    dlen = min(length, 8 * 2 ** int(np.ceil(np.log2(dist / 8)))) if pdms else length
    d = torch.full((n,), dlen, dtype=torch.int64, device=dev)
    lit = d - e
    suf_off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    suf_off[1:] = torch.cumsum(lit, 0)
    suf = torch.empty(int(suf_off[-1]), dtype=torch.uint8, device=dev)
    step = 1 << 22
    for q0 in range(0, n, step):
        q1 = min(n, q0 + step)
        L = lit[q0:q1]
        pos = torch.repeat_interleave(torch.arange(q0, q1, device=dev), L)
        t = torch.arange(int(suf_off[q0]), int(suf_off[q1]), device=dev) - suf_off[pos]
        suf[int(suf_off[q0]):int(suf_off[q1])] = s.bytes[ids[pos] * length + e[pos] + t]
    i32 = lambda x: x.to(torch.int32)
    return run_off, i32(e), i32(d), i32(ids), suf_off, suf
