"""ctypes wrapper around the CPU oracle (``oracle.c``) -- test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this package.  The GPU product path never imports it.
All arrays are host numpy arrays; results are returned as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.or_sort.argtypes = [P, P, U64, P]; L.or_sort.restype = I32
        L.or_lcp.argtypes = [P, P, U64, P, P]; L.or_lcp.restype = None
        L.or_dist_exact.argtypes = [P, U64, P, P, P]; L.or_dist_exact.restype = None
        L.or_dist_bruteforce.argtypes = [P, P, U64, P]; L.or_dist_bruteforce.restype = None
        L.or_kr_key.argtypes = [P, U64]; L.or_kr_key.restype = U64
        L.or_dist_prefix.argtypes = [P, P, U64, U32, U32, P, P, P]; L.or_dist_prefix.restype = I32
        L.or_select_splitters.argtypes = [U64, P, U32, P]; L.or_select_splitters.restype = I32
        L.or_select_splitters_chars.argtypes = [U64, P, P, P, U32, P]
        L.or_select_splitters_chars.restype = I32
        L.or_bucket_bounds.argtypes = [P, P, U64, P, P, P, U32, P]; L.or_bucket_bounds.restype = None
        L.or_fc_encode.argtypes = [P, P, U64, P, P, P, P, U32, P, P, P, P, P]
        L.or_fc_encode.restype = ctypes.c_int64
        L.or_fc_decode.argtypes = [U32, P, P, P, P, P, U64, P, P]; L.or_fc_decode.restype = None
        L.or_merge.argtypes = [U32, P, P, P, P, P, P, U64, P, P, P]; L.or_merge.restype = I32
        L.or_check_sorted.argtypes = [P, P, U64, P, P]; L.or_check_sorted.restype = ctypes.c_int64
        L.or_suffix_sort.argtypes = [P, U64, P, P]; L.or_suffix_sort.restype = I32
        L.or_check_suffixes.argtypes = [P, U64, P, P]; L.or_check_suffixes.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _host(bytes_, offsets):
    b = np.ascontiguousarray(np.asarray(bytes_, dtype=np.uint8))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if b.size == 0:
        b = np.zeros(1, dtype=np.uint8)
    return b, o


def strings_np(s):
    """(bytes, offsets) numpy views of a ``synth.StringSet`` (copied to host)."""
    return _host(s.bytes.cpu().numpy(), s.offsets.cpu().numpy().view(np.uint64))


def sort(bytes_, offsets) -> np.ndarray:
    b, o = _host(bytes_, offsets)
    n = o.size - 1
    perm = np.empty(max(n, 1), dtype=np.uint32)
    if lib().or_sort(_p(b), _p(o), n, _p(perm)) != 0:
        raise MemoryError("oracle sort")
    return perm[:n]


def lcp(bytes_, offsets, perm) -> np.ndarray:
    """LCP array of the order ``perm`` (its values index ``offsets``)."""
    b, o = _host(bytes_, offsets)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    n = perm.size
    out = np.empty(max(n, 1), dtype=np.uint32)
    lib().or_lcp(_p(b), _p(o), n, _p(perm), _p(out))
    return out[:n]


def dist_exact(offsets, perm, lcp_) -> np.ndarray:
    o = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = o.size - 1
    out = np.empty(max(n, 1), dtype=np.uint32)
    lib().or_dist_exact(_p(o), n, _p(np.ascontiguousarray(perm, dtype=np.uint32)),
                        _p(np.ascontiguousarray(lcp_, dtype=np.uint32)), _p(out))
    return out[:n]


def dist_bruteforce(bytes_, offsets) -> np.ndarray:
    b, o = _host(bytes_, offsets)
    n = o.size - 1
    out = np.empty(max(n, 1), dtype=np.uint32)
    lib().or_dist_bruteforce(_p(b), _p(o), n, _p(out))
    return out[:n]


def kr_key(data: bytes, m: int | None = None) -> int:
    a = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8).copy()
    return int(lib().or_kr_key(_p(a), len(data) if m is None else m))


def dist_prefix(bytes_, offsets, init_len=8, hash_bits=64):
    """Returns (dist_approx by input index, rounds, collisions)."""
    b, o = _host(bytes_, offsets)
    n = o.size - 1
    out = np.empty(max(n, 1), dtype=np.uint32)
    rounds = ctypes.c_uint32(0)
    coll = ctypes.c_uint64(0)
    rc = lib().or_dist_prefix(_p(b), _p(o), n, init_len, hash_bits, _p(out),
                              ctypes.byref(rounds), ctypes.byref(coll))
    if rc != 0:
        raise ValueError(f"oracle dist_prefix rc={rc}")
    return out[:n], int(rounds.value), int(coll.value)


def select_splitters(n, perm, r) -> np.ndarray:
    ids = np.empty(max(r - 1, 1), dtype=np.uint32)
    if lib().or_select_splitters(n, _p(np.ascontiguousarray(perm, dtype=np.uint32)), r, _p(ids)) != 0:
        raise ValueError("select_splitters")
    return ids[:r - 1]


def select_splitters_chars(perm, offsets, r, weights=None) -> np.ndarray:
    """Character-based regular sampling of one sorted array (r - 1 samples)."""
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    o = np.ascontiguousarray(offsets, dtype=np.uint64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
    ids = np.empty(max(r - 1, 1), dtype=np.uint32)
    if lib().or_select_splitters_chars(perm.size, _p(perm), _p(o), _p(w), r, _p(ids)) != 0:
        raise ValueError("select_splitters_chars")
    return ids[:r - 1]


def bucket_bounds(bytes_, offsets, perm, spl_bytes, spl_offsets) -> np.ndarray:
    b, o = _host(bytes_, offsets)
    sb, so = _host(spl_bytes, spl_offsets)
    n = len(perm)
    r = so.size  # r-1 splitters -> r buckets
    out = np.empty(r + 1, dtype=np.uint64)
    lib().or_bucket_bounds(_p(b), _p(o), n, _p(np.ascontiguousarray(perm, dtype=np.uint32)),
                           _p(sb), _p(so), r, _p(out))
    return out


def fc_encode(bytes_, offsets, perm, lcp_, dist, bounds):
    """Returns dict(lcp, len, id, suf_off, suf)."""
    b, o = _host(bytes_, offsets)
    n = len(perm)
    r = len(bounds) - 1
    bounds = np.ascontiguousarray(bounds, dtype=np.uint64)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp_ = np.ascontiguousarray(lcp_, dtype=np.uint32)
    dist = None if dist is None else np.ascontiguousarray(dist, dtype=np.uint32)
    fl = np.empty(max(n, 1), np.uint32); fd = np.empty(max(n, 1), np.uint32)
    fi = np.empty(max(n, 1), np.uint32); so = np.empty(n + 1, np.uint64)
    cap = int(b.size) + 1
    suf = np.empty(cap, np.uint8)
    tot = lib().or_fc_encode(_p(b), _p(o), n, _p(perm), _p(lcp_), _p(dist), _p(bounds), r,
                             _p(fl), _p(fd), _p(fi), _p(so), _p(suf))
    if tot < 0:
        raise ValueError("fc_encode: e > d")
    return dict(lcp=fl[:n], len=fd[:n], id=fi[:n], suf_off=so, suf=suf[:tot], run_off=bounds)


def fc_decode(run_off, fc_lcp, fc_len, suf_off, suf):
    run_off = np.ascontiguousarray(run_off, dtype=np.uint64)
    fc_lcp = np.ascontiguousarray(fc_lcp, dtype=np.uint32)
    fc_len = np.ascontiguousarray(fc_len, dtype=np.uint32)
    suf_off = np.ascontiguousarray(suf_off, dtype=np.uint64)
    suf = np.ascontiguousarray(suf, dtype=np.uint8)
    if suf.size == 0:
        suf = np.zeros(1, np.uint8)
    n = fc_lcp.size
    out_off = np.empty(n + 1, np.uint64)
    out = np.empty(int(fc_len.astype(np.uint64).sum()) + 1, np.uint8)
    lib().or_fc_decode(len(run_off) - 1, _p(run_off), _p(fc_lcp), _p(fc_len), _p(suf_off), _p(suf), n,
                       _p(out_off), _p(out))
    return out[:int(out_off[-1])], out_off


def merge(run_off, fc_lcp, fc_len, fc_id, suf_off, suf):
    """Returns (src u64, id u32, lcp u32)."""
    run_off = np.ascontiguousarray(run_off, dtype=np.uint64)
    n = int(run_off[-1])
    arrs = [np.ascontiguousarray(a, dtype=t) for a, t in
            ((fc_lcp, np.uint32), (fc_len, np.uint32), (fc_id, np.uint32), (suf_off, np.uint64))]
    suf = np.ascontiguousarray(suf, dtype=np.uint8)
    if suf.size == 0:
        suf = np.zeros(1, np.uint8)
    src = np.empty(max(n, 1), np.uint64); idv = np.empty(max(n, 1), np.uint32)
    lc = np.empty(max(n, 1), np.uint32)
    rc = lib().or_merge(len(run_off) - 1, _p(run_off), _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]),
                        _p(suf), n, _p(src), _p(idv), _p(lc))
    if rc != 0:
        raise MemoryError("oracle merge")
    return src[:n], idv[:n], lc[:n]


def check_sorted(bytes_, offsets, perm, lcp_=None) -> int:
    """-1 if perm is the stable sorted order (and lcp, if given, is exact)."""
    b, o = _host(bytes_, offsets)
    n = o.size - 1
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lc = None if lcp_ is None else np.ascontiguousarray(lcp_, dtype=np.uint32)
    return int(lib().or_check_sorted(_p(b), _p(o), n, _p(perm), _p(lc)))


def suffix_sort(text) -> tuple[np.ndarray, np.ndarray]:
    """Suffix array and LCP array of one text (numpy uint8)."""
    t = np.ascontiguousarray(np.asarray(text, dtype=np.uint8))
    N = t.size
    if N == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    sa = np.empty(N, np.uint32)
    lc = np.empty(N, np.uint32)
    lib().or_suffix_sort(_p(t), N, _p(sa), _p(lc))
    return sa, lc


def check_suffixes(text, sa, lcp_=None) -> int:
    """-1 if sa is the suffix array of text (and lcp, if given, exact)."""
    t = np.ascontiguousarray(np.asarray(text, dtype=np.uint8))
    sa = np.ascontiguousarray(sa, dtype=np.uint32)
    lc = None if lcp_ is None else np.ascontiguousarray(lcp_, dtype=np.uint32)
    return int(lib().or_check_suffixes(_p(t), t.size, _p(sa), _p(lc)))
