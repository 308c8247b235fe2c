"""Seeded synthetic string workloads shaped like the paper's inputs.

This module only draws inputs.  It holds none of the sorting method's
arithmetic: no comparison, LCP, hashing of prefixes, bucketing or coding.
Both the CPU oracle tests and the GPU path take their inputs from here.

Every random quantity comes from a counter-based generator (the SplitMix64
finaliser of Steele, Lea and Flood, 2014) evaluated on (stream, index)
counters, so any subset can be regenerated on its own and the CPU and GPU
produce the same bytes.  Only the permutation of the D/N generator is drawn
with ``torch.randperm`` on the CPU (seeded) and then moved to the device.

Workloads (all byte strings, ``bytes`` u8 + ``offsets`` int64[n+1]):

* ``dn_strings``   -- fixed-length strings with a chosen D/N ratio, the shape of
  the paper's DNData weak-scaling inputs (Section 5): a run of 'A' filler, the
  base-26 code of a random permutation index (most significant digit first),
  then uniform letters.  Sorted order, LCPs and distinguishing prefixes of this
  family have closed forms, which the tests use as pins.
* ``text_strings`` -- variable-length text-like strings: log-normal lengths,
  Zipf-distributed printable bytes and a share of exact duplicates.  It stands
  in for the paper's CommonCrawl / Wikipedia / WikiText sets, which are not
  available here.
* ``random_sets``  -- many independent sets (log-uniform sizes, uniform lengths,
  uniform letters) for batched execution.
* ``poisson_requests`` -- a seeded request trace for the serving loop.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

_MASK64 = (1 << 64) - 1


def _s64(c: int) -> int:
    """Unsigned 64-bit constant -> the int64 with the same bits."""
    c &= _MASK64
    return c - (1 << 64) if c >= (1 << 63) else c


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_M1 = _s64(0xBF58476D1CE4E5B9)
_M2 = _s64(0x94D049BB133111EB)

# stream identifiers (arbitrary distinct constants)
_ST_TAIL = 0x11
_ST_LEN = 0x21
_ST_DUP = 0x31
_ST_DUPJ = 0x32
_ST_BYTE = 0x41
_ST_SETLEN = 0x51
_ST_SETBYTE = 0x52
_ST_RUN = 0x61


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function applied to int64 counters (wrapping arithmetic)."""
    z = x + _GOLDEN
    z = (z ^ _lsr(z, 30)) * _M1
    z = (z ^ _lsr(z, 27)) * _M2
    return z ^ _lsr(z, 31)


def mix64_py(x: int) -> int:
    """Plain-integer twin of :func:`mix64` (unsigned result), for self-checks."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _stream_base(seed: int, stream: int) -> int:
    return _s64(mix64_py(((seed & 0xFFFFFFFF) << 32) ^ (stream << 8) ^ 0x5EED))


def _u32(seed: int, stream: int, ctr: torch.Tensor) -> torch.Tensor:
    """Uniform 32-bit integers (as int64) for the given counters."""
    return _lsr(mix64(ctr + _stream_base(seed, stream)), 32)


@dataclass
class StringSet:
    """A string array: concatenated bytes plus ``offsets`` (n+1 entries)."""

    bytes: torch.Tensor          # uint8 [N]
    offsets: torch.Tensor        # int64 [n+1]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.offsets.numel() - 1

    @property
    def N(self) -> int:
        return self.bytes.numel()

    def to(self, device) -> "StringSet":
        return StringSet(self.bytes.to(device), self.offsets.to(device), dict(self.meta))

    def lengths(self) -> torch.Tensor:
        return self.offsets[1:] - self.offsets[:-1]

    def get(self, i: int) -> bytes:
        o = self.offsets
        return bytes(self.bytes[int(o[i]):int(o[i + 1])].cpu().numpy().tobytes())

    def as_list(self) -> list[bytes]:
        b = self.bytes.cpu().numpy().tobytes()
        o = self.offsets.cpu().tolist()
        return [b[o[i]:o[i + 1]] for i in range(len(o) - 1)]


def from_list(strings: list[bytes], device="cpu") -> StringSet:
    lens = [len(s) for s in strings]
    offs = [0]
    for L in lens:
        offs.append(offs[-1] + L)
    data = b"".join(strings)
    bt = torch.frombuffer(bytearray(data), dtype=torch.uint8) if data else torch.empty(0, dtype=torch.uint8)
    return StringSet(bt.clone().to(device), torch.tensor(offs, dtype=torch.int64, device=device))


def concat(sets: list[StringSet]) -> tuple[StringSet, torch.Tensor]:
    """Concatenate string sets; returns the union and the set boundaries (string index, B+1)."""
    bts, offs, bounds = [], [], [0]
    base = 0
    for s in sets:
        bts.append(s.bytes)
        offs.append(s.offsets[:-1] + base)
        base += s.N
        bounds.append(bounds[-1] + s.n)
    dev = sets[0].bytes.device if sets else "cpu"
    offs.append(torch.tensor([base], dtype=torch.int64, device=dev))
    return (StringSet(torch.cat(bts) if bts else torch.empty(0, dtype=torch.uint8, device=dev), torch.cat(offs)),
            torch.tensor(bounds, dtype=torch.int64))


# ---------------------------------------------------------------------------
# D/N-ratio strings (the paper's DNData shape)
# ---------------------------------------------------------------------------

def dn_digits(n: int) -> int:
    """Number of base-26 digits that encode 0..n-1 (at least 1)."""
    k = 1
    while 26 ** k < n:
        k += 1
    return k


def dn_filler(n: int, length: int, ratio: float) -> int:
    k = dn_digits(n)
    f = max(0, int(math.floor(ratio * length + 0.5)) - k)
    if f + k > length:
        raise ValueError("string length too short for the permutation code")
    return f


def dn_perm(n: int, seed: int) -> torch.Tensor:
    g = torch.Generator().manual_seed(int(seed))
    return torch.randperm(n, generator=g, dtype=torch.int64)


def dn_strings(n: int, length: int, ratio: float, seed: int = 0, device="cpu",
               chunk: int = 1 << 20) -> StringSet:
    """``n`` strings of exactly ``length`` letters 'A'..'Z'.

    String i = 'A' * F, then the k-digit base-26 code of pi(i) written
    'A'+digit, most significant first, then uniform letters, where pi is a
    seeded random permutation of 0..n-1, k = ceil(log26 n) and
    F = max(0, round(ratio*length) - k).  ``meta['pi']`` holds pi (CPU).
    """
    k = dn_digits(max(n, 1))
    F = dn_filler(max(n, 1), length, ratio)
    pi = dn_perm(n, seed)
    out = torch.empty(n * length, dtype=torch.uint8, device=device)
    view = out.view(n, length) if n else out.view(0, length)
    if n:
        view[:, :F] = ord("A")
    T = length - F - k
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        p = pi[c0:c1].to(device)
        for d in range(k):
            view[c0:c1, F + d] = (65 + (p // (26 ** (k - 1 - d))) % 26).to(torch.uint8)
        if T > 0:
            i = torch.arange(c0, c1, dtype=torch.int64, device=device)
            j = torch.arange(T, dtype=torch.int64, device=device)
            ctr = i[:, None] * T + j[None, :]
            view[c0:c1, F + k:] = (65 + _u32(seed, _ST_TAIL, ctr) % 26).to(torch.uint8)
    offsets = torch.arange(n + 1, dtype=torch.int64, device=device) * length
    return StringSet(out, offsets, {"kind": "dn", "n": n, "length": length, "ratio": ratio,
                                    "seed": seed, "k": k, "filler": F, "pi": pi})


# ---------------------------------------------------------------------------
# text-like strings (log-normal lengths, Zipf bytes, exact duplicates)
# ---------------------------------------------------------------------------

def _lognormal_len_thresholds(median: float, sigma: float, max_len: int) -> torch.Tensor:
    # len = clamp(round(exp(ln median + sigma Z)), 1, max_len); P(len <= L) for L = 1..max_len-1
    th = []
    for L in range(1, max_len):
        z = (math.log(L + 0.5) - math.log(median)) / sigma
        cdf = 0.5 * math.erfc(-z / math.sqrt(2.0))
        th.append(min(int(math.floor(cdf * 4294967296.0)), 4294967296))
    return torch.tensor(th, dtype=torch.int64)


def _zipf_thresholds(s: float, ncodes: int) -> torch.Tensor:
    w = [r ** (-s) for r in range(1, ncodes + 1)]
    tot = sum(w)
    acc, th = 0.0, []
    for r in range(ncodes - 1):
        acc += w[r]
        th.append(min(int(math.floor(acc / tot * 4294967296.0)), 4294967296))
    return torch.tensor(th, dtype=torch.int64)


def text_strings(n: int, seed: int = 0, median: float = 40.0, sigma: float = 1.0,
                 max_len: int = 4096, zipf_s: float = 1.1, ncodes: int = 96,
                 first_code: int = 0x20, dup_frac: float = 0.2, device="cpu",
                 chunk_bytes: int = 1 << 26) -> StringSet:
    """Variable-length text-like strings.

    Lengths: round(exp(ln median + sigma Z)) clipped to [1, max_len].
    Bytes: Zipf(zipf_s) over ``ncodes`` codes starting at ``first_code``
    (rank r -> byte first_code + r - 1).  Each string i >= 1 is, with
    probability ``dup_frac``, an exact copy of a uniformly chosen earlier
    string (copies of copies resolve to the original).
    """
    dev = torch.device(device)
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    # duplicates
    is_dup = (_u32(seed, _ST_DUP, idx) < int(math.floor(dup_frac * 4294967296.0))) & (idx >= 1)
    j = _lsr(mix64(idx + _stream_base(seed, _ST_DUPJ)), 11) % torch.clamp(idx, min=1)
    src = torch.where(is_dup, j, idx)
    for _ in range(64):
        nxt = src[src]
        if torch.equal(nxt, src):
            break
        src = nxt
    lth = _lognormal_len_thresholds(median, sigma, max_len).to(dev)
    lens = 1 + torch.searchsorted(lth, _u32(seed, _ST_LEN, src), right=True)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    offsets[1:] = torch.cumsum(lens, 0)
    N = int(offsets[-1])
    out = torch.empty(N, dtype=torch.uint8, device=dev)
    zth = _zipf_thresholds(zipf_s, ncodes).to(dev)
    # generate in chunks of strings holding about chunk_bytes bytes
    c0 = 0
    while c0 < n:
        target = int(offsets[c0]) + chunk_bytes
        c1 = int(torch.searchsorted(offsets, torch.tensor([target], device=dev), right=True)[0]) - 1
        c1 = max(c0 + 1, min(n, c1))
        b0, b1 = int(offsets[c0]), int(offsets[c1])
        sid = torch.repeat_interleave(torch.arange(c0, c1, device=dev), lens[c0:c1])
        t = torch.arange(b0, b1, device=dev, dtype=torch.int64) - offsets[sid]
        ctr = src[sid] * max_len + t
        out[b0:b1] = (first_code + torch.searchsorted(zth, _u32(seed, _ST_BYTE, ctr), right=True)).to(torch.uint8)
        c0 = c1
    return StringSet(out, offsets, {"kind": "text", "n": n, "seed": seed, "dup_src": src.cpu()})


# ---------------------------------------------------------------------------
# many independent sets (batched execution)
# ---------------------------------------------------------------------------

def log_uniform_sizes(count: int, lo: float, hi: float, seed: int) -> list[int]:
    g = torch.Generator().manual_seed(int(seed) + 7)
    u = torch.rand(count, generator=g, dtype=torch.float64)
    v = torch.floor(torch.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))) + 0.5)
    return [int(x) for x in v.tolist()]


def random_sets(num_sets: int, size_lo: float, size_hi: float, len_lo: int = 8, len_hi: int = 256,
                seed: int = 0, device="cpu") -> tuple[StringSet, torch.Tensor]:
    """``num_sets`` independent sets, sizes log-uniform in [size_lo, size_hi],
    lengths uniform in [len_lo, len_hi], uniform letters 'A'..'Z'.
    Returns the concatenated strings and set boundaries (string index, B+1)."""
    dev = torch.device(device)
    sizes = log_uniform_sizes(num_sets, size_lo, size_hi, seed)
    bounds = torch.zeros(num_sets + 1, dtype=torch.int64)
    bounds[1:] = torch.cumsum(torch.tensor(sizes, dtype=torch.int64), 0)
    n = int(bounds[-1])
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    lens = len_lo + _u32(seed, _ST_SETLEN, idx) % (len_hi - len_lo + 1)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    offsets[1:] = torch.cumsum(lens, 0)
    N = int(offsets[-1])
    out = torch.empty(N, dtype=torch.uint8, device=dev)
    step = 1 << 27
    for b0 in range(0, N, step):
        b1 = min(N, b0 + step)
        ctr = torch.arange(b0, b1, dtype=torch.int64, device=dev)
        out[b0:b1] = (65 + _u32(seed, _ST_SETBYTE, ctr) % 26).to(torch.uint8)
    return StringSet(out, offsets, {"kind": "sets", "sizes": sizes}), bounds


def random_runs(n: int, k: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """A uniformly random run index in [0, k) for each of n strings (the k-way
    merge workload: strings dealt to k runs at random)."""
    idx = torch.arange(n, dtype=torch.int64, device=torch.device(device))
    return _u32(seed, _ST_RUN, idx) % k


# ---------------------------------------------------------------------------
# serving trace
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    kind: str            # "dn" or "text"
    ratio: float         # for "dn"
    seed: int


def poisson_requests(count: int, qps: float, size_lo: float = 1e3, size_hi: float = 1e7,
                     seed: int = 0) -> list[Request]:
    """Poisson arrivals at ``qps``; sizes log-uniform; half fixed-length-100
    D/N strings with ratio in {0.1, 0.5, 0.9}, half text-like strings."""
    g = torch.Generator().manual_seed(int(seed) + 11)
    gaps = -torch.log1p(-torch.rand(count, generator=g, dtype=torch.float64)) / qps
    t = torch.cumsum(gaps, 0).tolist()
    sizes = log_uniform_sizes(count, size_lo, size_hi, seed + 13)
    kinds = torch.randint(0, 2, (count,), generator=g).tolist()
    ratios = torch.randint(0, 3, (count,), generator=g).tolist()
    return [Request(i, t[i], sizes[i], "dn" if kinds[i] == 0 else "text",
                    (0.1, 0.5, 0.9)[ratios[i]], seed * 100003 + i) for i in range(count)]


def request_strings(req: Request, device="cpu") -> StringSet:
    if req.kind == "dn":
        return dn_strings(req.n, 100, req.ratio, seed=req.seed, device=device)
    return text_strings(req.n, seed=req.seed, device=device)
