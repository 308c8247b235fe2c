"""Suffix sorting on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_16517_amd as ss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def _fib(n):
    a, b = b"b", b"a"
    while len(b) < n:
        a, b = b, b + a
    return b[:n]


def _texts():
    rng = np.random.default_rng(0)
    yield "one", b"x"
    yield "two", b"ba"
    yield "banana", b"banana"
    yield "zeros_in_text", bytes(rng.integers(0, 3, 5000).astype(np.uint8))
    yield "dna_200k", bytes(rng.choice(np.frombuffer(b"ACGT", np.uint8), 200_000))
    yield "bytes_300k", bytes(rng.integers(0, 256, 300_000).astype(np.uint8))
    yield "unary_20k", b"a" * 20_000
    yield "periodic_20k", b"abcab" * 4_000
    yield "fibonacci_20k", _fib(20_000)
    yield "small_255", bytes(rng.integers(65, 68, 255).astype(np.uint8))
    yield "small_257", bytes(rng.integers(65, 68, 257).astype(np.uint8))


@pytest.mark.parametrize("name,text", list(_texts()), ids=lambda x: x if isinstance(x, str) and len(x) < 40 else "")
def test_suffix_array_and_lcp_match_oracle(name, text):
    t = torch.frombuffer(bytearray(text), dtype=torch.uint8).to(DEV)
    sa, lcp, steps = ss.suffix_sort(t)
    torch.cuda.synchronize()
    esa, elcp = oracle.suffix_sort(np.frombuffer(text, np.uint8))
    np.testing.assert_array_equal(u32(sa), esa)
    np.testing.assert_array_equal(u32(lcp), elcp)
    assert steps >= 1


def test_suffix_array_with_eight_byte_rank_pairs():
    """N >= 2^28: rank pairs take 8 bytes; checked pair by pair by the oracle."""
    N = (1 << 28) + 4099
    g = torch.Generator(device=DEV).manual_seed(1)
    t = torch.randint(0, 4, (N,), dtype=torch.uint8, device=DEV, generator=g) + 65
    sa, lcp, steps = ss.suffix_sort(t)
    torch.cuda.synchronize()
    print(f"[suffix] N={N} steps={steps}", flush=True)
    assert oracle.check_suffixes(t.cpu().numpy(), u32(sa), u32(lcp)) == -1
