"""Writes kr_vectors.txt: frozen Karp-Rabin prefix keys computed by the CPU oracle.

Run from the repository root: python tests/golden/make_kr_vectors.py
The vectors cover word-boundary lengths (0..17, 31..33, 63..65), zero bytes,
0xFF bytes and a long input; they freeze the hash so that GPU parity tests and
the oracle agree on every (bytes, length) pair.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

CASES = []
for m in list(range(0, 18)) + [31, 32, 33, 63, 64, 65, 255, 256, 257]:
    CASES.append(bytes((7 * i + 65) & 0xFF for i in range(m)))
CASES += [b"\x00", b"\x00\x00\x00\x00\x00", b"\xff" * 9, b"A\x00", b"AB\x00\x00", bytes(range(256)) * 4]

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kr_vectors.txt")
    with open(out, "w") as f:
        f.write("# hex(prefix bytes) key  -- Karp-Rabin mod 2^61-1, base 0x0B3C4D5E6F708192,\n")
        f.write("# 4-byte little-endian limbs, length appended; written by make_kr_vectors.py (oracle)\n")
        for c in CASES:
            f.write(f"{c.hex() if c else '-'} {oracle.kr_key(c):016x}\n")
    print("wrote", out, len(CASES))
