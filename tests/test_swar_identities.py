"""The word arithmetic behind the distance-table compares of the pruning
scans, checked exhaustively on the CPU (the GPU parity tests check the
kernels that use it end to end):

* the general byte compare: bit 7 of each byte of the result is set exactly
  when that byte of x is <= t, for every t in 0..254 (the largest finite
  table byte) and every byte value, without carries between bytes;
* the short form for t <= 126: with every byte of x ORed with 0x80, the
  subtraction of (t + 1) in every byte borrows within no byte;
* the gather of two words' flags into one byte with a single multiply.

Each formula is written here as the kernels state it (uint32 arithmetic)."""
import numpy as np

M32 = 0xFFFFFFFF
H = 0x80808080


def flags_general(x, t):
    tt = t * 0x01010101
    s = ((tt | H) - (x & ~H & M32)) & M32
    return ((tt & ~x) | (~(tt ^ x) & s)) & H & M32


def flags_small(x, t):
    t1 = (t + 1) * 0x01010101
    return ~((((x | H) - t1) & M32) | x) & H & M32


def gather8(a, b):
    return ((((a >> 7) | (b >> 3)) * 0x01020408) & M32) >> 24


def expected_flags(x, t):
    return sum(0x80 << (8 * i) for i in range(4) if ((x >> (8 * i)) & 255) <= t)


def test_general_compare_every_threshold_and_byte():
    xs = np.arange(256, dtype=np.uint64) * 0x01010101
    for t in range(255):
        for x in xs.tolist():
            assert flags_general(x, t) == expected_flags(x, t), (t, x)


def test_short_compare_every_threshold_and_byte():
    for t in range(127):
        for b in range(256):
            x = b * 0x01010101
            assert flags_small(x, t) == expected_flags(x, t), (t, b)


def test_compares_keep_bytes_apart():
    """Mixed words: every byte is decided on its own (no borrow or carry
    between bytes), including bytes next to the threshold and 255."""
    rng = np.random.default_rng(7)
    for _ in range(20000):
        t = int(rng.integers(0, 255))
        picks = [int(rng.integers(0, 256)), t, min(t + 1, 255), 255, 0, 127, 128]
        bs = [picks[int(rng.integers(0, len(picks)))] for _ in range(4)]
        x = sum(v << (8 * i) for i, v in enumerate(bs))
        assert flags_general(x, t) == expected_flags(x, t)
        if t <= 126:
            assert flags_small(x, t) == expected_flags(x, t)


def test_gather_of_two_words_flags():
    for ma in range(16):
        for mb in range(16):
            a = sum(0x80 << (8 * i) for i in range(4) if (ma >> i) & 1)
            b = sum(0x80 << (8 * i) for i in range(4) if (mb >> i) & 1)
            assert gather8(a, b) == ma | (mb << 4), (ma, mb)
