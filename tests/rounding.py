"""Round-to-nearest-even conversion to BF16 written on the FP64 bit pattern (test helper)."""
import numpy as np


def bf16_rne_bits(x):
    """BF16 bits (uint16) of positive normal FP64 values, rounded to nearest, ties to even.

    Integer arithmetic on the FP64 pattern: keep the top 7 of the 52 fraction bits and round on the
    other 45 (half = 2^44); a carry out of the fraction raises the exponent."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert np.all(x > 0) and np.all(x < 3e38) and np.all(x > 1.2e-38), "test values stay normal in BF16"
    b = x.view(np.uint64)
    e = ((b >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023 + 127
    m = b & np.uint64((1 << 52) - 1)
    q = (m >> np.uint64(45)).astype(np.int64)
    rem = (m & np.uint64((1 << 45) - 1)).astype(np.int64)
    half = 1 << 44
    up = (rem > half) | ((rem == half) & ((q & 1) == 1))
    q = q + up
    carry = q == 128
    q = np.where(carry, 0, q)
    e = e + carry
    return ((e << 7) | q).astype(np.uint16)
