"""CPU pins of the tests' own BF16 rounding (hand-computed bit patterns)."""
import numpy as np

from rounding import bf16_rne_bits


def test_bf16_reference_rounding_pins():
    """The test's own BF16 rounding against hand-computed bit patterns (CPU arithmetic only)."""
    t = 2.0 ** -8
    cases = {1.0: 0x3F80, 1 + t: 0x3F80, 1 + 3 * t: 0x3F82, 1 + t + 2.0 ** -30: 0x3F81, 2 - 2.0 ** -9: 0x4000,
             1 + 2 * t - 2.0 ** -20: 0x3F81, 0.5: 0x3F00, 3.0: 0x4040}
    got = bf16_rne_bits(np.array(list(cases.keys())))
    assert [int(v) for v in got] == list(cases.values())
