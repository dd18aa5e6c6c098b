"""The autotuner returns a valid decomposition and caches it."""
import pytest

pytestmark = pytest.mark.gpu


def test_autotune_valid_and_cached():
    import paper_1008_3699_amd as P
    from gpu_util import dev
    dev()
    for n in (64, 200):
        p, us = P.autotune(2, (n, n), "f32", "ssor")
        assert 1 <= p[0] <= n // 2 and 1 <= p[1] <= n // 2 and us > 0
        assert (n + p[1] - 1) // p[1] <= 128  # tiles fit the pipelined path
        p2, us2 = P.autotune(2, (n, n), "f32", "ssor")
        assert p2 == p and us2 == -1.0
