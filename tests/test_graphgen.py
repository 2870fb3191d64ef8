"""Host checks of the synthetic graph generators (no GPU)."""
import numpy as np

import graphgen


def test_rmat_chunked_independent_of_workers():
    """Chunk k draws from its own stream, so the pairs do not depend on how
    many processes fill the chunks."""
    a = graphgen.rmat_chunked(10, 8, 0.57, 0.19, 0.19, seed=3, workers=1, chunk=1000)
    b = graphgen.rmat_chunked(10, 8, 0.57, 0.19, 0.19, seed=3, workers=3, chunk=1000)
    assert a.n == 1024 and a.src.size == 8 * 1024
    np.testing.assert_array_equal(a.src, b.src)
    np.testing.assert_array_equal(a.dst, b.dst)
    assert a.src.min() >= 0 and a.src.max() < a.n and a.dst.min() >= 0 and a.dst.max() < a.n


def test_rmat_chunked_matches_the_serial_distribution():
    """The same quadrant probabilities as the one-stream generator: the edge
    count per vertex, sorted, follows the same heavy tail (the largest degrees
    agree within a factor of two, the self-pair share within 20%)."""
    a = graphgen.rmat_chunked(13, 16, 0.57, 0.19, 0.19, seed=5, workers=2, chunk=20000)
    b = graphgen.rmat(13, 16, 0.57, 0.19, 0.19, seed=5)
    da = np.sort(np.bincount(np.concatenate([a.src, a.dst]), minlength=a.n))[::-1]
    db = np.sort(np.bincount(np.concatenate([b.src, b.dst]), minlength=b.n))[::-1]
    for k in (0, 10, 100, 1000):
        assert 0.5 < da[k] / db[k] < 2.0, k
    sa, sb = np.mean(a.src == a.dst), np.mean(b.src == b.dst)
    assert abs(sa - sb) < 0.2 * sb
