"""Pins of the noise oracle: the counter-based generator reproduces its published known-answer
vectors, and its outputs are uniform, independent and a bijection of the counter; the Gaussian
deviates and the noise model have the stated moments."""
import os

import numpy as np
import scipy.stats

from oracle import noise as N

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_reproduces_published_known_answer_vectors():
    """Philox-4x32-10 against the known-answer vectors published with the generator (Salmon et
    al., SC 2011; tests/golden/philox4x32_10_kat.txt): a wrong multiplier, Weyl constant, round
    count or word order changes every output word."""
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for v in rows:
        ctr = [np.array([c], dtype=np.uint64) for c in v[:4]]
        out = N.philox4x32_10(ctr, (v[4], v[5]))
        assert [int(o[0]) for o in out] == v[6:], [hex(int(o[0])) for o in out]


def test_philox_outputs_are_uniform_and_a_bijection_of_the_counter():
    n = 200_000
    i = np.arange(n, dtype=np.uint64)
    out = N.philox4x32_10((i, np.zeros(n, np.uint64), np.zeros(n, np.uint64),
                           np.zeros(n, np.uint64)), (0x12345678, 0x9ABCDEF0))
    words = np.stack(out)
    assert words.max() < 2 ** 32
    # a keyed bijection of the 128-bit counter: distinct counters, distinct outputs
    assert np.unique(words[0] * np.uint64(2 ** 32) + words[1]).size == n
    for w in words:                                        # each word uniform on 16 bins
        h = np.bincount((w >> np.uint64(28)).astype(np.int64), minlength=16)
        assert scipy.stats.chisquare(h).pvalue > 1e-4
    # neighbouring counters are uncorrelated
    u = words[0].astype(np.float64) / 2 ** 32
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.01
    # the key matters, and the result is a pure function of (counter, key)
    other = N.philox4x32_10((i[:100], 0 * i[:100], 0 * i[:100], 0 * i[:100]), (1, 0))
    assert not np.array_equal(other[0], words[0][:100])
    again = N.philox4x32_10((i[:100], 0 * i[:100], 0 * i[:100], 0 * i[:100]),
                            (0x12345678, 0x9ABCDEF0))
    assert np.array_equal(again[0], words[0][:100])


def test_normals_are_standard_normal():
    e = N.normals(400_000, seed=2024, stream=3)
    assert abs(e.mean()) < 5 * 1 / np.sqrt(e.size)
    assert abs(e.var() - 1) < 5 * np.sqrt(2 / e.size)
    assert scipy.stats.kstest(e[:50_000], "norm").pvalue > 1e-4
    assert not np.array_equal(e[:1000], N.normals(1000, seed=2024, stream=4))
    assert np.array_equal(e[:1000], N.normals(1000, seed=2024, stream=3))


def test_normals_of_one_block_are_independent_and_prefix_stable():
    """The four deviates of a Philox block (two Box-Muller pairs) are uncorrelated with each
    other and with the next block's; their squares sum to -2 ln u per pair (the pair's radius).
    Drawing fewer voxels returns a prefix of the same sequence."""
    e = N.normals(400_000, seed=11, stream=0).reshape(-1, 4)
    c = np.corrcoef(np.concatenate([e[:-1], e[1:]], axis=1).T)
    off = c[~np.eye(8, dtype=bool)]
    assert np.abs(off).max() < 0.01
    # the pair (cos, sin) of one radius: e0^2 + e1^2 = r0^2 = -2 ln u0 is Exp(1/2) distributed
    r2 = e[:, 0] ** 2 + e[:, 1] ** 2
    assert scipy.stats.kstest(r2[:50_000], "expon", args=(0, 2)).pvalue > 1e-4
    x = N.philox4x32_10((np.arange(5, dtype=np.uint64), np.zeros(5, np.uint64),
                         np.zeros(5, np.uint64), np.zeros(5, np.uint64)), (11, 0))
    u0 = (x[0].astype(np.float64) + 0.5) * 2.0 ** -32
    np.testing.assert_allclose(r2[:5], -2.0 * np.log(u0), rtol=1e-13)
    for n in (1, 2, 3, 5, 7, 4001):
        assert np.array_equal(N.normals(n, 11, 0), e.ravel()[:n])


def test_noise_model_moments():
    rng = np.random.default_rng(0)
    cube = np.where(rng.uniform(size=(40, 50, 200)) < 0.5, 0.0, 37.0)
    gain, floor = 0.8, 2.5
    d = N.add_noise(cube, seed=7, stream=0, gain=gain, sigma_floor=floor) - cube
    for level in (0.0, 37.0):
        m = cube == level
        var = gain * level + floor ** 2
        assert abs(d[m].mean()) < 5 * np.sqrt(var / m.sum())
        assert abs(d[m].var() / var - 1) < 5 * np.sqrt(2 / m.sum())
    # negative voxels (possible after a signed loss gradient) only see the floor
    neg = N.add_noise(-np.ones(1000), 1, 0, 5.0, 0.0)
    assert np.array_equal(neg, -np.ones(1000))
