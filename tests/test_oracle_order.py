"""Pins of the random ordering's oracle (Sec. IV-A orders the points at random).

The ordering sorts the indices by the splitmix64 finaliser of seed XOR i.  The finaliser is pinned to
the first five published outputs of the SplitMix64 generator started from state 0 (state advances by
0x9e3779b97f4a7c15 and each output is the finaliser of the state), so a wrong constant or shift fails;
the order itself must be a permutation, must change with the seed, and must carry no trace of the
input order.
"""
import numpy as np
import pytest

import oracle

GOLDEN = 0x9E3779B97F4A7C15
# SplitMix64 from state 0: the published first outputs of the generator
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC,
                    0x1B39896A51A8749B]


def test_finaliser_reproduces_published_splitmix64_outputs():
    for k, want in enumerate(SPLITMIX64_SEED0, start=1):
        assert oracle.mix64((k * GOLDEN) % 2 ** 64) == want, k


@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000, 100_003])
def test_random_order_is_a_permutation(n):
    p = oracle.random_order(n, seed=11)
    assert p.shape == (n,)
    assert np.array_equal(np.sort(p), np.arange(n))


def test_random_order_depends_on_the_seed_and_forgets_the_input_order():
    n = 50_000
    a, b = oracle.random_order(n, 1), oracle.random_order(n, 2)
    assert not np.array_equal(a, b)
    # rank correlation between position and index is that of a random permutation (sd 1/sqrt(n))
    pos = np.arange(n)
    for p in (a, b):
        r = np.corrcoef(pos, p)[0, 1]
        assert abs(r) < 5 / np.sqrt(n), r
    # the first 1% of the order covers the index range evenly (each decile holds about 10%)
    head = a[: n // 100]
    counts = np.bincount(head * 10 // n, minlength=10)
    assert counts.min() > 0.6 * counts.mean() and counts.max() < 1.4 * counts.mean()


def test_random_order_sorts_by_the_keys():
    n = 500
    p = oracle.random_order(n, 7)
    keys = [oracle.mix64(7 ^ int(i)) for i in p]
    assert all(keys[q] < keys[q + 1] for q in range(n - 1))
