"""Input generators: Philox known-answer vectors and graph constructions."""
import numpy as np
import pytest

import tcolgen


def test_philox_known_answers():
    # Known-answer vectors published with the Random123 library (Philox4x32, 10 rounds)
    kat = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in kat:
        out = tcolgen.philox4x32_10(np.array([ctr], np.uint32), key)[0]
        assert tuple(int(x) for x in out) == want


def test_random_words_offsets_consistent():
    a = tcolgen.random_words(7, 1, 40)
    b = tcolgen.random_words(7, 1, 13, offset=9)
    assert np.array_equal(a[9:22], b)


def test_gnp_symmetric_density():
    A = tcolgen.gnp(300, 0.5, 1)
    assert A.dtype == np.uint8
    assert np.array_equal(A, A.T) and not A.diagonal().any()
    dens = A.sum() / (300 * 299)
    assert abs(dens - 0.5) < 0.01
    assert np.array_equal(A, tcolgen.gnp(300, 0.5, 1))
    assert not np.array_equal(A, tcolgen.gnp(300, 0.5, 2))


def test_planted_is_legal_and_dense():
    P = tcolgen.planted(1000, 28, 3)
    # expected global density 0.5 -> cross-class probability 0.5180
    assert P.p_cross == pytest.approx(249750 / 482140, rel=1e-9)
    A = P.A
    assert np.array_equal(A, A.T) and not A.diagonal().any()
    sizes = np.bincount(P.classes, minlength=28)
    assert sorted(sizes.tolist()) == [35] * 8 + [36] * 20
    same = P.classes[:, None] == P.classes[None, :]
    assert not (A.astype(bool) & same).any()
    assert abs(A.sum() / (1000 * 999) - 0.5) < 0.01


def test_mycielski_sizes():
    # M_m has 3*2^(m-2) - 1 vertices; edges 1, 5, 20, 71, 236 for m = 2..6
    for m, e in zip(range(2, 7), [1, 5, 20, 71, 236]):
        A = tcolgen.mycielski(m)
        assert A.shape[0] == 3 * 2 ** (m - 2) - 1
        assert A.sum() // 2 == e
        assert np.array_equal(A, A.T) and not A.diagonal().any()
        # triangle-free
        assert np.trace(np.linalg.matrix_power(A.astype(np.int64), 3)) == 0


def test_weights0_distribution():
    W = tcolgen.weights0(4, 100, 30, seed=0)
    assert W.dtype == np.float32 and W.shape == (4, 100, 30)
    assert abs(float(W.std()) - 0.01) < 5e-4
    assert abs(float(W.mean())) < 5e-4
    assert np.array_equal(W, tcolgen.weights0(4, 100, 30, seed=0))


def test_greedy_count_is_legal_bound():
    A = tcolgen.gnp(80, 0.5, 4)
    k = tcolgen.greedy_colour_count(A)
    assert 5 <= k <= 80
