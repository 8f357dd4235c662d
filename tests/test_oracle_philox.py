"""Pins of the oracle's Philox4x32-10 against the generator's published
known-answer vectors (Salmon et al., SC'11) and basic uniformity."""
import os
import numpy as np
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox(ctr, key) == out


def test_uniforms_open_interval_and_moments():
    u = np.array([oracle.uniform2(7, i, 3, 5, 1 << 24) for i in range(20000)]).ravel()
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert abs(u.mean() - 0.5) < 0.006
    assert abs(u.var() - 1.0 / 12.0) < 0.003


def test_uniform_word_mapping():
    # uniform = ((hi << 21 | lo >> 11) + 0.5) * 2^-53 of each word pair
    w = oracle.philox([11, 22, 33, 44], [5, 0])
    u = oracle.uniform2(5, 11, 22, 33, 44)
    exp0 = (((w[0] << 21) | (w[1] >> 11)) + 0.5) / 2.0 ** 53
    exp1 = (((w[2] << 21) | (w[3] >> 11)) + 0.5) / 2.0 ** 53
    assert u[0] == exp0 and u[1] == exp1
