"""Oracle random numbers against the published Philox definition (CPU)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert orc.philox(ctr, key) == out


def test_uniform_open_interval_and_layout(orc):
    # draw d uses block d>>1 and words (2j, 2j+1), j = d&1, of Philox(ctr=(k0,k1,step,d>>1), key=(seed,k2))
    seed, key, step = 7, [11, 22, 33], 5
    for d in range(6):
        o = orc.philox([key[0], key[1], step, d >> 1], [seed, key[2]])
        j = d & 1
        w = (o[2 * j] << 32) | o[2 * j + 1]
        expect = ((w >> 12) + 0.5) * 2.0 ** -52
        assert orc.uniform(seed, key, step, d) == expect
    u = np.array([orc.uniform(seed, [i, 2 * i, 3 * i], i, i % 7) for i in range(20000)])
    assert u.min() > 0.0 and u.max() < 1.0
    # mean and variance of U(0,1) within 5 sigma
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / len(u))


def test_extreme_words_map_inside_unit_interval(orc):
    # the mapping of the largest and smallest 64-bit words
    assert ((0 >> 12) + 0.5) * 2.0 ** -52 > 0.0
    assert (((2 ** 64 - 1) >> 12) + 0.5) * 2.0 ** -52 < 1.0


def test_keys_distinct_and_deterministic(orc):
    keys = {tuple(orc.primary_key(2, e, i)) for e in range(200) for i in range(5)}
    assert len(keys) == 1000
    p = orc.primary_key(2, 3, 0)
    c0 = orc.child_key(2, p, 10, 0)
    c1 = orc.child_key(2, p, 10, 1)
    c2 = orc.child_key(2, p, 11, 0)
    assert len({tuple(c0), tuple(c1), tuple(c2), tuple(p)}) == 4
    assert orc.child_key(2, p, 10, 0) == c0
    # definition: first three words of Philox(ctr=(k0,k1,k2,step), key=(seed, 0xB7E15162 ^ ordinal))
    assert c1 == orc.philox([p[0], p[1], p[2], 10], [2, 0xB7E15162 ^ 1])[:3]
    assert p == orc.philox([3, 0, 0, 0], [2, 0x243F6A88])[:3]
