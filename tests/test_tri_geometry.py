"""Block geometry of the three-field walk, on the host: a lane's 2^m blocks
(m >= 4) go in levels of triples (b + T, b + Q + T, b + 2Q + T), T < Q, with
Q = 2^(m-2), 2^(m-4), ... >= 2 and b = 2^m - 4Q, and the 2 (m odd) or 4
(m even) blocks left after the last level are walked exactly.  The walk
relies on four facts, checked here for every m the search can use:

- the levels and the tail cover every block exactly once;
- the three blocks of a triple have the parity of T (the top low spin's sign
  pattern, and the carried-step recurrence, which alternates with T);
- for 0 < T < Q the three blocks' boundary steps flip the same high spin
  (trailing zeros of T), so one high field serves all three;
- the old value of that spin is bit c + 1 of each block's own index (the
  Gray code of consecutive block indices), which the walk reads per block.
"""

import pytest


def levels(m):
    out = []
    base, q = 0, 1 << (m - 2)
    while q >= 2:
        out.append((base, q))
        base += 3 * q
        q >>= 2
    return out, base


def gray(x):
    return x ^ (x >> 1)


def ctz(x):
    return (x & -x).bit_length() - 1


@pytest.mark.parametrize("m", range(4, 13))
def test_levels_tile_the_lane(m):
    lv, tail = levels(m)
    seen = []
    for base, q in lv:
        assert base % (4 * q) == 0
        for t in range(q):
            seen += [base + t, base + q + t, base + 2 * q + t]
    rest = list(range(tail, 1 << m))
    assert len(rest) == (2 if m % 2 else 4)
    assert sorted(seen + rest) == list(range(1 << m))


@pytest.mark.parametrize("m", range(4, 13))
def test_triples_share_parity_and_boundary_spin(m):
    lv, _ = levels(m)
    for base, q in lv:
        for t in range(q):
            blocks = (base + t, base + q + t, base + 2 * q + t)
            assert {b & 1 for b in blocks} == {t & 1}
            if t == 0:
                continue
            c = ctz(t)
            for b in blocks:
                # the high spin that changes between blocks b - 1 and b is
                # spin c of the block index's Gray code, the same for all three
                assert gray(b) ^ gray(b - 1) == 1 << c
                # its old value (+1 iff set before the flip) is bit c + 1 of b
                old_up = (gray(b - 1) >> c) & 1
                assert old_up == (b >> (c + 1)) & 1


@pytest.mark.parametrize("m", range(4, 13))
def test_parity_alternates_across_levels(m):
    """The carried top-spin step flips its lane part's sign from one triple
    to the next; that needs the parity of consecutive triples to alternate,
    also from a level's last triple (T = Q - 1, odd) to the next level's
    first (T = 0, even)."""
    lv, _ = levels(m)
    seq = [base + t for base, q in lv for t in range(q)]
    assert all(((a ^ b) & 1) == 1 for a, b in zip(seq, seq[1:]))
    assert seq[0] % 2 == 0
