"""Pins of the BCC trial draws (reading; the paper fixes neither the random
numbers nor how a swap partner is chosen beyond its being a nearest
neighbour).

Each trial takes one 32-bit word of a Philox4x32-10 call keyed by the lane's
base cell as its acceptance draw; the partner direction is drawn once per
(sweep, colour, sub-colour) set (x step from one per-colour draw, y and z
steps from another).  Checked here by enumeration over whole lattices, not
by restating the formulas:
  * no two trials of a sweep share a random word, and no trial counter
    equals a per-colour partner-bit counter or the shift counter;
  * inside one set every partner has the same direction;
  * the direction, counted once per set, is uniform over the 8 first
    neighbours (chi-square over sets and sweeps), its x step independent of
    its y and z steps;
  * the acceptance draw is uniform on [0, 2^32) (chi-square, and its low
    bit balanced);
  * the partner is a first neighbour of the site (Cartesian distance).
"""
import numpy as np
import pytest


def chi2_uniform(counts):
    counts = np.asarray(counts, dtype=np.float64)
    e = counts.sum() / counts.size
    return float(((counts - e) ** 2 / e).sum()), counts.size - 1


@pytest.mark.parametrize("L,B", [((4, 4, 4), (12, 12, 12)), ((7, 6, 5), (2, 3, 4)),
                                 ((13, 9, 22), (12, 12, 12)), ((24, 25, 26), (12, 12, 12)),
                                 ((2, 2, 2), (2, 2, 2))])
def test_draw_words_unique(orc, L, B):
    for s in (0, 3, 1000):
        ctr, word, dirs, u = orc.bcc_draws(L, B, 4242, s)
        keys = np.concatenate([ctr, word[:, None].astype(np.uint32)], axis=1)
        assert np.unique(keys, axis=0).shape[0] == keys.shape[0]
        assert np.all(ctr[:, 2] == s)
        # one call serves at most 4 trials, through distinct words
        _, per_call = np.unique(ctr, axis=0, return_counts=True)
        assert per_call.max() <= 4
        # never the counter of a partner-bit draw (0, 0, s, 32 + c) and
        # (0, 0, s, 40 + c) or of the origin shift (0, 0, s, 8)
        low = (ctr[:, 0] == 0) & (ctr[:, 1] == 0)
        assert not np.any(low & (((ctr[:, 3] >= 32) & (ctr[:, 3] < 48)) | (ctr[:, 3] == 8)))


def test_partner_steps_shared_per_set(orc):
    L, B = (13, 9, 22), (12, 12, 12)
    for s in (0, 7):
        col, sub, _ = orc.schedule(L, B, 99, s)
        _, _, dirs, _ = orc.bcc_draws(L, B, 99, s)
        key = col.astype(np.int64) * 54 + sub
        for k in np.unique(key):
            assert np.unique(dirs[key == k]).size == 1, (s, k)
        # and different sets do not all agree
        assert np.unique(dirs).size == 8


def set_directions(orc, L, B, seed, sweeps):
    """The direction of every (sweep, colour, sub-colour) set, once per set."""
    out = []
    for s in sweeps:
        col, sub, _ = orc.schedule(L, B, seed, s)
        _, _, dirs, _ = orc.bcc_draws(L, B, seed, s)
        key = col.astype(np.int64) * 54 + sub
        _, first = np.unique(key, return_index=True)
        out.append(dirs[first])
    return np.concatenate(out).astype(np.int64)


def test_direction_uniform_and_x_independent(orc):
    L, B = (6, 6, 6), (12, 12, 12)
    d = set_directions(orc, L, B, 7, range(120))     # 120 sweeps x 8 colours x 54 sets
    hist = np.zeros((2, 4), np.int64)
    np.add.at(hist, (d & 1, d >> 1), 1)
    chi2, dof = chi2_uniform(hist.ravel())
    assert chi2 < dof + 6 * np.sqrt(2 * dof), hist
    # independence of the x step from the (y, z) steps: 2 x 4 contingency
    row, colm, n = hist.sum(1, keepdims=True), hist.sum(0, keepdims=True), hist.sum()
    e = row * colm / n
    chi2 = float(((hist - e) ** 2 / e).sum())
    assert chi2 < 3 + 6 * np.sqrt(6), hist


def test_acceptance_draw_uniform(orc):
    L, B = (10, 10, 10), (12, 12, 12)
    us = np.concatenate([orc.bcc_draws(L, B, 31, s)[3] for s in range(20)])
    counts = np.bincount((us >> 26).astype(np.int64), minlength=64)
    chi2, dof = chi2_uniform(counts)
    assert chi2 < dof + 6 * np.sqrt(2 * dof)
    # all 32 bits are drawn: the low bit too is balanced
    odd = int(np.count_nonzero(us & 1))
    assert abs(odd - us.size / 2) < 6 * np.sqrt(us.size / 4)


def test_partner_is_a_first_neighbour(orc):
    L, B = (7, 6, 5), (12, 12, 12)
    _, _, dirs, _ = orc.bcc_draws(L, B, 5, 2)
    N = 2 * int(np.prod(L))
    i = np.arange(N)
    j = np.array([orc.neighbour(L, int(a), int(d)) for a, d in zip(i, dirs)])

    def pos(k):
        b, c = k % 2, k // 2
        x, y, z = c % L[0], (c // L[0]) % L[1], c // (L[0] * L[1])
        return np.stack([2 * x + b, 2 * y + b, 2 * z + b], axis=-1)

    d = (pos(j) - pos(i)) % (2 * np.asarray(L))
    d = np.where(d > np.asarray(L), d - 2 * np.asarray(L), d)
    assert np.all(np.abs(d) == 1)
    # sign of each component follows the direction bits
    want = np.stack([(dirs.astype(np.int64) >> a) & 1 for a in range(3)], axis=-1) * 2 - 1
    assert np.array_equal(d, want)


# ---- FCC (the partner of every trial of a set is drawn once per set) ----

def fcc_pos(L, k):
    sub = np.array([(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])
    b, c = k % 4, k // 4
    x, y, z = c % L[0], (c // L[0]) % L[1], c // (L[0] * L[1])
    return np.stack([2 * x, 2 * y, 2 * z], axis=-1) + sub[b]


def fcc_disp(L, i, j):
    d = (fcc_pos(L, j) - fcc_pos(L, i)) % (2 * np.asarray(L))
    return np.where(d > np.asarray(L), d - 2 * np.asarray(L), d)


def test_fcc_partner_is_first_neighbour_and_shared_per_set(orc):
    L, B = (7, 6, 5), (12, 12, 12)
    N = 4 * int(np.prod(L))
    i = np.arange(N)
    for s in (0, 4):
        j, u = orc.fcc_draws(L, B, 21, s)
        d = fcc_disp(L, i, j)
        assert np.all((d * d).sum(-1) == 2)          # first shell: (+-1, +-1, 0) and permutations
        col, sub, _ = orc.schedule(L, B, 21, s, lattice=orc.FCC)
        key = col.astype(np.int64) * 108 + sub
        for k in np.unique(key):
            assert np.unique(d[key == k], axis=0).shape[0] == 1, (s, k)
        # acceptance words: one Philox call per cell, a different word per site
        assert np.unique(u).size > 0.99 * N


def test_fcc_partner_uniform_over_the_twelve(orc):
    """One displacement per (colour, sub-colour) set, counted once per set."""
    L, B = (6, 6, 6), (12, 12, 12)
    N = 4 * int(np.prod(L))
    i = np.arange(N)
    counts = {}
    for s in range(200):
        j, _ = orc.fcc_draws(L, B, 5, s)
        d = fcc_disp(L, i, j)
        col, sub, _ = orc.schedule(L, B, 5, s, lattice=orc.FCC)
        key = col.astype(np.int64) * 108 + sub
        _, first = np.unique(key, return_index=True)   # one draw per set
        for v, c in zip(*np.unique(d[first], axis=0, return_counts=True)):
            counts[tuple(v)] = counts.get(tuple(v), 0) + c
    assert len(counts) == 12
    chi2, dof = chi2_uniform(list(counts.values()))
    assert chi2 < dof + 6 * np.sqrt(2 * dof), counts
