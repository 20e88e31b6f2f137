"""Pins of the oracle on the FCC lattice (the lattice of the paper's
Fe29Co29Ni28Al7Ti7 alloy and its L1_2 precipitates, Section "Evolution of
chemical defects").  FCC: four sites per cubic cell, first/second/third
shells of 12/6/24 neighbours.

Pins that do not reuse the oracle's displacement tables: the L1_2 (A3B)
closed form worked out by hand, a brute-force pair sum classified by
Cartesian minimum-image distance, the energy change against full energies,
a Cartesian conflict audit of the schedule, and exact enumeration of a
32-site cell.
"""
import math

import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W

FCC = 1
Z = (12, 6, 24)
KB = 86.17333262
SUB = np.array([(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])


def n_sites(L):
    return 4 * int(np.prod(L))


def positions(L):
    Lx, Ly, Lz = L
    z, y, x, b = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), np.arange(4), indexing="ij")
    return (np.stack([2 * x, 2 * y, 2 * z], axis=-1) + SUB[b]).reshape(-1, 3)


def site_index(L, X):
    Lx, Ly, Lz = L
    X = X % (2 * np.asarray(L))
    par = (X[..., 0] & 1) | (X[..., 1] & 1) << 1 | (X[..., 2] & 1) << 2
    b = np.array([0, -1, -1, 1, -1, 2, 3, -1])[par]
    assert np.all(b >= 0)
    cell = ((X[..., 2] >> 1) * Ly + (X[..., 1] >> 1)) * Lx + (X[..., 0] >> 1)
    return cell * 4 + b


def brute_force_counts(L, S, K, sigma):
    P = positions(L)
    box = 2 * np.asarray(L)
    d2_of_shell = (2, 4, 6)
    counts = np.zeros((S, K, K), np.int64)
    for i in range(len(P)):
        d = (P - P[i] + box // 2) % box - box // 2
        d2 = (d * d).sum(axis=1)
        for s in range(S):
            for j in np.nonzero(d2 == d2_of_shell[s])[0]:
                counts[s, sigma[i], sigma[j]] += 1
    return counts


def test_shell_sizes_and_geometry(orc):
    assert [orc.shell_size(s, FCC) for s in range(3)] == [12, 6, 24]
    L = (5, 4, 6)
    P = positions(L)
    box = 2 * np.asarray(L)
    for i in [0, 1, 2, 3, 57, n_sites(L) - 1]:
        for k in range(42):
            j = orc.neighbour(L, i, k, FCC)
            d = (P[j] - P[i] + box // 2) % box - box // 2
            shell = 0 if k < 12 else (1 if k < 18 else 2)
            assert int((d * d).sum()) == (2, 4, 6)[shell]


@pytest.mark.parametrize("L", [(2, 2, 2), (3, 4, 5), (4, 4, 4)])
def test_l12_closed_form(orc, L):
    """A3B in the L1_2 arrangement: B on cube corners, A on face centres.
    Per cell: 2E = 24 V1ab + 24 V1aa + 6 V2bb + 18 V2aa + 48 V3ab + 48 V3aa
    (a corner has 12 A first neighbours, 6 B second, 24 A third; a face
    centre 4 B + 8 A first, 6 A second, 8 B + 16 A third)."""
    rng = np.random.default_rng(3)
    epi = W.epi_table(3, 2, 40.0, rng).astype(np.int64)
    sigma = np.tile(np.array([1, 0, 0, 0], np.uint8), int(np.prod(L)))
    A, B = 0, 1
    twice = (24 * epi[0, A, B] + 24 * epi[0, A, A] + 6 * epi[1, B, B] + 18 * epi[1, A, A]
             + 48 * epi[2, A, B] + 48 * epi[2, A, A])
    assert orc.energy(L, epi.astype(np.int32), sigma, FCC) == int(np.prod(L)) * twice // 2


def test_l12_sro_hand_values(orc):
    """L1_2 A3B: c_A = 3/4, c_B = 1/4.  First shell around B: all A, so
    P(A|B) = 1 and alpha^{AB} = 1 - 1/(3/4) = -1/3; around A: 4 B of 12,
    P(B|A) = 1/3, alpha^{BA} = 1 - (1/3)/(1/4) = -1/3; P(B|B) = 0 gives
    alpha^{BB} = 1."""
    L = (3, 3, 3)
    sigma = np.tile(np.array([1, 0, 0, 0], np.uint8), 27)
    alpha, _ = orc.sro(L, 3, 2, sigma, FCC)
    assert np.isclose(alpha[0, 1, 0], -1.0 / 3.0) and np.isclose(alpha[0, 0, 1], -1.0 / 3.0)
    assert np.isclose(alpha[0, 1, 1], 1.0)
    assert np.isclose(alpha[0, 0, 0], 1.0 - (8.0 / 12.0) / 0.75)


@pytest.mark.parametrize("L,S,K", [((4, 4, 4), 3, 4), ((4, 5, 4), 2, 3), ((5, 4, 4), 1, 5)])
def test_energy_and_counts_match_brute_force(orc, L, S, K):
    rng = np.random.default_rng(sum(L) + K)
    epi = W.epi_table(S, K, 25.0, rng)
    sigma = rng.integers(0, K, size=n_sites(L)).astype(np.uint8)
    counts = brute_force_counts(L, S, K, sigma)
    assert np.array_equal(orc.pair_counts(L, S, K, sigma, FCC).astype(np.int64), counts)
    assert orc.energy(L, epi, sigma, FCC) == int((counts * epi.astype(np.int64)).sum()) // 2


@pytest.mark.parametrize("L", [(2, 2, 2), (2, 3, 4), (4, 4, 4), (5, 6, 5)])
@pytest.mark.parametrize("S,K", [(1, 2), (3, 5), (3, 8)])
def test_delta_energy_equals_full_difference(orc, L, S, K):
    rng = np.random.default_rng(hash((L, S, K)) % 997)
    epi = W.epi_table(S, K, 25.0, rng)
    sigma = rng.integers(0, K, size=n_sites(L)).astype(np.uint8)
    E0 = orc.energy(L, epi, sigma, FCC)
    for _ in range(10):
        i = int(rng.integers(0, sigma.size))
        j = orc.neighbour(L, i, int(rng.integers(0, 12)), FCC)
        s2 = sigma.copy()
        s2[i], s2[j] = s2[j], s2[i]
        assert orc.energy(L, epi, s2, FCC) - E0 == orc.delta_energy(L, epi, sigma, i, j, FCC)


def footprints(L, S=3):
    P = positions(L)
    first = np.array([v for v in [(1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0), (1, 0, 1), (1, 0, -1),
                                  (-1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1)]])
    w = np.concatenate([np.zeros((1, 3), int), first])
    r2max = (2, 4, 6)[S - 1]
    ball = np.array([(a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3)
                     if (a + b + c) % 2 == 0 and a * a + b * b + c * c <= r2max])
    r = np.unique((w[:, None, :] + ball[None, :, :]).reshape(-1, 3), axis=0)
    return site_index(L, P[:, None, :] + w[None, :, :]), site_index(L, P[:, None, :] + r[None, :, :])


@pytest.mark.parametrize("L,B", [((4, 4, 4), (2, 2, 2)), ((7, 5, 6), (3, 2, 3)), ((12, 13, 12), (12, 12, 12)),
                                 ((9, 8, 10), (4, 4, 5))])
def test_schedule_conflict_free(orc, L, B):
    N = n_sites(L)
    write, read = footprints(L)
    for s in range(2):
        col, sub, blk = orc.schedule(L, B, 321 + s, s, FCC)
        assert sub.max() < 108 and np.all(sub % 4 == np.arange(N) % 4)
        for c in range(8):
            in_c = np.nonzero(col == c)[0]
            for q in np.unique(sub[in_c]):
                T = in_c[sub[in_c] == q]
                rows = np.sort(read[T], axis=1)
                first = np.concatenate([np.ones((len(T), 1), bool), rows[:, 1:] != rows[:, :-1]], axis=1)
                nread = np.bincount(rows[first], minlength=N)
                wmask = np.zeros(N, bool)
                wmask[write[T].ravel()] = True
                assert not np.any(wmask & (nread >= 2)), (L, B, s, c, q)
            sites = read[in_c].ravel()
            owner = np.repeat(blk[in_c], read.shape[1])
            lo = np.full(N, np.iinfo(np.int64).max)
            hi = np.full(N, -1)
            np.minimum.at(lo, sites, owner)
            np.maximum.at(hi, sites, owner)
            wmask = np.zeros(N, bool)
            wmask[write[in_c].ravel()] = True
            assert not np.any(wmask & (hi >= 0) & (lo != hi)), (L, B, s, c)


@pytest.mark.parametrize("T", [700.0, 1600.0])
def test_32_site_cell_matches_enumeration(orc, T):
    """Exact canonical distribution (Eq. (1)) of a 2x2x2-cell FCC binary
    with 4 minority atoms, against the oracle's chain (batch means)."""
    L = (2, 2, 2)
    rng = np.random.default_rng(int(T) + 1)
    epi = W.epi_table(3, 2, 30.0, rng)
    comp = [28, 4]
    E_all, _ = orc.enumerate_configs(L, epi, comp, lattice=FCC)
    w = np.exp(-(E_all - E_all.min()) / (KB * T))
    w /= w.sum()
    exact = float((w * E_all).sum())
    st = orc.OracleState(L, (2, 2, 2), epi, W.configuration(comp, rng), 99 + int(T), lattice=FCC)
    Et, _ = st.sweep(T, 30000, trace_E=True)
    x = Et[500:].astype(np.float64)
    nb = 40
    m = x[: x.size // nb * nb].reshape(nb, -1).mean(axis=1)
    se = m.std(ddof=1) / math.sqrt(nb)
    assert abs(m.mean() - exact) < 5 * se, (m.mean(), exact, se)
    assert np.array_equal(np.bincount(st.sigma, minlength=2), comp)
    assert st.E[0] == orc.energy(L, epi, st.sigma, FCC)


def test_zero_interaction_swaps_every_unlike_pair(orc):
    """With V = 0 every proposed swap of unlike species is accepted: on an
    equiatomic binary about half of all trials change the configuration."""
    L = (6, 6, 6)
    rng = np.random.default_rng(4)
    K = 2
    sigma = W.configuration(W.equiatomic(K, n_sites(L)), rng)
    st = orc.OracleState(L, (3, 3, 3), np.zeros((1, K, K), np.int32), sigma, 5, lattice=FCC)
    st.sweep(1000.0, 20)
    # with V = 0 every unlike pair swaps: about half the trials
    frac = int(st.accepted[0]) / (20 * n_sites(L))
    assert 0.4 < frac < 0.6
