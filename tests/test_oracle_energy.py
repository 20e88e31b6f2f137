"""Pins of the oracle's EPI energy, energy change, pair counts and SRO.

The EPI model keeps pair interactions only (paper, Section "Results and
discussion").  Pins that do not reuse the oracle's displacement tables:
  * closed forms: a single-species lattice and the B2-ordered binary;
  * a brute-force sum over all site pairs classified by Cartesian
    minimum-image distance (sqrt(3)/2, 1, sqrt(2) lattice constants);
  * the incremental energy change equals the difference of two full
    energies, for every lattice size down to 2 cells;
  * Warren-Cowley SRO (Eq. (SRO)): sum_p c_p alpha^{pp'} = 0, symmetry,
    and the B2 values alpha = -1 / +1 worked out by hand.
"""
import itertools

import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W

Z = (8, 6, 12)


def positions(L):
    """Doubled coordinates (units of a/2) of every site in canonical order."""
    Lx, Ly, Lz = L
    out = np.zeros((2 * Lx * Ly * Lz, 3), np.int64)
    i = 0
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                for b in range(2):
                    out[i] = (2 * x + b, 2 * y + b, 2 * z + b)
                    i += 1
    return out


def brute_force_pairs(L, S, K, sigma):
    """Unordered pairs {i, j}, i != j, by minimum-image squared distance in
    (a/2)^2 units: 3 -> shell 1, 4 -> shell 2, 8 -> shell 3.  Needs L >= 4
    (each pair then has a unique nearest image within shell 3)."""
    P = positions(L)
    box = 2 * np.asarray(L)
    counts = np.zeros((S, K, K), np.int64)
    d2_of_shell = (3, 4, 8)
    for i in range(len(P)):
        d = P - P[i]
        d = (d + box // 2) % box - box // 2
        d2 = (d * d).sum(axis=1)
        for s in range(S):
            for j in np.nonzero(d2 == d2_of_shell[s])[0]:
                counts[s, sigma[i], sigma[j]] += 1
    return counts  # ordered (centre, neighbour) counts


def random_case(L, S, K, seed):
    rng = np.random.default_rng(seed)
    epi = W.epi_table(S, K, 25.0, rng)
    sigma = rng.integers(0, K, size=W.n_sites(L)).astype(np.uint8)
    return epi, sigma


@pytest.mark.parametrize("S", [1, 2, 3])
def test_uniform_lattice_closed_form(orc, S):
    L = (5, 4, 6)
    N = W.n_sites(L)
    rng = np.random.default_rng(S)
    epi = W.epi_table(S, 3, 40.0, rng)
    for p in range(3):
        sigma = np.full(N, p, np.uint8)
        want = sum(N * Z[s] * int(epi[s, p, p]) // 2 for s in range(S))
        assert orc.energy(L, epi, sigma) == want


@pytest.mark.parametrize("L", [(4, 4, 4), (6, 5, 4), (2, 2, 2), (3, 2, 5)])
def test_b2_ordered_binary_closed_form(orc, L):
    """Corners A, bodies B: every first-neighbour bond is A-B, second and
    third neighbours are alike.  E = N/4 [16 V1ab + 6 (V2aa + V2bb) + 12 (V3aa + V3bb)]."""
    N = W.n_sites(L)
    rng = np.random.default_rng(7)
    epi = W.epi_table(3, 2, 40.0, rng).astype(np.int64)
    sigma = np.tile(np.array([0, 1], np.uint8), N // 2)
    want = N * (16 * epi[0, 0, 1] + 6 * (epi[1, 0, 0] + epi[1, 1, 1])
                + 12 * (epi[2, 0, 0] + epi[2, 1, 1])) // 4
    assert orc.energy(L, epi.astype(np.int32), sigma) == want


@pytest.mark.parametrize("L,S,K", [((4, 4, 4), 3, 5), ((5, 4, 6), 2, 3), ((4, 5, 4), 1, 8),
                                   ((6, 6, 5), 3, 2)])
def test_energy_and_counts_match_brute_force_pairs(orc, L, S, K):
    epi, sigma = random_case(L, S, K, seed=sum(L) * 10 + K)
    counts = brute_force_pairs(L, S, K, sigma)
    assert np.array_equal(orc.pair_counts(L, S, K, sigma).astype(np.int64), counts)
    want = int((counts * epi.astype(np.int64)).sum()) // 2
    assert orc.energy(L, epi, sigma) == want


def test_neighbour_geometry(orc):
    """Every displacement lands at the stated distance on the stated sublattice."""
    L = (5, 6, 7)
    P = positions(L)
    box = 2 * np.asarray(L)
    for i in [0, 1, 17, 100, 2 * 5 * 6 * 7 - 1]:
        for k in range(26):
            j = orc.neighbour(L, i, k)
            d = (P[j] - P[i] + box // 2) % box - box // 2
            d2 = int((d * d).sum())
            shell = 0 if k < 8 else (1 if k < 14 else 2)
            assert d2 == (3, 4, 8)[shell]
            if k < 8:
                # shell-1 vector k: +1 on axis a iff bit a of k is set
                assert tuple(int(v) for v in d) == tuple(1 if (k >> a) & 1 else -1 for a in range(3))


@pytest.mark.parametrize("L", [(2, 2, 2), (3, 3, 3), (2, 3, 4), (4, 4, 4), (5, 7, 6), (9, 8, 9)])
@pytest.mark.parametrize("S,K", [(1, 2), (2, 4), (3, 5), (3, 8)])
def test_delta_energy_equals_full_difference(orc, L, S, K):
    epi, sigma = random_case(L, S, K, seed=hash((L, S, K)) % 1000)
    rng = np.random.default_rng(99)
    E0 = orc.energy(L, epi, sigma)
    for _ in range(12):
        i = int(rng.integers(0, sigma.size))
        j = orc.neighbour(L, i, int(rng.integers(0, 8)))
        dE = orc.delta_energy(L, epi, sigma, i, j)
        s2 = sigma.copy()
        s2[i], s2[j] = s2[j], s2[i]
        assert orc.energy(L, epi, s2) - E0 == dE


def test_sro_sum_rule_and_symmetry(orc):
    L = (6, 6, 6)
    K, S = 5, 3
    rng = np.random.default_rng(4)
    comp = W.dirichlet_counts(K, W.n_sites(L), 2.0, rng)
    sigma = W.configuration(comp, rng)
    alpha, counts = orc.sro(L, S, K, sigma)
    c = comp / comp.sum()
    for m in range(S):
        # sum_p c_p alpha^{p p'} = 0 for every centre p'
        assert np.allclose((alpha[m] * c[None, :]).sum(axis=1), 0.0, atol=1e-12)
        assert np.allclose(alpha[m], alpha[m].T, atol=1e-12)
        assert np.array_equal(counts[m], counts[m].T)
        assert counts[m].sum() == Z[m] * sigma.size


def test_sro_b2_hand_values(orc):
    """B2 binary, c_A = c_B = 1/2.  Shell 1: every neighbour of A is B, so
    P(B|A) = 1, alpha^{AB} = 1 - 1/(1/2) = -1 and alpha^{AA} = 1 - 0 = +1.
    Shells 2 and 3 connect like sites: alpha^{AA} = -1, alpha^{AB} = +1."""
    L = (4, 4, 4)
    sigma = np.tile(np.array([0, 1], np.uint8), W.n_sites(L) // 2)
    alpha, _ = orc.sro(L, 3, 2, sigma)
    assert np.allclose(alpha[0], [[1, -1], [-1, 1]])
    assert np.allclose(alpha[1], [[-1, 1], [1, -1]])
    assert np.allclose(alpha[2], [[-1, 1], [1, -1]])


def test_sro_missing_species_is_nan(orc):
    L = (4, 4, 4)
    sigma = np.tile(np.array([0, 1], np.uint8), W.n_sites(L) // 2)
    alpha, _ = orc.sro(L, 1, 3, sigma)
    assert np.isnan(alpha[0, 2, :]).all() and np.isnan(alpha[0, :, 2]).all()
    assert not np.isnan(alpha[0, :2, :2]).any()
