"""Detailed balance of one trial of the oracle.

A trial proposes the swap of a pair (i, j) of first neighbours chosen
without looking at the configuration: the draws depend on the seed, sweep,
colour and site only.  Reversibility with respect to Eq. (1) (Section
"Monte Carlo simulation") then reduces to the acceptance rule:
    pi(s) a(s -> s') = pi(s') a(s' -> s),  pi ~ exp(-E / k_B T).
For each pair this checks three things.
* The oracle's energy change equals E(s') - E(s) from an independent
  Cartesian pair sum, and the reverse move's change is its negative.
* The exact acceptance probability over the whole draw space satisfies
  a(s -> s') / a(s' -> s) = exp(-(E(s') - E(s)) / k_B T) to within the
  draw resolution, 2^-32 (the acceptance draw of both lattices is a whole
  32-bit word).  The probability is found by bisection on the oracle's test,
  which is monotone in the draw.
* Pairs are checked on random quinary configurations at 1 K to 5000 K.
"""
import math

import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W
from test_oracle_sampler_sets import multiplicity

KB = 86.17333262


def cartesian_energy(M, epi, sigma):
    S = epi.shape[0]
    V = epi.astype(np.int64)
    twice = 0
    for s in range(S):
        twice += int((M[s] * V[s][sigma[:, None], sigma[None, :]]).sum())
    assert twice % 2 == 0
    return twice // 2


def acceptance_probability(orc, dE, tab):
    """Fraction of the 2^32 draws u that the oracle accepts for an energy
    change dE: the test is u < threshold, so the accepted draws are a
    prefix; bisection finds its length."""
    n = 1 << 32
    lo, hi = 0, n                       # accepted count in [lo, hi]
    while lo < hi:
        mid = (lo + hi) // 2            # is draw `mid` accepted?
        if orc.accept(dE, mid, tab):
            lo = mid + 1
        else:
            hi = mid
    return lo / n


@pytest.mark.parametrize("lattice,L", [(0, (4, 5, 3)), (1, (3, 4, 3))])
@pytest.mark.parametrize("T", [1.0, 300.0, 800.0, 2000.0, 5000.0])
def test_single_trial_detailed_balance(orc, lattice, L, T):
    rng = np.random.default_rng(int(T) * 7 + lattice)
    K, S = 5, 3
    epi = W.epi_table(S, K, 30.0 if T > 100 else 0.2, rng)
    M = multiplicity(L, lattice, S)
    N = M.shape[1]
    tab = orc.thresholds(T)
    nfirst = 8 if lattice == 0 else 12
    checked = 0
    for _ in range(6):
        sigma = W.configuration(W.equiatomic(K, N), rng)
        E0 = cartesian_energy(M, epi, sigma)
        assert E0 == orc.energy(L, epi, sigma, lattice)
        for i in rng.choice(N, size=5, replace=False):
            for k in range(nfirst):
                j = orc.neighbour(L, int(i), k, lattice)
                if sigma[i] == sigma[j]:
                    continue
                dE = orc.delta_energy(L, epi, sigma, int(i), j, lattice)
                swapped = sigma.copy()
                swapped[i], swapped[j] = sigma[j], sigma[i]
                assert dE == cartesian_energy(M, epi, swapped) - E0
                assert orc.delta_energy(L, epi, swapped, j, int(i), lattice) == -dE
                a_fwd = acceptance_probability(orc, dE, tab)
                a_rev = acceptance_probability(orc, -dE, tab)
                resolution = 2.0 ** -32
                x = -dE / (KB * T)
                # pi(s) a(s->s') - pi(s') a(s'->s), scaled by pi(s) (both
                # probabilities are 1 for downhill moves)
                lhs, rhs = a_fwd, math.exp(min(x, 700.0)) * a_rev
                if dE > 0:
                    assert a_rev == 1.0
                    assert abs(a_fwd - math.exp(x)) <= resolution + 1e-12 * math.exp(x)
                elif dE < 0:
                    assert a_fwd == 1.0
                    assert abs(a_rev - math.exp(-x)) <= resolution + 1e-12 * math.exp(-x)
                else:
                    assert a_fwd == a_rev == 1.0
                assert abs(lhs - rhs) <= (resolution + 1e-12) * max(1.0, math.exp(min(x, 700.0)))
                checked += 1
    assert checked >= 60
