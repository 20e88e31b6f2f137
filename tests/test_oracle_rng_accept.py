"""Pins of the oracle's random numbers and Metropolis acceptance.

Philox: the oracle builds its 4x32 and 4x64 generators from one round body;
numpy.random.Philox (an independent implementation of the 4x64-10 variant of
Salmon et al., SC'11) pins that body.  Statistical checks cover the 4x32
instance used for trials.

Acceptance: Eq. (3) of the paper (min(1, exp(-beta dE))).  The table product
must equal 2^32 exp(-beta dE) to within a few ulp, dE <= 0 always accepts.
"""
import math

import numpy as np
import pytest


def _numpy_philox_block(ctr, key):
    # numpy advances its 256-bit counter before producing a block
    c = [int(x) for x in ctr]
    assert c[0] >= 1
    c[0] -= 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_round_body_matches_numpy(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        ctr = rng.integers(1, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr[1:] |= rng.integers(0, 2, size=3, dtype=np.uint64) << np.uint64(63)
        got = orc.philox4x64(ctr, key)
        want = _numpy_philox_block(ctr, key)
        assert np.array_equal(got, want)


def test_philox4x32_avalanche(orc):
    """Flipping any single input bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(5)
    flips = []
    for _ in range(64):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
        base = orc.philox4x32(ctr, key)
        for w in range(6):
            bit = int(rng.integers(0, 32))
            c2, k2 = ctr.copy(), key.copy()
            if w < 4:
                c2[w] ^= np.uint32(1 << bit)
            else:
                k2[w - 4] ^= np.uint32(1 << bit)
            out = orc.philox4x32(c2, k2)
            flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out)))
    mean = float(np.mean(flips))
    # 128 fair bits: mean 64, sd of the mean 8/sqrt(384) ~ 0.41
    assert abs(mean - 64.0) < 2.5


def test_philox4x32_uniform_words(orc):
    """Chi-square of the top byte of each output word over sequential counters."""
    n = 20000
    counts = np.zeros((4, 256), np.int64)
    bits = np.zeros((4, 32), np.int64)
    for c in range(n):
        out = orc.philox4x32([c, 0, 7, 3], [0x1234, 0x5678])
        for w in range(4):
            counts[w, int(out[w]) >> 24] += 1
            for b in range(32):
                bits[w, b] += (int(out[w]) >> b) & 1
    exp = n / 256.0
    for w in range(4):
        chi2 = float(((counts[w] - exp) ** 2 / exp).sum())
        # 255 dof: mean 255, sd ~22.6; 6 sd bound
        assert chi2 < 255 + 6 * 22.6
    # every bit fair: sd = sqrt(n)/2 ~ 70.7
    assert np.all(np.abs(bits - n / 2) < 6 * math.sqrt(n) / 2)


KB = 86.17333262  # micro-eV / K


@pytest.mark.parametrize("T", [1.0, 300.0, 800.0, 1000.0, 2000.0, 5000.0])
def test_threshold_table_is_exp(orc, T):
    tab = orc.thresholds(T)
    beta = 1.0 / (KB * T)
    rng = np.random.default_rng(int(T))
    dEs = np.concatenate([np.arange(1, 600), rng.integers(1, 1 << 24, 3000)])
    for dE in dEs:
        dE = int(dE)
        thr = (tab[512 + (dE >> 16)] * tab[256 + ((dE >> 8) & 255)]) * tab[dE & 255]
        want = math.ldexp(math.exp(-beta * dE), 32)
        # exp(-x) carries the rounding of x = beta*dE: relative error ~ x*eps
        x = beta * dE
        if want > 1e-290:
            assert abs(thr - want) <= (8.0 + 4.0 * x) * 2.0**-52 * want
        else:
            assert thr < 1e-280


def test_accept_rule_edges(orc):
    tab = orc.thresholds(800.0)
    beta = 1.0 / (KB * 800.0)
    for u in (0, 1, 2**31, 2**32 - 1):
        assert orc.accept(0, u, tab)
        assert orc.accept(-12345, u, tab)
        assert not orc.accept(1 << 24, u, tab)
        assert not orc.accept((1 << 24) + 5, u, tab)
    # dE with exp(-beta dE) = 1/2: accept exactly the lower half of the draws
    dE = int(round(math.log(2.0) / beta))
    p = math.exp(-beta * dE)
    cut = math.ldexp(p, 32)
    u_lo = int(math.floor(cut)) - 1
    u_hi = int(math.ceil(cut)) + 1
    assert orc.accept(dE, u_lo, tab)
    assert not orc.accept(dE, u_hi, tab)


def test_accept_frequency_matches_boltzmann_factor(orc):
    """Eq. (3): acceptance frequency of uphill moves is exp(-beta dE)."""
    tab = orc.thresholds(1000.0)
    beta = 1.0 / (KB * 1000.0)
    rng = np.random.default_rng(3)
    u = rng.integers(0, 2**32, size=40000, dtype=np.uint64)
    for dE in (1000, 20000, 60000, 150000):
        acc = sum(orc.accept(dE, int(x), tab) for x in u[:10000])
        p = math.exp(-beta * dE)
        sd = math.sqrt(10000 * p * (1 - p)) + 1e-9
        assert abs(acc - 10000 * p) < 6 * sd + 1
