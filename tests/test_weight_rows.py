"""CPU checks of the pair-weight rows the library builds.  This is host logic
that both sweep kernels read.

Each row form is checked: byte-dot digits, the last species folded in, and
full fields.  The kernel's weighing of packed neighbour counts is emulated
on the rows, in wrap-around 32-bit integers, and must give the energy change
of a swap computed directly from the pair energies.  A swap of species a at
site i with species b at its first neighbour j changes only the bonds of i
and j other than the i-j bond itself (Section "Monte Carlo simulation",
Eq. (3); the pairwise EPI model of Section "Results and discussion").
"""
import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W

BCC, FCC = 0, 1
Z = {BCC: (8, 6, 12), FCC: (12, 6, 24)}
DOT, FOLDED, FULL = 2, 1, 0


@pytest.fixture(scope="module")
def smcx():
    from paper_2509_20949_amd import smcx as m
    m.lib()
    return m


def to_int32(x):
    return ((int(x) + (1 << 31)) % (1 << 32)) - (1 << 31)


def direct_dE(epi, a, b, ni, nj):
    """ni[s], nj[s]: species of the neighbours of i and j in shell s; entry 0
    of shell 1 is the partner (j, species b, around i; i, species a, around j)."""
    dE = 0
    for s in range(len(ni)):
        for k, p in enumerate(ni[s]):
            if s == 0 and k == 0:
                continue
            dE += int(epi[s, b, p]) - int(epi[s, a, p])
        for k, p in enumerate(nj[s]):
            if s == 0 and k == 0:
                continue
            dE += int(epi[s, a, p]) - int(epi[s, b, p])
    return dE


def kernel_dE(form, row, kmax, S, lattice, ci, cj):
    """ci[s][p], cj[s][p]: species counts per shell (partner included), as the
    kernels' packed histograms hold them."""
    row = [int(v) for v in row]
    if form == DOT:
        acc = row[3 * S]
        for s in range(S):
            d = [32 + ci[s][p] - cj[s][p] if p < kmax - 1 else 32 for p in range(4)]
            for k in range(3):
                word = row[3 * s + k] & 0xFFFFFFFF
                digits = [((word >> (8 * p)) & 255) - (256 if (word >> (8 * p)) & 128 else 0) for p in range(4)]
                acc += (1 << (8 * k)) * sum(d[p] * digits[p] for p in range(4))
        return to_int32(acc)
    bias = 32 if lattice == FCC else (16 if kmax <= 6 else 0)
    nf = kmax - 1 if form == FOLDED else kmax
    acc = row[S * kmax]
    for s in range(S):
        for p in range(nf):
            acc += (bias + ci[s][p] - cj[s][p]) * row[s * kmax + p]
    return to_int32(acc)


def check_rows(smcx, lattice, K, S, epi, expect_form, rng, n_cases=300):
    form, rows = smcx.smcx_weight_rows(lattice, K, S, epi)
    assert form == expect_form
    kmax = int(round(np.sqrt(rows.shape[0])))
    for _ in range(n_cases):
        a, b = int(rng.integers(K)), int(rng.integers(K))
        ni = [list(rng.integers(0, K, Z[lattice][s])) for s in range(S)]
        nj = [list(rng.integers(0, K, Z[lattice][s])) for s in range(S)]
        ni[0][0], nj[0][0] = b, a
        ci = [np.bincount(ni[s], minlength=kmax) for s in range(S)]
        cj = [np.bincount(nj[s], minlength=kmax) for s in range(S)]
        got = kernel_dE(form, rows[a * kmax + b], kmax, S, lattice, ci, cj)
        assert got == direct_dE(epi, a, b, ni, nj), (lattice, K, S, a, b)


@pytest.mark.parametrize("lattice,K,S,form", [(BCC, 5, 3, DOT), (BCC, 2, 1, DOT), (BCC, 3, 2, DOT), (BCC, 4, 3, DOT),
                                              (BCC, 6, 3, FOLDED), (BCC, 8, 2, FOLDED), (FCC, 5, 3, DOT),
                                              (FCC, 3, 2, DOT), (FCC, 2, 1, DOT)])
def test_rows_reproduce_direct_energy_change(smcx, lattice, K, S, form):
    job = W.lattice_job((4, 4, 4), K, S, 30.0, np.full(1, 800.0), stream=500 + 10 * K + S, lattice=lattice)
    check_rows(smcx, lattice, K, S, job.epi, form, np.random.default_rng(K * 10 + S + lattice))


@pytest.mark.parametrize("lattice,K", [(BCC, 4), (BCC, 5), (FCC, 5)])
def test_extreme_pair_energies_take_full_rows(smcx, lattice, K):
    """+-(2^22 - 1) micro-eV put the folded weights outside three signed
    base-256 digits: the rows fall back to full fields, still exact."""
    rng = np.random.default_rng(K + 7 * lattice)
    S = 3
    v = rng.choice([-(1 << 22) + 1, (1 << 22) - 1, 0, 123456], size=(S, K, K)).astype(np.int32)
    epi = np.triu(v) + np.transpose(np.triu(v, 1), (0, 2, 1))
    check_rows(smcx, lattice, K, S, epi, FULL, rng)


def test_rows_reject_bad_tables(smcx):
    epi = np.zeros((1, 3, 3), np.int32)
    epi[0, 0, 1] = 5                      # not symmetric
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_weight_rows(BCC, 3, 1, epi)
    assert e.value.status == smcx.E_INVALID
    with pytest.raises(smcx.SmcxError):
        smcx.smcx_weight_rows(FCC, 6, 1, np.zeros((1, 6, 6), np.int32))   # FCC kernels take K <= 5
