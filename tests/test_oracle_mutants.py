"""Planted mistakes in the oracle are caught by its pins.

Each case copies oracle/smcx_oracle.c, plants one plausible mistake by a
text substitution, compiles the copy into a separate library, and runs a
few of the oracle's own pin tests against it through ``oracle.using``.  At
least one pin must fail for every mistake.  The unmodified oracle passes
the same pins (``test_unmodified_oracle_passes``).  Nothing here touches the
HIP library.  The mistakes are planted only in temporary copies of the
oracle, on the CPU.
"""
import os

import numpy as np
import pytest

import test_oracle_detailed_balance as DB
import test_oracle_energy as EN
import test_oracle_philox_kat as KAT
import test_oracle_rng_accept as RA
import test_oracle_sampler_sets as SETS
import test_oracle_schedule as SCH
from paper_2509_20949_amd import workloads as W


# ---- pins, each a call of an existing test with fixed parameters -------------
def pin_delta_energy(orc):
    for L in ((4, 4, 4), (5, 7, 6)):
        EN.test_delta_energy_equals_full_difference(orc, L, 3, 5)


def pin_closed_forms(orc):
    for S in (1, 2, 3):
        EN.test_uniform_lattice_closed_form(orc, S)
    EN.test_b2_ordered_binary_closed_form(orc, (4, 4, 4))


def pin_acceptance(orc):
    for T in (300.0, 2000.0):
        RA.test_threshold_table_is_exp(orc, T)
    RA.test_accept_frequency_matches_boltzmann_factor(orc)


def pin_detailed_balance(orc):
    for T in (800.0, 5000.0):
        DB.test_single_trial_detailed_balance(orc, 0, (4, 5, 3), T)


def pin_schedule(orc):
    SCH.test_conflict_free_small_blocks(orc, (8, 8, 8))


def pin_philox(orc):
    for ctr, key, want in KAT.RANDOM123_KAT:
        KAT.test_published_known_answers(orc, ctr, key, want)


def pin_sro(orc):
    EN.test_sro_sum_rule_and_symmetry(orc)
    EN.test_sro_b2_hand_values(orc)


def pin_sampler(orc):
    """The 64-site exact enumeration with two-trial sets, shortened."""
    rng = np.random.default_rng(64)
    epi = W.epi_table(3, 2, 30.0, rng)
    SETS.check_chain(orc, (8, 2, 2), (4, 2, 2), 0, epi, 4, 1000.0, seed=641, n_sweeps=20000)


MUTANTS = {
    "partner neighbourhood dropped from dE": (
        "        if (m != i) dE += epi[(s * K + si) * K + sigma[m]] - epi[(s * K + sj) * K + sigma[m]];\n",
        "        (void)m;\n",
        [pin_delta_energy, pin_detailed_balance]),
    "energy not halved": (
        "    return twiceE / 2;\n",
        "    return twiceE;\n",
        [pin_closed_forms]),
    "beta ten times too large": (
        "    double beta = 1.0 / (kB_ueV_per_K * T);\n",
        "    double beta = 10.0 / (kB_ueV_per_K * T);\n",
        [pin_acceptance, pin_detailed_balance]),
    "wrong byte of dE indexes the middle table": (
        "    double thr = (tab[512 + (dE >> 16)] * tab[256 + ((dE >> 8) & 255)]) * tab[dE & 255];\n",
        "    double thr = (tab[512 + (dE >> 16)] * tab[256 + ((dE >> 7) & 255)]) * tab[dE & 255];\n",
        [pin_detailed_balance]),
    "threshold halved": (
        "    return (double)u < thr;\n",
        "    return (double)u < 0.5 * thr;\n",
        [pin_acceptance, pin_detailed_balance]),
    "sub-colours from residues mod 2 along x": (
        "                uint8_t q = (uint8_t)((((lz % 3) * 3 + ly % 3) * 3 + lx % 3) * nsub);\n",
        "                uint8_t q = (uint8_t)((((lz % 3) * 3 + ly % 3) * 3 + lx % 2) * nsub);\n",
        [pin_schedule]),
    "Philox Weyl increment off by two": (
        "               0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)\n",
        "               0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE87u)\n",
        [pin_philox]),
    "SRO normalised by the wrong species": (
        "                double P = (double)c[(m * K + pc) * K + p] / ((double)or_shell_size(lat, m) * (double)Np[pc]);\n",
        "                double P = (double)c[(m * K + pc) * K + p] / ((double)or_shell_size(lat, m) * (double)Np[p]);\n",
        [pin_sro]),
    "minority atoms propose only -x partners": (
        "                    j = or_neighbour(0, L, i, dir);\n",
        "                    j = or_neighbour(0, L, i, sigma[i] == 1 ? (dir & 6) : dir);\n",
        [pin_sampler]),
}


@pytest.fixture(scope="module")
def source(orc):
    path = os.path.join(os.path.dirname(orc.__file__), "smcx_oracle.c")
    with open(path) as f:
        return f.read()


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(orc, source, tmp_path, name):
    old, new, pins = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = orc.build(force=True, src=str(src), out=str(tmp_path / "libmutant.so"))
    failed = []
    with orc.using(lib):
        for pin in pins:
            try:
                pin(orc)
            except AssertionError:
                failed.append(pin.__name__)
    assert failed, f"no pin caught the planted mistake '{name}'"


def test_unmodified_oracle_passes(orc):
    pins = {p for _, _, ps in MUTANTS.values() for p in ps}
    for pin in sorted(pins, key=lambda p: p.__name__):
        pin(orc)
