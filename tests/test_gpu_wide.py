"""GPU parity on large lattices.  Where cell indices leave the 24-bit
multiplier (Lx * Ly >= 2^24) the kernels switch to 64-bit addressing (staging
rows, write-back rows and the Philox base cells); the 512^3 benchmark lattice
is checked in the launch configuration the benchmark times."""
import os
import sys

import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def smcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20949_amd import smcx as m
    m.lib()
    return m


@pytest.fixture(scope="module", autouse=True)
def oracle_threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))
    yield
    orc.set_threads(1)


@pytest.mark.parametrize("lattice", [0, 1])
def test_wide_rows_use_64_bit_addressing(smcx, orc, lattice):
    L = (4096, 4097, 4)
    assert L[0] * L[1] >= 1 << 24
    job = W.lattice_job(L, 3, 2, 30.0, np.full(2, 1500.0), stream=400 + lattice, name=f"wide{lattice}",
                        lattice=lattice)
    note(f"wide rows lattice={lattice} L={L} sites={job.N}")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 1500.0, lattice=lattice)
    ref = orc.OracleState(job.L, (12, 12, 12), job.epi, job.sigma, job.seed, lattice=lattice)
    try:
        assert lat.energy() == int(ref.E[0])
        for t in range(2):
            lat.sweep(1)
            ref.sweep(1500.0, 1)
            got = lat.config()
            if not np.array_equal(got, ref.sigma):
                bad = np.nonzero(got != ref.sigma)[0]
                raise AssertionError(f"config differs after sweep {t + 1}: {bad.size} sites, first {bad[:8]}")
            assert lat.energy() == int(ref.E[0])
        assert lat.stats()["accepted"] == int(ref.accepted[0]) > 0
    finally:
        lat.close()


def test_benchmark_lattice_first_sweeps_equal_oracle(smcx, orc):
    """The 512^3 benchmark lattice (268,435,456 sites, K = 5 Dirichlet(5),
    S = 3, 800 K) in the launch configuration the benchmark times (B = 12):
    configuration, energy and accepted count equal to the oracle after each
    of the first five sweeps; then running energy = full recompute and the
    composition unchanged after ten more."""
    job = W.config3(n_sweeps=1)
    note(f"benchmark lattice L={job.L} sites={job.N}")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 800.0, block=(12, 12, 12))
    ref = orc.OracleState(job.L, (12, 12, 12), job.epi, job.sigma, job.seed)
    try:
        assert lat.energy() == int(ref.E[0])
        for t in range(5):
            note(f"  sweep {t + 1}")
            lat.sweep(1)
            ref.sweep(800.0, 1)
            got = lat.config()
            if not np.array_equal(got, ref.sigma):
                bad = np.nonzero(got != ref.sigma)[0]
                raise AssertionError(f"config differs after sweep {t + 1}: {bad.size} sites, first {bad[:8]}")
            assert lat.energy() == int(ref.E[0])
            assert lat.stats()["accepted"] == int(ref.accepted[0])
        lat.sweep(10)
        assert lat.energy() == lat.energy_recompute()
        assert np.array_equal(np.bincount(lat.config(), minlength=job.K), np.bincount(job.sigma, minlength=job.K))
    finally:
        lat.close()
