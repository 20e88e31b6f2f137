"""GPU parity of smcx_sweep_observed: sweeps with the pair counts (the SRO
numerators, Eq. (SRO)) and the energy recorded after every sweep on the
device, equal to the oracle's per-sweep trace entry by entry, across the
256-sweep read-back chunks, on both lattices and under an anneal schedule."""
import sys

import numpy as np
import pytest

from paper_2509_20949_amd import workloads as W

pytestmark = pytest.mark.gpu
BCC, FCC = 0, 1


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


@pytest.mark.parametrize("lattice,L,K,S,n,block", [
    (BCC, (16, 16, 16), 5, 3, 20, (12, 12, 12)),
    (BCC, (8, 9, 10), 4, 2, 300, (4, 5, 6)),     # two read-back chunks (256 + 44)
    (FCC, (8, 8, 8), 5, 3, 12, (12, 12, 12)),
])
def test_observed_sweeps_equal_oracle_trace(smcx, orc, lattice, L, K, S, n, block):
    T = W.linear_anneal(2000.0, 600.0, n)
    job = W.lattice_job(L, K, S, 30.0, T, stream=700 + n + lattice, name="observed", lattice=lattice)
    note(f"observed sweeps lattice={lattice} L={L} K={K} S={S} n={n}")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, float(T[0]), block=block, lattice=lattice)
    ref = orc.OracleState(job.L, block, job.epi, job.sigma, job.seed, lattice=lattice)
    try:
        lat.set_schedule(T)
        E, counts = lat.sweep_observed(n)
        E_ref, C_ref = ref.sweep(T, n, trace_E=True, trace_counts=True)
        assert np.array_equal(E, E_ref)
        assert np.array_equal(counts, C_ref)
        assert np.array_equal(lat.config(), ref.sigma)
        assert lat.energy() == int(E[-1])
        # a zero-length call does nothing
        E0, C0 = lat.sweep_observed(0)
        assert E0.size == 0 and C0.size == 0
        assert lat.stats()["sweeps"] == n
    finally:
        lat.close()
