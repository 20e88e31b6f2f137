"""GPU parity of the pair counts N_m[p'][p] (the energy recompute and the
Warren-Cowley SRO, Eq. (SRO)) on lattices of 2^22 cells and more, where the
library counts with bit planes: equal to the oracle's counts entry by entry,
with ragged x/y tiles, a z extent that leaves a short last z range, both
lattices, a composition with an absent species, and lattices narrower than
a tile (rows or x cells that wrap within one tile)."""
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


CASES = [
    # lattice, cells per axis, K, S, composition fractions (None: equiatomic)
    (BCC, (160, 162, 170), 5, 3, None),
    (BCC, (512, 256, 33), 3, 2, None),
    (BCC, (130, 131, 260), 2, 1, None),
    (BCC, (124, 186, 190), 5, 3, np.array([0.5, 0.3, 0.0, 0.15, 0.05])),
    (FCC, (130, 132, 250), 5, 3, None),
    (FCC, (200, 150, 141), 4, 2, None),
    # fewer rows than a tile's 64 bits (rows wrap several times in a word),
    # and fewer cells along x than a wavefront's lanes
    (BCC, (40000, 8, 14), 5, 3, None),
    (FCC, (6, 600, 1200), 5, 3, None),
]


@pytest.mark.parametrize("lattice,L,K,S,comp", CASES)
def test_pair_counts_large_lattices(smcx, orc, lattice, L, K, S, comp):
    assert L[0] * L[1] * L[2] >= 1 << 22
    counts = None if comp is None else W.counts_from_fractions(comp, W.n_sites(L, lattice))
    job = W.lattice_job(L, K, S, 30.0, np.full(1, 900.0), comp=counts, stream=600 + K + 10 * lattice,
                        name=f"pc{lattice}", lattice=lattice)
    note(f"pair counts lattice={lattice} L={L} K={K} S={S}")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 900.0, lattice=lattice)
    try:
        _, counts = lat.sro()
        ref = orc.pair_counts(job.L, S, K, job.sigma, lattice)
        assert np.array_equal(counts, ref)
        # and after a sweep (a configuration the sampler produced)
        lat.sweep(1)
        _, counts = lat.sro()
        ref = orc.pair_counts(job.L, S, K, lat.config(), lattice)
        assert np.array_equal(counts, ref)
    finally:
        lat.close()
