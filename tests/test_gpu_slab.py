"""GPU tests of z-slabs (lattice parallelism with ghost layers): the slab
kernel with its halo planes in the caller's buffer.

* One slab that is the whole lattice exchanges halos with itself
  (smcx_sweep): bit-identical to the oracle on the periodic lattice with the
  z-slab schedule (block grid not shifted along z).
* Several slabs of one lattice, each its own context and buffer, stepped one
  colour phase at a time (smcx_slab_phase) with the halo planes exchanged
  between them by device copies between phases: together bit-identical to
  the oracle on the whole lattice.  This is the decomposition one GPU per
  slab would run (there the copies are transfers between GPUs); here all
  slabs share one GPU.
"""
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


class Slabs:
    """G slabs of Lz planes each stacked along z, one context and buffer per
    slab (planes: 2 halo, Lz own, 2 halo), on one stream."""

    def __init__(self, smcx, job, G, B, T):
        import torch
        self.smcx, self.job, self.G = smcx, job, G
        Lx, Ly, Lz_all = job.L
        assert Lz_all % G == 0
        self.Lz = Lz_all // G
        self.P = 2 * Lx * Ly
        self.stream = torch.cuda.Stream()
        planes = job.sigma.reshape(Lz_all, self.P)
        self.bufs, self.ctxs = [], []
        with torch.cuda.stream(self.stream):
            for g in range(G):
                idx = [(g * self.Lz + k) % Lz_all for k in range(-2, self.Lz + 2)]
                self.bufs.append(torch.from_numpy(np.ascontiguousarray(planes[idx])).to("cuda:0"))
        self.stream.synchronize()
        for g in range(G):
            d = smcx.make_desc((Lx, Ly, self.Lz), job.K, job.S, B, job.seed)
            self.ctxs.append(smcx.smcx_create_slab(d, self.bufs[g].data_ptr(), g * self.Lz, job.epi, T,
                                                   self.stream.cuda_stream))

    def own(self, g):
        return self.bufs[g][2:self.Lz + 2]

    def exchange_before(self):
        import torch
        G, Lz = self.G, self.Lz
        with torch.cuda.stream(self.stream):
            for g in range(G):
                self.bufs[g][0:2].copy_(self.own((g - 1) % G)[Lz - 2:Lz])
                self.bufs[g][Lz + 2:Lz + 4].copy_(self.own((g + 1) % G)[0:2])

    def exchange_after(self, colour):
        import torch
        G, Lz = self.G, self.Lz
        with torch.cuda.stream(self.stream):
            for g in range(G):
                if (colour >> 2) & 1 == 0:   # lowest blocks ran: plane below the slab returns to slab g-1
                    self.own((g - 1) % G)[Lz - 1].copy_(self.bufs[g][1])
                else:                        # highest blocks ran: plane above returns to slab g+1
                    self.own((g + 1) % G)[0].copy_(self.bufs[g][Lz + 2])

    def sweep(self):
        for colour in range(8):
            self.exchange_before()
            for c in self.ctxs:
                self.smcx.smcx_slab_phase(c, 1)
            self.exchange_after(colour)

    def config(self):
        self.stream.synchronize()
        return np.concatenate([self.own(g).cpu().numpy().ravel() for g in range(self.G)])

    def delta_energy(self, E0):
        return sum(self.smcx.smcx_energy(c) for c in self.ctxs) - E0

    def close(self):
        for c in self.ctxs:
            self.smcx.smcx_destroy(c)
        self.ctxs = []


def compare(got, ref, what):
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{what}: {bad.size} sites differ, first {bad[:8]}")


@pytest.mark.parametrize("L,B", [((13, 12, 16), (4, 4, 4)), ((9, 10, 24), (3, 5, 12)), ((20, 17, 12), (12, 12, 6))])
def test_single_slab_equals_oracle(smcx, orc, L, B):
    job = W.lattice_job(L, 5, 3, 30.0, np.full(6, 950.0), stream=140, name="slab1")
    note(f"single slab L={L} B={B}")
    s = Slabs(smcx, job, 1, B, 950.0)
    ref = orc.OracleState(job.L, B, job.epi, job.sigma, job.seed, fixed_z=True)
    try:
        assert smcx.smcx_energy(s.ctxs[0]) == int(ref.E[0])
        for t in range(6):
            smcx.smcx_sweep(s.ctxs[0], 1)
            ref.sweep(950.0, 1)
            compare(s.config(), ref.sigma, f"sweep {t + 1}")
            assert smcx.smcx_energy(s.ctxs[0]) == int(ref.E[0])
        assert smcx.smcx_energy_recompute(s.ctxs[0]) == int(ref.E[0])
        assert smcx.smcx_get_stats(s.ctxs[0])["accepted"] == int(ref.accepted[0]) > 0
    finally:
        s.close()


@pytest.mark.parametrize("L,G,B", [((11, 10, 24), 2, (4, 4, 6)), ((12, 9, 36), 3, (12, 4, 6))])
def test_stacked_slabs_equal_whole_lattice(smcx, orc, L, G, B):
    assert orc.axis_blocks(L[2], B[2]) == G * orc.axis_blocks(L[2] // G, B[2])   # same z blocks
    job = W.lattice_job(L, 4, 3, 30.0, np.full(5, 1100.0), stream=141, name="slabs")
    note(f"{G} slabs of L={L} B={B}")
    s = Slabs(smcx, job, G, B, 1100.0)
    ref = orc.OracleState(job.L, B, job.epi, job.sigma, job.seed, fixed_z=True)
    E0 = int(ref.E[0])
    E0_slabs = sum(smcx.smcx_energy(c) for c in s.ctxs)
    try:
        for t in range(5):
            s.sweep()
            ref.sweep(1100.0, 1)
            compare(s.config(), ref.sigma, f"sweep {t + 1}")
            assert s.delta_energy(E0_slabs) == int(ref.E[0]) - E0
        acc = sum(smcx.smcx_get_stats(c)["accepted"] for c in s.ctxs)
        assert acc == int(ref.accepted[0]) > 0
        with pytest.raises(smcx.SmcxError) as e:   # no whole sweeps while a sweep is half done
            smcx.smcx_slab_phase(s.ctxs[0], 3)
            smcx.smcx_sweep(s.ctxs[0], 1)
        assert e.value.status == smcx.E_STATE
    finally:
        s.close()


def test_slab_512x512x64_equals_oracle(smcx, orc):
    """One GPU's share of the 512^3 benchmark lattice cut into 8 z-slabs, at
    its real shape (512 x 512 x 64 cells, 33,554,432 sites), as a slab that
    exchanges halos with itself: bit-identical to the oracle."""
    job = W.lattice_job((512, 512, 64), 5, 3, 30.0, np.full(3, 800.0), dirichlet=5.0, stream=3,
                        name="slab512x512x64")
    B = (12, 12, 11)
    note(f"slab {job.L} B={B}")
    s = Slabs(smcx, job, 1, B, 800.0)
    ref = orc.OracleState(job.L, B, job.epi, job.sigma, job.seed, fixed_z=True)
    try:
        for t in range(3):
            smcx.smcx_sweep(s.ctxs[0], 1)
            ref.sweep(800.0, 1)
            compare(s.config(), ref.sigma, f"sweep {t + 1}")
            assert smcx.smcx_energy(s.ctxs[0]) == int(ref.E[0])
            note(f"  sweep {t + 1} ok")
    finally:
        s.close()


def test_eight_slabs_of_the_benchmark_lattice_equal_oracle(smcx, orc):
    """The 512^3 benchmark lattice as 8 slabs of 512 x 512 x 64 (the split
    over 8 GPUs, all on this one), halos exchanged between colour phases:
    configuration and total energy change equal to the oracle's run of the
    whole lattice after each of two sweeps.  B_z = 11 gives each slab 6
    z-blocks and the whole lattice 48, with the same bounds."""
    job = W.config3(n_sweeps=1)
    B = (12, 12, 11)
    assert orc.axis_blocks(512, 11) == 8 * orc.axis_blocks(64, 11)
    note(f"8 slabs of {job.L}, B={B}")
    s = Slabs(smcx, job, 8, B, 800.0)
    ref = orc.OracleState(job.L, B, job.epi, job.sigma, job.seed, fixed_z=True)
    E0 = int(ref.E[0])
    E0_slabs = sum(smcx.smcx_energy(c) for c in s.ctxs)
    try:
        for t in range(2):
            s.sweep()
            ref.sweep(800.0, 1)
            compare(s.config(), ref.sigma, f"sweep {t + 1}")
            assert s.delta_energy(E0_slabs) == int(ref.E[0]) - E0
            note(f"  sweep {t + 1} ok")
    finally:
        s.close()
