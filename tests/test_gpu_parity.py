"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

The bar is bit-for-bit: species array and int64 energy after every sweep,
the accepted count, pair counts / SRO, the device's Philox words and FP64
threshold products.  Inputs come from the seeded generators in
paper_2509_20949_amd.workloads; the oracle never sees library output.
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


def run_parity(smcx, orc, job, block, n_sweeps, T=None, every=1, check_sro=False):
    """Advance GPU and oracle side by side; compare after every `every` sweeps."""
    T = job.T if T is None else T
    note(f"{job.name or 'lattice'} L={job.L} K={job.K} S={job.S} B={block} sweeps={n_sweeps}")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, float(T[0]), block=block)
    ref = orc.OracleState(job.L, block, job.epi, job.sigma, job.seed)
    try:
        if len(set(np.asarray(T[:n_sweeps]).tolist())) > 1:
            lat.set_schedule(T[:n_sweeps])
        assert lat.energy() == int(ref.E[0])
        done = 0
        while done < n_sweeps:
            k = min(every, n_sweeps - done)
            lat.sweep(k)
            ref.sweep(T[done:done + k], k)
            done += k
            got = lat.config()
            if not np.array_equal(got, ref.sigma):
                bad = np.nonzero(got != ref.sigma)[0]
                raise AssertionError(f"config differs after sweep {done}: {bad.size} sites, first {bad[:8]}")
            assert lat.energy() == int(ref.E[0]), f"energy differs after sweep {done}"
            if check_sro:
                alpha, counts = lat.sro()
                a_ref, c_ref = orc.sro(job.L, job.S, job.K, ref.sigma)
                assert np.array_equal(counts, c_ref)
                assert np.array_equal(np.isnan(alpha), np.isnan(a_ref))
                assert np.allclose(alpha, a_ref, rtol=0, atol=1e-12, equal_nan=True)
        st = lat.stats()
        assert st["accepted"] == int(ref.accepted[0])
        if job.K > 1 and len(np.unique(job.sigma)) > 1:
            # the trajectory really moved (guards against two idle sides)
            assert st["accepted"] > 0 and not np.array_equal(ref.sigma, job.sigma)
        assert st["attempted"] == n_sweeps * job.N
        assert lat.energy_recompute() == int(ref.E[0])
        return lat.energy(), st
    finally:
        lat.close()


def test_device_philox_matches_oracle(smcx, orc):
    note("device philox")
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([0xDEADBEEF, 0x12345678], np.uint32)
    got = smcx.smcx_device_philox(ctr, key)
    for k in range(0, 4096, 37):
        assert np.array_equal(got[k], orc.philox4x32(ctr[k], key))
    # the published Random123 known answers, on the device itself
    from test_oracle_philox_kat import RANDOM123_KAT
    for c, k, want in RANDOM123_KAT:
        out = smcx.smcx_device_philox(np.array([c], np.uint32), np.array(k, np.uint32))
        assert [int(v) for v in out[0]] == list(want)


@pytest.mark.parametrize("T", [1.0, 250.0, 800.0, 2000.0, 5000.0])
def test_device_fp64_threshold_products(smcx, orc, T):
    """The device's FP64 products of the byte tables equal the oracle's bits
    (IEEE round to nearest, no contraction), including tiny and denormal
    products at low temperature."""
    note(f"device thresholds T={T}")
    rng = np.random.default_rng(int(T))
    dE = np.concatenate([np.arange(1, 2000), rng.integers(1, 1 << 24, 20000),
                         [(1 << 24) - 1, 65535, 65536, 65537, 255, 256, 257]]).astype(np.int32)
    got = smcx.smcx_device_thresholds(T, dE)
    tab = orc.thresholds(T)
    want = np.array([(tab[512 + (e >> 16)] * tab[256 + ((e >> 8) & 255)]) * tab[e & 255] for e in dE.tolist()])
    assert got.tobytes() == want.tobytes()


@pytest.mark.parametrize("T", [1.0, 250.0, 800.0, 2000.0, 5000.0])
def test_device_accept_bounds_agree_with_table_test(smcx, orc, T):
    """The kernels decide an uphill swap without the threshold tables when dE
    lies outside (lo, hi]: every dE <= lo must pass the exact test of
    Eq. (3) (u < thr(dE) on the oracle's tables) and every dE > hi fail it.
    Checked next to both bounds for random and edge-case draws; the band in
    between stays a few micro-eV wide."""
    note(f"accept bounds T={T}")
    rng = np.random.default_rng(int(T) + 7)
    # any 32-bit word (the acceptance draw of both lattices), even and odd
    u = np.concatenate([rng.integers(1, 1 << 31, 40000) * 2, rng.integers(1, 1 << 32, 40000),
                        [1, 2, 3, 4, 5, 6, 8, 1 << 31, (1 << 32) - 1, (1 << 32) - 2, (1 << 32) - 4, 3 << 30,
                         (1 << 24) - 1, (1 << 24) + 1]]).astype(np.uint32)
    lo, hi = smcx.smcx_device_accept_bounds(T, u)
    tab = orc.thresholds(T)

    def passes(dE):   # exact test for 0 < dE < 2^24, vectorised like the oracle's expression
        e = dE.astype(np.int64)
        thr = (tab[512 + (e >> 16)] * tab[256 + ((e >> 8) & 255)]) * tab[e & 255]
        return u.astype(np.float64) < thr

    assert np.all(hi >= lo) and np.all(hi - lo <= 2 * 8 + 1)
    for k in range(4):
        d = lo.astype(np.int64) - k
        m = (d > 0) & (d < (1 << 24))
        assert np.all(passes(np.clip(d, 1, (1 << 24) - 1))[m]), (T, k)
        d = hi.astype(np.int64) + 1 + k
        m = (d > 0) & (d < (1 << 24))
        assert not np.any(passes(np.clip(d, 1, (1 << 24) - 1))[m]), (T, k)


@pytest.mark.parametrize("T", [1.0, 250.0, 800.0, 2000.0, 5000.0])
def test_accept_bounds_exhaustive(smcx, T):
    """Every 32-bit acceptance draw (all FCC draws, and the even BCC ones
    among them): the bounds the kernels decide with never contradict the
    exact FP64 table test of Eq. (3) at lo, lo - 1, hi + 1 or hi + 2, on the
    device's own table products (bit-equal to the oracle's, above).  The
    device's FP32 logarithm stays within the 2.0e-6 the bound derivation
    assumes, and the band that needs the table is at most 17 micro-eV wide."""
    note(f"exhaustive accept bounds T={T}")
    bad_lo, bad_hi, log_err, band = smcx.smcx_device_check_accept_bounds(T)
    assert bad_lo == 0 and bad_hi == 0, (bad_lo, bad_hi)
    assert 0.0 < log_err <= 2.0e-6, log_err
    assert band <= 17, band


def test_config1_parity_every_sweep(smcx, orc):
    job = W.config1(n_sweeps=100)
    run_parity(smcx, orc, job, (12, 12, 12), 100)


@pytest.mark.parametrize("block", [(2, 2, 2), (3, 4, 2), (4, 4, 4)])
def test_config1_parity_small_blocks(smcx, orc, block):
    job = W.config1(n_sweeps=30)
    run_parity(smcx, orc, job, block, 30)


def test_16cube_three_shells(smcx, orc):
    job = W.lattice_job((16, 16, 16), 5, 3, 30.0, np.full(40, 800.0), stream=31, name="bcc16_k5_s3")
    run_parity(smcx, orc, job, (12, 12, 12), 40, check_sro=True)


@pytest.mark.parametrize("L,block", [((13, 9, 22), (5, 4, 12)), ((4, 4, 4), (2, 2, 2)),
                                     ((5, 7, 31), (12, 3, 7)), ((26, 25, 27), (12, 12, 12)),
                                     ((37, 12, 9), (10, 6, 4))])
def test_ragged_lattices(smcx, orc, L, block):
    job = W.lattice_job(L, 3, 3, 40.0, np.full(12, 1100.0), stream=41, name="ragged")
    run_parity(smcx, orc, job, block, 12)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("S", [1, 2, 3])
def test_every_species_and_shell_count(smcx, orc, K, S):
    job = W.lattice_job((8, 9, 10), K, S, 25.0, np.full(5, 900.0), stream=50 + K, name=f"K{K}S{S}")
    run_parity(smcx, orc, job, (4, 5, 6), 5)


def test_extreme_interactions_and_temperatures(smcx, orc):
    rng = np.random.default_rng(9)
    K, S = 4, 3
    v = rng.choice([-(1 << 22) + 1, (1 << 22) - 1, 0, 123456], size=(S, K, K)).astype(np.int32)
    epi = np.triu(v) + np.transpose(np.triu(v, 1), (0, 2, 1))
    sigma = W.configuration(W.equiatomic(K, W.n_sites((10, 10, 10))), rng)
    for T in (1.0, 5000.0):
        job = W.Lattice((10, 10, 10), epi, sigma, 77, np.full(6, T), name=f"extreme T={T}")
        run_parity(smcx, orc, job, (5, 5, 5), 6)


def test_anneal_schedule_config2_full(smcx, orc):
    """64^3 quinary, 3 shells, the whole linear anneal 2000 K -> 600 K over
    1000 sweeps: after every sweep the configuration, the running energy and
    the pair counts / Warren-Cowley SRO equal the oracle's (the oracle's
    counts are taken inside its own sweep loop)."""
    job = W.config2(n_sweeps=1000)
    T = job.T
    note(f"config2 full anneal L={job.L} sweeps={T.size} T {T[0]:.0f} -> {T[-1]:.0f} K")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, float(T[0]), block=(12, 12, 12))
    ref = orc.OracleState(job.L, (12, 12, 12), job.epi, job.sigma, job.seed)
    try:
        lat.set_schedule(T)
        assert lat.energy() == int(ref.E[0])
        for k in range(T.size):
            lat.sweep(1)
            Et, Ct = ref.sweep(T[k:k + 1], 1, trace_E=True, trace_counts=True)
            got = lat.config()
            if not np.array_equal(got, ref.sigma):
                bad = np.nonzero(got != ref.sigma)[0]
                raise AssertionError(f"config differs after sweep {k + 1} (T = {T[k]:.1f} K): {bad.size} sites")
            assert lat.energy() == int(Et[0]) == int(ref.E[0]), f"energy differs after sweep {k + 1}"
            alpha, counts = lat.sro()
            assert np.array_equal(counts, Ct[0]), f"pair counts differ after sweep {k + 1}"
            if k % 100 == 99:
                a_ref, c_ref = orc.sro(job.L, job.S, job.K, ref.sigma)
                assert np.array_equal(c_ref, Ct[0])
                assert np.allclose(alpha, a_ref, rtol=0, atol=1e-12, equal_nan=True)
                note(f"  sweep {k + 1}: T = {T[k]:.1f} K, E = {int(ref.E[0])} micro-eV")
        st = lat.stats()
        assert st["accepted"] == int(ref.accepted[0]) > 0
        assert st["attempted"] == T.size * job.N
    finally:
        lat.close()


def test_checkpoint_resume_is_bit_identical(smcx, orc):
    job = W.lattice_job((12, 12, 12), 5, 3, 30.0, np.full(20, 900.0), stream=61, name="resume")
    note("resume")
    a = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 900.0)
    try:
        a.sweep(20)
        full = a.config()
        E_full = a.energy()
    finally:
        a.close()
    b = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 900.0)
    try:
        b.sweep(9)
        mid = b.config()
    finally:
        b.close()
    c = smcx.Lattice(job.L, job.epi, mid, job.seed, 900.0)
    try:
        smcx.smcx_set_state(c.ctx, mid, 9)
        c.sweep(11)
        assert np.array_equal(c.config(), full)
        assert c.energy() == E_full
    finally:
        c.close()


def test_zero_sweeps_and_uniform_lattice(smcx, orc):
    job = W.lattice_job((6, 6, 6), 1, 3, 30.0, np.full(3, 900.0), stream=62, name="uniform")
    note("uniform")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 900.0)
    try:
        E0 = lat.energy()
        lat.sweep(0)
        lat.sweep(3)
        assert lat.energy() == E0 and lat.stats()["accepted"] == 0
        assert np.array_equal(lat.config(), job.sigma)
    finally:
        lat.close()


def test_create_device_borrows_torch_memory(smcx, orc):
    import torch
    job = W.lattice_job((10, 11, 12), 4, 3, 30.0, np.full(6, 950.0), stream=63, name="device")
    note("create_device")
    dev = torch.from_numpy(job.sigma.copy()).to("cuda:0")
    stream = torch.cuda.Stream()
    d = smcx.make_desc(job.L, job.K, job.S, (5, 5, 5), job.seed)
    ctx = smcx.smcx_create_device(d, dev.data_ptr(), job.epi, 950.0, stream.cuda_stream)
    ref = orc.OracleState(job.L, (5, 5, 5), job.epi, job.sigma, job.seed)
    try:
        smcx.smcx_sweep(ctx, 6)
        ref.sweep(950.0, 6)
        smcx.smcx_synchronize(ctx)
        assert np.array_equal(dev.cpu().numpy(), ref.sigma)
        assert smcx.smcx_energy(ctx) == int(ref.E[0])
    finally:
        smcx.smcx_destroy(ctx)
    bad = torch.full((job.N,), 9, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_create_device(d, bad.data_ptr(), job.epi, 950.0, stream.cuda_stream)
    assert e.value.status == smcx.E_INVALID


def test_failed_table_upload_keeps_previous_tables(smcx, orc):
    """A temperature change whose table upload fails (forced from the host
    with SMCX_FAULT_TABLES) returns an error and leaves the context sweeping
    on its previous tables and schedule: the trajectory equals the oracle's
    at the old temperature."""
    job = W.lattice_job((10, 10, 10), 4, 3, 30.0, np.full(8, 900.0), stream=64, name="table-fault")
    note("table upload fault")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 900.0, block=(5, 5, 5))
    ref = orc.OracleState(job.L, (5, 5, 5), job.epi, job.sigma, job.seed)
    try:
        lat.sweep(3)
        ref.sweep(900.0, 3)
        os.environ["SMCX_FAULT_TABLES"] = "1"
        try:
            with pytest.raises(smcx.SmcxError):
                lat.set_temperature(1500.0)
            with pytest.raises(smcx.SmcxError):
                lat.set_schedule(np.linspace(2000.0, 1000.0, 50))
        finally:
            del os.environ["SMCX_FAULT_TABLES"]
        lat.sweep(5)
        ref.sweep(900.0, 5)
        assert np.array_equal(lat.config(), ref.sigma)
        assert lat.energy() == int(ref.E[0])
        # and a later change goes through
        lat.set_temperature(1200.0)
        lat.sweep(2)
        ref.sweep(1200.0, 2)
        assert np.array_equal(lat.config(), ref.sigma)
        assert lat.energy() == int(ref.E[0])
    finally:
        lat.close()
