"""smcx_sweep_noalloc (no device allocation; its state in the library's
fixed scratch array) against smcx_sweep on a context, through the C ABI.

Two calls in a row share the one scratch array: the second uses a smaller
lattice, fewer species and shells, another seed and a later sweep index,
so anything the first call left in the array and the second still read
would show.  The bar is bit-for-bit: configuration, energy change and
accepted count.  The first case is also checked against the oracle.
"""
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


def context_run(smcx, job, lattice, block, T, sweep0, n):
    """The existing entry points: a context set to sweep index sweep0, n sweeps."""
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, T, block=block, lattice=lattice)
    try:
        if sweep0:
            smcx.smcx_set_state(lat.ctx, job.sigma, sweep0)
        E0 = lat.energy()
        lat.sweep(n)
        return lat.config(), lat.energy() - E0, lat.stats()["accepted"]
    finally:
        lat.close()


def noalloc_run(smcx, job, lattice, block, T, sweep0, n, stream):
    import torch
    dev = torch.from_numpy(job.sigma.copy()).to("cuda:0")
    torch.cuda.synchronize()
    d = smcx.make_desc(job.L, job.K, job.S, block, job.seed, lattice)
    dE, acc = smcx.smcx_sweep_noalloc(d, dev.data_ptr(), job.epi, T, sweep0, n, stream.cuda_stream)
    return dev.cpu().numpy(), dE, acc


def test_noalloc_sweeps_equal_context_sweeps(smcx, orc):
    import torch
    stream = torch.cuda.Stream()
    cases = [
        # (job, lattice, block, T, sweep0, n): the second is smaller in every respect
        (W.lattice_job((10, 11, 12), 5, 3, 30.0, np.full(6, 950.0), stream=71, name="noalloc-a"),
         smcx.LATTICE_BCC, (5, 5, 5), 950.0, 0, 6),
        (W.lattice_job((8, 8, 9), 3, 2, 25.0, np.full(3, 1300.0), stream=72, name="noalloc-b"),
         smcx.LATTICE_BCC, (4, 4, 4), 1300.0, 7, 3),
    ]
    for k, (job, lattice, block, T, s0, n) in enumerate(cases):
        note(f"noalloc case {k}: L={job.L} K={job.K} S={job.S} B={block} sweep0={s0} n={n}")
        want_cfg, want_dE, want_acc = context_run(smcx, job, lattice, block, T, s0, n)
        got_cfg, got_dE, got_acc = noalloc_run(smcx, job, lattice, block, T, s0, n, stream)
        assert np.array_equal(got_cfg, want_cfg), k
        assert got_dE == want_dE, (k, got_dE, want_dE)
        assert got_acc == want_acc, (k, got_acc, want_acc)
        assert got_acc > 0 and not np.array_equal(got_cfg, job.sigma)
        if k == 0:
            orc.set_threads(4)
            ref = orc.OracleState(job.L, block, job.epi, job.sigma, job.seed)
            E0 = int(ref.E[0])
            ref.sweep(T, n)
            orc.set_threads(1)
            assert np.array_equal(got_cfg, ref.sigma)
            assert got_dE == int(ref.E[0]) - E0


def test_noalloc_fcc_and_rejections(smcx):
    import torch
    stream = torch.cuda.Stream()
    job = W.lattice_job((6, 5, 7), 4, 3, 30.0, np.full(4, 1100.0), stream=73, name="noalloc-fcc",
                        lattice=smcx.LATTICE_FCC)
    note("noalloc FCC")
    want = context_run(smcx, job, smcx.LATTICE_FCC, (0, 0, 0), 1100.0, 2, 4)
    got = noalloc_run(smcx, job, smcx.LATTICE_FCC, (0, 0, 0), 1100.0, 2, 4, stream)
    assert np.array_equal(got[0], want[0]) and got[1:] == want[1:]
    # invalid inputs are rejected before any kernel runs
    dev = torch.from_numpy(job.sigma.copy()).to("cuda:0")
    d = smcx.make_desc(job.L, job.K, job.S, (0, 0, 0), job.seed, smcx.LATTICE_FCC)
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_sweep_noalloc(d, dev.data_ptr(), job.epi, 9000.0, 0, 1, stream.cuda_stream)
    assert e.value.status == smcx.E_RANGE
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_sweep_noalloc(d, dev.data_ptr(), job.epi, 900.0, (1 << 32) - 1, 2, stream.cuda_stream)
    assert e.value.status == smcx.E_RANGE
    bad = torch.full((job.N,), 7, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_sweep_noalloc(d, bad.data_ptr(), job.epi, 900.0, 0, 1, stream.cuda_stream)
    assert e.value.status == smcx.E_INVALID
