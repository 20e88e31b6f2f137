"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/smcx.h declares, builds the same FP64 threshold tables as the
oracle, and rejects invalid arguments before touching a device.
No compute call is made here (there is no GPU on this host)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smcx.h")


@pytest.fixture(scope="module")
def smcx():
    from paper_2509_20949_amd import smcx as m
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smcx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("smcx_create", "smcx_sweep", "smcx_energy", "smcx_sro", "smcx_get_config",
                 "smcx_batch_create", "smcx_batch_run", "smcx_server_create", "smcx_server_step"):
        assert must in names


def test_library_exports_every_declared_symbol(smcx):
    lib = smcx.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_the_header(smcx):
    for n in declared_functions():
        if n in ("smcx_last_error", "smcx_global_error", "smcx_status_string", "smcx_server_last_error"):
            continue
        assert hasattr(smcx, n), n


def test_host_threshold_tables_equal_oracle(smcx, orc):
    for T in (1.0, 250.0, 300.0, 800.0, 1000.0, 1234.5, 2000.0, 5000.0):
        a = smcx.smcx_threshold_table(T)
        b = orc.thresholds(T)
        assert a.tobytes() == b.tobytes(), T


@pytest.mark.parametrize("T", [0.5, 0.0, -3.0, 5000.5, float("nan")])
def test_temperature_range_rejected(smcx, T):
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_threshold_table(T)
    assert e.value.status == smcx.E_RANGE


def _desc(smcx, L=(8, 8, 8), K=4, S=2, block=(0, 0, 0)):
    return smcx.make_desc(L, K, S, block, 1)


def test_create_validation_before_device(smcx):
    N = 1024
    sigma = np.zeros(N, np.uint8)
    epi = np.zeros((2, 4, 4), np.int32)
    cases = [
        (dict(L=(3, 8, 8)), sigma[:2 * 3 * 64], epi, 800.0, smcx.E_UNSUPPORTED),
        (dict(L=(1, 8, 8)), sigma[:128], epi, 800.0, smcx.E_INVALID),
        (dict(block=(13, 0, 0)), sigma, epi, 800.0, smcx.E_UNSUPPORTED),
        (dict(block=(1, 0, 0)), sigma, epi, 800.0, smcx.E_INVALID),
        (dict(K=9), sigma, np.zeros((2, 9, 9), np.int32), 800.0, smcx.E_UNSUPPORTED),
        (dict(S=4), sigma, np.zeros((4, 4, 4), np.int32), 800.0, smcx.E_UNSUPPORTED),
        (dict(), np.full(N, 4, np.uint8), epi, 800.0, smcx.E_INVALID),
        (dict(), sigma, epi, 6000.0, smcx.E_RANGE),
    ]
    asym = epi.copy()
    asym[0, 0, 1] = 5
    cases.append((dict(), sigma, asym, 800.0, smcx.E_INVALID))
    big = epi.copy()
    big[1, 2, 2] = 1 << 22
    cases.append((dict(), sigma, big, 800.0, smcx.E_RANGE))
    for kw, s, e, T, want in cases:
        d = _desc(smcx, **kw)
        with pytest.raises(smcx.SmcxError) as err:
            smcx.smcx_create(d, s, e, T)
        assert err.value.status == want, (kw, err.value)


def test_null_handles_are_rejected(smcx):
    lib = smcx.lib()
    assert lib.smcx_sweep(None, 1) == smcx.E_INVALID
    E = C.c_int64()
    assert lib.smcx_energy(None, C.byref(E)) == smcx.E_INVALID
    lib.smcx_destroy(None)   # no-op


def test_schedule_block_counts_match_oracle(smcx, orc):
    """The library's block-count rule (smcx_plan, computed by the library on
    the host) equals the oracle's for every axis length and width."""
    for L in range(4, 200, 3):
        for B in (2, 3, 5, 8, 11, 12):
            d = smcx.make_desc((L, 8, 9), 4, 3, (B, 4, 5), 1)
            blk, nb = smcx.smcx_plan(d)
            assert blk == (B, 4, 5)
            assert nb == (orc.axis_blocks(L, B), orc.axis_blocks(8, 4), orc.axis_blocks(9, 5)), (L, B)


def test_plan_depends_only_on_the_lattice_shape(smcx):
    """block = 0: the library's choice is a fixed function of (lattice, L, K),
    the same for every seed and shell count, and the same as the choice it
    reports for that axis length in any other position."""
    for lattice, Ks in ((0, (2, 4, 5, 8)), (1, (2, 5))):
        for L in (4, 7, 16, 25, 37, 48, 64, 96, 512):
            for K in Ks:
                choices = set()
                for S, seed in ((1, 1), (3, 99)):
                    d = smcx.make_desc((L, 16, 33), K, S, (0, 0, 0), seed, lattice)
                    blk, nb = smcx.smcx_plan(d)
                    d2 = smcx.make_desc((33, L, 16), K, S, (0, 0, 0), seed + 1, lattice)
                    blk2, _ = smcx.smcx_plan(d2)
                    assert blk2[1] == blk[0]
                    assert all(2 <= b <= 12 for b in blk) and all(n % 2 == 0 for n in nb)
                    choices.add(blk[0])
                assert len(choices) == 1, (lattice, L, K)


def test_fcc_validation(smcx):
    sigma = np.zeros(4 * 512, np.uint8)
    d = smcx.make_desc((8, 8, 8), 6, 3, (0, 0, 0), 1, smcx.LATTICE_FCC)
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_create(d, sigma, np.zeros((3, 6, 6), np.int32), 800.0)
    assert e.value.status == smcx.E_UNSUPPORTED
    d = smcx.make_desc((8, 8, 8), 3, 3, (0, 0, 0), 1, 7)
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_create(d, sigma, np.zeros((3, 3, 3), np.int32), 800.0)
    assert e.value.status == smcx.E_INVALID
    # a 4-site-per-cell species array is checked against K before any device call
    d = smcx.make_desc((8, 8, 8), 3, 3, (0, 0, 0), 1, smcx.LATTICE_FCC)
    bad = sigma.copy()
    bad[-1] = 3
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_create(d, bad, np.zeros((3, 3, 3), np.int32), 800.0)
    assert e.value.status == smcx.E_INVALID


def test_temperature_ladder_scales_as_inverse_sqrt_n(smcx):
    """Equation for Delta T: the spacing scales as 1/sqrt(N_atom); by default
    it reproduces the paper's example (0.1 K at 10^9 atoms)."""
    T = smcx.smcx_temperature_ladder(1000.0, 5, 10**9)
    assert np.allclose(np.diff(T), 0.1, rtol=0, atol=1e-12) and T[0] == 1000.0
    for N in (1024, 524288, 268435456, 1066867200):
        a = smcx.smcx_temperature_ladder(800.0, 3, N, 2.0, 1024)
        b = smcx.smcx_temperature_ladder(800.0, 3, 4 * N, 2.0, 1024)
        assert np.isclose(np.diff(a)[0], 2.0 * np.sqrt(1024 / N), rtol=1e-14)
        assert np.isclose(np.diff(b)[0] * 2, np.diff(a)[0], rtol=1e-14)   # 4x the atoms: half the spacing
    # the paper's 1.07e9-atom production lattice: about 0.097 K from the 1e9 example
    d = np.diff(smcx.smcx_temperature_ladder(1000.0, 2, 672 * 630 * 630 * 4))[0]
    assert 0.096 < d < 0.0975
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_temperature_ladder(4999.0, 3, 100, 1.0, 100)
    assert e.value.status == smcx.E_RANGE
    with pytest.raises(smcx.SmcxError) as e:
        smcx.smcx_temperature_ladder(800.0, 0, 100)
    assert e.value.status == smcx.E_INVALID
