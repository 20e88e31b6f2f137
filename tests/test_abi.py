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


def test_schedule_block_counts_match_oracle(orc):
    """The library's block-count rule (declared in smcx.h) is the oracle's."""
    import paper_2509_20949_amd.smcx  # noqa: F401
    for L in range(4, 200, 3):
        for B in (2, 3, 5, 8, 12):
            n = orc.axis_blocks(L, B)
            want = max(2, min(2 * -(-L // (2 * B)), 2 * (L // 4)))
            assert n == want


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
