"""ctypes front end of the plain sequential CPU oracle (smcx_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product library never loads
it.  ``build()`` compiles the C source with gcc (no fast-math, no FP
contraction, so the FP64 threshold products round exactly as written).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smcx_oracle.c")
LIB = os.path.join(HERE, "libsmcx_oracle.so")

_lib = None


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (by default smcx_oracle.c into oracle/libsmcx_oracle.so)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wextra", "-I", HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _bind(path: str):
    L = C.CDLL(path)
    p = C.POINTER
    L.or_set_threads.argtypes = [C.c_int]
    L.or_set_fixed_z.argtypes = [C.c_int]
    L.or_get_threads.restype = C.c_int
    L.or_philox4x32_10.argtypes = [p(C.c_uint32), p(C.c_uint32), p(C.c_uint32)]
    L.or_philox4x64_10.argtypes = [p(C.c_uint64), p(C.c_uint64), p(C.c_uint64)]
    L.or_thresholds.argtypes = [C.c_double, p(C.c_double)]
    L.or_accept.argtypes = [C.c_int64, C.c_uint32, p(C.c_double)]
    L.or_accept.restype = C.c_int
    L.or_axis_blocks.argtypes = [C.c_int, C.c_int]
    L.or_axis_blocks.restype = C.c_int
    L.or_axis_bounds.argtypes = [C.c_int, C.c_int, p(C.c_int32)]
    L.or_sweep_shift.argtypes = [p(C.c_int32), C.c_uint64, C.c_uint32, p(C.c_int32)]
    L.or_schedule.argtypes = [C.c_int, p(C.c_int32), p(C.c_int32), C.c_uint64, C.c_uint32,
                              p(C.c_uint8), p(C.c_uint8), p(C.c_int64)]
    L.or_neighbour.argtypes = [C.c_int, p(C.c_int32), C.c_int64, C.c_int]
    L.or_bcc_draws.argtypes = [p(C.c_int32), p(C.c_int32), C.c_uint64, C.c_uint32, p(C.c_uint32),
                               p(C.c_uint8), p(C.c_uint8), p(C.c_uint32)]
    L.or_bcc_draws.restype = C.c_int
    L.or_fcc_draws.argtypes = [p(C.c_int32), p(C.c_int32), C.c_uint64, C.c_uint32, p(C.c_int64), p(C.c_uint32)]
    L.or_fcc_draws.restype = C.c_int
    L.or_shell_size.argtypes = [C.c_int, C.c_int]
    L.or_n_sub.argtypes = [C.c_int]
    L.or_neighbour.restype = C.c_int64
    L.or_energy.argtypes = [C.c_int, p(C.c_int32), C.c_int, C.c_int, p(C.c_int32), p(C.c_uint8)]
    L.or_energy.restype = C.c_int64
    L.or_delta_energy.argtypes = [C.c_int, p(C.c_int32), C.c_int, C.c_int, p(C.c_int32), p(C.c_uint8),
                                  C.c_int64, C.c_int64]
    L.or_delta_energy.restype = C.c_int64
    L.or_pair_counts.argtypes = [C.c_int, p(C.c_int32), C.c_int, C.c_int, p(C.c_uint8), p(C.c_uint64)]
    L.or_sro.argtypes = [C.c_int, p(C.c_int32), C.c_int, C.c_int, p(C.c_uint8), p(C.c_double),
                         p(C.c_uint64)]
    L.or_sweep.argtypes = [C.c_int, p(C.c_int32), p(C.c_int32), C.c_int, C.c_int, p(C.c_int32),
                           C.c_uint64, C.c_uint32, C.c_int32, p(C.c_double), p(C.c_uint8),
                           p(C.c_int64), p(C.c_uint64), p(C.c_int64), p(C.c_uint64)]
    L.or_sweep.restype = C.c_int
    L.or_exchange_accept.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_uint64,
                                     C.c_uint32, C.c_uint64]
    L.or_exchange_accept.restype = C.c_int
    L.or_enumerate.argtypes = [C.c_int, p(C.c_int32), C.c_int, C.c_int, p(C.c_int32), p(C.c_int32),
                               C.c_int64, p(C.c_int64), p(C.c_uint64)]
    L.or_enumerate.restype = C.c_int64
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(LIB)
    return _lib


@contextlib.contextmanager
def using(path: str):
    """Route every call of this module through another build of the oracle
    (the planted-mistake tests load deliberately broken copies)."""
    global _lib
    saved = lib()
    _lib = _bind(path)
    try:
        yield
    finally:
        _lib = saved


def set_threads(n: int) -> None:
    """Worker threads of the oracle (results are identical for any count)."""
    lib().or_set_threads(int(n))


@contextlib.contextmanager
def fixed_z(on: bool = True):
    """Within the block: the z-slab schedule (block grid shifted along x and y
    only)."""
    lib().or_set_fixed_z(1 if on else 0)
    try:
        yield
    finally:
        lib().or_set_fixed_z(0)


def get_threads() -> int:
    return int(lib().or_get_threads())


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _L(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(3))


def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def thresholds(T):
    tab = np.zeros(768, np.float64)
    lib().or_thresholds(float(T), _ptr(tab, C.c_double))
    return tab


def accept(dE, u, tab):
    return bool(lib().or_accept(int(dE), int(u), _ptr(tab, C.c_double)))


def axis_blocks(L, B):
    return lib().or_axis_blocks(int(L), int(B))


def axis_bounds(L, B):
    n = axis_blocks(L, B)
    b = np.zeros(n + 1, np.int32)
    lib().or_axis_bounds(int(L), int(B), _ptr(b, C.c_int32))
    return b


def sweep_shift(L, seed, s):
    out = np.zeros(3, np.int32)
    lib().or_sweep_shift(_ptr(_L(L), C.c_int32), C.c_uint64(seed), C.c_uint32(s),
                         _ptr(out, C.c_int32))
    return out


BCC, FCC = 0, 1


def n_sub(lattice=BCC):
    return 4 if lattice == FCC else 2


def shell_size(s, lattice=BCC):
    return lib().or_shell_size(int(lattice), int(s))


def n_sites(L, lattice=BCC):
    return n_sub(lattice) * int(np.prod(np.asarray(L, dtype=np.int64)))


def schedule(L, B, seed, s, lattice=BCC):
    Lv = _L(L)
    N = n_sites(Lv, lattice)
    col = np.zeros(N, np.uint8)
    sub = np.zeros(N, np.uint8)
    blk = np.zeros(N, np.int64)
    lib().or_schedule(int(lattice), _ptr(Lv, C.c_int32), _ptr(_L(B), C.c_int32), C.c_uint64(seed),
                      C.c_uint32(s), _ptr(col, C.c_uint8), _ptr(sub, C.c_uint8),
                      _ptr(blk, C.c_int64))
    return col, sub, blk


def bcc_draws(L, B, seed, s):
    """Per-site BCC trial draws of sweep s: (counters [N, 4], word, dir, u_acc)."""
    Lv = _L(L)
    N = n_sites(Lv, BCC)
    ctr = np.zeros((N, 4), np.uint32)
    word = np.zeros(N, np.uint8)
    dirs = np.zeros(N, np.uint8)
    u = np.zeros(N, np.uint32)
    rc = lib().or_bcc_draws(_ptr(Lv, C.c_int32), _ptr(_L(B), C.c_int32), C.c_uint64(seed), C.c_uint32(s),
                            _ptr(ctr, C.c_uint32), _ptr(word, C.c_uint8), _ptr(dirs, C.c_uint8),
                            _ptr(u, C.c_uint32))
    if rc != 0:
        raise ValueError("invalid arguments")
    return ctr, word, dirs, u


def fcc_draws(L, B, seed, s):
    """Per-site FCC trial draws of sweep s: (partner site index, u_acc)."""
    Lv = _L(L)
    N = n_sites(Lv, FCC)
    partner = np.zeros(N, np.int64)
    u = np.zeros(N, np.uint32)
    rc = lib().or_fcc_draws(_ptr(Lv, C.c_int32), _ptr(_L(B), C.c_int32), C.c_uint64(seed), C.c_uint32(s),
                            _ptr(partner, C.c_int64), _ptr(u, C.c_uint32))
    if rc != 0:
        raise ValueError("invalid arguments")
    return partner, u


def neighbour(L, i, k, lattice=BCC):
    return lib().or_neighbour(int(lattice), _ptr(_L(L), C.c_int32), int(i), int(k))


def _epi(epi):
    return np.ascontiguousarray(epi, dtype=np.int32)


def energy(L, epi, sigma, lattice=BCC):
    e = _epi(epi)
    S, K = e.shape[0], e.shape[1]
    s = np.ascontiguousarray(sigma, dtype=np.uint8)
    return lib().or_energy(int(lattice), _ptr(_L(L), C.c_int32), S, K, _ptr(e, C.c_int32), _ptr(s, C.c_uint8))


def delta_energy(L, epi, sigma, i, j, lattice=BCC):
    e = _epi(epi)
    s = np.ascontiguousarray(sigma, dtype=np.uint8)
    return lib().or_delta_energy(int(lattice), _ptr(_L(L), C.c_int32), e.shape[0], e.shape[1],
                                 _ptr(e, C.c_int32), _ptr(s, C.c_uint8), int(i), int(j))


def pair_counts(L, S, K, sigma, lattice=BCC):
    s = np.ascontiguousarray(sigma, dtype=np.uint8)
    out = np.zeros((S, K, K), np.uint64)
    lib().or_pair_counts(int(lattice), _ptr(_L(L), C.c_int32), S, K, _ptr(s, C.c_uint8), _ptr(out, C.c_uint64))
    return out


def sro(L, S, K, sigma, lattice=BCC):
    s = np.ascontiguousarray(sigma, dtype=np.uint8)
    alpha = np.zeros((S, K, K), np.float64)
    counts = np.zeros((S, K, K), np.uint64)
    lib().or_sro(int(lattice), _ptr(_L(L), C.c_int32), S, K, _ptr(s, C.c_uint8), _ptr(alpha, C.c_double),
                 _ptr(counts, C.c_uint64))
    return alpha, counts


def exchange_accept(Ea, Eb, Ta, Tb, seed, k, round_):
    return bool(lib().or_exchange_accept(int(Ea), int(Eb), float(Ta), float(Tb), C.c_uint64(seed),
                                         C.c_uint32(k), C.c_uint64(round_)))


class OracleState:
    """A lattice advanced by the oracle, sweep by sweep."""

    def __init__(self, L, B, epi, sigma, seed, s0=0, lattice=BCC, fixed_z=False):
        self.fixed_z = bool(fixed_z)
        self.lattice = int(lattice)
        self.L = _L(L)
        self.B = _L(B)
        self.epi = _epi(epi)
        self.S, self.K = int(self.epi.shape[0]), int(self.epi.shape[1])
        self.sigma = np.array(sigma, dtype=np.uint8, copy=True)
        self.seed = int(seed)
        self.s = int(s0)
        self.E = np.zeros(1, np.int64)
        self.E[0] = energy(self.L, self.epi, self.sigma, self.lattice)
        self.accepted = np.zeros(1, np.uint64)

    def sweep(self, T, n=1, trace_E=False, trace_counts=False):
        Ts = np.ascontiguousarray(np.broadcast_to(np.asarray(T, np.float64), (n,)), np.float64)
        Et = np.zeros(n, np.int64) if trace_E else None
        Ct = np.zeros((n, self.S, self.K, self.K), np.uint64) if trace_counts else None
        with fixed_z(self.fixed_z):
            rc = self._sweep(n, Ts, Et, Ct)
        if rc != 0:
            raise ValueError("oracle rejected the sweep arguments")
        self.s += n
        return Et, Ct

    def _sweep(self, n, Ts, Et, Ct):
        return lib().or_sweep(
            self.lattice, _ptr(self.L, C.c_int32), _ptr(self.B, C.c_int32), self.S, self.K,
            _ptr(self.epi, C.c_int32), C.c_uint64(self.seed), C.c_uint32(self.s), n,
            _ptr(Ts, C.c_double), _ptr(self.sigma, C.c_uint8), _ptr(self.E, C.c_int64),
            _ptr(self.accepted, C.c_uint64),
            _ptr(Et, C.c_int64) if Et is not None else None,
            _ptr(Ct, C.c_uint64) if Ct is not None else None)


def enumerate_configs(L, epi, comp, max_cfg=5_000_000, with_counts=False, lattice=BCC):
    e = _epi(epi)
    S, K = e.shape[0], e.shape[1]
    c = np.ascontiguousarray(comp, dtype=np.int32)
    from math import factorial
    n = factorial(int(c.sum()))
    for x in c:
        n //= factorial(int(x))
    if n > max_cfg:
        raise ValueError("too many configurations")
    E = np.zeros(n, np.int64)
    counts = np.zeros((n, S, K, K), np.uint64) if with_counts else None
    got = lib().or_enumerate(int(lattice), _ptr(_L(L), C.c_int32), S, K, _ptr(e, C.c_int32),
                             _ptr(c, C.c_int32), n, _ptr(E, C.c_int64),
                             _ptr(counts, C.c_uint64) if counts is not None else None)
    if got != n:
        raise RuntimeError("enumeration count mismatch")
    return E, counts
