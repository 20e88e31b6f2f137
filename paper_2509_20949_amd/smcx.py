"""Thin ctypes binding of libsmcx (C ABI in include/smcx.h).

Functions keep the C names and only marshal arguments; every step of the
sweep runs in the HIP library.  There is no fallback: if libsmcx.so is
missing or cannot load, :func:`lib` raises.

PyTorch is used only for device memory and streams (``smcx_create_device``
takes a torch tensor's data pointer and a torch stream).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmcx.so")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_RANGE, E_STATE = 0, -1, -2, -3, -4, -5, -6
LATTICE_BCC, LATTICE_FCC = 0, 1
MAX_SPECIES, MAX_SHELLS, MAX_BLOCK = 8, 3, 12


class SmcxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"smcx status {status}: {msg}")
        self.status = status


class smcx_desc(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("L", C.c_int32 * 3), ("n_species", C.c_int32),
                ("n_shells", C.c_int32), ("block", C.c_int32 * 3), ("seed", C.c_uint64)]


_lib = None
_P = C.POINTER


def _sig(L, name, res, args):
    f = getattr(L, name)
    f.restype = res
    f.argtypes = args


def lib():
    """Load libsmcx.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2509_20949_amd/build.py")
    L = C.CDLL(LIB_PATH)
    st, vp, i32, i64, u64, dbl = C.c_int, C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    pd = _P(smcx_desc)
    _sig(L, "smcx_create", st, [pd, _P(C.c_uint8), _P(i32), dbl, _P(vp)])
    _sig(L, "smcx_create_device", st, [pd, vp, _P(i32), dbl, vp, _P(vp)])
    _sig(L, "smcx_create_slab", st, [pd, vp, C.c_uint32, _P(i32), dbl, vp, _P(vp)])
    _sig(L, "smcx_slab_phase", st, [vp, i32])
    _sig(L, "smcx_plan", st, [pd, _P(i32), _P(i32)])
    _sig(L, "smcx_set_temperature", st, [vp, dbl])
    _sig(L, "smcx_set_schedule", st, [vp, _P(dbl), i32])
    _sig(L, "smcx_sweep", st, [vp, i32])
    _sig(L, "smcx_sweep_observed", st, [vp, i32, _P(i64), _P(u64)])
    _sig(L, "smcx_energy", st, [vp, _P(i64)])
    _sig(L, "smcx_energy_recompute", st, [vp, _P(i64)])
    _sig(L, "smcx_sro", st, [vp, _P(dbl), _P(u64)])
    _sig(L, "smcx_get_config", st, [vp, _P(C.c_uint8), C.c_size_t])
    _sig(L, "smcx_get_stats", st, [vp, _P(u64), _P(u64), _P(u64), _P(i32)])
    _sig(L, "smcx_set_state", st, [vp, _P(C.c_uint8), u64])
    _sig(L, "smcx_synchronize", st, [vp])
    _sig(L, "smcx_profile", st, [vp, i32])
    _sig(L, "smcx_kernel_time", st, [vp, _P(dbl), _P(u64)])
    _sig(L, "smcx_destroy", None, [vp])
    _sig(L, "smcx_last_error", C.c_char_p, [vp])
    _sig(L, "smcx_global_error", C.c_char_p, [])
    _sig(L, "smcx_status_string", C.c_char_p, [st])
    _sig(L, "smcx_batch_create", st, [i32, pd, _P(_P(C.c_uint8)), _P(_P(i32)), _P(dbl), _P(vp)])
    _sig(L, "smcx_batch_run", st, [vp, _P(i32)])
    _sig(L, "smcx_batch_run_unbatched", st, [vp, _P(i32)])
    _sig(L, "smcx_batch_ctx", st, [vp, i32, _P(vp)])
    _sig(L, "smcx_batch_set_temperature", st, [vp, i32, dbl])
    _sig(L, "smcx_batch_exchange", st, [vp, _P(i32), _P(i32), i32, u64, u64, _P(i32)])
    _sig(L, "smcx_temperature_ladder", st, [dbl, i32, u64, dbl, u64, _P(dbl)])
    _sig(L, "smcx_batch_synchronize", st, [vp])
    _sig(L, "smcx_batch_destroy", None, [vp])
    _sig(L, "smcx_server_create", st, [C.c_size_t, i32, i32, _P(vp)])
    _sig(L, "smcx_server_submit", st, [vp, pd, _P(C.c_uint8), _P(i32), dbl, i32, _P(u64)])
    _sig(L, "smcx_server_step", st, [vp, _P(i32), _P(i32), _P(i32)])
    _sig(L, "smcx_server_poll", st, [vp, u64, _P(i32)])
    _sig(L, "smcx_server_result", st, [vp, u64, _P(i64), _P(u64), _P(C.c_uint8), C.c_size_t])
    _sig(L, "smcx_server_footprint", C.c_size_t, [pd])
    _sig(L, "smcx_server_destroy", None, [vp])
    _sig(L, "smcx_server_last_error", C.c_char_p, [vp])
    _sig(L, "smcx_threshold_table", st, [dbl, _P(dbl)])
    _sig(L, "smcx_device_thresholds", st, [dbl, _P(i32), i32, _P(dbl)])
    _sig(L, "smcx_device_philox", st, [_P(C.c_uint32), _P(C.c_uint32), i32, _P(C.c_uint32)])
    _sig(L, "smcx_device_accept_bounds", st, [dbl, _P(C.c_uint32), i32, _P(i32), _P(i32)])
    _sig(L, "smcx_sweep_noalloc", st, [pd, vp, _P(i32), dbl, u64, i32, vp, _P(i64), _P(u64)])
    _sig(L, "smcx_device_check_accept_bounds", st, [dbl, _P(u64), _P(u64), _P(dbl), _P(i32)])
    _sig(L, "smcx_weight_rows", st, [i32, i32, i32, _P(i32), _P(i32), _P(i32), _P(i32), _P(i32), C.c_size_t])
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != OK:
        L = lib()
        msg = (L.smcx_last_error(ctx) if ctx else L.smcx_global_error()) or b""
        raise SmcxError(status, msg.decode(errors="replace"))


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(a, t):
    return a.ctypes.data_as(_P(t))


def make_desc(L, K, S, block=(0, 0, 0), seed=0, lattice=LATTICE_BCC) -> smcx_desc:
    d = smcx_desc()
    d.lattice = int(lattice)
    d.L[:] = [int(v) for v in L]
    d.n_species = int(K)
    d.n_shells = int(S)
    d.block[:] = [int(v) for v in block]
    d.seed = int(seed) & (2**64 - 1)
    return d


# ---- C-named wrappers ---------------------------------------------------------

def smcx_create(desc: smcx_desc, species, epi_ueV, T_kelvin: float):
    s = _u8(species)
    e = np.ascontiguousarray(epi_ueV, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().smcx_create(C.byref(desc), _ptr(s, C.c_uint8), _ptr(e, C.c_int32), float(T_kelvin),
                             C.byref(out)))
    return out.value


def smcx_create_device(desc: smcx_desc, d_species_ptr: int, epi_ueV, T_kelvin: float, hip_stream: int = 0):
    e = np.ascontiguousarray(epi_ueV, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().smcx_create_device(C.byref(desc), C.c_void_p(d_species_ptr), _ptr(e, C.c_int32),
                                    float(T_kelvin), C.c_void_p(hip_stream or None), C.byref(out)))
    return out.value


def smcx_sweep_noalloc(desc: smcx_desc, d_species_ptr: int, epi_ueV, T_kelvin: float, sweep0: int, n: int,
                       hip_stream: int = 0):
    """n sweeps of the lattice at d_species_ptr from sweep index sweep0 with no
    device allocation; returns (energy change, accepted swaps)."""
    e = np.ascontiguousarray(epi_ueV, dtype=np.int32)
    dE, acc = C.c_int64(), C.c_uint64()
    _check(lib().smcx_sweep_noalloc(C.byref(desc), C.c_void_p(d_species_ptr), _ptr(e, C.c_int32), float(T_kelvin),
                                    int(sweep0), int(n), C.c_void_p(hip_stream or None), C.byref(dE),
                                    C.byref(acc)))
    return dE.value, acc.value


def smcx_create_slab(desc: smcx_desc, d_buffer_ptr: int, z_offset: int, epi_ueV, T_kelvin: float,
                     hip_stream: int = 0):
    e = np.ascontiguousarray(epi_ueV, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().smcx_create_slab(C.byref(desc), C.c_void_p(d_buffer_ptr), int(z_offset), _ptr(e, C.c_int32),
                                  float(T_kelvin), C.c_void_p(hip_stream or None), C.byref(out)))
    return out.value


def smcx_slab_phase(ctx, n: int):
    _check(lib().smcx_slab_phase(ctx, int(n)), ctx)


def smcx_plan(desc: smcx_desc):
    """(block width per axis, blocks per axis) of the schedule the library runs."""
    blk, nb = (C.c_int32 * 3)(), (C.c_int32 * 3)()
    _check(lib().smcx_plan(C.byref(desc), blk, nb))
    return tuple(blk), tuple(nb)


def smcx_set_temperature(ctx, T_kelvin: float):
    _check(lib().smcx_set_temperature(ctx, float(T_kelvin)), ctx)


def smcx_set_schedule(ctx, T_per_sweep):
    t = np.ascontiguousarray(T_per_sweep, dtype=np.float64)
    _check(lib().smcx_set_schedule(ctx, _ptr(t, C.c_double), int(t.size)), ctx)


def smcx_sweep(ctx, n: int):
    _check(lib().smcx_sweep(ctx, int(n)), ctx)


def smcx_sweep_observed(ctx, n: int, S: int, K: int):
    E = np.zeros(int(n), np.int64)
    counts = np.zeros((int(n), S, K, K), np.uint64)
    _check(lib().smcx_sweep_observed(ctx, int(n), _ptr(E, C.c_int64), _ptr(counts, C.c_uint64)), ctx)
    return E, counts


def smcx_energy(ctx) -> int:
    E = C.c_int64()
    _check(lib().smcx_energy(ctx, C.byref(E)), ctx)
    return E.value


def smcx_energy_recompute(ctx) -> int:
    E = C.c_int64()
    _check(lib().smcx_energy_recompute(ctx, C.byref(E)), ctx)
    return E.value


def smcx_sro(ctx, S: int, K: int):
    alpha = np.zeros((S, K, K), np.float64)
    counts = np.zeros((S, K, K), np.uint64)
    _check(lib().smcx_sro(ctx, _ptr(alpha, C.c_double), _ptr(counts, C.c_uint64)), ctx)
    return alpha, counts


def smcx_get_config(ctx, N: int) -> np.ndarray:
    out = np.empty(N, np.uint8)
    _check(lib().smcx_get_config(ctx, _ptr(out, C.c_uint8), N), ctx)
    return out


def smcx_get_stats(ctx):
    sw, at, ac = C.c_uint64(), C.c_uint64(), C.c_uint64()
    blk = (C.c_int32 * 3)()
    _check(lib().smcx_get_stats(ctx, C.byref(sw), C.byref(at), C.byref(ac), blk), ctx)
    return {"sweeps": sw.value, "attempted": at.value, "accepted": ac.value, "block": tuple(blk)}


def smcx_set_state(ctx, species, sweep_index: int):
    s = _u8(species)
    _check(lib().smcx_set_state(ctx, _ptr(s, C.c_uint8), int(sweep_index)), ctx)


def smcx_synchronize(ctx):
    _check(lib().smcx_synchronize(ctx), ctx)


def smcx_profile(ctx, enable: bool):
    _check(lib().smcx_profile(ctx, 1 if enable else 0), ctx)


def smcx_kernel_time(ctx):
    ms, n = C.c_double(), C.c_uint64()
    _check(lib().smcx_kernel_time(ctx, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def smcx_destroy(ctx):
    if ctx:
        lib().smcx_destroy(ctx)


def smcx_threshold_table(T_kelvin: float) -> np.ndarray:
    out = np.zeros(768, np.float64)
    _check(lib().smcx_threshold_table(float(T_kelvin), _ptr(out, C.c_double)))
    return out


def smcx_device_thresholds(T_kelvin: float, dE) -> np.ndarray:
    d = np.ascontiguousarray(dE, dtype=np.int32)
    out = np.zeros(d.size, np.float64)
    _check(lib().smcx_device_thresholds(float(T_kelvin), _ptr(d, C.c_int32), int(d.size), _ptr(out, C.c_double)))
    return out


def smcx_weight_rows(lattice: int, K: int, S: int, epi):
    """(form, table[kmax*kmax, row_len]) of the pair-weight rows the library builds."""
    e = np.ascontiguousarray(epi, dtype=np.int32)
    form, kmax, row_len = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().smcx_weight_rows(int(lattice), int(K), int(S), _ptr(e, C.c_int32), C.byref(form), C.byref(kmax),
                                  C.byref(row_len), None, 0))
    out = np.zeros(kmax.value * kmax.value * row_len.value, np.int32)
    _check(lib().smcx_weight_rows(int(lattice), int(K), int(S), _ptr(e, C.c_int32), C.byref(form), C.byref(kmax),
                                  C.byref(row_len), _ptr(out, C.c_int32), out.size))
    return form.value, out.reshape(kmax.value * kmax.value, row_len.value)


def smcx_device_accept_bounds(T_kelvin: float, u):
    """(lo, hi) per acceptance draw, as the sweep kernels compute them."""
    v = np.ascontiguousarray(u, dtype=np.uint32)
    lo = np.zeros(v.size, np.int32)
    hi = np.zeros(v.size, np.int32)
    _check(lib().smcx_device_accept_bounds(float(T_kelvin), _ptr(v, C.c_uint32), int(v.size), _ptr(lo, C.c_int32),
                                           _ptr(hi, C.c_int32)))
    return lo, hi


def smcx_device_check_accept_bounds(T_kelvin: float):
    """Exhaustive device check of the acceptance bounds over all 2^32 draws:
    (violations below, violations above, max log2 error, widest band)."""
    a, b, e, w = C.c_uint64(), C.c_uint64(), C.c_double(), C.c_int32()
    _check(lib().smcx_device_check_accept_bounds(float(T_kelvin), C.byref(a), C.byref(b), C.byref(e), C.byref(w)))
    return a.value, b.value, e.value, w.value


def smcx_device_philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    _check(lib().smcx_device_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), int(c.shape[0]),
                                    _ptr(out, C.c_uint32)))
    return out


# ---- batch -------------------------------------------------------------------

def smcx_batch_create(descs: Sequence[smcx_desc], species: Sequence[np.ndarray], epis: Sequence[np.ndarray],
                      T_kelvin: Sequence[float]):
    n = len(descs)
    arr = (smcx_desc * n)(*descs)
    sp = [_u8(s) for s in species]
    ep = [np.ascontiguousarray(e, dtype=np.int32) for e in epis]
    sp_ptrs = (_P(C.c_uint8) * n)(*[_ptr(s, C.c_uint8) for s in sp])
    ep_ptrs = (_P(C.c_int32) * n)(*[_ptr(e, C.c_int32) for e in ep])
    T = np.ascontiguousarray(T_kelvin, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().smcx_batch_create(n, arr, sp_ptrs, ep_ptrs, _ptr(T, C.c_double), C.byref(out)))
    return out.value


def smcx_batch_run(batch, n_sweeps):
    n = np.ascontiguousarray(n_sweeps, dtype=np.int32)
    _check(lib().smcx_batch_run(batch, _ptr(n, C.c_int32)))


def smcx_batch_run_unbatched(batch, n_sweeps):
    n = np.ascontiguousarray(n_sweeps, dtype=np.int32)
    _check(lib().smcx_batch_run_unbatched(batch, _ptr(n, C.c_int32)))


def smcx_batch_ctx(batch, r: int):
    out = C.c_void_p()
    _check(lib().smcx_batch_ctx(batch, int(r), C.byref(out)))
    return out.value


def smcx_batch_set_temperature(batch, r: int, T_kelvin: float):
    _check(lib().smcx_batch_set_temperature(batch, int(r), float(T_kelvin)))


def smcx_batch_exchange(batch, a, b, seed: int, round_: int):
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    acc = np.zeros(a.size, np.int32)
    _check(lib().smcx_batch_exchange(batch, _ptr(a, C.c_int32), _ptr(b, C.c_int32), int(a.size), int(seed),
                                     int(round_), _ptr(acc, C.c_int32)))
    return acc


def smcx_temperature_ladder(T0: float, n: int, n_atoms: int, dT_ref: float = 0.0, n_ref: int = 0) -> np.ndarray:
    out = np.zeros(int(n), np.float64)
    _check(lib().smcx_temperature_ladder(float(T0), int(n), int(n_atoms), float(dT_ref), int(n_ref),
                                         _ptr(out, C.c_double)))
    return out


def smcx_batch_synchronize(batch):
    _check(lib().smcx_batch_synchronize(batch))


def smcx_batch_destroy(batch):
    if batch:
        lib().smcx_batch_destroy(batch)


# ---- serving -------------------------------------------------------------------

def smcx_server_create(hbm_budget_bytes: int, max_slots: int, sweeps_per_step: int):
    out = C.c_void_p()
    _check(lib().smcx_server_create(int(hbm_budget_bytes), int(max_slots), int(sweeps_per_step), C.byref(out)))
    return out.value


def _srv_check(status, srv):
    if status != OK:
        msg = lib().smcx_server_last_error(srv) or b""
        raise SmcxError(status, msg.decode(errors="replace"))


def smcx_server_submit(srv, desc: smcx_desc, species, epi_ueV, T_kelvin: float, n_sweeps: int) -> int:
    s = _u8(species)
    e = np.ascontiguousarray(epi_ueV, dtype=np.int32)
    rid = C.c_uint64()
    _srv_check(lib().smcx_server_submit(srv, C.byref(desc), _ptr(s, C.c_uint8), _ptr(e, C.c_int32),
                                        float(T_kelvin), int(n_sweeps), C.byref(rid)), srv)
    return rid.value


def smcx_server_step(srv):
    r, w, f = C.c_int32(), C.c_int32(), C.c_int32()
    _srv_check(lib().smcx_server_step(srv, C.byref(r), C.byref(w), C.byref(f)), srv)
    return r.value, w.value, f.value


def smcx_server_poll(srv, rid: int) -> int:
    s = C.c_int32()
    _srv_check(lib().smcx_server_poll(srv, int(rid), C.byref(s)), srv)
    return s.value


def smcx_server_result(srv, rid: int, N: Optional[int] = None):
    E, acc = C.c_int64(), C.c_uint64()
    cfg = np.empty(N, np.uint8) if N else None
    _srv_check(lib().smcx_server_result(srv, int(rid), C.byref(E), C.byref(acc),
                                        _ptr(cfg, C.c_uint8) if cfg is not None else None,
                                        int(N or 0)), srv)
    return E.value, acc.value, cfg


def smcx_server_footprint(desc: smcx_desc) -> int:
    return int(lib().smcx_server_footprint(C.byref(desc)))


def smcx_server_destroy(srv):
    if srv:
        lib().smcx_server_destroy(srv)


# ---- convenience -----------------------------------------------------------------

class Lattice:
    """One lattice context (owns its device memory)."""

    def __init__(self, L, epi, sigma, seed, T, block=(0, 0, 0), lattice=LATTICE_BCC):
        epi = np.ascontiguousarray(epi, dtype=np.int32)
        self.S, self.K = int(epi.shape[0]), int(epi.shape[1])
        self.L = tuple(int(v) for v in L)
        self.lattice = int(lattice)
        self.N = (4 if lattice == LATTICE_FCC else 2) * self.L[0] * self.L[1] * self.L[2]
        self.desc = make_desc(self.L, self.K, self.S, block, seed, lattice)
        self.ctx = smcx_create(self.desc, sigma, epi, T)

    def sweep(self, n=1):
        smcx_sweep(self.ctx, n)

    def set_temperature(self, T):
        smcx_set_temperature(self.ctx, T)

    def set_schedule(self, T):
        smcx_set_schedule(self.ctx, T)

    def sweep_observed(self, n):
        """n sweeps; per sweep energy (n,) and pair counts (n, S, K, K)."""
        return smcx_sweep_observed(self.ctx, n, self.S, self.K)

    def energy(self):
        return smcx_energy(self.ctx)

    def energy_recompute(self):
        return smcx_energy_recompute(self.ctx)

    def config(self):
        return smcx_get_config(self.ctx, self.N)

    def sro(self):
        return smcx_sro(self.ctx, self.S, self.K)

    def stats(self):
        return smcx_get_stats(self.ctx)

    def close(self):
        smcx_destroy(self.ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
