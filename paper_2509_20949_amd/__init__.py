"""MI355X-native canonical-ensemble Monte Carlo swap sweeps (SMC-X hot path).

The compute path lives in the HIP library ``libsmcx.so`` (C ABI declared in
``include/smcx.h``); :mod:`paper_2509_20949_amd.smcx` is its thin ctypes
binding and :mod:`paper_2509_20949_amd.workloads` draws seeded inputs.
"""
__all__ = ["smcx", "workloads"]
