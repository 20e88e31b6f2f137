"""Seeded synthetic inputs shaped like the paper's alloy workloads.

This module only draws inputs (EPI tables, compositions, configurations,
temperature ladders and schedules).  It holds none of the sampling
arithmetic, so the HIP library and the CPU oracle can both be fed from it.

The paper's fitted FeCoNiAlTi EPI and its DFT data are not available, so
effective pair interactions are drawn from N(0, sigma) per shell and
rounded to integer micro-eV (round half to even), upper triangle mirrored.
Compositions are equiatomic or Dirichlet(alpha); fractions become integer
counts by largest remainder, ties to the lower species index.  A
configuration is a uniformly random arrangement of that multiset
(numpy PCG64 permutation).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BASE_SEED = 250920949

# the paper's alloy Fe29 Co29 Ni28 Al7 Ti7 (fractions), for optional use
FECONIALTI = (0.29, 0.29, 0.28, 0.07, 0.07)


BCC, FCC = 0, 1


def n_sites(L, lattice: int = BCC) -> int:
    Lx, Ly, Lz = (int(v) for v in L)
    return (4 if lattice == FCC else 2) * Lx * Ly * Lz


def epi_table(S: int, K: int, sigma_meV: float, rng: np.random.Generator) -> np.ndarray:
    """Symmetric [S][K][K] int32 micro-eV table, entries ~ N(0, sigma)."""
    V = np.zeros((S, K, K), dtype=np.int32)
    for s in range(S):
        for p in range(K):
            for q in range(p, K):
                v = np.rint(rng.normal(0.0, sigma_meV) * 1000.0)
                V[s, p, q] = V[s, q, p] = int(v)
    return V


def counts_from_fractions(frac, N: int) -> np.ndarray:
    """Largest-remainder rounding of N*frac; ties go to the lower index."""
    frac = np.asarray(frac, dtype=np.float64)
    frac = frac / frac.sum()
    raw = frac * N
    base = np.floor(raw).astype(np.int64)
    left = int(N - base.sum())
    rem = raw - base
    order = sorted(range(len(frac)), key=lambda k: (-rem[k], k))
    for k in order[:left]:
        base[k] += 1
    return base


def equiatomic(K: int, N: int) -> np.ndarray:
    return counts_from_fractions(np.ones(K), N)


def dirichlet_counts(K: int, N: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    return counts_from_fractions(rng.dirichlet(np.full(K, alpha)), N)


def configuration(counts, rng: np.random.Generator) -> np.ndarray:
    """Uniformly random arrangement (canonical site order) of the multiset
    (in-place Fisher-Yates shuffle of the sorted species array)."""
    sigma = np.repeat(np.arange(len(counts), dtype=np.uint8), np.asarray(counts))
    rng.shuffle(sigma)
    return sigma


def linear_anneal(T0: float, T1: float, n: int) -> np.ndarray:
    """T_s = T0 + (T1 - T0) s / (n - 1), s = 0..n-1."""
    if n == 1:
        return np.array([T0], dtype=np.float64)
    s = np.arange(n, dtype=np.float64)
    return T0 + (T1 - T0) * s / (n - 1)


def kernel_seed(rng: np.random.Generator) -> int:
    return int(rng.integers(0, 2**63 - 1, dtype=np.int64))


@dataclasses.dataclass
class Lattice:
    """One synthetic lattice job."""
    L: tuple
    epi: np.ndarray          # [S][K][K] int32 micro-eV
    sigma: np.ndarray        # N uint8, canonical site order
    seed: int                # Philox key
    T: np.ndarray            # per-sweep temperature, length n_sweeps
    name: str = ""
    lattice: int = BCC

    @property
    def S(self) -> int:
        return int(self.epi.shape[0])

    @property
    def K(self) -> int:
        return int(self.epi.shape[1])

    @property
    def N(self) -> int:
        return n_sites(self.L, self.lattice)

    @property
    def n_sweeps(self) -> int:
        return int(self.T.size)


def _streams(k: int):
    ss = np.random.SeedSequence(BASE_SEED + k)
    return [np.random.default_rng(c) for c in ss.spawn(5)]


def lattice_job(L, K: int, S: int, sigma_meV: float, T, comp: Optional[np.ndarray] = None,
                dirichlet: Optional[float] = None, stream: int = 0, name: str = "",
                lattice: int = BCC) -> Lattice:
    """Generic seeded lattice: EPI, composition, permutation and kernel seed
    come from four independent child streams of SeedSequence(BASE_SEED+stream)."""
    r_epi, r_comp, r_perm, _r_ladder, r_seed = _streams(stream)
    N = n_sites(L, lattice)
    epi = epi_table(S, K, sigma_meV, r_epi)
    if comp is None:
        comp = dirichlet_counts(K, N, dirichlet, r_comp) if dirichlet else equiatomic(K, N)
    sigma = configuration(comp, r_perm)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    return Lattice(tuple(int(v) for v in L), epi, sigma, kernel_seed(r_seed), T, name, lattice)


# --- the five workload shapes ------------------------------------------------

def fcc_alloy(L=(64, 64, 64), n_sweeps: int = 100, T: float = 1000.0, stream: int = 6) -> Lattice:
    """FCC quinary with the paper's alloy composition Fe29Co29Ni28Al7Ti7
    (fractions), shells 1-3, sigma 30 meV (the paper's production lattice
    is FCC; its fitted EPI is not available)."""
    N = n_sites(L, FCC)
    return lattice_job(L, 5, 3, 30.0, np.full(n_sweeps, T), comp=counts_from_fractions(FECONIALTI, N),
                       stream=stream, name=f"fcc{L[0]}_feconialti", lattice=FCC)


def config1(n_sweeps: int = 100) -> Lattice:
    """8^3 cells (1,024 sites), K=4 equiatomic, shells 1-2, sigma 20 meV, 1000 K."""
    return lattice_job((8, 8, 8), 4, 2, 20.0, np.full(n_sweeps, 1000.0), stream=1,
                       name="bcc8_k4_s2_1000K")


def config2(n_sweeps: int = 1000) -> Lattice:
    """64^3 cells (524,288 sites), K=5 equiatomic, shells 1-3, sigma 30 meV,
    linear anneal 2000 K -> 600 K over 1,000 sweeps."""
    T = linear_anneal(2000.0, 600.0, 1000)[:n_sweeps]
    return lattice_job((64, 64, 64), 5, 3, 30.0, T, stream=2, name="bcc64_k5_s3_anneal")


def config3(n_sweeps: int = 200, L: int = 512) -> Lattice:
    """512^3 cells (268,435,456 sites), K=5 Dirichlet(5), shells 1-3,
    sigma 30 meV, 800 K."""
    return lattice_job((L, L, L), 5, 3, 30.0, np.full(n_sweeps, 800.0), dirichlet=5.0,
                       stream=3, name=f"bcc{L}_k5_s3_800K")


def config4(n_replicas: int = 256, n_sweeps: int = 500, Lmin: int = 16, Lmax: int = 96) -> List[Lattice]:
    """Independent replicas: edge L ~ U{Lmin..Lmax}, K in {4,5}, T ~ U(300, 2000) K,
    Dirichlet(3) compositions, one shared 3-shell 5x5 EPI (K=4 uses its
    top-left 4x4 block)."""
    r_epi, r_comp, r_perm, r_ladder, r_seed = _streams(4)
    epi5 = epi_table(3, 5, 30.0, r_epi)
    jobs = []
    for r in range(n_replicas):
        L = int(r_ladder.integers(Lmin, Lmax + 1))
        K = int(r_ladder.integers(4, 6))
        T = float(r_ladder.uniform(300.0, 2000.0))
        N = n_sites((L, L, L))
        comp = dirichlet_counts(K, N, 3.0, r_comp)
        sigma = configuration(comp, r_perm)
        epi = np.ascontiguousarray(epi5[:, :K, :K])
        jobs.append(Lattice((L, L, L), epi, sigma, kernel_seed(r_seed), np.full(n_sweeps, T),
                            name=f"replica{r}"))
    return jobs


@dataclasses.dataclass
class Request:
    arrival_s: float
    job: Lattice


def config5(rate_hz: float = 50.0, window_s: float = 60.0, min_sites: float = 1e4,
            max_sites: float = 1e8, min_sweeps: float = 10, max_sweeps: float = 1000,
            stream: int = 5, materialize: bool = True) -> List[Request]:
    """Poisson request stream: sites log-U(min_sites, max_sites) -> cubic
    L = max(4, round((n/2)^(1/3))), K=5 Dirichlet(5), T ~ U(300, 2000) K,
    sweeps log-U(min_sweeps, max_sweeps) rounded, shared 3-shell EPI."""
    r_epi, r_comp, r_perm, r_arr, r_seed = _streams(stream)
    epi = epi_table(3, 5, 30.0, r_epi)
    out = []
    t = 0.0
    while True:
        t += float(r_arr.exponential(1.0 / rate_hz))
        if t >= window_s:
            break
        n = float(np.exp(r_arr.uniform(np.log(min_sites), np.log(max_sites))))
        L = max(4, int(round((n / 2.0) ** (1.0 / 3.0))))
        T = float(r_arr.uniform(300.0, 2000.0))
        sw = int(round(float(np.exp(r_arr.uniform(np.log(min_sweeps), np.log(max_sweeps))))))
        seed = kernel_seed(r_seed)
        N = n_sites((L, L, L))
        comp = dirichlet_counts(5, N, 5.0, r_comp)
        sigma = configuration(comp, r_perm) if materialize else np.empty(0, np.uint8)
        out.append(Request(t, Lattice((L, L, L), epi, sigma, seed, np.full(sw, T),
                                      name=f"req{len(out)}")))
    return out
