/*
 * smcx_oracle.h -- plain, slow, sequential CPU oracle for canonical-ensemble
 * Metropolis swap sweeps on a multicomponent BCC lattice with an
 * effective-pair-interaction (EPI) energy (Liu, Yang, Zhou, Xu, "SMC-X: A
 * Distributed Scalable Monte Carlo Simulation Method for Chemically Complex
 * Alloys", arXiv:2509.20949).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this code: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against an
 * independent, obviously correct reference.  It shares no source with the
 * library under paper_2509_20949_amd/.
 *
 * What each function follows:
 *   - Boltzmann target and Metropolis rule: Section "Monte Carlo simulation",
 *     Eq. (1) (canonical probability) and Eq. (3) (acceptance
 *     min(1, exp(-beta dE))).
 *   - Sweep = one trial per lattice site: same section, text after Eq. (3).
 *   - Swap moves between neighbouring sites conserve composition
 *     (Introduction; canonical ensemble, Eq. (1)).
 *   - Link-cell (block) decomposition that visits every site once per step:
 *     Section "Distributed SMC-X", equation for P_LC.  The paper does not
 *     state how the link cells are built; the reading used here (a per-sweep
 *     random origin shift of an even block grid, 8 block colours, 54 local
 *     sub-colours) is documented in the design notes and in smcx_oracle.c.
 *   - EPI energy: Section "Results and discussion" (pairwise interactions
 *     only).  The functional form E = 1/2 sum_i sum_delta V_s(sigma_i,
 *     sigma_{i+delta}) with integer micro-eV tables is a reading; the paper
 *     gives no formula.
 *   - Warren-Cowley SRO: Section "Evolution of chemical defects", Eq. (SRO):
 *     alpha_m^{pp'} = 1 - P_m^{p|p'} / c_p, centre species p'.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     written here from the published round function.  The paper names no
 *     generator.
 *
 * Conventions (all readings, see smcx_oracle.c):
 *   lat       0 = BCC (2 sites per cubic cell), 1 = FCC (4 sites per cell)
 *   site id   i = ((z*Ly + y)*Lx + x)*n_sub + b
 *   energies  int32 micro-eV per pair, table epi[s][p][q], s = shell 0..S-1
 *   k_B       86.17333262 micro-eV/K (CODATA 2018)
 */
#ifndef SMCX_ORACLE_H
#define SMCX_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Threads for the trials of one (colour, sub-colour) set and for pair sums;
 * results are bit-identical for every thread count. */
void or_set_threads(int n);
/* 1: the block grid shifts along x and y only (z-slab decomposition). */
void or_set_fixed_z(int on);
int or_get_threads(void);

/* Philox4x32-10 and its 4x64-10 sibling (same round structure, wider words). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Acceptance threshold tables for temperature T (kelvin):
 * tab[0..255] = T0, tab[256..511] = T1, tab[512..767] = T2. */
void or_thresholds(double T, double tab[768]);
/* Metropolis decision for an energy change dE (micro-eV) and a uniform
 * 32-bit draw u.  Returns 1 to accept. */
int or_accept(int64_t dE, uint32_t u, const double tab[768]);

/* Number of blocks along one axis and the block bounds b_0..b_n. */
int or_axis_blocks(int L, int B);
void or_axis_bounds(int L, int B, int32_t* bounds /* n+1 */);

/* Origin shift of sweep s. */
void or_sweep_shift(const int32_t L[3], uint64_t seed, uint32_t s, int32_t shift[3]);

/* Per-site schedule of sweep s: colour (0..7), sub-colour (0..53) and the
 * linear index of the block the site belongs to. */
void or_schedule(int lat, const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s,
                 uint8_t* colour, uint8_t* subcolour, int64_t* block);

/* BCC trial draws of sweep s for every site i: Philox counter ctr[4i..4i+3],
 * the word used, the first-neighbour vector number (bit a set = +1 on axis
 * a) and the acceptance draw.  Returns 0, or -1 on invalid arguments. */
int or_bcc_draws(const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s, uint32_t* ctr,
                 uint8_t* word, uint8_t* dir, uint32_t* u_acc);

/* FCC trial draws of sweep s for every site i: the partner's site index
 * and the acceptance draw.  Returns 0, or -1 on invalid arguments. */
int or_fcc_draws(const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s, int64_t* partner,
                 uint32_t* u_acc);

/* Site index of neighbour `k` of site i, k indexing the displacement set of
 * shells 1..S in the order documented in smcx_oracle.c. */
int64_t or_neighbour(int lat, const int32_t L[3], int64_t i, int k);
int or_shell_size(int lat, int s);
int or_n_sub(int lat);

/* Total energy (micro-eV), pair counts and Warren-Cowley SRO. */
int64_t or_energy(int lat, const int32_t L[3], int S, int K, const int32_t* epi, const uint8_t* sigma);
int64_t or_delta_energy(int lat, const int32_t L[3], int S, int K, const int32_t* epi,
                        const uint8_t* sigma, int64_t i, int64_t j);
void or_pair_counts(int lat, const int32_t L[3], int S, int K, const uint8_t* sigma, uint64_t* counts);
void or_sro(int lat, const int32_t L[3], int S, int K, const uint8_t* sigma, double* alpha,
            uint64_t* counts /* nullable */);

/* Run n sweeps, sweep indices s0 .. s0+n-1, temperature T[k] for sweep s0+k.
 * sigma is updated in place; *E (running energy) and *accepted are advanced.
 * E_trace (nullable) receives the energy after every sweep; counts_trace
 * (nullable) the pair counts [S][K][K] after every sweep.
 * Returns 0, or -1 on invalid arguments. */
int or_sweep(int lat, const int32_t L[3], const int32_t B[3], int S, int K, const int32_t* epi,
             uint64_t seed, uint32_t s0, int32_t n, const double* T, uint8_t* sigma,
             int64_t* E, uint64_t* accepted, int64_t* E_trace, uint64_t* counts_trace);

/* Replica-exchange decision for pair k of exchange round `round`. */
int or_exchange_accept(int64_t Ea, int64_t Eb, double Ta, double Tb, uint64_t seed, uint32_t k,
                       uint64_t round);

/* Exact enumeration over every configuration with the given composition.
 * Fills E_all[cfg] (nullable) and returns the number of configurations, or
 * -1 if it exceeds max_cfg. */
int64_t or_enumerate(int lat, const int32_t L[3], int S, int K, const int32_t* epi,
                     const int32_t* comp, int64_t max_cfg, int64_t* E_all,
                     uint64_t* counts_all /* nullable: [cfg][S][K][K] */);

#ifdef __cplusplus
}
#endif
#endif
