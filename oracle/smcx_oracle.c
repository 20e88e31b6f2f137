/*
 * smcx_oracle.c -- plain sequential CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares nothing with the HIP library: no headers, no
 * tables, no helpers.  Every function is written for readability, not speed.
 *
 * Paper: arXiv:2509.20949 (SMC-X).  Citations name the section and equation.
 *
 * ---------------------------------------------------------------------------
 * Geometry (reading; the paper's production lattice is FCC, the benchmark
 * lattice is BCC; both are implemented)
 *   Cells (x, y, z), 0 <= x < Lx etc., n_sub sites per cell: BCC 2 (corner,
 *   body centre), FCC 4 (corner, three face centres).  In "doubled"
 *   coordinates (units of half the lattice constant) site b of a cell sits at
 *   (2x, 2y, 2z) + SUB[b].  Periodic on every axis (the paper simulates
 *   supercells; it states no boundary condition).
 *   Site id i = ((z*Ly + y)*Lx + x)*n_sub + b.
 *
 * Neighbour shells in doubled coordinates:
 *   BCC: 8 (+-1,+-1,+-1); 6 (+-2,0,0); 12 (+-2,+-2,0) and permutations
 *   FCC: 12 (+-1,+-1,0); 6 (+-2,0,0); 24 (+-2,+-1,+-1) and permutations
 *   BCC first-shell vector number `dir` (0..7) has component +1 on axis a
 *   when bit a of dir is set, -1 otherwise.
 *
 * Energy (reading of the EPI model, Section "Results and discussion": pair
 * interactions only):  E = 1/2 sum_i sum_{delta in shells 1..S}
 *   V_{shell(delta)}(sigma_i, sigma_{i+delta}),  V symmetric int32 micro-eV.
 *   A bond whose periodic images coincide (L = 2) is counted once per
 *   displacement vector.
 * ---------------------------------------------------------------------------
 */
#include "smcx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Worker threads for the trials of one (colour, sub-colour) set and for the
 * pair sums.  The trials of one set never read what another writes (the
 * schedule guarantees it, the audit test checks it) and the sums are exact
 * integers, so any thread count gives the same bits as one thread. */
static int g_threads = 1;

void or_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int or_get_threads(void) { return g_threads; }

/* Lattice parallelism with ghost layers (Section "Distributed SMC-X"): a
 * lattice cut into z-slabs keeps its link cells aligned to the slab
 * boundaries, so the per-sweep origin shift of the block grid is applied
 * along x and y only.  or_set_fixed_z(1) selects that schedule. */
static int g_fixed_z = 0;
void or_set_fixed_z(int on) { g_fixed_z = on != 0; }

/* ------------------------------------------------------------------------ */
/* Philox (Salmon et al., SC'11, "Parallel random numbers: as easy as 1, 2,  */
/* 3").  State: four counter words and two key words.  One round multiplies */
/* words 0 and 2 by two fixed odd constants, keeping both halves of each     */
/* double-width product; the new words are                                   */
/*   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0)).    */
/* Between rounds the key is bumped by two Weyl constants.  Ten rounds.      */
/* ------------------------------------------------------------------------ */
/* Both widths are generated from one body, so that the 64-bit instance,
 * which numpy.random.Philox also implements, pins the round structure shared
 * with the 32-bit instance used for the trials. */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    /* schoolbook 64x64 -> 128 from 32-bit halves */
    uint64_t a0 = a & 0xffffffffu, a1 = a >> 32;
    uint64_t b0 = b & 0xffffffffu, b1 = b >> 32;
    uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
    uint64_t mid = (p00 >> 32) + (p01 & 0xffffffffu) + (p10 & 0xffffffffu);
    *lo = (p00 & 0xffffffffu) | (mid << 32);
    *hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

#define DEFINE_PHILOX4(NAME, WORD, MULHILO, M0, M1, W0, W1)                 \
    void NAME(const WORD ctr[4], const WORD key[2], WORD out[4])            \
    {                                                                       \
        WORD x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];            \
        WORD k0 = key[0], k1 = key[1];                                      \
        for (int r = 0; r < 10; ++r) {                                      \
            if (r > 0) { k0 += (W0); k1 += (W1); }                          \
            WORD hi0, lo0, hi1, lo1;                                        \
            MULHILO((M0), x0, &hi0, &lo0);                                  \
            MULHILO((M1), x2, &hi1, &lo1);                                  \
            WORD n0 = hi1 ^ x1 ^ k0;                                        \
            WORD n1 = lo1;                                                  \
            WORD n2 = hi0 ^ x3 ^ k1;                                        \
            WORD n3 = lo0;                                                  \
            x0 = n0; x1 = n1; x2 = n2; x3 = n3;                             \
        }                                                                   \
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;                 \
    }

/* constants of the SC'11 paper: multipliers, then Weyl key increments
 * (golden ratio and sqrt(3) - 1 in fixed point) */
DEFINE_PHILOX4(or_philox4x32_10, uint32_t, mulhilo32,
               0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
DEFINE_PHILOX4(or_philox4x64_10, uint64_t, mulhilo64,
               0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
               0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* ------------------------------------------------------------------------ */
/* Metropolis acceptance, Eq. (3): accept with probability 1 if dE <= 0,    */
/* exp(-beta dE) otherwise.  Reading for exact reproducibility: a uniform   */
/* 32-bit draw u is accepted iff (double)u < 2^32 exp(-beta dE), where the  */
/* right-hand side is assembled from three 256-entry FP64 tables indexed by */
/* the bytes of dE, multiplied in a fixed order.  dE >= 2^24 is rejected    */
/* (for T <= 5000 K its probability is below 2^-32).                        */
/* ------------------------------------------------------------------------ */
void or_thresholds(double T, double tab[768])
{
    const double kB_ueV_per_K = 86.17333262; /* CODATA 2018, micro-eV / K */
    double beta = 1.0 / (kB_ueV_per_K * T);
    for (int l = 0; l < 256; ++l) {
        tab[l] = exp(-((double)l * beta));
        tab[256 + l] = exp(-((double)(l * 256) * beta));
        tab[512 + l] = ldexp(exp(-((double)(l * 65536) * beta)), 32);
    }
}

int or_accept(int64_t dE, uint32_t u, const double tab[768])
{
    if (dE <= 0) return 1;
    if (dE >= (1 << 24)) return 0;
    double thr = (tab[512 + (dE >> 16)] * tab[256 + ((dE >> 8) & 255)]) * tab[dE & 255];
    return (double)u < thr;
}

/* ------------------------------------------------------------------------ */
/* Geometry.  lat = 0: BCC, two sites per cubic cell (corner, body centre);  */
/* lat = 1: FCC, four sites per cubic cell (corner and three face centres). */
/* In doubled coordinates (units of half the lattice constant) site b of   */
/* cell (x, y, z) sits at (2x, 2y, 2z) + SUB[b].  Site id = cell * n_sub + b, */
/* cell = (z*Ly + y)*Lx + x.                                                 */
/* ------------------------------------------------------------------------ */
static const int SUB_BCC[2][3] = {{0, 0, 0}, {1, 1, 1}};
static const int SUB_FCC[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};

/* BCC shells: 8 first neighbours (+-1,+-1,+-1) -- vector number dir has +1
 * on axis a when bit a of dir is set --, 6 second (+-2,0,0), 12 third
 * (+-2,+-2,0). */
static const int BCC1[8][3] = {
    {-1, -1, -1}, {+1, -1, -1}, {-1, +1, -1}, {+1, +1, -1},
    {-1, -1, +1}, {+1, -1, +1}, {-1, +1, +1}, {+1, +1, +1}};
static const int SHELL2[6][3] = {
    {+2, 0, 0}, {-2, 0, 0}, {0, +2, 0}, {0, -2, 0}, {0, 0, +2}, {0, 0, -2}};
static const int BCC3[12][3] = {
    {+2, +2, 0}, {+2, -2, 0}, {-2, +2, 0}, {-2, -2, 0},
    {+2, 0, +2}, {+2, 0, -2}, {-2, 0, +2}, {-2, 0, -2},
    {0, +2, +2}, {0, +2, -2}, {0, -2, +2}, {0, -2, -2}};
/* FCC shells: 12 first neighbours (+-1,+-1,0) and permutations, 6 second
 * (+-2,0,0), 24 third (+-2,+-1,+-1) and permutations. */
static const int FCC1[12][3] = {
    {+1, +1, 0}, {+1, -1, 0}, {-1, +1, 0}, {-1, -1, 0},
    {+1, 0, +1}, {+1, 0, -1}, {-1, 0, +1}, {-1, 0, -1},
    {0, +1, +1}, {0, +1, -1}, {0, -1, +1}, {0, -1, -1}};
static const int FCC3[24][3] = {
    {+2, +1, +1}, {+2, +1, -1}, {+2, -1, +1}, {+2, -1, -1},
    {-2, +1, +1}, {-2, +1, -1}, {-2, -1, +1}, {-2, -1, -1},
    {+1, +2, +1}, {+1, +2, -1}, {-1, +2, +1}, {-1, +2, -1},
    {+1, -2, +1}, {+1, -2, -1}, {-1, -2, +1}, {-1, -2, -1},
    {+1, +1, +2}, {+1, -1, +2}, {-1, +1, +2}, {-1, -1, +2},
    {+1, +1, -2}, {+1, -1, -2}, {-1, +1, -2}, {-1, -1, -2}};

int or_n_sub(int lat) { return lat == 1 ? 4 : 2; }

int or_shell_size(int lat, int s)
{
    if (lat == 1) return s == 0 ? 12 : (s == 1 ? 6 : 24);
    return s == 0 ? 8 : (s == 1 ? 6 : 12);
}

/* displacement k of the concatenated list shell1 ++ shell2 ++ shell3 */
static const int* displacement(int lat, int k, int* shell)
{
    int n1 = or_shell_size(lat, 0), n2 = or_shell_size(lat, 1);
    if (k < n1) { *shell = 0; return lat == 1 ? FCC1[k] : BCC1[k]; }
    if (k < n1 + n2) { *shell = 1; return SHELL2[k - n1]; }
    *shell = 2;
    return lat == 1 ? FCC3[k - n1 - n2] : BCC3[k - n1 - n2];
}

static int64_t wrap(int64_t v, int64_t m) { v %= m; return v < 0 ? v + m : v; }

/* A site in decoded form: doubled coordinates X, Y, Z. */
typedef struct { int64_t X, Y, Z; } site_xyz;

static site_xyz decode_site(int lat, const int32_t L[3], int64_t i)
{
    int nsub = or_n_sub(lat);
    int64_t b = i % nsub, cell = i / nsub;
    int64_t x = cell % L[0], y = (cell / L[0]) % L[1], z = cell / ((int64_t)L[0] * L[1]);
    const int* o = lat == 1 ? SUB_FCC[b] : SUB_BCC[b];
    site_xyz p = {2 * x + o[0], 2 * y + o[1], 2 * z + o[2]};
    return p;
}

/* periodic add of a displacement component in [-2, 2] to X in [0, 2L) */
static int64_t wrap_small(int64_t v, int64_t twoL) { return v < 0 ? v + twoL : (v >= twoL ? v - twoL : v); }

static int64_t site_at(int lat, const int32_t L[3], site_xyz p, const int* d)
{
    int64_t X = wrap_small(p.X + d[0], 2 * (int64_t)L[0]);
    int64_t Y = wrap_small(p.Y + d[1], 2 * (int64_t)L[1]);
    int64_t Z = wrap_small(p.Z + d[2], 2 * (int64_t)L[2]);
    int64_t cell = ((Z >> 1) * L[1] + (Y >> 1)) * L[0] + (X >> 1);
    int parity = (int)((X & 1) | (Y & 1) << 1 | (Z & 1) << 2);
    int b;
    if (lat == 1) {
        static const int SUB_OF_PARITY[8] = {0, -1, -1, 1, -1, 2, 3, -1};
        b = SUB_OF_PARITY[parity];
    } else {
        b = parity == 7 ? 1 : 0;
    }
    return cell * or_n_sub(lat) + b;
}

int64_t or_neighbour(int lat, const int32_t L[3], int64_t i, int k)
{
    int shell;
    const int* d = displacement(lat, k, &shell);
    return site_at(lat, L, decode_site(lat, L, i), d);
}

static int n_displacements(int lat, int S)
{
    int n = 0;
    for (int s = 0; s < S; ++s) n += or_shell_size(lat, s);
    return n;
}

static int64_t n_sites(int lat, const int32_t L[3]) { return or_n_sub(lat) * (int64_t)L[0] * L[1] * L[2]; }

/* ------------------------------------------------------------------------ */
/* Energy, energy change, pair counts, SRO                                   */
/* ------------------------------------------------------------------------ */
int64_t or_energy(int lat, const int32_t L[3], int S, int K, const int32_t* epi, const uint8_t* sigma)
{
    int64_t N = n_sites(lat, L), twiceE = 0;
    int nd = n_displacements(lat, S);
#pragma omp parallel for reduction(+ : twiceE) num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        site_xyz p = decode_site(lat, L, i);
        for (int k = 0; k < nd; ++k) {
            int s;
            const int* d = displacement(lat, k, &s);
            int64_t n = site_at(lat, L, p, d);
            twiceE += epi[(s * K + sigma[i]) * K + sigma[n]];
        }
    }
    return twiceE / 2;
}

/* Energy change of exchanging the species of sites i and j (j a first
 * neighbour of i).  Only bonds touching i or j change; the bond i-j itself
 * is unchanged because V is symmetric:
 *   dE = sum_{delta, i+delta != j} [V(sj, s_{i+delta}) - V(si, s_{i+delta})]
 *      + sum_{delta, j+delta != i} [V(si, s_{j+delta}) - V(sj, s_{j+delta})]  */
int64_t or_delta_energy(int lat, const int32_t L[3], int S, int K, const int32_t* epi,
                        const uint8_t* sigma, int64_t i, int64_t j)
{
    int nd = n_displacements(lat, S);
    int si = sigma[i], sj = sigma[j];
    site_xyz pi = decode_site(lat, L, i), pj = decode_site(lat, L, j);
    int64_t dE = 0;
    for (int k = 0; k < nd; ++k) {
        int s;
        const int* d = displacement(lat, k, &s);
        int64_t n = site_at(lat, L, pi, d);
        if (n != j) dE += epi[(s * K + sj) * K + sigma[n]] - epi[(s * K + si) * K + sigma[n]];
        int64_t m = site_at(lat, L, pj, d);
        if (m != i) dE += epi[(s * K + si) * K + sigma[m]] - epi[(s * K + sj) * K + sigma[m]];
    }
    return dE;
}

/* counts[m][p'][p] = number of (centre i of species p', displacement of
 * shell m, neighbour of species p). */
void or_pair_counts(int lat, const int32_t L[3], int S, int K, const uint8_t* sigma, uint64_t* counts)
{
    int64_t N = n_sites(lat, L);
    int nd = n_displacements(lat, S);
    size_t nc = (size_t)S * K * K;
    memset(counts, 0, sizeof(uint64_t) * nc);
#pragma omp parallel num_threads(g_threads)
    {
        uint64_t* mine = (uint64_t*)calloc(nc, sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            site_xyz p = decode_site(lat, L, i);
            for (int k = 0; k < nd; ++k) {
                int s;
                const int* d = displacement(lat, k, &s);
                int64_t n = site_at(lat, L, p, d);
                mine[(s * K + sigma[i]) * K + sigma[n]] += 1;
            }
        }
#pragma omp critical
        for (size_t c = 0; c < nc; ++c) counts[c] += mine[c];
        free(mine);
    }
}

/* Warren-Cowley SRO, Eq. (SRO): alpha_m^{pp'} = 1 - P_m^{p|p'} / c_p with
 * P_m^{p|p'} = counts[m][p'][p] / (Z_m N_{p'}), c_p = N_p / N.  Stored at
 * alpha[(m*K + p')*K + p].  NaN when N_p or N_{p'} is zero (reading). */
void or_sro(int lat, const int32_t L[3], int S, int K, const uint8_t* sigma, double* alpha, uint64_t* counts)
{
    int64_t N = n_sites(lat, L);
    uint64_t* c = counts ? counts : (uint64_t*)malloc(sizeof(uint64_t) * S * K * K);
    or_pair_counts(lat, L, S, K, sigma, c);
    int64_t Np[256] = {0};
    for (int64_t i = 0; i < N; ++i) Np[sigma[i]] += 1;
    for (int m = 0; m < S; ++m)
        for (int pc = 0; pc < K; ++pc)
            for (int p = 0; p < K; ++p) {
                double P = (double)c[(m * K + pc) * K + p] / ((double)or_shell_size(lat, m) * (double)Np[pc]);
                double cp = (double)Np[p] / (double)N;
                alpha[(m * K + pc) * K + p] = (Np[p] == 0 || Np[pc] == 0) ? NAN : 1.0 - P / cp;
            }
    if (!counts) free(c);
}

/* ------------------------------------------------------------------------ */
/* Schedule of one sweep (reading of the dynamical link cells, Section      */
/* "Distributed SMC-X": every site is visited exactly once per step, and     */
/* sites updated together are separated by more than the interaction range).*/
/*                                                                           */
/* Per axis with L cells and block-width parameter B:                        */
/*   n = 1 if L < 4, else n = max(2, min(2*ceil(L/(2B)), 2*floor(L/4)))      */
/*   (even, every block at least 2 and at most max(B, 4) cells wide),        */
/*   bounds b_k = floor(k*L/n).                                              */
/* Sweep s draws an origin shift o_a = (r_a * L_a) >> 32 from                */
/*   Philox4x32-10(key = seed, counter = (0, 0, s, 8)).                      */
/* Cell coordinate x_a maps to u_a = (x_a - o_a) mod L_a, block k_a with     */
/* b_k <= u_a < b_{k+1}, local coordinate l_a = u_a - b_k.                   */
/* Colour c = (k_x & 1) | (k_y & 1) << 1 | (k_z & 1) << 2, phases c = 0..7.  */
/* Sub-colour q = (((l_z%3)*3 + l_y%3)*3 + l_x%3)*n_sub + b: 54 rounds      */
/* (BCC) or 108 (FCC).                                                      */
/* Trials run colour by colour, sub-colour by sub-colour, and inside one     */
/* (c, q) set in ascending site id (the trials of one set commute).          */
/* ------------------------------------------------------------------------ */
int or_axis_blocks(int L, int B)
{
    if (L < 4) return 1;
    int n = 2 * ((L + 2 * B - 1) / (2 * B));
    int cap = 2 * (L / 4);
    if (n > cap) n = cap;
    if (n < 2) n = 2;
    return n;
}

void or_axis_bounds(int L, int B, int32_t* bounds)
{
    int n = or_axis_blocks(L, B);
    for (int k = 0; k <= n; ++k) bounds[k] = (int32_t)(((int64_t)k * L) / n);
}

void or_sweep_shift(const int32_t L[3], uint64_t seed, uint32_t s, int32_t shift[3])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {0u, 0u, s, 8u};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    for (int a = 0; a < 3; ++a) shift[a] = (int32_t)(((uint64_t)r[a] * (uint64_t)L[a]) >> 32);
    if (g_fixed_z) shift[2] = 0;
}

/* base (nullable, one entry per cell): the cell whose local coordinates are
 * 3 * floor(l / 3) on every axis, in the same block (the cell of residue 0
 * in the cell's group of 3 x 3 x 3 residues). */
static void schedule_full(int lat, const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s,
                          uint8_t* colour, uint8_t* subcolour, int64_t* block, int64_t* base)
{
    const int nsub = or_n_sub(lat);
    int32_t shift[3];
    or_sweep_shift(L, seed, s, shift);
    /* per axis and cell coordinate x: block index k and local coordinate l */
    int n[3];
    int32_t* kof[3];
    int32_t* lof[3];
    for (int a = 0; a < 3; ++a) {
        n[a] = or_axis_blocks(L[a], B[a]);
        int32_t* bounds = (int32_t*)malloc(sizeof(int32_t) * (n[a] + 1));
        or_axis_bounds(L[a], B[a], bounds);
        kof[a] = (int32_t*)malloc(sizeof(int32_t) * L[a]);
        lof[a] = (int32_t*)malloc(sizeof(int32_t) * L[a]);
        for (int32_t x = 0; x < L[a]; ++x) {
            int64_t u = wrap((int64_t)x - shift[a], L[a]);
            int kk = 0;
            while (!(bounds[kk] <= u && u < bounds[kk + 1])) ++kk;
            kof[a][x] = kk;
            lof[a][x] = (int32_t)(u - bounds[kk]);
        }
        free(bounds);
    }
    int64_t cell = 0;
    for (int64_t z = 0; z < L[2]; ++z)
        for (int64_t y = 0; y < L[1]; ++y)
            for (int64_t x = 0; x < L[0]; ++x, ++cell) {
                int kx = kof[0][x], ky = kof[1][y], kz = kof[2][z];
                int lx = lof[0][x], ly = lof[1][y], lz = lof[2][z];
                uint8_t c = (uint8_t)((kx & 1) | ((ky & 1) << 1) | ((kz & 1) << 2));
                uint8_t q = (uint8_t)((((lz % 3) * 3 + ly % 3) * 3 + lx % 3) * nsub);
                for (int b = 0; b < nsub; ++b) {
                    colour[nsub * cell + b] = c;
                    subcolour[nsub * cell + b] = (uint8_t)(q + b);
                    if (block) block[nsub * cell + b] = ((int64_t)kz * n[1] + ky) * n[0] + kx;
                }
                if (base) {
                    int64_t bx = wrap(x - lx % 3, L[0]), by = wrap(y - ly % 3, L[1]), bz = wrap(z - lz % 3, L[2]);
                    base[cell] = (bz * L[1] + by) * L[0] + bx;
                }
            }
    for (int a = 0; a < 3; ++a) { free(kof[a]); free(lof[a]); }
}

void or_schedule(int lat, const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s,
                 uint8_t* colour, uint8_t* subcolour, int64_t* block)
{
    schedule_full(lat, L, B, seed, s, colour, subcolour, block, NULL);
}

/* BCC trial draws (reading; the paper fixes neither the random numbers nor
 * how a swap partner is picked beyond its being a nearest neighbour).
 *   A trial at site (cell, b) with residue m = ((l_z%3)*3 + l_y%3)*3 + l_x%3
 *   (sub-colour q = 2m + b) takes the 32-bit word 2*(m & 1) + b of
 *   Philox4x32-10(key = seed, counter = (g lo, g hi, s, c + 256*(m >> 1))),
 *   g = the cell's base cell (see schedule_full): one call serves the four
 *   trials of residues 2k and 2k+1 of one base cell.  The word is the
 *   trial's acceptance draw, compared as in or_accept.
 *   Partner: first-neighbour vector number dir (bit a set = +1 on axis a),
 *   shared by all trials of one (sweep, colour, sub-colour) set, as for
 *   FCC: bit 0 (x) is bit q of the 128-bit string X_c =
 *   Philox4x32-10(key, (0, 0, s, 40 + c)); bits 1 (y) and 2 (z) are bits 2q
 *   and 2q+1 of R_c = Philox4x32-10(key, (0, 0, s, 32 + c)), bit t of a
 *   string being bit t%32 of word t/32.  Every trial still proposes the
 *   swap of one fixed pair, chosen without looking at the configuration, so
 *   each trial is a Metropolis step reversible with respect to Eq. (1); over
 *   the set draws dir is uniform on 0..7. */
static int set_bit(const uint32_t R[4], int t) { return (int)((R[t >> 5] >> (t & 31)) & 1u); }

/* R: R_c (words 0..3) and X_c (words 4..7) of the trial's colour */
static void bcc_draw(const uint32_t key[2], uint32_t s, int c, int q, int64_t g, const uint32_t R[8],
                     uint32_t ctr[4], int* word, int* dir, uint32_t* u_acc)
{
    int m = q >> 1, b = q & 1;
    ctr[0] = (uint32_t)g;
    ctr[1] = (uint32_t)((uint64_t)g >> 32);
    ctr[2] = s;
    ctr[3] = (uint32_t)c + 256u * (uint32_t)(m >> 1);
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    *word = 2 * (m & 1) + b;
    *dir = set_bit(R + 4, q) | set_bit(R, 2 * q) << 1 | set_bit(R, 2 * q + 1) << 2;
    *u_acc = r[*word];
}

static void bcc_set_bits(const uint32_t key[2], uint32_t s, int c, uint32_t R[8])
{
    uint32_t ctr[4] = {0u, 0u, s, 32u + (uint32_t)c};
    or_philox4x32_10(ctr, key, R);
    uint32_t cx[4] = {0u, 0u, s, 40u + (uint32_t)c};
    or_philox4x32_10(cx, key, R + 4);
}

int or_bcc_draws(const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s, uint32_t* ctr,
                 uint8_t* word, uint8_t* dir, uint32_t* u_acc)
{
    for (int a = 0; a < 3; ++a)
        if (L[a] < 2 || B[a] < 2) return -1;
    int64_t N = n_sites(0, L), ncell = N / 2;
    uint8_t* colour = (uint8_t*)malloc(N);
    uint8_t* sub = (uint8_t*)malloc(N);
    int64_t* base = (int64_t*)malloc(sizeof(int64_t) * ncell);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t R[8][8];
    schedule_full(0, L, B, seed, s, colour, sub, NULL, base);
    for (int c = 0; c < 8; ++c) bcc_set_bits(key, s, c, R[c]);
    for (int64_t i = 0; i < N; ++i) {
        int w, d;
        uint32_t u;
        bcc_draw(key, s, colour[i], sub[i], base[i / 2], R[colour[i]], ctr + 4 * i, &w, &d, &u);
        word[i] = (uint8_t)w;
        dir[i] = (uint8_t)d;
        u_acc[i] = u;
    }
    free(colour);
    free(sub);
    free(base);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sweeps                                                                    */
/* ------------------------------------------------------------------------ */
static int valid_inputs(const int32_t L[3], const int32_t B[3], int S, int K, const int32_t* epi)
{
    if (S < 1 || S > 3 || K < 1 || K > 255) return 0;
    for (int a = 0; a < 3; ++a)
        if (L[a] < 2 || B[a] < 2) return 0;
    for (int s = 0; s < S; ++s)
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q)
                if (epi[(s * K + p) * K + q] != epi[(s * K + q) * K + p]) return 0;
    return 1;
}

/* FCC partner choice (reading; the paper states none).  A site of
 * sublattice b has 12 first neighbours, 4 in each other sublattice.  The
 * partner of every trial of one (sweep s, colour c, sub-colour q) set is
 * drawn once, from r = Philox4x32-10(key, (q, 0, s, c + 64)): the partner
 * sublattice b' = the k-th sublattice other than b in increasing order,
 * k = (r0 * 3) >> 32, and on the two axes where b and b' differ the
 * neighbour (+-1, +-1) with the signs given by bits 30 (first axis) and 31
 * (second axis) of r1, set = +1.  Every trial still swaps one fixed pair
 * chosen without looking at the configuration (a reversible Metropolis
 * step of Eq. (1)); over the set draw the partner is uniform over the 12.
 * The trial's own draw is only its acceptance word (see or_sweep). */
static int fcc_partner_sublattice(const uint32_t key[2], uint32_t s, int c, int q, uint32_t* signs)
{
    uint32_t ctr[4] = {(uint32_t)q, 0u, s, (uint32_t)c + 64u};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    *signs = r[1];
    int b = q % 4, k = (int)(((uint64_t)r[0] * 3u) >> 32);
    for (int bp = 0; bp < 4; ++bp) {
        if (bp == b) continue;
        if (k-- == 0) return bp;
    }
    return -1;
}

static int64_t fcc_partner(const int32_t L[3], int64_t i, int bp, uint32_t signs)
{
    int b = (int)(i % 4);
    int d[3] = {0, 0, 0};
    int bit = 30;
    for (int a = 0; a < 3; ++a)
        if (SUB_FCC[b][a] != SUB_FCC[bp][a]) {
            d[a] = ((signs >> bit) & 1u) ? +1 : -1;
            ++bit;
        }
    return site_at(1, L, decode_site(1, L, i), d);
}

int or_fcc_draws(const int32_t L[3], const int32_t B[3], uint64_t seed, uint32_t s, int64_t* partner,
                 uint32_t* u_acc)
{
    for (int a = 0; a < 3; ++a)
        if (L[a] < 2 || B[a] < 2) return -1;
    int64_t N = n_sites(1, L);
    uint8_t* colour = (uint8_t*)malloc(N);
    uint8_t* sub = (uint8_t*)malloc(N);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int psub[8 * 108];
    uint32_t psign[8 * 108];
    schedule_full(1, L, B, seed, s, colour, sub, NULL, NULL);
    for (int g = 0; g < 8 * 108; ++g) psub[g] = fcc_partner_sublattice(key, s, g / 108, g % 108, &psign[g]);
    for (int64_t i = 0; i < N; ++i) {
        int64_t cell = i / 4;
        int g = colour[i] * 108 + sub[i];
        uint32_t ctr[4] = {(uint32_t)cell, (uint32_t)(cell >> 32), s, (uint32_t)colour[i]};
        uint32_t rnd[4];
        or_philox4x32_10(ctr, key, rnd);
        u_acc[i] = rnd[i % 4];
        partner[i] = fcc_partner(L, i, psub[g], psign[g]);
    }
    free(colour);
    free(sub);
    return 0;
}

int or_sweep(int lat, const int32_t L[3], const int32_t B[3], int S, int K, const int32_t* epi,
             uint64_t seed, uint32_t s0, int32_t n, const double* T, uint8_t* sigma,
             int64_t* E, uint64_t* accepted, int64_t* E_trace, uint64_t* counts_trace)
{
    if ((lat != 0 && lat != 1) || !valid_inputs(L, B, S, K, epi) || n < 0) return -1;
    const int nsub = or_n_sub(lat);
    const int ngroups = 8 * 27 * nsub;
    int64_t N = n_sites(lat, L);
    for (int64_t i = 0; i < N; ++i)
        if (sigma[i] >= K) return -1;
    uint8_t* colour = (uint8_t*)malloc(N);
    uint8_t* sub = (uint8_t*)malloc(N);
    int64_t* base = lat == 0 ? (int64_t*)malloc(sizeof(int64_t) * (N / 2)) : NULL;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * N);
    uint32_t R[8][8];
    int64_t start[8 * 27 * 4 + 1];
    int partner_sub[8 * 27 * 4];
    uint32_t partner_signs[8 * 27 * 4];
    double tab[768];
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};

    for (int32_t t = 0; t < n; ++t) {
        uint32_t s = s0 + (uint32_t)t;
        or_thresholds(T[t], tab);
        schedule_full(lat, L, B, seed, s, colour, sub, NULL, base);
        if (lat == 0)
            for (int c = 0; c < 8; ++c) bcc_set_bits(key, s, c, R[c]);
        /* order: counting sort on (colour, sub-colour), stable in site id */
        memset(start, 0, sizeof(start));
        for (int64_t i = 0; i < N; ++i) start[colour[i] * 27 * nsub + sub[i] + 1] += 1;
        for (int g = 0; g < ngroups; ++g) start[g + 1] += start[g];
        for (int64_t i = 0; i < N; ++i) order[start[colour[i] * 27 * nsub + sub[i]]++] = i;

        /* FCC: one partner sublattice per (colour, sub-colour) set */
        if (lat == 1)
            for (int g = 0; g < ngroups; ++g)
                partner_sub[g] = fcc_partner_sublattice(key, s, g / (27 * nsub), g % (27 * nsub), &partner_signs[g]);
        for (int g = 0; g < ngroups; ++g) {
            int64_t lo = g == 0 ? 0 : start[g - 1], hi = start[g];
            int64_t dE_set = 0;
            uint64_t acc_set = 0;
#pragma omp parallel for reduction(+ : dE_set, acc_set) num_threads(g_threads) schedule(static) \
    if (hi - lo > 512)
            for (int64_t r = lo; r < hi; ++r) {
                int64_t i = order[r];
                int64_t cell = i / nsub;
                int b = (int)(i % nsub);
                int64_t j;
                uint32_t u_acc;
                if (lat == 0) {
                    uint32_t ctr[4];
                    int word, dir;
                    bcc_draw(key, s, colour[i], sub[i], base[cell], R[colour[i]], ctr, &word, &dir, &u_acc);
                    j = or_neighbour(0, L, i, dir);
                } else {
                    /* FCC: the four sites of a cell share one Philox call,
                     * site b taking word b as its acceptance draw */
                    uint32_t ctr[4] = {(uint32_t)cell, (uint32_t)(cell >> 32), s, (uint32_t)colour[i]};
                    uint32_t rnd[4];
                    or_philox4x32_10(ctr, key, rnd);
                    u_acc = rnd[b];
                    j = fcc_partner(L, i, partner_sub[g], partner_signs[g]);
                }
                if (sigma[i] == sigma[j]) continue;
                int64_t dE = or_delta_energy(lat, L, S, K, epi, sigma, i, j);
                if (or_accept(dE, u_acc, tab)) {
                    uint8_t tmp = sigma[i];
                    sigma[i] = sigma[j];
                    sigma[j] = tmp;
                    dE_set += dE;
                    acc_set += 1;
                }
            }
            *E += dE_set;
            *accepted += acc_set;
        }
        if (E_trace) E_trace[t] = *E;
        if (counts_trace) or_pair_counts(lat, L, S, K, sigma, counts_trace + (size_t)t * S * K * K);
    }
    free(colour);
    free(sub);
    free(base);
    free(order);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact enumeration (Eq. (1) evaluated by brute force on tiny cells).       */
/* Visits every arrangement of the multiset given by comp[] in lexicographic */
/* order (next permutation of a sorted sequence).                            */
/* ------------------------------------------------------------------------ */
static int next_multiset_permutation(uint8_t* a, int64_t n)
{
    int64_t k = n - 2;
    while (k >= 0 && a[k] >= a[k + 1]) --k;
    if (k < 0) return 0;
    int64_t l = n - 1;
    while (a[l] <= a[k]) --l;
    uint8_t t = a[k]; a[k] = a[l]; a[l] = t;
    for (int64_t p = k + 1, q = n - 1; p < q; ++p, --q) { t = a[p]; a[p] = a[q]; a[q] = t; }
    return 1;
}

int64_t or_enumerate(int lat, const int32_t L[3], int S, int K, const int32_t* epi,
                     const int32_t* comp, int64_t max_cfg, int64_t* E_all, uint64_t* counts_all)
{
    int64_t N = n_sites(lat, L), tot = 0;
    for (int p = 0; p < K; ++p) tot += comp[p];
    if (tot != N) return -1;
    uint8_t* a = (uint8_t*)malloc(N);
    int64_t pos = 0;
    for (int p = 0; p < K; ++p)
        for (int32_t c = 0; c < comp[p]; ++c) a[pos++] = (uint8_t)p;
    int64_t cfg = 0;
    do {
        if (cfg >= max_cfg) { free(a); return -1; }
        if (E_all) E_all[cfg] = or_energy(lat, L, S, K, epi, a);
        if (counts_all) or_pair_counts(lat, L, S, K, a, counts_all + (size_t)cfg * S * K * K);
        ++cfg;
    } while (next_multiset_permutation(a, N));
    free(a);
    return cfg;
}

/* ------------------------------------------------------------------------ */
/* Replica exchange (Section "Distributed SMC-X", equations for P_swap and  */
/* Delta): configurations at T_a and T_b with energies E_a, E_b swap with   */
/* probability min(1, exp(Delta)), Delta = (1/k_B)(1/T_a - 1/T_b)(E_a - E_b).*/
/* Reading for reproducibility: pair k of exchange round `round` draws       */
/* u = word 0 of Philox4x32-10(key = seed, counter = (k, round lo, round hi, */
/* 9)) and accepts iff (double)u < 2^32 min(1, exp(Delta)).                  */
/* ------------------------------------------------------------------------ */
int or_exchange_accept(int64_t Ea, int64_t Eb, double Ta, double Tb, uint64_t seed, uint32_t k,
                       uint64_t round)
{
    const double kB_ueV_per_K = 86.17333262;
    double delta = (1.0 / kB_ueV_per_K) * (1.0 / Ta - 1.0 / Tb) * ((double)Ea - (double)Eb);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {k, (uint32_t)round, (uint32_t)(round >> 32), 9u};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    double p = delta >= 0.0 ? 1.0 : exp(delta);
    return (double)r[0] < ldexp(p, 32);
}
