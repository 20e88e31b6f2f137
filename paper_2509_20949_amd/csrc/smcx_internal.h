// smcx_internal.h -- types shared by the host and device parts of libsmcx.
//
// Nothing here is part of the C ABI (include/smcx.h).  The library is written
// for gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace smcx {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerGroup = 4;    // blocks (one per wave) per workgroup, BCC
constexpr int kWavesPerGroupFcc = 2; // FCC: its 13.9 KB block images fit 5 workgroups of 2 per CU
constexpr int kWavesPerGroupFccWide = 11;   // FCC single lattice: 11 images fill a CU's 160 KB of LDS
constexpr int kMaxBlock = 12;        // widest block: 4 x 4 x 4 cells per sub-colour round
constexpr int kMaxK = 8;
constexpr int kMaxS = 3;

// LDS image of one block: two byte arrays (corner and body sublattice) of
// 15 x 15 x 15 cells.  Corner array covers local cells -1..13, body array
// -2..12, so a block of width <= 12 plus its interaction halo fits.
// The plane pitch is padded from 225 to 231 bytes: with the lane-to-cell map
// of lane_cell() (device_common.h), the 64 bytes a wave reads at one common
// offset then lie in distinct 4-byte LDS banks of each half-wave (or share a
// dword), for every offset a trial uses; at 225 they collide 3-way.
constexpr int kP = 15;               // row pitch (cells)
constexpr int kPP = 231;             // plane pitch (15 rows + 6 bytes of padding)
constexpr int kArr = 3460;           // bytes per sublattice array (last byte 14*231 + 14*15 + 14)
// Bytes per wave: the two arrays.
constexpr int kWaveLds = 2 * kArr;
static_assert(kPP >= 15 * kP && kArr > 14 * kPP + 14 * kP + 14, "LDS array too small");

// Threshold tables: T0 | T1 | T2, 256 doubles each, then ln(2) k_B T in
// micro-eV (the scale of the acceptance bounds, device_common.h) and a pad.
constexpr int kTab = 770;
constexpr int kTabLn2kT = 768;

// Row of the pair-weight table for one (sigma_i, sigma_j) = (a, b):
// W[s][p] = V_s(b, p) - V_s(a, p) for s < SMAX, p < KMAX, then a constant;
// or, in the byte-dot form (tables.cpp), 3 SMAX packed digit words and a
// constant.  Entries per row, padded to a multiple of 4:
__host__ __device__ constexpr int wrow_entries(int kmax, int smax)
{
    return (smax * kmax > 3 * smax ? smax * kmax : 3 * smax) + 1;
}
__host__ __device__ constexpr int wrow(int kmax, int smax) { return (wrow_entries(kmax, smax) + 3) & ~3; }

// DevLattice::drop_last: the form of the weight rows (tables.cpp).
constexpr int kWtabFull = 0;   // KMAX fields per shell
constexpr int kWtabDrop = 1;   // KMAX-1 fields, the last species folded in
constexpr int kWtabDot = 2;    // byte-dot digits (KMAX <= 5)

// Running energy (micro-eV, int64) and accepted-swap count (uint64) of one
// lattice, spread over kSpread slots one cache line apart: the wave of block
// f adds its totals to slot f % kSpread, so one launch's thousands of
// device-scope atomics do not all meet on a single address (they serialise
// there).  The values are the sums over the slots; state_init/state_sum
// (tables.cpp) write and read the host image.
constexpr int kSpread = 128;
constexpr int kSlotWords = 8;                        // 64 bytes per slot: energy, accepted, padding
constexpr int kStateWords = kSpread * kSlotWords;    // int64 words per lattice
void state_init(int64_t* h /* kStateWords */, int64_t E, uint64_t accepted);
void state_sum(const int64_t* h /* kStateWords */, int64_t* E, uint64_t* accepted);

// Pair counts N_m[p'][p] as the pair-count kernel leaves them: kCountSlots
// copies of [kMaxS][kMaxK][kMaxK] uint64, workgroup b adding into copy
// b % kCountSlots (its atomics then meet few others on an address); the
// counts are the sums over the copies (count_sum, tables.cpp).
constexpr int kCountWords = kMaxS * kMaxK * kMaxK;
constexpr int kCountSlots = 16;
constexpr size_t kCountBytes = sizeof(unsigned long long) * kCountWords * kCountSlots;
void count_sum(const unsigned long long* slots /* kCountSlots * kCountWords */, unsigned long long* out /* kCountWords */);

// Per-lattice state the kernels read (device memory).
struct DevLattice {
    uint8_t* species;        // 2*Lx*Ly*Lz bytes, canonical order (slab: 2*Lx*Ly*(Lz+4), see below)
    const double* tabs;      // n_tabs x 768 thresholds
    const int32_t* wtab;     // KMAX*KMAX rows of wrow(KMAX, SMAX) ints
    int64_t* state;          // running energy and accepted count, kStateWords words (see below)
    int32_t L[3];
    int32_t nb[3];           // blocks per axis (even)
    uint32_t key[2];
    uint32_t sweep0;         // sweep index of launch step t = 0
    uint32_t tab_s0;         // sweep index of tabs[0]
    int32_t n_tabs;          // later sweeps reuse the last table
    int32_t K;
    int32_t blocks_per_colour;
    int32_t lattice;         // 0 BCC, 1 FCC
    int32_t drop_last;       // form of the weight rows: kWtabFull, kWtabDrop or kWtabDot
    int32_t slab;            // 1: z-slab of a larger lattice (BCC); species points at 2 halo planes below it,
                             // 2 more follow it, z is not shifted and not wrapped
    uint32_t z_off;          // slab: global z of the slab's first plane (random-number cell ids)
};

// One workgroup's share of a batched phase: kWavesPerGroup consecutive
// same-colour blocks of one lattice.
struct WorkItem {
    int32_t lattice;
    int32_t first_block;     // index among that lattice's blocks of the colour
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies; key bumped by the Weyl constants between rounds.  On the
// device each round's two three-way XORs are single v_bitop3 instructions.
__host__ __device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    uint32_t x0 = c[0], x1 = c[1], x2 = c[2], x3 = c[3];
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    c[0] = x0; c[1] = x1; c[2] = x2; c[3] = x3;
}

// Per-axis schedule: number of blocks for L cells and width parameter B.
__host__ __device__ inline int axis_blocks(int L, int B)
{
    int n = 2 * ((L + 2 * B - 1) / (2 * B));
    const int cap = 2 * (L / 4);
    if (n > cap) n = cap;
    if (n < 2) n = 2;
    return n;
}

// Block-width parameter the library uses along an axis of L cells when the
// caller leaves it to the library (tables.cpp).
int plan_block(int lattice, int L, int K);
// Blocks per workgroup of a single lattice's colour launches with
// blocks_per_colour blocks on a device of n_cu compute units (tables.cpp);
// work placement only, never the trajectory.
int plan_waves_per_group(int lattice, int blocks_per_colour, int n_cu);

// Host helpers (tables.cpp).
void build_thresholds(double T, double* out /* kTab */);
// bias: the per-field offset the kernel packs into its histogram words
// (16 for BCC with K <= 6, 0 for BCC with K <= 8, 32 for FCC).  Returns the
// value of DevLattice::drop_last the rows are built for.
// dot_ok: the byte-dot form may be used (taken when kmax <= 5 and the
// weights have three-digit forms; both lattice kernels read it).
int build_wtab(const int32_t* epi, int K, int S, int kmax, int smax, int bias, bool dot_ok, int32_t* out);

// Launchers (kernels.hip, kernels_fcc.hip, pair_counts.hip).  Return hipSuccess or the launch error.
// slab: d_lat describes a z-slab (BCC only; one lattice, no work items).
// wpg: blocks per workgroup, 0 for the lattice type's default
// (waves_per_group); single FCC lattices may take kWavesPerGroupFccWide
// (plan_waves_per_group).
hipError_t launch_sweep_phase(int lattice, const DevLattice* d_lat, const WorkItem* d_items, int n_groups,
                              int t, int colour, int kmax, int smax, hipStream_t stream, bool slab = false,
                              int wpg = 0);
hipError_t launch_pair_counts(int lattice, const uint8_t* species, const int32_t L[3], int K, int S,
                              unsigned long long* d_counts, hipStream_t stream);
hipError_t launch_sweep_phase_fcc(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t,
                                  int colour, int smax, hipStream_t stream, int wpg);
hipError_t launch_species_max(const uint8_t* species, size_t n, unsigned int* d_max, hipStream_t stream);
hipError_t launch_thresholds(const double* d_tab, const int32_t* d_dE, int n, double* d_out, hipStream_t stream);
hipError_t launch_accept_bounds(const double* d_tab, const uint32_t* d_u, int n, int32_t* d_lo, int32_t* d_hi,
                                hipStream_t stream);
hipError_t launch_accept_bounds_check(const double* d_tab, unsigned long long* d_out, hipStream_t stream);
hipError_t launch_philox(const uint32_t* d_ctr, uint32_t k0, uint32_t k1, int n, uint32_t* d_out,
                         hipStream_t stream);

// Kernel template keys: the smallest instantiated KMAX >= K (BCC); FCC
// kernels are built for K <= 5.
int kmax_for(int K);
inline int kmax_for(int lattice, int K) { return lattice == 1 ? 5 : kmax_for(K); }
inline int wtab_bias(int lattice, int kmax) { return lattice == 1 ? 32 : (kmax <= 6 ? 16 : 0); }
inline int sites_per_cell(int lattice) { return lattice == 1 ? 4 : 2; }
inline int waves_per_group(int lattice) { return lattice == 1 ? kWavesPerGroupFcc : kWavesPerGroup; }
inline int first_shell(int lattice) { return lattice == 1 ? 12 : 8; }
inline int shell_size(int lattice, int s)
{
    return lattice == 1 ? (s == 0 ? 12 : s == 1 ? 6 : 24) : (s == 0 ? 8 : s == 1 ? 6 : 12);
}

}  // namespace smcx
