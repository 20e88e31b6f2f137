// device_common.h -- small device helpers shared by the BCC and FCC sweep
// kernels.
#pragma once

#include "smcx_internal.h"

namespace smcx {

// Species codes in LDS: species v is stored as (F + 32) * v, F the width of
// its histogram field; the top 3 bits give v back.
__device__ __forceinline__ uint32_t decode(uint32_t code) { return code >> 5; }

// acc + a * b on the 24-bit multiplier (a, b signed 24-bit), modulo 2^32
__device__ __forceinline__ uint32_t mad24(uint32_t a, int32_t b, uint32_t acc)
{
    return (uint32_t)__mul24((int32_t)a, b) + acc;
}

// Cell (3 ix, 3 iy, 3 iz) of a 4 x 4 x 4 sub-colour round taken by `lane`:
// lane bits 0 and 5 give ix, bits 1-2 iy, bits 3-4 iz.  Each half-wave then
// covers two x columns, which with the 231-byte plane pitch puts its 32 byte
// reads at any common offset into distinct LDS banks.
__device__ __forceinline__ void lane_cell(int lane, int& ix, int& iy, int& iz)
{
    ix = (lane & 1) | ((lane >> 4) & 2);
    iy = (lane >> 1) & 3;
    iz = (lane >> 3) & 3;
}

// An empty asm on the accumulator keeps the counting chain sequential:
// otherwise the adds are reassociated into a tree, and each shift then needs
// its own mask and instruction instead of one shift-add.
__device__ __forceinline__ void keep(uint32_t& h) { asm("" : "+v"(h)); }

// Add +1 (NEG: -1) in the field of code c to h: one v_lshl_add_u32, whose
// shift takes the low 5 bits of c.  Written out, so that no mask of c is
// materialised: the compiler folds c & 31 into the shift only when both sit
// in one basic block, and the sweep kernels count codes that were loaded in
// other blocks (codes carried from the previous trial, in a loop).  (The
// instruction also keeps each count a chain of shift-adds, as keep() does.)
template <bool NEG> __device__ __forceinline__ void count1(uint32_t& h, uint32_t c)
{
    if constexpr (NEG) asm("v_lshl_add_u32 %0, -1, %1, %0" : "+v"(h) : "v"(c));
    else asm("v_lshl_add_u32 %0, 1, %1, %0" : "+v"(h) : "v"(c));
}

// LDS form of the pair-weight table: entry f of row (a, b) (f = s*KMAX + p
// for a weight, SMAX*KMAX for the constant) sits in plane f at position
// a*KMAX + b, planes wplane(KMAX) dwords apart.  The lanes of a wave read one
// plane per instruction, each at its own row: distinct rows fall in distinct
// 4-byte banks, equal rows broadcast (a row-per-lane layout made most lanes
// collide, its rows all starting on the same few banks).
constexpr int wplane(int kmax) { return ((kmax * kmax + 31) / 32) * 32; }
constexpr int wplanes(int kmax, int smax) { return wrow_entries(kmax, smax); }

// Fill the LDS planes (PS dwords apart, PS >= KMAX*KMAX) from the
// row-major table of wrow(KMAX, SMAX) ints per row.
template <int KMAX, int SMAX, int PS = wplane(KMAX)>
__device__ __forceinline__ void load_wplanes(int32_t* s_w, const int32_t* wtab)
{
    constexpr int WR = wrow(KMAX, SMAX);
    for (int k = threadIdx.x; k < wplanes(KMAX, SMAX) * PS; k += blockDim.x) {
        const int f = k / PS, row = k - f * PS;
        s_w[k] = row < KMAX * KMAX ? wtab[row * WR + f] : 0;
    }
}

// Byte-dot codes (weight rows in kWtabDot form, KMAX <= 5): species
// v < KMAX-1 is stored as 40 v, i.e. counted by a shift of 8 v into byte v
// of the histogram word; the last species as 31 + 32 v, counted into bit 31,
// which the weighing masks off.  The top 3 bits still give v back.  For up
// to four species bytes at once.
template <int KMAX>
__device__ __forceinline__ uint32_t encode4_dot(uint32_t v)
{
    static_assert(KMAX <= 5, "byte-dot codes need KMAX <= 5");
    constexpr uint32_t c = 8 - (KMAX - 1);                 // v + c >= 8 iff v == KMAX-1
    const uint32_t last = ((v + c * 0x01010101u) >> 3) & 0x01010101u;
    constexpr uint32_t k = (uint32_t)(31 - 8 * (KMAX - 1)); // code change of the last species, mod 2^32
    return (v << 5) + (v << 3) + last * k;                   // no carries or borrows between bytes
}

// Lower bound floor(k L / n) of block k of n along an axis of L cells
// (0 <= k <= n <= L).  k L <= L^2 < 2^32 whenever L <= 65535; wider axes
// divide in 64 bits.  Called with wave-uniform arguments, so it runs on the scalar unit.
__device__ __forceinline__ int block_lo(int k, int L, int n)
{
    return L <= 65535 ? (int)(((uint32_t)k * (uint32_t)L) / (uint32_t)n) : (int)(((int64_t)k * L) / n);
}

// The index of the calling lane's wavefront in its workgroup, as a value the
// compiler knows to be the same for all lanes: everything derived from it
// (block coordinates, row bases) is then computed once per wave in scalar
// registers rather than per lane.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)); }

// Accesses to the lattice in HBM.  A pointer loaded from a struct is generic
// to the compiler, and generic (flat) accesses also count against the LDS
// wait counter; through an address-space-1 pointer they are global loads
// and stores.
template <class T> __device__ __forceinline__ T gload(const uint8_t* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T> __device__ __forceinline__ void gstore(uint8_t* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// Raw buffer resource over the n bytes from p (stride 0; the third word is
// the gfx9 32-bit data format).  The hardware checks every buffer access
// against n: loads past it return 0, stores past it are dropped.  The
// staging and write-back of the sweep kernels address a lattice plane by
// a resource whose base is that plane (scalar registers) and a 32-bit
// per-lane offset, so their rows need no 64-bit vector arithmetic.
constexpr int kRsrcWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t byte_rsrc(uint8_t* p, uint64_t n)
{
    // min(n, 2^32 - 1), on the scalar unit (it has no 64-bit ordered compare)
    const uint32_t nr = (uint32_t)(n >> 32) != 0u ? 0xffffffffu : (uint32_t)n;
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)nr, kRsrcWord3);
}
__device__ __forceinline__ uint32_t bload32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v)
{
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, r, (int)off, 0, 0);
}

// Bounds of the Metropolis test (Eq. (3)) for an acceptance draw u.
// The exact test accepts an uphill change dE iff u < thr(dE), thr the FP64
// table product, equal to 2^32 exp(-dE / k_B T) to a relative 1e-12.  Let x
// be the energy with 2^32 exp(-x / k_B T) = u, x = (32 - log2 u) ln2 k_B T.
// e below is x in FP32 from v_log_f32.  Over every u > 0 the device's
// 32 - log2(float(u)) is within 2.0e-6 of 32 - log2(u) (checked for all
// 2^32 draws by smcx_device_check_accept_bounds), so with c = ln2 k_B T
// rounded to FP32 and x <= 32 c:  |e - x| <= 2.0e-6 c + 2^-23 x <= 1.8
// micro-eV for T <= 5000 K.  e -+ M rounds to FP32 within 0.5 (e < 2^24)
// and truncates to an integer, so with M = 8 the bound lo lies more than
// 5.7 micro-eV below x and hi + 1 more than 4.7 above it: every dE <= lo
// passes the exact test and every dE > hi fails it.  Only lo < dE <= hi
// (and u = 0, where x is infinite but thr may underflow) need the table.
// c = ln2 k_B T in micro-eV, as a float.
// The sweep kernels compare float(dE) with the edges elo = e - M and
// ehi = e + M: for an integer dE in (0, 2^24), float(dE) is exact, and
// float(dE) <= elo iff dE <= lo = floor(elo), likewise for hi.  (u = 0:
// e = +inf.)
constexpr float kAcceptMargin = 8.0f;
__device__ __forceinline__ void accept_edges(uint32_t u, float c, float& elo, float& ehi)
{
    const float e = (32.0f - __builtin_amdgcn_logf((float)u)) * c;
    elo = e - kAcceptMargin;
    ehi = e + kAcceptMargin;
}
// The same bounds as integers, lo = floor(elo) and hi = floor(ehi) (at most
// 1e9; e >= 0, and the truncation is the floor wherever the bound is
// positive, the only place it is used).
__device__ __forceinline__ void accept_bounds(uint32_t u, float c, int& lo, int& hi)
{
    float elo, ehi;
    accept_edges(u, c, elo, ehi);
    lo = (int)fminf(elo, 1.0e9f);
    hi = (int)fminf(ehi, 1.0e9f);
}

// XCD-aware workgroup order of a sweep launch.  Workgroups are
// handed to the 8 XCDs of the chip in turn (workgroup b to XCD b % 8), each
// XCD with its own L2.  Workgroup b therefore takes group
// (b % 8) * chunk + b / 8 of the n groups (chunk = ceil(n / 8), grid =
// 8 * chunk): each XCD works through one contiguous range of blocks, the
// same range in every colour launch, so the halo a block stages was mostly
// written by blocks of the previous colour that ran on the same XCD and may
// still sit in its L2 (in a batched launch, consecutive work items are the
// blocks of one replica).  Any order is correct; returns -1 for workgroups
// beyond n.
__device__ __forceinline__ int xcd_group(int n)
{
    const int chunk = (n + 7) / 8;
    const int g = (int)(blockIdx.x % 8u) * chunk + (int)(blockIdx.x / 8u);
    return g < n ? g : -1;
}
inline int xcd_grid(int n) { return 8 * ((n + 7) / 8); }

__device__ __forceinline__ int wrap_add(int v, int L)   // v in [-L, 2L)
{
    v = v < 0 ? v + L : v;
    return v >= L ? v - L : v;
}

}  // namespace smcx
