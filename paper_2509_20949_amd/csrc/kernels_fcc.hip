// kernels_fcc.hip -- the sweep kernel on the FCC lattice
// (the lattice of the paper's quinary alloy and its L1_2 precipitates).
//
// Four sublattices per cubic cell at doubled offsets SUB[b]; 12/6/24
// neighbours in shells 1/2/3.  One wavefront per block as on BCC; the LDS
// image holds one 15^3 byte array per sublattice, array b covering local
// cells -1-SUB[b][a] .. 13-SUB[b][a] along axis a, so every neighbour offset
// is a compile-time constant for a given (sublattice, displacement).  A
// round is one (residue class, sublattice) pair: 27 x 4 = 108 rounds.
//
// Partner choice: the partner of all trials of one (sweep, colour,
// sub-colour) set -- its sublattice and the signs of the step on the two
// axes where the sublattices differ -- is drawn once (the same draw on
// every wave), so a scalar branch selects a trial specialised on it, which
// reads only the cells its energy change needs (the symmetric difference of
// the site's and the partner's shells), every read of a wave at one common
// offset.  A trial's own draw is its acceptance word: one Philox call per
// cell serves the cell's four sites.  (The FCC pair counts are in
// pair_counts.hip.)
#include "device_common.h"

namespace smcx {
namespace fcc {

constexpr int SUB[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
constexpr int SH1[12][3] = {{+1, +1, 0}, {+1, -1, 0}, {-1, +1, 0}, {-1, -1, 0}, {+1, 0, +1}, {+1, 0, -1},
                            {-1, 0, +1}, {-1, 0, -1}, {0, +1, +1}, {0, +1, -1}, {0, -1, +1}, {0, -1, -1}};
constexpr int SH2[6][3] = {{+2, 0, 0}, {-2, 0, 0}, {0, +2, 0}, {0, -2, 0}, {0, 0, +2}, {0, 0, -2}};
constexpr int SH3[24][3] = {{+2, +1, +1}, {+2, +1, -1}, {+2, -1, +1}, {+2, -1, -1}, {-2, +1, +1}, {-2, +1, -1},
                            {-2, -1, +1}, {-2, -1, -1}, {+1, +2, +1}, {+1, +2, -1}, {-1, +2, +1}, {-1, +2, -1},
                            {+1, -2, +1}, {+1, -2, -1}, {-1, -2, +1}, {-1, -2, -1}, {+1, +1, +2}, {+1, -1, +2},
                            {-1, +1, +2}, {-1, -1, +2}, {+1, +1, -2}, {+1, -1, -2}, {-1, +1, -2}, {-1, -1, -2}};
constexpr int kArrays = 4;
constexpr int kBpOff = kArrays * kArr;      // per-wave partner-sublattice table (108 bytes)
constexpr int kWaveLdsF = kBpOff + 112;

constexpr int origin(int b, int a) { return 1 + SUB[b][a]; }
constexpr int stride(int a) { return a == 0 ? 1 : (a == 1 ? kP : kPP); }
constexpr int sub_of_parity(int px, int py, int pz)
{
    return (px == 0 && py == 0 && pz == 0) ? 0 : (px && py && !pz) ? 1 : (px && !py && pz) ? 2 : 3;
}
constexpr int fdiv2(int t) { return t >= 0 ? t / 2 : -((-t + 1) / 2); }
constexpr int mod2(int t) { return t & 1; }

// LDS offset from the site (b, cell) to the site at doubled displacement d.
constexpr int offset(int b, int dx, int dy, int dz)
{
    const int d[3] = {dx, dy, dz};
    int par[3] = {0, 0, 0}, cd[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const int t = SUB[b][a] + d[a];
        par[a] = mod2(t);
        cd[a] = fdiv2(t);
    }
    const int bp = sub_of_parity(par[0], par[1], par[2]);
    int off = (bp - b) * kArr;
    for (int a = 0; a < 3; ++a) off += (cd[a] + origin(bp, a) - origin(b, a)) * stride(a);
    return off;
}

// The two axes on which sublattices B and BP differ.
constexpr int axis1(int B, int BP) { return SUB[B][0] != SUB[BP][0] ? 0 : 1; }
constexpr int axis2(int B, int BP) { return SUB[B][2] != SUB[BP][2] ? 2 : 1; }

// The cells a trial must load, for the site in sublattice B and its partner
// in sublattice BP with signs SG (bit 0: first differing axis, bit 1:
// second; set = +1), counting shells s < S.  In doubled coordinates the
// partner is at dj, and what the energy change needs per shell s is
// sum over N_s of e(i + v) - sum over N_s of e(i + dj + v): cells in both
// N_s(i) and N_s(j) cancel.  The rest, the symmetric differences, are 50
// distinct cells for S = 3 (against 2 x 42 neighbours), some counted in two
// shells.  plus/minus: bit s set = +1 / -1 in shell s.  The partner (dj, in
// i's first shell) and the site itself (in j's first shell) are among them.
struct DiffCells {
    int n;
    int off[64];
    int plus[64], minus[64];
    int i_site, i_partner;   // indices of the site and of the partner
    int off_partner;         // LDS offset of the partner
};

constexpr int find_cell(const int (&d)[64][3], int n, int x, int y, int z)
{
    for (int k = 0; k < n; ++k)
        if (d[k][0] == x && d[k][1] == y && d[k][2] == z) return k;
    return -1;
}

constexpr bool in_shell(int s, int x, int y, int z)
{
    const int r = x * x + y * y + z * z;
    return ((x + y + z) & 1) == 0 && r == (s == 0 ? 2 : s == 1 ? 4 : 6);
}

constexpr DiffCells make_diff(int B, int BP, int SG, int S)
{
    DiffCells c{};
    int d[64][3] = {};
    int dj[3] = {0, 0, 0};
    dj[axis1(B, BP)] = (SG & 1) ? 1 : -1;
    dj[axis2(B, BP)] = (SG & 2) ? 1 : -1;
    for (int s = 0; s < S; ++s) {
        const int n = s == 0 ? 12 : s == 1 ? 6 : 24;
        for (int k = 0; k < n; ++k) {
            const int* v = s == 0 ? SH1[k] : s == 1 ? SH2[k] : SH3[k];
            // i's neighbour v, unless it is also j's neighbour in shell s
            if (!in_shell(s, v[0] - dj[0], v[1] - dj[1], v[2] - dj[2])) {
                int t = find_cell(d, c.n, v[0], v[1], v[2]);
                if (t < 0) { t = c.n++; d[t][0] = v[0]; d[t][1] = v[1]; d[t][2] = v[2]; }
                c.plus[t] |= 1 << s;
            }
            // j's neighbour dj + v, unless it is also i's neighbour in shell s
            const int w0 = dj[0] + v[0], w1 = dj[1] + v[1], w2 = dj[2] + v[2];
            if (!in_shell(s, w0, w1, w2)) {
                int t = find_cell(d, c.n, w0, w1, w2);
                if (t < 0) { t = c.n++; d[t][0] = w0; d[t][1] = w1; d[t][2] = w2; }
                c.minus[t] |= 1 << s;
            }
        }
    }
    for (int k = 0; k < c.n; ++k) c.off[k] = offset(B, d[k][0], d[k][1], d[k][2]);
    c.i_site = find_cell(d, c.n, 0, 0, 0);
    c.i_partner = find_cell(d, c.n, dj[0], dj[1], dj[2]);
    c.off_partner = offset(B, dj[0], dj[1], dj[2]);
    return c;
}

template <int B, int BP, int SG, int S> struct Diff { static constexpr DiffCells v = make_diff(B, BP, SG, S); };

// Species fields: 6 bits each (up to 24 neighbours per shell), 5 species,
// biased by 32 so that 32 + n_i - n_j never borrows.
constexpr int F = 6;
constexpr int KMAXF = 5;
constexpr uint32_t kBias = 32u * (1u | 1u << 6 | 1u << 12 | 1u << 18 | 1u << 24);

// One trial: site at LDS byte ai (sublattice B), partner in sublattice BP
// with the signs SG (bit 0: first differing axis, bit 1: second; set = +1),
// all three wave-uniform, acceptance draw u_acc.
// mode: the form of the weight rows (wave-uniform): kWtabDot or kWtabFull.
template <int SMAX, int B, int BP, int SG>
__device__ __forceinline__ void trial(uint8_t* lat, int ai, uint32_t u_acc, bool valid, int mode,
                                      const int32_t* wtab, const double* tab, float ln2kT, int64_t& dEsum,
                                      uint32_t& nacc)
{
    int e_lo, e_hi;
    accept_bounds(u_acc, ln2kT, e_lo, e_hi);   // depends on the draw only
    constexpr int PS = wplane(KMAXF);
    constexpr DiffCells C = Diff<B, BP, SG, SMAX>::v;
    static_assert(C.n <= 64 && C.i_site >= 0 && C.i_partner >= 0, "cell table");
    // packed per-shell fields bias + n_i - n_j over the symmetric
    // differences (6-bit fields, or bytes in the byte-dot form), with the
    // codes of the site and of the partner
    uint32_t h[kMaxS];
#pragma unroll
    for (int s = 0; s < kMaxS; ++s) h[s] = mode == kWtabDot ? 0x20202020u : kBias;
    uint32_t ci = 0u, cj = 0u;
#pragma unroll
    for (int k = 0; k < C.n; ++k) {
        const uint32_t c = lat[ai + C.off[k]];
        if (k == C.i_site) ci = c;
        if (k == C.i_partner) cj = c;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
            if (C.plus[k] >> s & 1) count1<false>(h[s], c);
            if (C.minus[k] >> s & 1) count1<true>(h[s], c);
        }
    }
    const int aj = ai + C.off_partner;
    const uint32_t a = min(decode(ci), (uint32_t)(KMAXF - 1)), b = min(decode(cj), (uint32_t)(KMAXF - 1));
    const int32_t* w = wtab + (a * KMAXF + b);   // row (a, b) of the weight planes
    // (kmax = 5: the table builder gives the byte-dot rows or, when the
    // weights are too large for them, full rows of KMAXF fields per shell)
    uint32_t acc;
    if (mode == kWtabDot) {
        // bytes 32 + n_i - n_j (bit 31, the last species, masked off) dotted
        // with the three base-256 digits of the folded weights, in one
        // chain: ((A2 * 256 + A1) * 256 + constant) + A0
        int32_t dd[kMaxS];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) dd[s] = (int32_t)(h[s] & 0x7fffffffu);
        int32_t X = 0;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(dd[s], w[(3 * s + 2) * PS], X, false);
        X = (int32_t)((uint32_t)X << 8);
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(dd[s], w[(3 * s + 1) * PS], X, false);
        X = (int32_t)(((uint32_t)X << 8) + (uint32_t)w[3 * SMAX * PS]);
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(dd[s], w[(3 * s + 0) * PS], X, false);
        acc = (uint32_t)X;
    } else {
        acc = (uint32_t)w[SMAX * KMAXF * PS];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
#pragma unroll
            for (int p = 0; p < KMAXF; ++p) acc = mad24((h[s] >> (F * p)) & 63u, w[(s * KMAXF + p) * PS], acc);
        }
    }
    const int32_t dE = (int32_t)acc;
    // Metropolis decision, Eq. (3): the exact table test (tables in global
    // memory) only for lanes between their bounds
    const bool up = (dE > 0) & (dE < (1 << 24));
    const bool near = up & (((dE > e_lo) & (dE <= e_hi)) | (u_acc == 0u));
    bool up_ok = up & (dE <= e_lo);
    if (__builtin_amdgcn_ballot_w64(near)) {
        const int e = dE < 1 ? 1 : (dE > (1 << 24) - 1 ? (1 << 24) - 1 : dE);
        const uint8_t* tb = (const uint8_t*)tab;
        const double thr = (gload<double>(tb + 8 * (512 + (e >> 16))) * gload<double>(tb + 8 * (256 + ((e >> 8) & 255)))) *
                           gload<double>(tb + 8 * (e & 255));
        up_ok = near ? (double)u_acc < thr : up_ok;
    }
    const bool accept = valid & (ci != cj) & ((dE <= 0) | up_ok);
    // both bytes stored by every lane (unchanged unless accepted): no two
    // lanes of a round touch the same byte
    lat[ai] = (uint8_t)(accept ? cj : ci);
    lat[aj] = (uint8_t)(accept ? ci : cj);
    dEsum += (int64_t)(accept ? dE : 0);
    nacc += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(accept));   // wave-uniform
}

// The partner sublattice BP and signs (wave-uniform values) select one
// instantiation.
template <int SMAX, int B, int BP>
__device__ __forceinline__ void trial_signs(int signs, uint8_t* lat, int ai, uint32_t u_acc, bool valid, int drop,
                                            const int32_t* wtab, const double* tab, float ln2kT, int64_t& dEsum,
                                            uint32_t& nacc)
{
    switch (signs) {
    case 0: trial<SMAX, B, BP, 0>(lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); break;
    case 1: trial<SMAX, B, BP, 1>(lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); break;
    case 2: trial<SMAX, B, BP, 2>(lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); break;
    default: trial<SMAX, B, BP, 3>(lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); break;
    }
}

template <int SMAX, int B>
__device__ __forceinline__ void trial_any(int bp, uint8_t* lat, int ai, int signs, uint32_t u_acc, bool valid, int drop,
                                          const int32_t* wtab, const double* tab, float ln2kT, int64_t& dEsum,
                                          uint32_t& nacc)
{
    if constexpr (B != 0) { if (bp == 0) { trial_signs<SMAX, B, 0>(signs, lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); return; } }
    if constexpr (B != 1) { if (bp == 1) { trial_signs<SMAX, B, 1>(signs, lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); return; } }
    if constexpr (B != 2) { if (bp == 2) { trial_signs<SMAX, B, 2>(signs, lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); return; } }
    if constexpr (B != 3) { if (bp == 3) { trial_signs<SMAX, B, 3>(signs, lat, ai, u_acc, valid, drop, wtab, tab, ln2kT, dEsum, nacc); return; } }
}

template <int B>
__device__ __forceinline__ int site_addr(int lx, int ly, int lz)
{
    return B * kArr + (lz + origin(B, 2)) * kPP + (ly + origin(B, 1)) * kP + (lx + origin(B, 0));
}

// Site b of cell l is staged when l_a lies in -1-SUB[b][a] .. w_a+1-SUB[b][a]
// and written back when l_a lies in -SUB[b][a] .. w_a-SUB[b][a] (the block's
// own cells and the partners its trials can reach).
__device__ __forceinline__ bool in_halo(int b, int lx, int ly, int lz, int wx, int wy, int wz)
{
    const int sx = SUB[b][0], sy = SUB[b][1], sz = SUB[b][2];
    return lx >= -1 - sx && lx <= wx + 1 - sx && ly >= -1 - sy && ly <= wy + 1 - sy && lz >= -1 - sz &&
           lz <= wz + 1 - sz;
}

__device__ __forceinline__ bool in_write_box(int b, int lx, int ly, int lz, int wx, int wy, int wz)
{
    const int sx = SUB[b][0], sy = SUB[b][1], sz = SUB[b][2];
    return lx >= -sx && lx <= wx - sx && ly >= -sy && ly <= wy - sy && lz >= -sz && lz <= wz - sz;
}

__device__ __forceinline__ int lds_index(int b, int lx, int ly, int lz)
{
    return b * kArr + (lz + 1 + SUB[b][2]) * kPP + (ly + 1 + SUB[b][1]) * kP + (lx + 1 + SUB[b][0]);
}

}  // namespace fcc

// WPG waves (blocks) per workgroup: 2 (five workgroups per CU, LDS-bound), or
// kWavesPerGroupFccWide for a single lattice whose colour then fits the chip
// in fewer generations (one workgroup of 11 block images fills a CU's LDS).
template <int SMAX, int WPG>
__global__ __launch_bounds__(kWave * WPG)
void sweep_phase_fcc_kernel(const DevLattice* __restrict__ lats, const WorkItem* __restrict__ items, int n_groups,
                            int t, int colour)
{
    using namespace fcc;
    __shared__ int32_t s_w[wplanes(KMAXF, SMAX) * wplane(KMAXF)];
    __shared__ __attribute__((aligned(16))) uint8_t s_lat[WPG * kWaveLdsF];

    const int wave = wave_id();
    const int lane = threadIdx.x % kWave;
    // group grp of the launch's n_groups (XCD-aware order): work item g of a
    // batched launch, or blocks WPG g .. WPG g + WPG - 1 of a single lattice
    const int grp = xcd_group(n_groups);
    if (grp < 0) return;   // no later barrier in a workgroup without a group
    int li = 0, f = grp * WPG;
    if (items) {
        li = items[grp].lattice;
        f = items[grp].first_block;
    }
    const DevLattice& D = lats[li];
    const uint32_t s = D.sweep0 + (uint32_t)t;
    // weight planes in LDS; the threshold tables stay in global memory
    load_wplanes<KMAXF, SMAX>(s_w, D.wtab);
    __syncthreads();
    int ti = (int)(s - D.tab_s0);
    ti = ti < 0 ? 0 : (ti >= D.n_tabs ? D.n_tabs - 1 : ti);
    const double* g_tab = D.tabs + (size_t)ti * kTab;
    const float ln2kT = (float)g_tab[kTabLn2kT];
    f += wave;
    if (f >= D.blocks_per_colour) return;   // no later barrier

    const int hx = D.nb[0] >> 1, hy = D.nb[1] >> 1;
    const int kx = 2 * (f % hx) + (colour & 1);
    const int ky = 2 * ((f / hx) % hy) + ((colour >> 1) & 1);
    const int kz = 2 * (f / (hx * hy)) + ((colour >> 2) & 1);
    const int Lx = D.L[0], Ly = D.L[1], Lz = D.L[2];
    uint32_t sh[4] = {0u, 0u, s, 8u};
    philox4x32_10(sh, D.key[0], D.key[1]);
    const int ox = (int)(((uint64_t)sh[0] * (uint32_t)Lx) >> 32);
    const int oy = (int)(((uint64_t)sh[1] * (uint32_t)Ly) >> 32);
    const int oz = (int)(((uint64_t)sh[2] * (uint32_t)Lz) >> 32);
    const int x0 = block_lo(kx, Lx, D.nb[0]), wx = block_lo(kx + 1, Lx, D.nb[0]) - x0;
    const int y0 = block_lo(ky, Ly, D.nb[1]), wy = block_lo(ky + 1, Ly, D.nb[1]) - y0;
    const int z0 = block_lo(kz, Lz, D.nb[2]), wz = block_lo(kz + 1, Lz, D.nb[2]) - z0;
    const int gx0 = wrap_add(x0 + ox, Lx), gy0 = wrap_add(y0 + oy, Ly), gz0 = wrap_add(z0 + oz, Lz);
    const uint32_t k0 = D.key[0], k1 = D.key[1];

    uint8_t* lat = s_lat + wave * kWaveLdsF;
    uint8_t* __restrict__ g = D.species;

    // partner of every (colour, sub-colour q) set of this sweep, from
    // r = Philox(key, (q, 0, s, c + 64)): sublattice = the k-th other than
    // the set's own, k = (r0 * 3) >> 32 (low 2 bits of the byte), signs =
    // bits 30 and 31 of r1 (bits 2 and 3)
    for (int q = lane; q < 108; q += kWave) {
        uint32_t r[4] = {(uint32_t)q, 0u, s, (uint32_t)colour + 64u};
        philox4x32_10(r, k0, k1);
        const int b = q & 3, k = (int)(((uint64_t)r[0] * 3u) >> 32);
        lat[kBpOff + q] = (uint8_t)((k + (k >= b ? 1 : 0)) | (int)(r[1] >> 30) << 2);
    }

    const bool dot_codes = D.drop_last == kWtabDot;   // LDS codes for the byte-dot weight rows
    // ---- stage block + halo: one cell (4 sublattice bytes, one dword) per lane ----
    // Rows r = (lane >> 4) + 4 it; the loads of 16 rows are issued together
    // (lanes and rows outside the halo load a clamped in-range cell).
    {
        const int lx = (lane & 15) - 2;
        const bool okx = lx <= wx + 1;
        const int gx = wrap_add(gx0 + (okx ? lx : -2), Lx);
        for (int it0 = 0; it0 < 64; it0 += 16) {
            uint32_t v16[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int it = it0 + u;
                const int ly = min((lane >> 4) + 4 * (it & 3) - 2, wy + 1), lz = min((it >> 2) - 2, wz + 1);
                const int gy = wrap_add(gy0 + ly, Ly), gz = wrap_add(gz0 + lz, Lz);
                v16[u] = gload<uint32_t>(g + 4 * (((size_t)gz * Ly + gy) * Lx + gx));
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int it = it0 + u;
                const int ly = (lane >> 4) + 4 * (it & 3) - 2, lz = (it >> 2) - 2;
                if (!okx || ly > wy + 1 || lz > wz + 1) continue;
                uint32_t v = v16[u];
                v = dot_codes ? encode4_dot<KMAXF>(v) : (v << 5) + (v << 2) + (v << 1);   // else (6 + 32) * species
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (in_halo(b, lx, ly, lz, wx, wy, wz)) lat[lds_index(b, lx, ly, lz)] = (uint8_t)(v >> (8 * b));
            }
        }
    }

    // ---- 27 residue classes x 4 sublattices = 108 rounds ----
    int ix, iy, iz;
    lane_cell(lane, ix, iy, iz);
    const uint32_t bx = (uint32_t)(gx0 + 3 * ix), by = (uint32_t)(gy0 + 3 * iy), bz = (uint32_t)(gz0 + 3 * iz);
    const uint32_t LxLy = (uint32_t)Lx * (uint32_t)Ly;
    const bool narrow = LxLy < (1u << 24) && (uint64_t)LxLy * (uint32_t)Lz < (1ull << 32);
    int64_t dEsum = 0;
    uint32_t nacc = 0;
    const int drop = D.drop_last;   // the form of the weight rows
    for (int m = 0; m < 27; ++m) {
        const int rx = m % 3, ry = (m / 3) % 3, rz = m / 9;
        const int lx = rx + 3 * ix, ly = ry + 3 * iy, lz = rz + 3 * iz;
        const bool valid = (lx < wx) & (ly < wy) & (lz < wz);
        uint32_t gx = bx + rx, gy = by + ry, gz = bz + rz;
        gx = min(gx, gx - (uint32_t)Lx);
        gy = min(gy, gy - (uint32_t)Ly);
        gz = min(gz, gz - (uint32_t)Lz);
        uint64_t cell;
        if (narrow)
            cell = __umul24(gz, LxLy) + __umul24(gy, (uint32_t)Lx) + gx;
        else
            cell = ((uint64_t)gz * (uint32_t)Ly + gy) * (uint32_t)Lx + gx;
        // one Philox call per cell: site b accepts with word b
        uint32_t ra[4] = {(uint32_t)cell, (uint32_t)(cell >> 32), s, (uint32_t)colour};
        philox4x32_10(ra, k0, k1);
        const int q0 = 4 * m;
        int pb = __builtin_amdgcn_readfirstlane(lat[kBpOff + q0]);
        trial_any<SMAX, 0>(pb & 3, lat, site_addr<0>(lx, ly, lz), pb >> 2, ra[0], valid, drop, s_w, g_tab, ln2kT, dEsum, nacc);
        __builtin_amdgcn_wave_barrier();
        pb = __builtin_amdgcn_readfirstlane(lat[kBpOff + q0 + 1]);
        trial_any<SMAX, 1>(pb & 3, lat, site_addr<1>(lx, ly, lz), pb >> 2, ra[1], valid, drop, s_w, g_tab, ln2kT, dEsum, nacc);
        __builtin_amdgcn_wave_barrier();
        pb = __builtin_amdgcn_readfirstlane(lat[kBpOff + q0 + 2]);
        trial_any<SMAX, 2>(pb & 3, lat, site_addr<2>(lx, ly, lz), pb >> 2, ra[2], valid, drop, s_w, g_tab, ln2kT, dEsum, nacc);
        __builtin_amdgcn_wave_barrier();
        pb = __builtin_amdgcn_readfirstlane(lat[kBpOff + q0 + 3]);
        trial_any<SMAX, 3>(pb & 3, lat, site_addr<3>(lx, ly, lz), pb >> 2, ra[3], valid, drop, s_w, g_tab, ln2kT, dEsum, nacc);
        __builtin_amdgcn_wave_barrier();
    }

    // ---- write back: sublattice b over cells -SUB[b][a] .. w_a - SUB[b][a] ----
    // Rows r = (lane >> 4) + 4 it; the 16 LDS reads of four rows are issued
    // together (rows and cells outside the boxes read clamped in-image bytes
    // and store nothing).
    {
        const int lx = (lane & 15) - 1;
        const bool okx = lx <= wx;
        const int lxc = okx ? lx : 0;
        const int gx = wrap_add(gx0 + lx, Lx);
        const int nit = 4 * (wz + 2);               // rows with lz <= wz
        for (int it0 = 0; it0 < nit; it0 += 4) {
            uint32_t c[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int it = it0 + u;
                const int lyc = min((lane >> 4) + 4 * (it & 3) - 1, wy), lzc = min((it >> 2) - 1, wz);
#pragma unroll
                for (int b = 0; b < 4; ++b) c[u][b] = lat[lds_index(b, lxc, lyc, lzc)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int it = it0 + u;
                const int ly = (lane >> 4) + 4 * (it & 3) - 1, lz = (it >> 2) - 1;
                if (!okx || ly > wy || lz > wz) continue;
                bool v[4];
                uint32_t e = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    v[b] = in_write_box(b, lx, ly, lz, wx, wy, wz);
                    e |= decode(c[u][b]) << (8 * b);
                }
                if (!(v[0] || v[1] || v[2] || v[3])) continue;
                const int gy = wrap_add(gy0 + ly, Ly), gz = wrap_add(gz0 + lz, Lz);
                uint8_t* q = g + 4 * (((size_t)gz * Ly + gy) * Lx + gx);
                if (v[0] && v[1] && v[2] && v[3]) {
                    gstore<uint32_t>(q, e);
                } else {
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (v[b]) gstore<uint8_t>(q + b, (uint8_t)(e >> (8 * b)));
                }
            }
        }
    }

    uint64_t sum = (uint64_t)dEsum;
    const uint32_t cnt = nacc;   // already the wave's total
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)sum, o, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(sum >> 32), o, kWave);
        sum += (uint64_t)lo | ((uint64_t)hi << 32);
    }
    if (lane == 0) {
        unsigned long long* slot = (unsigned long long*)(D.state + (f % kSpread) * kSlotWords);
        if (sum) atomicAdd(slot, (unsigned long long)sum);
        if (cnt) atomicAdd(slot + 1, (unsigned long long)cnt);
    }
}

template <int WPG>
static hipError_t launch_fcc(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t, int colour,
                             int smax, hipStream_t stream)
{
    const dim3 grid(xcd_grid(n_groups)), block(kWave * WPG);
    switch (smax) {
    case 1: hipLaunchKernelGGL((sweep_phase_fcc_kernel<1, WPG>), grid, block, 0, stream, d_lat, d_items, n_groups, t,
                               colour); break;
    case 2: hipLaunchKernelGGL((sweep_phase_fcc_kernel<2, WPG>), grid, block, 0, stream, d_lat, d_items, n_groups, t,
                               colour); break;
    case 3: hipLaunchKernelGGL((sweep_phase_fcc_kernel<3, WPG>), grid, block, 0, stream, d_lat, d_items, n_groups, t,
                               colour); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_phase_fcc(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t, int colour,
                                  int smax, hipStream_t stream, int wpg)
{
    if (n_groups <= 0) return hipSuccess;
    if (wpg == kWavesPerGroupFccWide) {
        if (d_items) return hipErrorInvalidValue;   // work items cover kWavesPerGroupFcc blocks each
        return launch_fcc<kWavesPerGroupFccWide>(d_lat, d_items, n_groups, t, colour, smax, stream);
    }
    if (wpg != kWavesPerGroupFcc) return hipErrorInvalidValue;
    return launch_fcc<kWavesPerGroupFcc>(d_lat, d_items, n_groups, t, colour, smax, stream);
}

}  // namespace smcx
