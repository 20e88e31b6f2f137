// pair_counts.hip -- pair counts N_m[p'][p] = #{(i, delta in shell m):
// sigma_i = p', sigma_{i+delta} = p} of a lattice: the numerator of the
// Warren-Cowley parameters (Eq. (SRO)) and, as E = 1/2 sum N_m[p'][p]
// V_m(p', p), the energy of the EPI model.  One kernel serves both lattice
// types (BCC and FCC).
//
// Each bond is counted once, from the half of every shell's displacement
// vectors whose first nonzero component is positive: with B_m[a][b] the
// count of (i, delta in that half) with sigma_i = a, sigma_{i+delta} = b,
// the other half gives B_m transposed (substitute j = i + delta), so
// N_m = B_m + B_m^T.  That halves the neighbour reads of a full count.
//
// Work: a task is a run of 64 cells along x of one (y, z) row, one cell per
// lane; a wavefront takes tasks in turn.  The row and its neighbour rows are
// wave-uniform (scalar addresses).  A lane loads every neighbour cell its
// sites' half-shells reach (one word per cell: the cell's 2 or 4 site bytes),
// forms per site and shell a packed histogram of the neighbour species, and
// adds it into its own counters in LDS (16-bit fields, two species per
// dword, one ds_add per dword).  Counters belong to one lane, so the adds
// never collide; at the end the workgroup sums each counter over its lanes
// and adds B and B^T into the 64-bit totals with a few global atomics.
#include <algorithm>
#include <utility>

#include "device_common.h"

namespace smcx {
namespace pc {

// Geometry in doubled coordinates (units of a/2).
struct Geo {
    int nsub;
    int sub[4][3];     // site offsets in the cell
    int nvec[3];       // shell sizes
    int vec[3][24][3]; // shell vectors
};

constexpr Geo bcc_geo()
{
    Geo g{};
    g.nsub = 2;
    g.sub[1][0] = g.sub[1][1] = g.sub[1][2] = 1;
    int n = 0;
    for (int e = 0; e < 8; ++e) {   // shell 1: (+-1, +-1, +-1)
        g.vec[0][n][0] = e & 1 ? 1 : -1;
        g.vec[0][n][1] = e & 2 ? 1 : -1;
        g.vec[0][n][2] = e & 4 ? 1 : -1;
        ++n;
    }
    g.nvec[0] = n;
    n = 0;
    for (int a = 0; a < 3; ++a)     // shell 2: (+-2, 0, 0) and permutations
        for (int s = -1; s <= 1; s += 2) {
            g.vec[1][n][a] = 2 * s;
            ++n;
        }
    g.nvec[1] = n;
    n = 0;
    for (int a = 0; a < 3; ++a)     // shell 3: (+-2, +-2, 0) and permutations
        for (int s = -1; s <= 1; s += 2)
            for (int t = -1; t <= 1; t += 2) {
                g.vec[2][n][a] = 2 * s;
                g.vec[2][n][(a + 1) % 3] = 2 * t;
                ++n;
            }
    g.nvec[2] = n;
    return g;
}

constexpr Geo fcc_geo()
{
    Geo g{};
    g.nsub = 4;
    const int sub[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 3; ++a) g.sub[b][a] = sub[b][a];
    int n = 0;
    for (int a = 0; a < 3; ++a)     // shell 1: (+-1, +-1, 0) and permutations
        for (int s = -1; s <= 1; s += 2)
            for (int t = -1; t <= 1; t += 2) {
                g.vec[0][n][a] = s;
                g.vec[0][n][(a + 1) % 3] = t;
                ++n;
            }
    g.nvec[0] = n;
    n = 0;
    for (int a = 0; a < 3; ++a)     // shell 2: (+-2, 0, 0) and permutations
        for (int s = -1; s <= 1; s += 2) {
            g.vec[1][n][a] = 2 * s;
            ++n;
        }
    g.nvec[1] = n;
    n = 0;
    for (int a = 0; a < 3; ++a)     // shell 3: (+-2, +-1, +-1) and permutations
        for (int s = -1; s <= 1; s += 2)
            for (int t = -1; t <= 1; t += 2)
                for (int u = -1; u <= 1; u += 2) {
                    g.vec[2][n][a] = 2 * s;
                    g.vec[2][n][(a + 1) % 3] = t;
                    g.vec[2][n][(a + 2) % 3] = u;
                    ++n;
                }
    g.nvec[2] = n;
    return g;
}

constexpr int fdiv2(int t) { return t >= 0 ? t / 2 : -((-t + 1) / 2); }

// Neighbour cells are numbered (dz+1)*9 + (dy+1)*3 + (dx+1), d in {-1,0,1}^3.
struct Bond {
    int cell;
    int sub;
};
struct Bonds {
    int n[4][3];
    Bond b[4][3][12];
    bool used[27];
};

constexpr Bonds make_bonds(const Geo g)
{
    Bonds r{};
    for (int b = 0; b < g.nsub; ++b)
        for (int m = 0; m < 3; ++m) {
            int n = 0;
            for (int k = 0; k < g.nvec[m]; ++k) {
                const int* v = g.vec[m][k];
                const int first = v[0] != 0 ? v[0] : (v[1] != 0 ? v[1] : v[2]);
                if (first < 0) continue;   // the other half: B^T
                int cd[3] = {0, 0, 0}, par[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a) {
                    const int t = g.sub[b][a] + v[a];
                    cd[a] = fdiv2(t);
                    par[a] = t - 2 * cd[a];
                }
                int bp = -1;
                for (int q = 0; q < g.nsub; ++q)
                    if (g.sub[q][0] == par[0] && g.sub[q][1] == par[1] && g.sub[q][2] == par[2]) bp = q;
                const int cell = (cd[2] + 1) * 9 + (cd[1] + 1) * 3 + (cd[0] + 1);
                r.b[b][m][n] = Bond{cell, bp};
                r.used[cell] = true;
                ++n;
            }
            r.n[b][m] = n;
        }
    r.used[13] = true;   // the cell itself
    return r;
}

template <int LAT> struct Tables {
    static constexpr Geo geo = LAT == 1 ? fcc_geo() : bcc_geo();
    static constexpr Bonds bonds = make_bonds(geo);
};

// Counters are 16 bits wide and shared by the two lanes l and l + 32 of a
// wave.  A task adds at most 2 * n_sub * 12 to one of them (two lanes, each
// with four FCC sites of one species and the 12 half-shell-3 neighbours of
// that species), so a wave takes at most this many tasks before its
// counters could wrap.
constexpr uint32_t kMaxTasksPerWave = 512;
static_assert(kMaxTasksPerWave * 2 * 4 * 12 < 65536, "pair-count counters could wrap");
constexpr int kBinLanes = 32;   // counter columns per wave

// Packed histogram of site B's neighbours in shell M (the half-shell
// bonds), F bits per species: bond K of the list reads byte sub of
// neighbour-cell word cell.  Expanded at compile time.
template <int LAT, int F, int B, int M, int... Ks>
__device__ __forceinline__ uint32_t half_shell(const uint32_t (&v)[27], std::integer_sequence<int, Ks...>)
{
    using T = Tables<LAT>;
    uint32_t h = 0u;
    ((h += 1u << (F * ((v[T::bonds.b[B][M][Ks].cell] >> (8 * T::bonds.b[B][M][Ks].sub)) & 255u))), ...);
    return h;
}

// Loads of one task: the words of every neighbour cell the half-shells of
// the cell at x reach, rows (y + dy, z + dz) (wave-uniform).
template <int LAT, int... Os>
__device__ __forceinline__ void load_cells(const uint8_t* g, int Lx, int Ly, int Lz, int y, int z, const int (&xo)[3],
                                           uint32_t (&v)[27], std::integer_sequence<int, Os...>)
{
    using T = Tables<LAT>;
    constexpr int NSUB = T::geo.nsub;
    auto one = [&](auto oc) {
        constexpr int o = decltype(oc)::value;
        if constexpr (T::bonds.used[o]) {
            constexpr int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            const int yy = wrap_add(y + dy, Ly), zz = wrap_add(z + dz, Lz);
            const size_t row = ((size_t)zz * (uint32_t)Ly + (uint32_t)yy) * (uint32_t)Lx;   // wave-uniform
            const uint8_t* p = g + NSUB * (row + (uint32_t)xo[dx + 1]);
            v[o] = NSUB == 4 ? gload<uint32_t>(p) : (uint32_t)gload<uint16_t>(p);
        }
    };
    (one(std::integral_constant<int, Os>{}), ...);
}

}  // namespace pc

// F: bits per species field of a histogram word (8 for K <= 4, 4 for
// K <= 8).  D counter dwords per (shell, centre species): dword k holds
// species k (low half) and species k + 16/F (high half).
template <int LAT, int F, int SMAX>
__global__ __launch_bounds__(256)
void pair_counts_kernel(const uint8_t* __restrict__ g, int Lx, int Ly, int Lz, int K, uint32_t n_tasks,
                        unsigned long long* __restrict__ counts)
{
    using T = pc::Tables<LAT>;
    constexpr int NSUB = T::geo.nsub;
    constexpr int D = F == 8 ? 2 : 4;
    constexpr int HI = 16 / F;                       // species offset of the high half
    constexpr uint32_t MASK = F == 8 ? 0x00FF00FFu : 0x000F000Fu;
    constexpr int C = pc::kBinLanes;
    extern __shared__ uint32_t bins[];               // [wave][nb][C]

    const int lane = threadIdx.x % kWave;
    const int wave = wave_id();
    const int nwv = blockDim.x / kWave;
    const int nb = SMAX * K * D;
    uint32_t* mine = bins + (size_t)wave * nb * C + (lane % C);
    if (lane < C)
        for (int d = 0; d < nb; ++d) mine[d * C] = 0u;

    // Waves take contiguous runs of tasks (row after row, so the neighbour
    // rows of the next task were mostly just read), and workgroups are
    // numbered XCD-aware (xcd_group): the runs of one XCD are adjacent and
    // share its L2.
    const uint32_t nwaves = gridDim.x * (uint32_t)nwv;
    const uint32_t per_wave = (n_tasks + nwaves - 1) / nwaves;
    const int grp = xcd_group((int)gridDim.x);
    const uint32_t t_begin = grp < 0 ? n_tasks : (uint32_t)(grp * nwv + wave) * per_wave;
    const uint32_t t_end = min(n_tasks, t_begin + per_wave);
    const uint32_t nchunk = (uint32_t)(Lx + kWave - 1) / kWave;
    // task t: cells (t % nchunk) * 64 + lane of row t / nchunk
    auto locate = [&](uint32_t t, int& y, int& z, int (&xo)[3]) -> bool {
        const uint32_t c = t % nchunk, r = t / nchunk;
        y = (int)(r % (uint32_t)Ly);
        z = (int)(r / (uint32_t)Ly);
        const int x = (int)c * kWave + lane;
        const int xc = x < Lx ? x : Lx - 1;
        xo[0] = xc == 0 ? Lx - 1 : xc - 1;
        xo[1] = xc;
        xo[2] = xc == Lx - 1 ? 0 : xc + 1;
        return x < Lx;
    };
    const auto cells = std::make_integer_sequence<int, 27>{};
    uint32_t t = t_begin;
    uint32_t v[27], vn[27];
    int y, z, xo[3];
    bool valid = false;
    if (t < t_end) {
        valid = locate(t, y, z, xo);
        pc::load_cells<LAT>(g, Lx, Ly, Lz, y, z, xo, v, cells);
    }
    while (t < t_end) {
        // the next task's loads go out before this task's counting
        const uint32_t tn = t + 1;
        bool valid_n = false;
        if (tn < t_end) {
            int yn, zn, xon[3];
            valid_n = locate(tn, yn, zn, xon);
            pc::load_cells<LAT>(g, Lx, Ly, Lz, yn, zn, xon, vn, cells);
        }
        if (valid) {
            auto site = [&](auto bc) {
                constexpr int b = decltype(bc)::value;
                const uint32_t a = min((v[13] >> (8 * b)) & 255u, (uint32_t)(K - 1));
                uint32_t* base = mine + a * (D * C);
                auto shell = [&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (m < SMAX) {
                        const uint32_t h = pc::half_shell<LAT, F, b, m>(
                            v, std::make_integer_sequence<int, T::bonds.n[b][m]>{});
#pragma unroll
                        for (int k = 0; k < D; ++k) atomicAdd(base + (m * K * D + k) * C, (h >> (F * k)) & MASK);
                    }
                };
                shell(std::integral_constant<int, 0>{});
                shell(std::integral_constant<int, 1>{});
                shell(std::integral_constant<int, 2>{});
            };
            site(std::integral_constant<int, 0>{});
            site(std::integral_constant<int, 1>{});
            if constexpr (NSUB == 4) {
                site(std::integral_constant<int, 2>{});
                site(std::integral_constant<int, 3>{});
            }
        }
#pragma unroll
        for (int o = 0; o < 27; ++o) v[o] = vn[o];
        valid = valid_n;
        t = tn;
    }
    __syncthreads();
    // Workgroup totals of each counter word; B and B^T into the 64-bit sums.
    for (int d = threadIdx.x; d < nb; d += blockDim.x) {
        uint32_t lo = 0u, hi = 0u;
        for (int w = 0; w < nwv; ++w) {
            const uint32_t* row = bins + ((size_t)w * nb + d) * C;
            for (int j = 0; j < C; ++j) {
                const uint32_t val = row[(j + d) & (C - 1)];   // rotated: lanes hit distinct banks
                lo += val & 0xffffu;
                hi += val >> 16;
            }
        }
        const int m = d / (K * D), a = (d / D) % K, k = d % D;
        unsigned long long* out = counts + (blockIdx.x % kCountSlots) * kCountWords;   // spread over the slots
        if (lo) {
            atomicAdd(&out[(m * kMaxK + a) * kMaxK + k], (unsigned long long)lo);
            atomicAdd(&out[(m * kMaxK + k) * kMaxK + a], (unsigned long long)lo);
        }
        if (hi) {
            atomicAdd(&out[(m * kMaxK + a) * kMaxK + k + HI], (unsigned long long)hi);
            atomicAdd(&out[(m * kMaxK + k + HI) * kMaxK + a], (unsigned long long)hi);
        }
    }
}

// ---------------------------------------------------------------------------
// K <= 5 species (BCC and FCC): bit planes.  A wavefront takes a tile of
// 64 x 64 cells of a z range: lane l holds x = x0 - 1 + l, bit b of a word
// pair holds y = y0 - 1 + b (both wrapped; lanes 0 and 63 and bits 0 and 63
// are the halo, the 62 x 62 cells inside are the tile's own).  Per z plane
// and sublattice the wave builds one 64-bit plane per species b < K - 1
// (bit y set iff the site at (x, y) holds b): the species' three bits are
// gathered row by row, and each species plane is one three-input logic
// operation of them.  A half-shell bond (cell offset d, neighbour sublattice
// q) then counts the pairs (a, b) of 64 sites with two ANDs and two bit
// counts, popcount(P_a(z) & shift(P_b(z + dz))): the y step a shift of the
// word pair, the x step a lane shift (DPP), the z step one of two planes
// held in registers.  The half shells here are the vectors whose first
// nonzero component in the order z, y, x is positive, so every bond reaches
// the same z plane or the next (dz = 0 or 1).  Pairs with the last species
// follow from the row sums sum_b N_m[a][b] = Z_m n_a (every site has Z_m
// neighbours in shell m).
namespace pc {
template <class Fn, int... Ks>
__device__ __forceinline__ void for_each_index(Fn&& fn, std::integer_sequence<int, Ks...>)
{
    (fn(std::integral_constant<int, Ks>{}), ...);
}
constexpr int kTile = 62;   // cells a tile owns along x and y
constexpr int kZm[2][3] = {{8, 6, 12}, {12, 6, 24}};   // shell sizes, BCC and FCC

// Half-shell bonds with the z-first rule: neighbour cell offset (dx, dy in
// -1..1, dz in 0..1) and sublattice.
struct ZBond {
    int dx, dy, dz, sub;
};
struct ZBonds {
    int n[4][3];
    ZBond b[4][3][12];
};
constexpr ZBonds make_zbonds(const Geo g)
{
    ZBonds r{};
    for (int b = 0; b < g.nsub; ++b)
        for (int m = 0; m < 3; ++m) {
            int n = 0;
            for (int k = 0; k < g.nvec[m]; ++k) {
                const int* v = g.vec[m][k];
                const int first = v[2] != 0 ? v[2] : (v[1] != 0 ? v[1] : v[0]);
                if (first < 0) continue;   // the other half: B^T
                int cd[3] = {0, 0, 0}, par[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a) {
                    const int t = g.sub[b][a] + v[a];
                    cd[a] = fdiv2(t);
                    par[a] = t - 2 * cd[a];
                }
                int bp = -1;
                for (int q = 0; q < g.nsub; ++q)
                    if (g.sub[q][0] == par[0] && g.sub[q][1] == par[1] && g.sub[q][2] == par[2]) bp = q;
                r.b[b][m][n] = ZBond{cd[0], cd[1], cd[2], bp};
                ++n;
            }
            r.n[b][m] = n;
        }
    return r;
}
template <int LAT> struct ZTables {
    static constexpr Geo geo = LAT == 1 ? fcc_geo() : bcc_geo();
    static constexpr ZBonds bonds = make_zbonds(geo);
};
constexpr bool zbonds_ok(const ZBonds& r, int nsub)
{
    for (int b = 0; b < nsub; ++b)
        for (int m = 0; m < 3; ++m)
            for (int k = 0; k < r.n[b][m]; ++k) {
                const ZBond& d = r.b[b][m][k];
                if (d.dx < -1 || d.dx > 1 || d.dy < -1 || d.dy > 1 || d.dz < 0 || d.dz > 1 || d.sub < 0) return false;
            }
    return true;
}
static_assert(zbonds_ok(ZTables<0>::bonds, 2) && zbonds_ok(ZTables<1>::bonds, 4), "z-first half shells");
static_assert(ZTables<0>::bonds.n[0][0] + ZTables<0>::bonds.n[1][0] == 8, "BCC: 8 first-shell bonds per cell");
static_assert(ZTables<1>::bonds.n[0][2] + ZTables<1>::bonds.n[3][2] == 24, "FCC: 12 third-shell bonds per site");
}  // namespace pc

template <int NSUB, int KM1>
struct Planes {
    uint32_t p[NSUB][KM1 > 0 ? KM1 : 1][2];   // [sublattice][species][half]
};

// Species planes of one z plane, the plane addressed by a buffer resource:
// row b (bit b) is row y = ystart + b (wrapped) at byte offset NSUB y Lx +
// xo, stepped row by row on the scalar unit; one row per instruction, 8 rows
// ahead of their use.
template <int NSUB, int KM1>
__device__ __forceinline__ void build_planes(__amdgpu_buffer_rsrc_t rs, int ystart, int Ly, uint32_t row_bytes,
                                             uint32_t xo, Planes<NSUB, KM1>& P)
{
    int y = ystart;
    uint32_t so = (uint32_t)ystart * row_bytes;
    auto load = [&](int) -> uint32_t {
        const uint32_t v = NSUB == 4 ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)xo, (int)so, 0)
                                     : (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, (int)xo, (int)so, 0);
        if (++y == Ly) {
            y = 0;
            so = 0;
        } else {
            so += row_bytes;
        }
        return v;
    };
    uint32_t S[NSUB][3][2] = {};   // [sublattice][species bit][half]
    constexpr int R = 8;           // rows per group
    uint32_t c[R], cn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) c[r] = load(r);
#pragma unroll
    for (int grp = 0; grp < 64 / R; ++grp) {
        if (grp < 64 / R - 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) cn[r] = load(R * (grp + 1) + r);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int b = R * grp + r;
#pragma unroll
            for (int sub = 0; sub < NSUB; ++sub)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    // one v_bfe and one v_lshl_or per bit, in a chain per
                    // word (not an OR tree, which holds every term at once)
                    S[sub][i][b >> 5] |= ((c[r] >> (8 * sub + i)) & 1u) << (b & 31);
                    keep(S[sub][i][b >> 5]);
                }
        }
        if (grp < 64 / R - 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) c[r] = cn[r];
        }
        // keep the scheduler from hoisting later groups' loads (each would
        // hold a register until its row is used)
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int sub = 0; sub < NSUB; ++sub)
#pragma unroll
        for (int sp = 0; sp < KM1; ++sp)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t m0 = sp & 1 ? 0u : ~0u, m1 = sp & 2 ? 0u : ~0u, m2 = sp & 4 ? 0u : ~0u;
                P.p[sub][sp][h] = (S[sub][0][h] ^ m0) & (S[sub][1][h] ^ m1) & (S[sub][2][h] ^ m2);
            }
}

// The word pair shifted so that bit y holds bit y + DY (DY = -1, 0, 1).
template <int DY> __device__ __forceinline__ void yshift(uint32_t& lo, uint32_t& hi)
{
    if constexpr (DY == 1) {
        lo = __builtin_amdgcn_alignbit(hi, lo, 1);
        hi = hi >> 1;
    } else if constexpr (DY == -1) {
        hi = __builtin_amdgcn_alignbit(hi, lo, 31);
        lo = lo << 1;
    }
}
// The value of lane l + DX in lane l (DX = -1, 0, 1; wavefront shifts).
template <int DX> __device__ __forceinline__ uint32_t xshift(uint32_t v)
{
    if constexpr (DX == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);
    else if constexpr (DX == -1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);
    else return v;
}

// Waves per SIMD: 3 (BCC), 2 (FCC: four sublattices' planes in registers).
template <int LAT> constexpr int kPlanesWaves = LAT == 1 ? 2 : 3;

template <int LAT, int KM1, int SMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPlanesWaves<LAT>)))
void pair_counts_planes_kernel(const uint8_t* __restrict__ g, int Lx, int Ly, int Lz, int ntx, int nty, int zc,
                               uint32_t n_items, unsigned long long* __restrict__ counts)
{
    using T = pc::ZTables<LAT>;
    constexpr int NSUB = T::geo.nsub;
    constexpr int KA = KM1 > 0 ? KM1 : 1;
    const int lane = threadIdx.x % kWave;
    const int grp = xcd_group((int)gridDim.x);
    if (grp < 0) return;   // no barriers in this kernel
    const uint32_t item = (uint32_t)grp * (blockDim.x / kWave) + (uint32_t)wave_id();
    if (item >= n_items) return;
    const int tx = (int)(item % (uint32_t)ntx), ty = (int)((item / (uint32_t)ntx) % (uint32_t)nty);
    const int zi = (int)(item / ((uint32_t)ntx * (uint32_t)nty));
    const int x0 = tx * pc::kTile, y0 = ty * pc::kTile;
    const int zb = zi * zc, ze = min(Lz, zb + zc);
    const int wx = min(pc::kTile, Lx - x0), wy = min(pc::kTile, Ly - y0);
    const int xl = (x0 - 1 + lane + Lx) % Lx;
    const int ystart = (y0 - 1 + Ly) % Ly;
    const uint32_t row_bytes = (uint32_t)NSUB * (uint32_t)Lx;
    const uint32_t xo = (uint32_t)NSUB * (uint32_t)xl;
    // the tile's own sites: lanes 1..wx, bits 1..wy
    const uint32_t xmask = (lane >= 1 && lane <= wx) ? ~0u : 0u;
    const uint64_t ym = ((1ull << (wy + 1)) - 1) & ~1ull;
    const uint32_t ymask[2] = {(uint32_t)ym & xmask, (uint32_t)(ym >> 32) & xmask};
    const uint64_t plane = (uint64_t)NSUB * (uint32_t)Lx * (uint32_t)Ly;   // bytes per z plane (< 2^32: checked on launch)
    auto zrsrc = [&](int z) {
        z = z >= Lz ? z - Lz : z;
        return byte_rsrc((uint8_t*)g + (uint64_t)z * plane, plane);
    };

    Planes<NSUB, KM1> W0, W1;   // planes z and z + 1
    build_planes<NSUB, KM1>(zrsrc(zb), ystart, Ly, row_bytes, xo, W0);
    uint32_t acc[SMAX][KA][KA] = {};
    uint32_t nsp[KA] = {};
#pragma nounroll
    for (int z = zb; z < ze; ++z) {
        build_planes<NSUB, KM1>(zrsrc(z + 1), ystart, Ly, row_bytes, xo, W1);
        auto centre = [&](auto sc) {
            constexpr int s = decltype(sc)::value;
            uint32_t C[KA][2];
#pragma unroll
            for (int a = 0; a < KM1; ++a) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    C[a][h] = W0.p[s][a][h] & ymask[h];
                    nsp[a] += (uint32_t)__popc(C[a][h]);
                }
            }
            auto shell = [&](auto mc) {
                constexpr int m = decltype(mc)::value;
                if constexpr (m < SMAX) {
                    auto bond = [&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        constexpr pc::ZBond d = T::bonds.b[s][m][k];
                        const Planes<NSUB, KM1>& N = d.dz ? W1 : W0;
#pragma unroll
                        for (int b = 0; b < KM1; ++b) {
                            uint32_t lo = N.p[d.sub][b][0], hi = N.p[d.sub][b][1];
                            yshift<d.dy>(lo, hi);
                            lo = xshift<d.dx>(lo);
                            hi = xshift<d.dx>(hi);
#pragma unroll
                            for (int a = 0; a < KM1; ++a)
                                acc[m][a][b] += (uint32_t)__popc(C[a][0] & lo) + (uint32_t)__popc(C[a][1] & hi);
                        }
                        // one bond at a time (its 2 (K - 1)^2 ANDs and bit
                        // counts are independent work enough): shifted planes
                        // of later bonds are not computed ahead
                        __builtin_amdgcn_sched_barrier(0);
                    };
                    pc::for_each_index(bond, std::make_integer_sequence<int, T::bonds.n[s][m]>{});
                }
            };
            shell(std::integral_constant<int, 0>{});
            shell(std::integral_constant<int, 1>{});
            shell(std::integral_constant<int, 2>{});
        };
        pc::for_each_index(centre, std::make_integer_sequence<int, NSUB>{});
        W0 = W1;
    }

    // wave sums, then this wave's share of every N_m[a][b] into copy
    // item % kCountSlots (two's-complement adds: a share may be negative,
    // the totals are exact)
    auto wsum = [&](uint32_t v) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, kWave);
        return v;
    };
    int64_t n[KA];
    int64_t nlast = (int64_t)NSUB * wx * wy * (ze - zb);   // sites of the tile and z range
#pragma unroll
    for (int a = 0; a < KM1; ++a) {
        n[a] = (int64_t)wsum(nsp[a]);
        nlast -= n[a];
    }
    constexpr int L = KM1;   // the last species
    unsigned long long* out = counts + (item % kCountSlots) * kCountWords;
    auto add = [&](int m, int a, int b, int64_t v) {
        if (v != 0) atomicAdd(&out[(m * kMaxK + a) * kMaxK + b], (unsigned long long)v);
    };
#pragma unroll
    for (int m = 0; m < SMAX; ++m) {
        int64_t B[KA][KA];
#pragma unroll
        for (int a = 0; a < KM1; ++a)
#pragma unroll
            for (int b = 0; b < KM1; ++b) B[a][b] = (int64_t)wsum(acc[m][a][b]);
        if (lane == 0) {
            const int64_t Z = pc::kZm[LAT][m];
            int64_t lastrow = Z * nlast;
#pragma unroll
            for (int a = 0; a < KM1; ++a) {
                int64_t row = 0;
#pragma unroll
                for (int b = 0; b < KM1; ++b) {
                    const int64_t v = B[a][b] + B[b][a];
                    row += v;
                    if (b >= a) {
                        add(m, a, b, v);
                        if (b > a) add(m, b, a, v);
                    }
                }
                const int64_t vl = Z * n[a] - row;   // N_m[a][last]
                add(m, a, L, vl);
                add(m, L, a, vl);
                lastrow -= vl;
            }
            add(m, L, L, lastrow);
        }
    }
}

template <int LAT, int F>
static hipError_t launch_pc(const uint8_t* species, const int32_t L[3], int K, int S, unsigned long long* d_counts,
                            hipStream_t stream)
{
    constexpr int D = F == 8 ? 2 : 4;
    const int nb = S * K * D;
    // LDS per workgroup: waves x nb counters x 32 columns x 4 bytes
    const int waves_per_group = 4;
    const uint64_t nchunk = ((uint64_t)L[0] + kWave - 1) / kWave;
    const uint64_t tasks = nchunk * (uint64_t)L[1] * (uint64_t)L[2];
    if (tasks > 0xffffffffull) return hipErrorInvalidValue;
    // enough waves for the chip (4096) and for the counters' range, at least
    // 4 tasks each where the lattice is small (each wave ends in a flush;
    // measured per synchronous call on 64^3 BCC: 32 us at 4 tasks per wave,
    // 35 us at 8, 42 us at 16; 2 and 1 tasks measured the same as 4)
    uint64_t waves = (tasks + pc::kMaxTasksPerWave - 1) / pc::kMaxTasksPerWave;
    waves = std::max<uint64_t>(waves, std::min<uint64_t>((tasks + 3) / 4, 4096));
    const uint64_t groups = (waves + waves_per_group - 1) / waves_per_group;
    const size_t lds = (size_t)waves_per_group * nb * pc::kBinLanes * sizeof(uint32_t);
    const dim3 grid((unsigned)xcd_grid((int)groups)), block((unsigned)(waves_per_group * kWave));
    switch (S) {
    case 1: hipLaunchKernelGGL((pair_counts_kernel<LAT, F, 1>), grid, block, lds, stream, species, L[0], L[1], L[2], K,
                               (uint32_t)tasks, d_counts); break;
    case 2: hipLaunchKernelGGL((pair_counts_kernel<LAT, F, 2>), grid, block, lds, stream, species, L[0], L[1], L[2], K,
                               (uint32_t)tasks, d_counts); break;
    case 3: hipLaunchKernelGGL((pair_counts_kernel<LAT, F, 3>), grid, block, lds, stream, species, L[0], L[1], L[2], K,
                               (uint32_t)tasks, d_counts); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// 2 <= K <= 5: the bit-plane kernel.  Work items are (x tile, y tile,
// z range); the z ranges are sized so that the launch has about one
// wavefront per wave slot of the chip (1,024 SIMDs x kPlanesWaves), each
// with at least 4 planes.
template <int LAT>
static hipError_t launch_planes(const uint8_t* species, const int32_t L[3], int K, int S,
                                unsigned long long* d_counts, hipStream_t stream)
{
    const int ntx = (L[0] + pc::kTile - 1) / pc::kTile, nty = (L[1] + pc::kTile - 1) / pc::kTile;
    const uint64_t tiles = (uint64_t)ntx * (uint64_t)nty;
    const uint64_t target = 1024 * kPlanesWaves<LAT>;
    uint64_t zc = (tiles * (uint64_t)L[2] + target - 1) / target;
    zc = std::max<uint64_t>(zc, 4);
    zc = std::min<uint64_t>(zc, (uint64_t)L[2]);
    const uint64_t nz = ((uint64_t)L[2] + zc - 1) / zc;
    const uint64_t items = tiles * nz;
    if (items > 0x7fffffffull) return hipErrorInvalidValue;
    const int waves_per_group = 4;
    const uint64_t groups = (items + waves_per_group - 1) / waves_per_group;
    const dim3 grid((unsigned)xcd_grid((int)groups)), block((unsigned)(waves_per_group * kWave));
#define SMCX_PC_PLANES(KM1, SM)                                                                                    \
    hipLaunchKernelGGL((pair_counts_planes_kernel<LAT, KM1, SM>), grid, block, 0, stream, species, L[0], L[1], L[2], \
                       ntx, nty, (int)zc, (uint32_t)items, d_counts)
    switch ((K - 1) * 4 + S) {
    case 1 * 4 + 1: SMCX_PC_PLANES(1, 1); break;
    case 1 * 4 + 2: SMCX_PC_PLANES(1, 2); break;
    case 1 * 4 + 3: SMCX_PC_PLANES(1, 3); break;
    case 2 * 4 + 1: SMCX_PC_PLANES(2, 1); break;
    case 2 * 4 + 2: SMCX_PC_PLANES(2, 2); break;
    case 2 * 4 + 3: SMCX_PC_PLANES(2, 3); break;
    case 3 * 4 + 1: SMCX_PC_PLANES(3, 1); break;
    case 3 * 4 + 2: SMCX_PC_PLANES(3, 2); break;
    case 3 * 4 + 3: SMCX_PC_PLANES(3, 3); break;
    case 4 * 4 + 1: SMCX_PC_PLANES(4, 1); break;
    case 4 * 4 + 2: SMCX_PC_PLANES(4, 2); break;
    case 4 * 4 + 3: SMCX_PC_PLANES(4, 3); break;
    default: return hipErrorInvalidValue;
    }
#undef SMCX_PC_PLANES
    return hipGetLastError();
}

// d_counts (kCountSlots copies of [kMaxS][kMaxK][kMaxK] uint64) receives
// N_m[p'][p] added to what it holds, split over the copies; the caller
// clears it first and sums the copies (count_sum).
hipError_t launch_pair_counts(int lattice, const uint8_t* species, const int32_t L[3], int K, int S,
                              unsigned long long* d_counts, hipStream_t stream)
{
    if (K < 1 || K > kMaxK || S < 1 || S > kMaxS) return hipErrorInvalidValue;
    // Bit planes for lattices of 2^22 cells and more: below that a launch
    // has too few tiles to fill the chip, and the per-lane kernel, with a
    // wavefront per 64 cells of a row, was faster (per call, measured: 128^3
    // BCC 47 against 55-71 us, 256^3 133 against 107 us).
    const uint64_t plane_bytes = (lattice == 1 ? 4ull : 2ull) * (uint32_t)L[0] * (uint32_t)L[1];
    const uint64_t cells = (uint64_t)(uint32_t)L[0] * (uint32_t)L[1] * (uint32_t)L[2];
    if (K >= 2 && K <= 5 && plane_bytes < (1ull << 32) && cells >= (1ull << 22))
        return lattice == 1 ? launch_planes<1>(species, L, K, S, d_counts, stream)
                            : launch_planes<0>(species, L, K, S, d_counts, stream);
    if (lattice == 1) return K <= 4 ? launch_pc<1, 8>(species, L, K, S, d_counts, stream)
                                    : launch_pc<1, 4>(species, L, K, S, d_counts, stream);
    return K <= 4 ? launch_pc<0, 8>(species, L, K, S, d_counts, stream)
                  : launch_pc<0, 4>(species, L, K, S, d_counts, stream);
}

}  // namespace smcx
