// tables.cpp -- host-built tables of libsmcx.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "smcx_internal.h"

namespace smcx {

// Metropolis thresholds (paper, Eq. (3)): an uphill change dE (micro-eV,
// 0 < dE < 2^24) is accepted iff (double)u < (T2[dE>>16]*T1[(dE>>8)&255])*T0[dE&255]
// for a uniform 32-bit u, i.e. with probability exp(-beta dE) to within
// 2^-32 plus a few ulp.  k_B = 86.17333262 micro-eV/K (CODATA 2018).
void build_thresholds(double T, double* out)
{
    const double kB = 86.17333262;
    const double beta = 1.0 / (kB * T);
    for (int l = 0; l < 256; ++l) {
        out[l] = std::exp(-((double)l * beta));
        out[256 + l] = std::exp(-((double)(l * 256) * beta));
        out[512 + l] = std::ldexp(std::exp(-((double)(l * 65536) * beta)), 32);
    }
    out[kTabLn2kT] = std::log(2.0) * kB * T;
    out[kTabLn2kT + 1] = 0.0;
}

// Pair-weight rows for the swap of species a (at site i) and b (at its
// first neighbour j).  With n_i[s][p], n_j[s][p] the species counts in shell
// s around i and j (each including the other site of the pair),
//   dE = sum_{s,p} (n_i[s][p] - n_j[s][p]) W[s][p] - (V_1(a,a) + V_1(b,b) - 2 V_1(a,b)),
//   W[s][p] = V_s(b,p) - V_s(a,p),
// the last term removing the i-j bond that both counts include.  Both sites
// have the same number of neighbours in every shell, so the differences
// d[s][p] = n_i[s][p] - n_j[s][p] sum to zero over p and the last species
// p = kmax-1 can be dropped: dE = sum_{s, p < kmax-1} d[s][p] (W[s][p] -
// W[s][kmax-1]) + the bond term.  The kernel multiplies on the 24-bit
// multiplier, so the folded rows are used only when every W[s][p] -
// W[s][kmax-1] fits in 24 signed bits (always when |V| < 2^21); otherwise
// the rows keep all kmax fields (|W| < 2^23 holds for |V| < 2^22).  The
// kernel packs bias + d[s][p] per field, so the constant also removes bias
// times the sum of the weights it reads.  Row layout: weight (s, p) at
// s*kmax + p, the constant at smax*kmax, all modulo 2^32 (the kernel sums
// modulo 2^32).
//
// Byte-dot rows (returned value kWtabDot; kmax <= 5): the kernel
// counts species p < kmax-1 in byte p of a 32-bit word (the last species
// in bit 31, which it masks off), forms bytes 32 + d[s][p] and takes dot
// products of 4 signed bytes.  Each folded weight W'[s][p] = W[s][p] -
// W[s][kmax-1] is written in three signed base-256 digits, W' = w0 + 2^8 w1
// + 2^16 w2 with w0, w1, w2 in [-128, 127]; row entry 3s + k packs digit k
// of W'[s][0..3] into bytes 0..3, and entry 3 smax holds the constant (the
// bond term less 32 times the sum of the W').  Used when every W' has such
// digits (|W'| < 2^23 - 2^15 suffices).
static bool digits3(int64_t w, int32_t d[3])
{
    for (int k = 0; k < 3; ++k) {
        const int64_t r = (int64_t)(int8_t)(uint8_t)(uint64_t)w;   // low digit in [-128, 127]
        d[k] = (int32_t)r;
        w = (w - r) / 256;
    }
    return w == 0;
}

int build_wtab(const int32_t* epi, int K, int S, int kmax, int smax, int bias, bool dot_ok, int32_t* out)
{
    const int wr = wrow(kmax, smax);
    auto W = [&](int a, int b, int s, int p) -> int64_t {   // zero for species beyond K
        return p < K ? (int64_t)epi[(s * K + b) * K + p] - epi[(s * K + a) * K + p] : 0;
    };
    if (dot_ok && kmax <= 5) {
        bool fits = true;
        int32_t dg[3];
        for (int a = 0; a < K && fits; ++a)
            for (int b = 0; b < K && fits; ++b)
                for (int s = 0; s < S && fits; ++s)
                    for (int p = 0; p < kmax - 1 && fits; ++p)
                        fits = digits3(W(a, b, s, p) - W(a, b, s, kmax - 1), dg);
        if (fits) {
            std::memset(out, 0, sizeof(int32_t) * (size_t)kmax * kmax * wr);
            for (int a = 0; a < K; ++a)
                for (int b = 0; b < K; ++b) {
                    int32_t* row = out + (size_t)(a * kmax + b) * wr;
                    int64_t sum = 0;
                    for (int s = 0; s < S; ++s)
                        for (int p = 0; p < kmax - 1; ++p) {
                            const int64_t w = W(a, b, s, p) - W(a, b, s, kmax - 1);
                            digits3(w, dg);
                            for (int k = 0; k < 3; ++k)
                                row[3 * s + k] = (int32_t)((uint32_t)row[3 * s + k] | ((uint32_t)(uint8_t)dg[k] << (8 * p)));
                            sum += w;
                        }
                    const int64_t corr = -((int64_t)epi[a * K + a] + epi[b * K + b] - 2 * (int64_t)epi[a * K + b]);
                    row[3 * smax] = (int32_t)(uint32_t)(uint64_t)(corr - 32 * sum);
                }
            return kWtabDot;
        }
    }
    // (the BCC kernels for kmax <= 5 take the byte-dot or the full rows)
    int drop = dot_ok && kmax <= 5 ? 0 : 1;
    for (int a = 0; a < K && drop; ++a)
        for (int b = 0; b < K && drop; ++b)
            for (int s = 0; s < S && drop; ++s)
                for (int p = 0; p < kmax - 1; ++p) {
                    const int64_t w = W(a, b, s, p) - W(a, b, s, kmax - 1);
                    if (w < -(int64_t)(1 << 23) || w >= (int64_t)(1 << 23)) { drop = 0; break; }
                }
    std::memset(out, 0, sizeof(int32_t) * (size_t)kmax * kmax * wr);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            int32_t* row = out + (size_t)(a * kmax + b) * wr;
            int64_t sum = 0;
            for (int s = 0; s < S; ++s) {
                const int64_t last = drop ? W(a, b, s, kmax - 1) : 0;
                for (int p = 0; p < kmax - drop; ++p) {
                    const int64_t w = W(a, b, s, p) - last;
                    row[s * kmax + p] = (int32_t)(uint32_t)(uint64_t)w;
                    sum += w;
                }
            }
            const int64_t corr = -((int64_t)epi[a * K + a] + epi[b * K + b] - 2 * (int64_t)epi[a * K + b]);
            const int64_t c = -(int64_t)bias * sum + corr;
            row[smax * kmax] = (int32_t)(uint32_t)(uint64_t)c;
        }
    return drop;
}

// Block width chosen for an axis of L cells when the caller leaves it to the
// library.  A wavefront runs one block's 54 rounds whatever the block's
// width, so a launch costs about the same per block, and the widest allowed
// block (12 cells, the 4 x 4 x 4-lane round) gives the fewest blocks and the
// most trials per wavefront.  Measured for batched replicas of every edge
// 16..96 and every B = 4..12 (bench.py --tune-blocks): the widths with the
// fewest blocks are the fastest at every edge, by 9 % or more, and B = 12
// always gives them.  The choice depends on nothing else, so a trajectory
// with block = 0 is reproducible.
int plan_block(int lattice, int L, int K)
{
    (void)lattice;
    (void)L;
    (void)K;
    return kMaxBlock;
}

// A colour launch of a single lattice runs its blocks in "generations" of
// the wave slots the chip holds; a partly filled last generation leaves
// most of the chip idle at the end of every launch.  FCC blocks fill 10
// slots per CU in workgroups of 2 (LDS-bound), or 11 in one workgroup of 11
// images (160 KB of LDS): the wide form is taken when it needs fewer
// generations, e.g. 2,744 blocks (the 336 x 315 x 315 lattice) take one
// generation of 2,816 slots instead of 1.07 of 2,560 (measured 196 us per
// launch against 273).  BCC keeps its 4-wave workgroups: on the 512^3
// lattice, workgroups of 7 and 11 blocks (21 and 22 waves per CU) measured
// no faster.
int plan_waves_per_group(int lattice, int blocks_per_colour, int n_cu)
{
    if (const char* f = std::getenv("SMCX_WAVES_PER_GROUP")) {   // measurement override (bench.py --tune-wpg)
        const int w = std::atoi(f);
        if (lattice == 1 && (w == kWavesPerGroupFcc || w == kWavesPerGroupFccWide)) return w;
    }
    if (lattice != 1 || n_cu < 1) return lattice == 1 ? kWavesPerGroupFcc : kWavesPerGroup;
    const long narrow = 10L * n_cu, wide = (long)kWavesPerGroupFccWide * n_cu;
    const long g_narrow = (blocks_per_colour + narrow - 1) / narrow, g_wide = (blocks_per_colour + wide - 1) / wide;
    return g_wide < g_narrow ? kWavesPerGroupFccWide : kWavesPerGroupFcc;
}

void count_sum(const unsigned long long* slots, unsigned long long* out)
{
    for (int k = 0; k < kCountWords; ++k) {
        unsigned long long v = 0;
        for (int c = 0; c < kCountSlots; ++c) v += slots[(size_t)c * kCountWords + k];
        out[k] = v;
    }
}

void state_init(int64_t* h, int64_t E, uint64_t accepted)
{
    std::memset(h, 0, sizeof(int64_t) * kStateWords);
    h[0] = E;
    h[1] = (int64_t)accepted;
}

void state_sum(const int64_t* h, int64_t* E, uint64_t* accepted)
{
    uint64_t e = 0, a = 0;   // modulo 2^64: partial slots may wrap, the sum does not
    for (int k = 0; k < kSpread; ++k) {
        e += (uint64_t)h[k * kSlotWords];
        a += (uint64_t)h[k * kSlotWords + 1];
    }
    if (E) *E = (int64_t)e;
    if (accepted) *accepted = a;
}

}  // namespace smcx
