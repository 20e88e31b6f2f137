// tables.cpp -- host-built tables of libsmcx.
#include <cmath>
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
int build_wtab(const int32_t* epi, int K, int S, int kmax, int smax, int bias, int32_t* out)
{
    const int wr = wrow(kmax, smax);
    auto W = [&](int a, int b, int s, int p) -> int64_t {   // zero for species beyond K
        return p < K ? (int64_t)epi[(s * K + b) * K + p] - epi[(s * K + a) * K + p] : 0;
    };
    int drop = 1;
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
