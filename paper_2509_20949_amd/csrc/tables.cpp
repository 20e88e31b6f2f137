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
//   dE = sum_{s,p} (n_i[s][p] - n_j[s][p]) (V_s(b,p) - V_s(a,p))
//        - (V_1(a,a) + V_1(b,b) - 2 V_1(a,b)),
// the last term removing the i-j bond that both counts include.  When the
// kernel packs bias + n_i - n_j per field, the constant also removes
// bias * sum W.
void build_wtab(const int32_t* epi, int K, int S, int kmax, int smax, int bias, int32_t* out)
{
    const int wr = wrow(kmax, smax);
    std::memset(out, 0, sizeof(int32_t) * (size_t)kmax * kmax * wr);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            int32_t* row = out + (size_t)(a * kmax + b) * wr;
            int64_t sum = 0;
            for (int s = 0; s < S; ++s)
                for (int p = 0; p < K; ++p) {
                    const int32_t w = epi[(s * K + b) * K + p] - epi[(s * K + a) * K + p];
                    row[s * kmax + p] = w;
                    sum += w;
                }
            const int64_t corr = -((int64_t)epi[a * K + a] + epi[b * K + b] - 2 * (int64_t)epi[a * K + b]);
            // stored modulo 2^32; the kernel sums modulo 2^32 as well
            const int64_t c = -(int64_t)bias * sum + corr;
            row[smax * kmax] = (int32_t)(uint32_t)(uint64_t)c;
        }
}

}  // namespace smcx
