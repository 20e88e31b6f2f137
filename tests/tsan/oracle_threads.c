/* Driver for a ThreadSanitizer run of the oracle's OpenMP paths on the CPU.
 * Builds random multicomponent lattices (BCC and FCC), runs sweeps with one thread
 * and with four, and checks that the configurations, energies, accept
 * counts and pair counts agree; the threaded run happens under TSan (with
 * LLVM's OpenMP race detector), which reports any data race it observes.
 * Exit status 0 iff every comparison holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "smcx_oracle.h"

static uint64_t lcg(uint64_t* s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return *s >> 33;
}

static int run(int lat, int L0, int K, int S)
{
    const int32_t L[3] = {L0, L0 + 1, L0 + 2};
    const int32_t B[3] = {4, 4, 4};
    const int nsub = lat ? 4 : 2;
    const size_t N = (size_t)nsub * L[0] * L[1] * L[2];
    uint64_t r = 12345u + (uint64_t)lat;
    int32_t* epi = (int32_t*)malloc(sizeof(int32_t) * S * K * K);
    for (int s = 0; s < S; ++s)
        for (int p = 0; p < K; ++p)
            for (int q = p; q < K; ++q) {
                const int32_t v = (int32_t)(lcg(&r) % 60001) - 30000;
                epi[(s * K + p) * K + q] = epi[(s * K + q) * K + p] = v;
            }
    uint8_t* a = (uint8_t*)malloc(N);
    uint8_t* b = (uint8_t*)malloc(N);
    for (size_t i = 0; i < N; ++i) a[i] = (uint8_t)(i % (size_t)K);
    for (size_t i = N - 1; i > 0; --i) {   /* shuffle */
        const size_t j = (size_t)(lcg(&r) % (i + 1));
        const uint8_t t = a[i];
        a[i] = a[j];
        a[j] = t;
    }
    memcpy(b, a, N);
    const int n = 3;
    double T[3] = {900.0, 700.0, 1500.0};
    int64_t Ea = or_energy(lat, L, S, K, epi, a), Eb = Ea;
    uint64_t acc_a = 0, acc_b = 0;
    uint64_t* ca = (uint64_t*)calloc((size_t)n * S * K * K, sizeof(uint64_t));
    uint64_t* cb = (uint64_t*)calloc((size_t)n * S * K * K, sizeof(uint64_t));
    or_set_threads(1);
    int rc = or_sweep(lat, L, B, S, K, epi, 99, 0, n, T, a, &Ea, &acc_a, NULL, ca);
    or_set_threads(4);
    rc |= or_sweep(lat, L, B, S, K, epi, 99, 0, n, T, b, &Eb, &acc_b, NULL, cb);
    or_set_threads(1);
    const int same = rc == 0 && memcmp(a, b, N) == 0 && Ea == Eb && acc_a == acc_b &&
                     memcmp(ca, cb, sizeof(uint64_t) * (size_t)n * S * K * K) == 0 && acc_a > 0;
    printf("lattice %d L=%d K=%d S=%d: %s (E %lld, accepted %llu)\n", lat, L0, K, S, same ? "same" : "DIFFERENT",
           (long long)Ea, (unsigned long long)acc_a);
    free(epi);
    free(a);
    free(b);
    free(ca);
    free(cb);
    return same ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    /* large enough that every (colour, sub-colour) set holds more than the
       512 trials above which the oracle runs a set on several threads */
    bad |= run(0, 56, 5, 3);
    bad |= run(1, 50, 4, 3);
    return bad;
}
