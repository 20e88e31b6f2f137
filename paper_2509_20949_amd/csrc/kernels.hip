// kernels.hip -- gfx950 kernels of libsmcx.
//
// sweep_phase: one colour phase of a Metropolis swap sweep (paper: Section
//   "Monte Carlo simulation", Eq. (3); link cells of Section "Distributed
//   SMC-X").  One wavefront owns one block of the shifted block grid: it
//   stages the block and its interaction halo from HBM into LDS, runs the 54
//   sub-colour rounds (64 lanes = the 4 x 4 x 4 same-residue cells of a 12-wide
//   block, one trial each), writes the block and the first-neighbour ring
//   back, and reduces its accepted energy changes.  Lanes of one round never
//   touch each other's sites, and LDS operations of one wavefront complete in
//   program order, so no barrier separates the rounds.
#include <type_traits>

#include "device_common.h"

namespace smcx {

// ---------------------------------------------------------------------------
// Species codes in LDS.  A site of species v is stored as (F + 32) * v, with
// F = 5 bits per species field when KMAX <= 6 and F = 4 otherwise: the low 5
// bits (the only bits a 32-bit shift reads) equal F * v, the top 3 bits equal
// v.  One shift-add per neighbour then counts species into packed fields.
template <int KMAX> struct Field { static constexpr int F = KMAX <= 6 ? 5 : 4; };

__device__ __forceinline__ uint32_t encode4(uint32_t species, int F)
{
    // up to four species bytes v_k -> bytes (F+32) v_k: no carries, as
    // (F+32) v <= 255 for every species the field width admits (all four
    // bytes are used, so no 24-bit multiply)
    return (species << 5) + species * (uint32_t)F;
}

// LDS layout of one block (see smcx_internal.h): corner array at offset 0,
// body array at kArr.  Local cell (x, y, z):
//   corner: (z+1)*kPP + (y+1)*kP + (x+1)       x in -1..13
//   body:   kArr + (z+2)*kPP + (y+2)*kP + (x+2) x in -2..12
// Offsets of the first shell from a corner site (body sites at cell offsets
// {-1,0}^3) and from a body site (corner sites at {0,+1}^3):
constexpr int kS1Corner = kArr;                      // + ex + ey*kP + ez*kPP, e in {0,1}
constexpr int kS1Body = -kArr - (kPP + kP + 1);      // + ex + ey*kP + ez*kPP, e in {0,1}

template <int SUB> __device__ __forceinline__ constexpr int s1base() { return SUB == 0 ? kS1Corner : kS1Body; }

// Waves per SIMD the BCC sweep kernel is compiled for (registers); LDS
// (4 block images and the weight planes per workgroup) admits 5 workgroups
// of 4 waves per CU.
constexpr int kSweepWavesPerSimd = 5;
// Rows whose loads a lane issues together when staging a block (registers
// bound it: one aligned word per row once the two loads are joined).
constexpr int kStageBatch = 16;

// Weight planes of the BCC kernel: row (a, b) at position a*KMAX + b of a
// 64-entry plane, so that the position of any two 3-bit codes (a lane
// without a site may decode a stale halo byte) stays inside its plane.  The
// KMAX^2 rows of real species then lie in distinct LDS banks (positions
// 8a + b, one multiply fewer, put species 4 and 0 of K = 5 on the same
// banks: 16 % of the LDS cycles went to those conflicts).
constexpr int kPlane = 64;
static_assert(7 * kMaxK + 7 < kPlane, "weight plane too narrow");

// Shell offsets inside one sublattice array.
__device__ __forceinline__ constexpr int s2off(int k)
{
    return k == 0 ? 1 : k == 1 ? -1 : k == 2 ? kP : k == 3 ? -kP : k == 4 ? kPP : -kPP;
}
__device__ __forceinline__ constexpr int s3off(int k)
{
    // (+-1, +-1, 0), (+-1, 0, +-1), (0, +-1, +-1)
    return k == 0 ? 1 + kP : k == 1 ? 1 - kP : k == 2 ? -1 + kP : k == 3 ? -1 - kP
         : k == 4 ? 1 + kPP : k == 5 ? 1 - kPP : k == 6 ? -1 + kPP : k == 7 ? -1 - kPP
         : k == 8 ? kP + kPP : k == 9 ? kP - kPP : k == 10 ? -kP + kPP : -kP - kPP;
}


// Counts of the second and third shells of the site at LDS byte a (its own
// sublattice), added to h[1] and h[2]; the codes of the 6 second and 12
// third neighbours are returned in r2 and r3 (index k: offsets s2off(k),
// s3off(k)).
template <int SMAX, bool NEG>
__device__ __forceinline__ void count_outer(const uint8_t* lat, int a, uint32_t (&h)[kMaxS], uint32_t (&r2)[6],
                                            uint32_t (&r3)[12])
{
    if constexpr (SMAX >= 2) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            r2[k] = lat[a + s2off(k)];
            count1<NEG>(h[1], r2[k]);
        }
    }
    if constexpr (SMAX >= 3) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            r3[k] = lat[a + s3off(k)];
            count1<NEG>(h[2], r3[k]);
        }
    }
}

// First-shell offset (from the site) of neighbour e = ex + 2 ey + 4 ez.
template <int SUB> __device__ __forceinline__ constexpr int s1off(int e)
{
    return s1base<SUB>() + (e & 1) + ((e >> 1) & 1) * kP + ((e >> 2) & 1) * kPP;
}

// acc + sum over shells s < SMAX and fields p < NF of field(s, p) * w[s*KMAX + p],
// modulo 2^32: field = bias + n_i - n_j read from the packed difference
// (F = 5), or n_i - n_j from the two 4-bit fields (F = 4).  The constant may
// leave the int32 range for extreme tables while the true dE (|dE| < 2^29)
// never does: the 32-bit multiply-adds wrap, and the wrapped sum is exact.
template <int KMAX, int SMAX, int NF>
__device__ __forceinline__ uint32_t weigh(const uint32_t (&hi)[kMaxS], const uint32_t (&hj)[kMaxS],
                                          const int32_t* w, uint32_t acc)
{
    constexpr int PS = kPlane;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if constexpr (Field<KMAX>::F == 5) {
            const uint32_t d = hi[s] - hj[s];   // fields 16 + n_i - n_j, no borrows
#pragma unroll
            for (int p = 0; p < NF; ++p)
                acc = mad24((d >> (5 * p)) & 31u, w[(s * KMAX + p) * PS], acc);
        } else {
#pragma unroll
            for (int p = 0; p < NF; ++p)
                acc = mad24((uint32_t)((int32_t)((hi[s] >> (4 * p)) & 15u) - (int32_t)((hj[s] >> (4 * p)) & 15u)),
                            w[(s * KMAX + p) * PS], acc);
        }
    }
    return acc;
}

// The partner part of a three-shell trial for the direction E (a
// compile-time value; the trial switches on its wave-uniform direction):
// half of the partner's neighbourhood is cells the site's own counts
// already hold.  In half-cell units j = i + s, s_a = +-1 the signs of E.
// j's first shell is i + (0 or 2 s_a per axis): i, the site's second
// neighbours i + 2 s_a along the three axes, its third neighbours in the
// three planes with the same signs, and the far cell i + 2 s (loaded).  j's
// second and third shells hold the site's first-shell cells k with one or
// two direction bits flipped (popcount(k ^ E) = 1 or 2) and 3 and 9 cells
// beyond (loaded).  With T0, T1 the site's first-shell counts over indices
// of even and odd popcount, those two sets are T[par E ^ 1] less cell
// E ^ 7 and T[par E] less cell E (the partner).  Sets cj (the partner's
// code) and adds j's counts to h (+1 per neighbour, or -1 with NEG).
template <int SUB, int E, bool NEG>
__device__ __forceinline__ void partner3(const uint8_t* lat, int ai, const uint32_t (&s1)[8], uint32_t ci,
                                         const uint32_t (&r2)[6], const uint32_t (&r3)[12], uint32_t T0,
                                         uint32_t T1, uint32_t& cj, uint32_t (&h)[kMaxS])
{
    constexpr int ex = E & 1, ey = (E >> 1) & 1, ez = (E >> 2) & 1;
    constexpr int dx = ex ? 1 : -1, dy = ey ? kP : -kP, dz = ez ? kPP : -kPP;
    constexpr bool odd = (ex + ey + ez) & 1;
    const int aj = ai + s1off<SUB>(E);
    cj = s1[E];
    uint32_t t_same = odd ? T1 : T0, t_other = odd ? T0 : T1;
    count1<true>(t_same, s1[E]);        // j's third-shell cells among the site's first shell
    count1<true>(t_other, s1[E ^ 7]);   // j's second-shell cells among them
    // j's first shell
    count1<NEG>(h[0], ci);
    count1<NEG>(h[0], r2[ex ? 0 : 1]);
    count1<NEG>(h[0], r2[ey ? 2 : 3]);
    count1<NEG>(h[0], r2[ez ? 4 : 5]);
    count1<NEG>(h[0], r3[(ex ? 0 : 2) + (ey ? 0 : 1)]);
    count1<NEG>(h[0], r3[4 + (ex ? 0 : 2) + (ez ? 0 : 1)]);
    count1<NEG>(h[0], r3[8 + (ey ? 0 : 2) + (ez ? 0 : 1)]);
    count1<NEG>(h[0], lat[ai + dx + dy + dz]);
    // j's second and third shells
    h[1] = NEG ? h[1] - t_other : h[1] + t_other;
    h[2] = NEG ? h[2] - t_same : h[2] + t_same;
    count1<NEG>(h[1], lat[aj + dx]);
    count1<NEG>(h[1], lat[aj + dy]);
    count1<NEG>(h[1], lat[aj + dz]);
    count1<NEG>(h[2], lat[aj + dx + dy]);
    count1<NEG>(h[2], lat[aj + dx - dy]);
    count1<NEG>(h[2], lat[aj - dx + dy]);
    count1<NEG>(h[2], lat[aj + dx + dz]);
    count1<NEG>(h[2], lat[aj + dx - dz]);
    count1<NEG>(h[2], lat[aj - dx + dz]);
    count1<NEG>(h[2], lat[aj + dy + dz]);
    count1<NEG>(h[2], lat[aj + dy - dz]);
    count1<NEG>(h[2], lat[aj - dy + dz]);
}

// Codes a trial hands to the next one (registers), so that the next trial
// reads neither its own site, nor its partner, nor 7 of its 8 first
// neighbours from LDS.  The next site is the other sublattice's site of the
// lane's cell: after a corner trial at corner(x, y, z) the body trial at
// body(x, y, z), whose first shell is corner(x + ex, y + ey, z + ez); after a
// body trial at body(x, y, z) the corner trial of the next residue class
// when that is corner(x + 1, y, z), whose first shell is body(x + ex,
// y - 1 + ey, z - 1 + ez).  Of these 8 cells one is the trial's own site
// (its new code), 6 are second or third neighbours of it that the trial
// reads, and one more cell of its sublattice it loads for the next trial
// (corner(x + 1, y + 1, z + 1), or body(x + 1, y - 1, z - 1)).  Nothing in
// the trial's round changes those 7 (only sites of its residue class and
// their partners, of the other sublattice, change).  The next site itself
// is a first neighbour of the trial's site: only this lane's trial can have
// swapped it.  Between the two trials no other lane changes any of these
// cells (a lane's cells lie within one cell of its own sites, lanes are
// three cells apart).
struct Carry {
    uint32_t s1[8];   // first-shell codes of the next site, index e = ex + 2 ey + 4 ez
    uint32_t own;     // code of the next site
};
// One trial: site at LDS byte ai (sublattice SUB) with its 32-bit
// acceptance draw u.  The partner is first-shell neighbour e = ex + 2 ey +
// 4 ez, the direction shared by the whole round (wave-uniform).  CIN: the
// site's code and its first shell come from the previous trial (cy);
// otherwise they are loaded.  COUT: cy is set for the next trial.
// Adds the accepted energy change to the lane's dEsum and the wave's
// accepted count to nacc (the same in every lane); updates the LDS image in
// place.
// E >= 0: the direction as a compile-time value (three shells), else e_rt.
template <int KMAX, int SMAX, int SUB, int MODE, bool CIN, bool COUT, int E>
__device__ __forceinline__ void trial_dir(uint8_t* lat, int ai, uint32_t u, int e_rt, bool valid,
                                          const int32_t* wtab, const double* tab, float ln2kT, int64_t& dEsum,
                                          uint32_t& nacc, Carry& cy)
{
    static_assert(SMAX < 3 || E >= 0, "three-shell trials take a compile-time direction");
    const int e = E >= 0 ? E : e_rt;
    constexpr int F = Field<KMAX>::F;
    constexpr bool DOT = MODE == kWtabDot;
    // 5-bit fields (and the byte-dot form) hold bias + n_i - n_j without
    // borrows: one packed difference per shell.  4-bit fields (KMAX = 8)
    // count the two neighbourhoods apart.
    constexpr bool DIFF = DOT || F == 5;
    const uint32_t u_acc = u;
    float elo, ehi;
    accept_edges(u_acc, ln2kT, elo, ehi);   // depends on the draw only: off the critical path
    const int aj = ai + s1base<SUB>() + (e & 1) + ((e >> 1) & 1) * kP + ((e >> 2) & 1) * kPP;

    // the site, its first shell, and the partner (first-shell cell e)
    uint32_t s1[8];
    uint32_t ci;
    if constexpr (CIN) {
#pragma unroll
        for (int e = 0; e < 8; ++e) s1[e] = cy.s1[e];
        ci = cy.own;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) s1[e] = lat[ai + s1off<SUB>(e)];
        ci = lat[ai];
    }
    // Species histograms of both neighbourhoods (the partner is counted in
    // the first shell of i and i in that of j; the constant term undoes it).
    // In the difference form j's chains subtract and are added to i's
    // (fields then hold bias + n_i - n_j).
    uint32_t hi[kMaxS], hj[kMaxS];
    constexpr uint32_t bias = DOT ? 0x20202020u
                            : F == 5 ? 0x10u * (1u | 1u << 5 | 1u << 10 | 1u << 15 | 1u << 20 | 1u << 25) : 0u;
#pragma unroll
    for (int s = 0; s < kMaxS; ++s) { hi[s] = bias; hj[s] = 0u; }
    uint32_t r2[6], r3[12];
    uint32_t cj;
    if constexpr (SMAX < 3) {
        // the partner by seven v_cndmask on the bits of e (held in a vector
        // register, e's selects stay in the trial's basic block instead of
        // becoming branches, which would keep the loads below from being
        // issued ahead)
        uint32_t ev = (uint32_t)e;
        asm volatile("" : "+v"(ev));
        const uint32_t x0 = ev & 1u ? s1[1] : s1[0], x1 = ev & 1u ? s1[3] : s1[2];
        const uint32_t x2 = ev & 1u ? s1[5] : s1[4], x3 = ev & 1u ? s1[7] : s1[6];
        const uint32_t y0 = ev & 2u ? x1 : x0, y1 = ev & 2u ? x3 : x2;
        cj = ev & 4u ? y1 : y0;
#pragma unroll
        for (int k = 0; k < 8; ++k) count1<false>(hi[0], s1[k]);
        count_outer<SMAX, false>(lat, ai, hi, r2, r3);
#pragma unroll
        for (int k = 0; k < 8; ++k) count1<DIFF>(hj[0], lat[aj + s1off<1 - SUB>(k)]);
        uint32_t q2[6], q3[12];
        count_outer<SMAX, DIFF>(lat, aj, hj, q2, q3);
    } else {
        uint32_t T0 = 0u, T1 = 0u;   // the site's first shell, indices of even / odd popcount
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (__builtin_popcount(k) & 1) count1<false>(T1, s1[k]);
            else count1<false>(T0, s1[k]);
        }
        hi[0] += T0 + T1;
        count_outer<3, false>(lat, ai, hi, r2, r3);
        // j's counts: subtracted from i's chains in the difference form
        auto& hp = *(DIFF ? &hi : &hj);
        partner3<SUB, (E >= 0 ? E : 0), DIFF>(lat, ai, s1, ci, r2, r3, T0, T1, cj, hp);
    }
    // Row (a, b) of the weight planes, a = ci >> 5 and b = cj >> 5, at byte
    // 4 (a*KMAX + b) of a plane.  (Lanes without a site in this round may
    // decode stale halo bytes: their row still lies inside the planes, and
    // their result is discarded.)
    const uint32_t row4 = __umul24(ci >> 5, 4u * KMAX) + ((cj >> 5) << 2);
    const int32_t* w = (const int32_t*)((const uint8_t*)wtab + row4);
    // the cell of this sublattice the next trial's first shell needs besides
    // these: corner(x + 1, y + 1, z + 1) or body(x + 1, y - 1, z - 1)
    const uint32_t fresh = COUT ? (uint32_t)lat[ai + (SUB == 0 ? 1 + kP + kPP : 1 - kP - kPP)] : 0u;
    if constexpr (DIFF) {
#pragma unroll
        for (int s = 0; s < kMaxS; ++s) { hi[s] += hj[s]; hj[s] = 0u; }
    }

    uint32_t acc;
    if constexpr (DOT) {
        // bytes 32 + n_i - n_j (bit 31, the last species, masked off) dotted
        // with the three base-256 digits of the folded weights, in one
        // chain: ((A2 * 256 + A1) * 256 + constant) + A0
        constexpr int PS = kPlane;
        int32_t d[kMaxS];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) d[s] = (int32_t)(hi[s] & 0x7fffffffu);
        int32_t X = 0;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(d[s], w[(3 * s + 2) * PS], X, false);
        X = (int32_t)((uint32_t)X << 8);
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(d[s], w[(3 * s + 1) * PS], X, false);
        X = (int32_t)(((uint32_t)X << 8) + (uint32_t)w[3 * SMAX * PS]);
#pragma unroll
        for (int s = 0; s < SMAX; ++s) X = __builtin_amdgcn_sdot4(d[s], w[(3 * s + 0) * PS], X, false);
        acc = (uint32_t)X;
    } else {
        // With kWtabDrop the rows fold in the last species, whose count
        // differences follow from the others (both sites have the same
        // number of neighbours per shell): only fields 0 .. KMAX-2 are read.
        acc = weigh<KMAX, SMAX, MODE == kWtabDrop ? KMAX - 1 : KMAX>(hi, hj, w,
                                                                      (uint32_t)w[SMAX * KMAX * kPlane]);
    }
    const int32_t dE = (int32_t)acc;

    // Metropolis decision, Eq. (3): the exact test on the FP64 byte tables,
    // evaluated only when a lane's dE falls between its bounds (a
    // wave-uniform branch, taken by a few percent of the rounds).  float(dE)
    // is exact wherever `up` holds.
    const float fdE = (float)dE;
    const bool up = (dE > 0) & (dE < (1 << 24));
    const bool sure = fdE <= elo;
    const bool near = up & ((!sure & (fdE <= ehi)) | (u_acc == 0u));
    bool up_ok = up & sure;
    if (__builtin_amdgcn_ballot_w64(near)) {
        const int e = dE < 1 ? 1 : (dE > (1 << 24) - 1 ? (1 << 24) - 1 : dE);
        const uint8_t* tb = (const uint8_t*)tab;   // global memory (L2-resident)
        const double thr = (gload<double>(tb + 8 * (512 + (e >> 16))) * gload<double>(tb + 8 * (256 + ((e >> 8) & 255)))) *
                           gload<double>(tb + 8 * (e & 255));
        up_ok = near ? (double)u_acc < thr : up_ok;
    }
    const bool accept = valid & (ci != cj) & ((dE <= 0) | up_ok);
    // Both bytes are stored by every lane (unchanged unless accepted): no
    // two lanes of a round touch the same byte, and a branch-free trial
    // keeps the whole round in one basic block for the scheduler.
    const uint32_t ci_new = accept ? cj : ci;
    lat[ai] = (uint8_t)ci_new;
    lat[aj] = (uint8_t)(accept ? ci : cj);
    dEsum += (int64_t)(accept ? dE : 0);
    nacc += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(accept));   // wave-uniform: counted on the scalar unit

    if constexpr (COUT) {
        // the next site is first-shell cell kNext of this site; it changed
        // iff it was the partner of an accepted swap
        constexpr int kNext = SUB == 0 ? 7 : 1;
        cy.own = accept && e == kNext ? ci : s1[kNext];
        if constexpr (SUB == 0) {   // next: body(x, y, z); its first shell corner(x + ex, y + ey, z + ez)
            cy.s1[0] = ci_new;
            cy.s1[1] = r2[0];   // +x
            cy.s1[2] = r2[2];   // +y
            cy.s1[3] = r3[0];   // +x +y
            cy.s1[4] = r2[4];   // +z
            cy.s1[5] = r3[4];   // +x +z
            cy.s1[6] = r3[8];   // +y +z
            cy.s1[7] = fresh;   // +x +y +z
        } else {                    // next: corner(x + 1, y, z); its first shell body(x + ex, y - 1 + ey, z - 1 + ez)
            cy.s1[0] = r3[11];  // -y -z
            cy.s1[1] = fresh;   // +x -y -z
            cy.s1[2] = r2[5];   // -z
            cy.s1[3] = r3[5];   // +x -z
            cy.s1[4] = r2[3];   // -y
            cy.s1[5] = r3[1];   // +x -y
            cy.s1[6] = ci_new;  // the site itself
            cy.s1[7] = r2[0];   // +x
        }
    }
}

// One trial with the round's direction e (wave-uniform).  Three-shell trials
// switch on it before anything else: each case is then one straight-line
// trial whose loads (the site's and the partner's cells) the compiler can
// issue together.
template <int KMAX, int SMAX, int SUB, int MODE, bool CIN, bool COUT>
__device__ __forceinline__ void trial(uint8_t* lat, int ai, uint32_t u, int e, bool valid, const int32_t* wtab,
                                      const double* tab, float ln2kT, int64_t& dEsum, uint32_t& nacc, Carry& cy)
{
    if constexpr (SMAX == 3) {
        switch (e) {
        case 0: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 0>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 1: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 1>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 2: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 2>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 3: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 3>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 4: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 4>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 5: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 5>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        case 6: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 6>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        default: trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, 7>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy); break;
        }
    } else {
        trial_dir<KMAX, SMAX, SUB, MODE, CIN, COUT, -1>(lat, ai, u, e, valid, wtab, tab, ln2kT, dEsum, nacc, cy);
    }
}

// ---------------------------------------------------------------------------
// SLAB: the lattice is a z-slab (DevLattice::slab) -- its own instance, so
// the periodic kernel carries none of the slab's addressing.  WPG: blocks
// (waves) per workgroup, kWavesPerGroup (5 workgroups, 20 waves per CU,
// bound by LDS).  Wider workgroups (3 of 7 or 2 of 11 per CU, 21 and 22
// waves) fill the wave slots of a 512^3 colour launch more evenly but
// measured no faster: a CU is busy issuing at 20 waves.
template <int KMAX, int SMAX, bool SLAB, int WPG>
__global__ __launch_bounds__(kWave * WPG) __attribute__((amdgpu_waves_per_eu(kSweepWavesPerSimd)))
void sweep_phase_kernel(const DevLattice* __restrict__ lats, const WorkItem* __restrict__ items, int n_groups,
                        int t, int colour)
{
    constexpr int F = Field<KMAX>::F;
    // One LDS buffer: the weight planes at offset 0 (so a plane's LDS offset
    // fits the st64 immediates of ds_read2st64_b32 and row addresses need no
    // base added), then the block images.
    constexpr int kWBytes = wplanes(KMAX, SMAX) * kPlane * 4;
    __shared__ __attribute__((aligned(16))) uint8_t s_mem[kWBytes + WPG * kWaveLds];
    int32_t* s_w = (int32_t*)s_mem;
    uint8_t* s_lat = s_mem + kWBytes;

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

    // Weight planes in LDS; the threshold tables of sweep s stay in global
    // memory (read only for the few draws whose decision needs them), which
    // leaves LDS for five workgroups per CU.
    load_wplanes<KMAX, SMAX, kPlane>(s_w, D.wtab);
    __syncthreads();
    int ti = (int)(s - D.tab_s0);
    ti = ti < 0 ? 0 : (ti >= D.n_tabs ? D.n_tabs - 1 : ti);
    const double* g_tab = D.tabs + (size_t)ti * kTab;

    f += wave;
    if (f >= D.blocks_per_colour) return;   // no later barrier

    // block coordinates: same-colour blocks are every other block per axis
    const int hx = D.nb[0] >> 1, hy = D.nb[1] >> 1;
    const int kx = 2 * (f % hx) + (colour & 1);
    const int ky = 2 * ((f / hx) % hy) + ((colour >> 1) & 1);
    const int kz = 2 * (f / (hx * hy)) + ((colour >> 2) & 1);
    const int Lx = D.L[0], Ly = D.L[1], Lz = D.L[2];

    // origin shift of sweep s (same for every wave of the sweep)
    uint32_t sh[4] = {0u, 0u, s, 8u};
    philox4x32_10(sh, D.key[0], D.key[1]);
    const int ox = (int)(((uint64_t)sh[0] * (uint32_t)Lx) >> 32);
    const int oy = (int)(((uint64_t)sh[1] * (uint32_t)Ly) >> 32);
    // a z-slab keeps its blocks aligned to its boundaries: no z shift
    constexpr bool slab = SLAB;
    const int oz = slab ? 0 : (int)(((uint64_t)sh[2] * (uint32_t)Lz) >> 32);

    const int x0 = block_lo(kx, Lx, D.nb[0]), wx = block_lo(kx + 1, Lx, D.nb[0]) - x0;
    const int y0 = block_lo(ky, Ly, D.nb[1]), wy = block_lo(ky + 1, Ly, D.nb[1]) - y0;
    const int z0 = block_lo(kz, Lz, D.nb[2]), wz = block_lo(kz + 1, Lz, D.nb[2]) - z0;
    // global coordinate of local cell 0
    const int gx0 = wrap_add(x0 + ox, Lx), gy0 = wrap_add(y0 + oy, Ly), gz0 = wrap_add(z0 + oz, Lz);

    uint8_t* lat = s_lat + wave * kWaveLds;
    uint8_t* __restrict__ g = D.species;
    // plane of the lattice array that holds local z plane lz of the block:
    // periodic wrap, or on a slab the plane two further on (the array starts
    // with the two halo planes below the slab)
    auto zplane = [&](int lz) -> int { return slab ? gz0 + lz + 2 : wrap_add(gz0 + lz, Lz); };

    // cell ids (and, on a slab, global cell ids) fit 32 bits and the 24-bit
    // multiplier (the usual case)
    const uint32_t LxLy = (uint32_t)Lx * (uint32_t)Ly;
    const uint64_t zspan = slab ? (uint64_t)Lz + 4 + D.z_off : (uint64_t)Lz;
    const bool narrow = LxLy < (1u << 24) && (uint64_t)LxLy * zspan < (1ull << 32);

    // species bytes -> LDS codes for this lattice's form of the weight rows
    const bool dot_codes = KMAX <= 5 && D.drop_last == kWtabDot;
    auto encode = [&](uint32_t v) -> uint32_t {
        if constexpr (KMAX <= 5) {
            if (dot_codes) return encode4_dot<KMAX>(v);
        }
        return encode4(v, F);
    };
    // The same map as a byte table for v_perm_b32, code_hi:code_lo = codes
    // of species 7..0 (species >= KMAX never occur: table byte 0).
    uint32_t code_lo = 0u, code_hi = 0u;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const uint32_t c = v < KMAX ? encode((uint32_t)v) & 0xffu : 0u;
        if (v < 4) code_lo |= c << (8 * v);
        else code_hi |= c << (8 * (v - 4));
    }
    // v_perm_b32 reads at most one scalar operand: hold one word in a vector
    // register for the whole staging rather than copying it there per row
    asm volatile("" : "+v"(code_lo));

    // A plane of the lattice (or the slab buffer) and its byte count from
    // there to the end of the buffer: the resource of the plane's rows.
    const uint64_t plane_bytes = 2ull * LxLy;
    const uint64_t buf_bytes = plane_bytes * (uint64_t)(slab ? Lz + 4 : Lz);
    const bool plane32 = plane_bytes < (1ull << 31);   // a row's byte offsets fit 31 bits

    // ---- stage block + halo: local cells -2..w+1 on each axis ----
    // Fast path (the block's x-range does not cross the periodic boundary):
    // 8 lanes per row, each taking cells lx0, lx0 + 1 (lx0 = 2 (lane & 7) - 2),
    // i.e. the bytes corner, body, corner, body at byte `at` of the row; it
    // loads the aligned dwords at `at & ~3` and 4 bytes on and aligns them.
    // Lane row lr = lane >> 3 takes rows ly = lr - 2 + 8 h (h = 0, 1) of each
    // plane lz = -2 .. 13.  Per lane, the in-plane byte offsets and LDS
    // positions of its two rows are set up once; a row adds only its plane,
    // which is wave-uniform (the buffer resource's base, scalar registers).
    // All 16 loads of a batch are issued before any LDS write.  Rows, planes
    // and cells past the halo (w < 12) load an in-range cell and write it to
    // image positions past w + 1, which no trial with a site and no
    // write-back reads; only positions outside the 15^3 arrays (corner -2,
    // body 13) are not written.  Every load stays inside the row's plane.
    if (plane32 && gx0 >= 3 && gx0 + wx + 4 <= Lx) {
        const int c8 = lane & 7, lr = lane >> 3;
        const int lx0 = 2 * c8 - 2;
        const int lxa = lx0 <= wx + 1 ? lx0 : -2;   // cells the lane loads
        uint32_t yoff[2];
        int cl[2];
        bool mc0[2], mc1[2], mb0[2], mb1[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ly = lr - 2 + 8 * h;
            const uint32_t gy = (uint32_t)wrap_add(gy0 + min(ly, wy + 1), Ly);
            yoff[h] = 2u * (gy * (uint32_t)Lx + (uint32_t)(gx0 + lxa));
            cl[h] = (ly + 1) * kP + (lx0 + 1);      // corner(lx0, ly, -1), less a plane
            mc0[h] = ly >= -1 && c8 >= 1;
            mc1[h] = ly >= -1;
            mb0[h] = ly <= 12;
            mb1[h] = ly <= 12 && c8 <= 6;
        }
#pragma unroll
        for (int it0 = 0; it0 < 32; it0 += kStageBatch) {
            uint32_t v[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int it = it0 + u, h = it & 1, lz = (it >> 1) - 2;
                const uint64_t zb = plane_bytes * (uint32_t)zplane(min(lz, wz + 1));
                const uint64_t base = zb & ~(uint64_t)3;
                const __amdgpu_buffer_rsrc_t r = byte_rsrc(g + base, buf_bytes - base);
                const uint32_t at = yoff[h] + ((uint32_t)zb & 2u);
                const uint32_t A = at & ~3u;
                v[u] = __builtin_amdgcn_perm(code_hi, code_lo,
                                             __builtin_amdgcn_alignbyte(bload32(r, A + 4), bload32(r, A), at));
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int it = it0 + u, h = it & 1, lz = (it >> 1) - 2;
                uint8_t* p = lat + cl[h] + (lz + 1) * kPP;   // corner(lx0, ly, lz)
                uint8_t* q = p + (kArr + kPP + kP + 1);      // body(lx0, ly, lz)
                const uint32_t w8 = v[u] >> 8;
                if (lz >= -1) {
                    if (mc0[h]) p[0] = (uint8_t)v[u];
                    if (mc1[h]) p[1] = (uint8_t)(v[u] >> 16);
                }
                if (lz <= 12) {
                    if (mb0[h]) q[0] = (uint8_t)w8;
                    if (mb1[h]) q[1] = (uint8_t)(w8 >> 16);
                }
            }
        }
    } else if (plane32) {
        // The x-range crosses the periodic boundary: the rows and LDS
        // positions of the fast path, but each lane loads its two cells
        // separately, one 16-bit load each at its own wrapped x, so that a
        // pair may straddle the boundary.  The plane's byte remainder
        // (zb & 2) goes into the scalar offset of both loads.
        const int c8 = lane & 7, lr = lane >> 3;
        const int lx0 = 2 * c8 - 2;
        const int lxa = lx0 <= wx + 1 ? lx0 : -2;   // cells the lane loads
        // gx0 + lxa + 1 <= (Lx - 1) + (wx + 2) < 2 Lx, as wx + 2 <= Lx
        const uint32_t gxa = (uint32_t)wrap_add(gx0 + lxa, Lx), gxb = (uint32_t)wrap_add(gx0 + lxa + 1, Lx);
        uint32_t oa[2], ob[2];
        int cl[2];
        bool mc0[2], mc1[2], mb0[2], mb1[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ly = lr - 2 + 8 * h;
            const uint32_t row = (uint32_t)wrap_add(gy0 + min(ly, wy + 1), Ly) * (uint32_t)Lx;
            oa[h] = 2u * (row + gxa);
            ob[h] = 2u * (row + gxb);
            cl[h] = (ly + 1) * kP + (lx0 + 1);
            mc0[h] = ly >= -1 && c8 >= 1;
            mc1[h] = ly >= -1;
            mb0[h] = ly <= 12;
            mb1[h] = ly <= 12 && c8 <= 6;
        }
#pragma unroll
        for (int it0 = 0; it0 < 32; it0 += kStageBatch) {
            uint32_t v[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int it = it0 + u, h = it & 1, lz = (it >> 1) - 2;
                const uint64_t zb = plane_bytes * (uint32_t)zplane(min(lz, wz + 1));
                const uint64_t base = zb & ~(uint64_t)3;
                const __amdgpu_buffer_rsrc_t r = byte_rsrc(g + base, buf_bytes - base);
                const int so = (int)((uint32_t)zb & 2u);
                const uint32_t a = __builtin_amdgcn_raw_buffer_load_b16(r, (int)oa[h], so, 0);
                const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)ob[h], so, 0);
                v[u] = __builtin_amdgcn_perm(code_hi, code_lo, a | b << 16);
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int it = it0 + u, h = it & 1, lz = (it >> 1) - 2;
                uint8_t* p = lat + cl[h] + (lz + 1) * kPP;
                uint8_t* q = p + (kArr + kPP + kP + 1);
                const uint32_t w8 = v[u] >> 8;
                if (lz >= -1) {
                    if (mc0[h]) p[0] = (uint8_t)v[u];
                    if (mc1[h]) p[1] = (uint8_t)(v[u] >> 16);
                }
                if (lz <= 12) {
                    if (mb0[h]) q[0] = (uint8_t)w8;
                    if (mb1[h]) q[1] = (uint8_t)(w8 >> 16);
                }
            }
        }
    } else {
        // planes of 2 GiB or more: one cell (two bytes) per lane, rows
        // r = (lane >> 4) + 4 it, 64-bit addresses; all 64 loads of a lane
        // are issued before any LDS write, as on the fast path (lanes and
        // rows outside the halo load a clamped in-range cell)
        const int lx = (lane & 15) - 2;
        const bool okx = lx <= wx + 1;
        const int gx = wrap_add(gx0 + (okx ? lx : -2), Lx);
#pragma unroll
        for (int it0 = 0; it0 < 64; it0 += 2 * kStageBatch) {
            uint32_t v2[2 * kStageBatch];
#pragma unroll
            for (int u = 0; u < 2 * kStageBatch; ++u) {
                const int it = it0 + u;
                const int ly = min((lane >> 4) + 4 * (it & 3) - 2, wy + 1), lz = min((it >> 2) - 2, wz + 1);
                const int gy = wrap_add(gy0 + ly, Ly);
                const size_t cell = ((size_t)zplane(lz) * Ly + gy) * Lx + gx;
                v2[u] = gload<uint16_t>(g + 2 * cell);
            }
#pragma unroll
            for (int u = 0; u < 2 * kStageBatch; ++u) {
                const int it = it0 + u;
                const int ly = (lane >> 4) + 4 * (it & 3) - 2, lz = (it >> 2) - 2;
                if (!okx || ly > wy + 1 || lz > wz + 1) continue;
                const uint32_t v = encode(v2[u]);
                if (lx >= -1 && ly >= -1 && lz >= -1)
                    lat[(lz + 1) * kPP + (ly + 1) * kP + (lx + 1)] = (uint8_t)v;
                if (lx <= wx && ly <= wy && lz <= wz)
                    lat[kArr + (lz + 2) * kPP + (ly + 2) * kP + (lx + 2)] = (uint8_t)(v >> 8);
            }
        }
    }

    // ---- 27 residue classes x 2 sublattices = 54 rounds ----
    // Lane (ix, iy, iz) takes local cell (rx + 3 ix, ry + 3 iy, rz + 3 iz) of
    // residue class m = (rz*3 + ry)*3 + rx; lanes past the block edge only
    // compute.  Acceptance draws: one Philox call per lane and residue pair
    // (2k, 2k+1), counter (base cell, s, colour + 256 k), the base cell being
    // the lane's cell of class 0; class 2k takes words 0 (corner) and 1
    // (body), class 2k+1 words 2 and 3.  The partner direction of sub-colour
    // q = 2m + b, the same for all blocks of the colour: x step bit q of the
    // Philox call (0, 0, s, 40 + colour), y and z steps bits 2q and 2q+1 of
    // the call (0, 0, s, 32 + colour).
    int ix, iy, iz;
    lane_cell(lane, ix, iy, iz);
    const int lane_c = (3 * iz + 1) * kPP + (3 * iy + 1) * kP + (3 * ix + 1);
    constexpr int kBodyFromCorner = kArr + kPP + kP + 1;
    const uint32_t k0 = D.key[0], k1 = D.key[1];
    uint32_t base_lo, base_hi;
    {
        // a lane that holds a site has gx0 + 3 ix < 2 Lx: one conditional
        // subtraction wraps it (other lanes only feed their draws to no trial)
        uint32_t bx = (uint32_t)(gx0 + 3 * ix), by = (uint32_t)(gy0 + 3 * iy), bz = (uint32_t)(gz0 + 3 * iz);
        bx = min(bx, bx - (uint32_t)Lx);
        by = min(by, by - (uint32_t)Ly);
        bz = slab ? bz + D.z_off : min(bz, bz - (uint32_t)Lz);   // a slab's cells are numbered globally
        const uint64_t cell = narrow ? (uint64_t)(__umul24(bz, LxLy) + __umul24(by, (uint32_t)Lx) + bx)
                                     : ((uint64_t)bz * (uint32_t)Ly + by) * (uint32_t)Lx + bx;
        base_lo = (uint32_t)cell;
        base_hi = (uint32_t)(cell >> 32);
    }
    uint64_t yz_lo, yz_hi, x_bits;   // partner steps, wave-uniform
    {
        uint32_t R[4] = {0u, 0u, s, 32u + (uint32_t)colour};
        philox4x32_10(R, k0, k1);
        // (readfirstlane returns int: widen through uint32_t, not by sign)
        yz_lo = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(R[0]) |
                (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(R[1]) << 32;
        yz_hi = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(R[2]) |
                (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(R[3]) << 32;
        uint32_t X[4] = {0u, 0u, s, 40u + (uint32_t)colour};
        philox4x32_10(X, k0, k1);
        x_bits = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(X[0]) |
                 (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(X[1]) << 32;
    }
    int64_t dEsum = 0;
    uint32_t nacc = 0;
    const float ln2kT = (float)g_tab[kTabLn2kT];
    // The rounds, instantiated for each form of the weight rows (byte-dot or
    // full for KMAX <= 5, folded or full above): the form is per lattice, so
    // each instance stays branch-free.
    auto all_rounds = [&](auto mode_tag) {
        constexpr int MODE = decltype(mode_tag)::value;
        // rounds of residue class m (corner then body) with draws uc, ub, the
        // y/z steps of sub-colours 2m, 2m+1 in b4 (bits 0-1, 2-3) and their x
        // steps in bits 2m, 2m+1 of x_bits
        // Carries (three shells only: they hand on second and third
        // neighbours): corner -> body of every class, and body -> corner of
        // the next class when that is one cell on in x (rx = 1, 2).
        constexpr bool CARRY = SMAX == 3;
        Carry cy;
        auto rounds = [&](int m, uint32_t uc, uint32_t ub, uint32_t b4) {
            const int rx = m % 3, ry = (m / 3) % 3, rz = m / 9;
            const bool valid = (3 * ix < wx - rx) & (3 * iy < wy - ry) & (3 * iz < wz - rz);
            const int ac = lane_c + (rz * kPP + ry * kP + rx);
            const uint32_t xb = (uint32_t)(x_bits >> (2 * m));
            const int e0 = (int)(xb & 1u) | (int)(b4 & 3u) << 1;
            const int e1 = (int)((xb >> 1) & 1u) | (int)((b4 >> 2) & 3u) << 1;
            if (CARRY && rx == 0) {   // wave-uniform: no carry into the first class of an x row
#pragma unroll
                for (int e = 0; e < 8; ++e) cy.s1[e] = lat[ac + s1off<0>(e)];
                cy.own = lat[ac];
            }
            trial<KMAX, SMAX, 0, MODE, CARRY, CARRY>(lat, ac, uc, e0, valid, s_w, g_tab, ln2kT, dEsum, nacc, cy);
            __builtin_amdgcn_wave_barrier();
            trial<KMAX, SMAX, 1, MODE, CARRY, CARRY>(lat, ac + kBodyFromCorner, ub, e1, valid, s_w, g_tab, ln2kT,
                                                     dEsum, nacc, cy);
            __builtin_amdgcn_wave_barrier();
        };
        // One copy of the round code serves all 27 classes (loops that are
        // not unrolled): the code a wave runs per round then stays small
        // enough for the instruction cache, which the CU's waves, each at
        // its own round, share.  The call for the next pair is made ahead
        // of the pair's rounds (for class 26 it is made and not used).
        uint32_t w[4] = {base_lo, base_hi, s, (uint32_t)colour};
        philox4x32_10(w, k0, k1);
#pragma nounroll
        for (int k = 0; k < 14; ++k) {
            uint32_t u0 = w[0], u1 = w[1], u2 = w[2], u3 = w[3];
            w[0] = base_lo; w[1] = base_hi; w[2] = s; w[3] = (uint32_t)colour + 256u * (uint32_t)(k + 1);
            philox4x32_10(w, k0, k1);
            // partner bits of sub-colours 4k .. 4k+3: bits 8k .. 8k+7
            uint32_t bits = (uint32_t)(8 * k < 64 ? yz_lo >> (8 * k) : yz_hi >> (8 * k - 64));
            const int nj = k < 13 ? 2 : 1;
#pragma nounroll
            for (int j = 0; j < nj; ++j) {
                rounds(2 * k + j, u0, u1, bits);
                u0 = u2;
                u1 = u3;
                bits >>= 4;
            }
        }
    };
    if constexpr (KMAX <= 5) {
        if (D.drop_last == kWtabDot)
            all_rounds(std::integral_constant<int, kWtabDot>{});
        else
            all_rounds(std::integral_constant<int, kWtabFull>{});
    } else {
        if (D.drop_last == kWtabDrop)
            all_rounds(std::integral_constant<int, kWtabDrop>{});
        else
            all_rounds(std::integral_constant<int, kWtabFull>{});
    }

    // ---- write back ----
    // A trial changes only corner cells 0..w and body cells -1..w-1 of the
    // block (its sites and their first neighbours).  Row path (planes under
    // 2 GiB): every cell of the box -1..w on each axis is written
    // whole (corner and body byte, one 16-bit store), the cells no trial
    // could change with the value staged from them.  That is the value they
    // still hold: no block of the same colour changes them (same-colour
    // blocks are one block of width >= 2 apart along some axis, and their
    // changes reach one cell beyond their own cells), and the cells of the
    // box are distinct (L >= w + 2 on each axis: at least 2 blocks of width
    // >= 2).  16 lanes per row (lx = (lane & 15) - 1) and 4 rows per
    // instruction: lane row lys = lane >> 4 takes rows ly = 4 yg + lys - 1
    // (yg = 0..3) of each plane lz = -1..w.  Per lane, the in-plane byte
    // offsets and LDS positions of its four rows are set up once; lanes past
    // the box read a clamped in-image cell and store nothing.  A lane's x is
    // wrapped once here, so blocks whose x-range crosses the periodic
    // boundary take this path too (same-colour blocks are as far apart
    // across the boundary as anywhere else, nb being even).
    if (plane32) {
        const int lx = (lane & 15) - 1, lys = lane >> 4;
        const int lxc = min(lx, wx);
        uint32_t yo[4];
        int cw[4];
        bool ok[4];
#pragma unroll
        for (int yg = 0; yg < 4; ++yg) {
            const int ly = 4 * yg + lys - 1, lyc = min(ly, wy);
            ok[yg] = lx <= wx && ly <= wy;
            const uint32_t gy = (uint32_t)wrap_add(gy0 + lyc, Ly);
            yo[yg] = 2u * (gy * (uint32_t)Lx + (uint32_t)wrap_add(gx0 + lxc, Lx));
            cw[yg] = (lyc + 1) * kP + (lxc + 1);   // corner(lxc, lyc, -1), less a plane
        }
#pragma unroll
        for (int lz = -1; lz <= kMaxBlock; ++lz) {
            if (lz > wz) continue;   // (wave-uniform)
            const uint64_t zb = plane_bytes * (uint32_t)zplane(lz);
            const __amdgpu_buffer_rsrc_t r = byte_rsrc(g + zb, buf_bytes - zb);
            uint32_t e[4];
#pragma unroll
            for (int yg = 0; yg < 4; ++yg) {
                const uint8_t* p = lat + cw[yg] + (lz + 1) * kPP;   // corner(lxc, lyc, lz)
                e[yg] = (uint32_t)p[0] | (uint32_t)p[kArr + kPP + kP + 1] << 8;
            }
#pragma unroll
            for (int yg = 0; yg < 4; ++yg)
                if (ok[yg]) bstore16(r, yo[yg], (e[yg] >> 5) & 0x0707u);
        }
    } else {
        // planes of 2 GiB or more: one cell (two bytes) per lane, rows
        // r = (lane >> 4) + 4 it, 64-bit addresses; the LDS reads of 8 rows
        // are issued together (rows and cells outside the boxes read clamped in-image
        // bytes and store nothing)
        const int lx = (lane & 15) - 1;
        const bool okx = lx <= wx;
        const int lxc = okx ? lx : wx;
        const int gx = wrap_add(gx0 + lxc, Lx);
        const int nit = 4 * (wz + 2);               // rows with lz <= wz
        for (int it0 = 0; it0 < nit; it0 += 8) {
            uint32_t vc[8], vb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int it = it0 + u;
                const int lyc = min((lane >> 4) + 4 * (it & 3) - 1, wy), lzc = min((it >> 2) - 1, wz);
                vc[u] = lat[(lzc + 1) * kPP + (lyc + 1) * kP + (lxc + 1)];
                vb[u] = lat[kArr + (lzc + 2) * kPP + (lyc + 2) * kP + (lxc + 2)];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int it = it0 + u;
                const int ly = (lane >> 4) + 4 * (it & 3) - 1, lz = (it >> 2) - 1;
                if (!okx || ly > wy || lz > wz) continue;
                const bool corner = lx >= 0 && ly >= 0 && lz >= 0;
                const bool body = lx < wx && ly < wy && lz < wz;
                if (!corner && !body) continue;
                const int gy = wrap_add(gy0 + ly, Ly);
                const size_t cell = ((size_t)zplane(lz) * Ly + gy) * Lx + gx;
                if (corner && body)
                    gstore<uint16_t>(g + 2 * cell, (uint16_t)(decode(vc[u]) | decode(vb[u]) << 8));
                else if (corner)
                    gstore<uint8_t>(g + 2 * cell, (uint8_t)decode(vc[u]));
                else
                    gstore<uint8_t>(g + 2 * cell + 1, (uint8_t)decode(vb[u]));
            }
        }
    }

    // ---- wavefront reduction of the energy change and accepted count ----
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

int kmax_for(int K)
{
    if (K <= 2) return 2;
    if (K <= 3) return 3;
    if (K <= 4) return 4;
    if (K <= 5) return 5;
    if (K <= 6) return 6;
    return 8;
}

template <int KMAX, int SMAX, bool SLAB, int WPG>
static hipError_t launch_t(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t,
                           int colour, hipStream_t stream)
{
    hipLaunchKernelGGL((sweep_phase_kernel<KMAX, SMAX, SLAB, WPG>), dim3(xcd_grid(n_groups)), dim3(kWave * WPG),
                       0, stream, d_lat, d_items, n_groups, t, colour);
    return hipGetLastError();
}

template <int KMAX, bool SLAB, int WPG>
static hipError_t launch_k(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t,
                           int colour, int smax, hipStream_t stream)
{
    switch (smax) {
    case 1: return launch_t<KMAX, 1, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, stream);
    case 2: return launch_t<KMAX, 2, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, stream);
    case 3: return launch_t<KMAX, 3, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, stream);
    }
    return hipErrorInvalidValue;
}

template <bool SLAB, int WPG>
static hipError_t launch_bcc(const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t, int colour,
                             int kmax, int smax, hipStream_t stream)
{
    switch (kmax) {
    case 2: return launch_k<2, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    case 3: return launch_k<3, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    case 4: return launch_k<4, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    case 5: return launch_k<5, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    case 6: return launch_k<6, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    case 8: return launch_k<8, SLAB, WPG>(d_lat, d_items, n_groups, t, colour, smax, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_phase(int lattice, const DevLattice* d_lat, const WorkItem* d_items, int n_groups, int t,
                              int colour, int kmax, int smax, hipStream_t stream, bool slab, int wpg)
{
    if (n_groups <= 0) return hipSuccess;
    if (lattice == 1)
        return slab ? hipErrorInvalidValue
                    : launch_sweep_phase_fcc(d_lat, d_items, n_groups, t, colour, smax, stream,
                                             wpg ? wpg : kWavesPerGroupFcc);
    if (slab) return wpg && wpg != kWavesPerGroup ? hipErrorInvalidValue
                                                   : launch_bcc<true, kWavesPerGroup>(d_lat, d_items, n_groups, t,
                                                                                     colour, kmax, smax, stream);
    if (wpg && wpg != kWavesPerGroup) return hipErrorInvalidValue;
    return launch_bcc<false, kWavesPerGroup>(d_lat, d_items, n_groups, t, colour, kmax, smax, stream);
}

__global__ void species_max_kernel(const uint8_t* __restrict__ g, size_t n, unsigned int* __restrict__ out)
{
    unsigned int m = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = max(m, (unsigned int)g[i]);
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned int)__shfl_xor(m, o, kWave));
    if ((threadIdx.x % kWave) == 0) atomicMax(out, m);
}

hipError_t launch_species_max(const uint8_t* species, size_t n, unsigned int* d_max, hipStream_t stream)
{
    size_t groups = (n + 255) / 256;
    if (groups > 4096) groups = 4096;
    if (groups == 0) groups = 1;
    hipLaunchKernelGGL(species_max_kernel, dim3((unsigned)groups), dim3(256), 0, stream, species, n, d_max);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Verification hooks: the device's FP64 threshold products and Philox.
__global__ void thresholds_kernel(const double* __restrict__ tab, const int32_t* __restrict__ dE, int n,
                                  double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int e = dE[k] < 1 ? 1 : (dE[k] > (1 << 24) - 1 ? (1 << 24) - 1 : dE[k]);
    out[k] = (tab[512 + (e >> 16)] * tab[256 + ((e >> 8) & 255)]) * tab[e & 255];
}

hipError_t launch_thresholds(const double* d_tab, const int32_t* d_dE, int n, double* d_out, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(thresholds_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, d_tab, d_dE, n, d_out);
    return hipGetLastError();
}

__global__ void accept_bounds_kernel(const double* __restrict__ tab, const uint32_t* __restrict__ u, int n,
                                     int32_t* __restrict__ lo, int32_t* __restrict__ hi)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int a, b;
    accept_bounds(u[k], (float)tab[kTabLn2kT], a, b);
    lo[k] = a;
    hi[k] = b;
}

hipError_t launch_accept_bounds(const double* d_tab, const uint32_t* d_u, int n, int32_t* d_lo, int32_t* d_hi,
                                hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(accept_bounds_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, d_tab, d_u, n, d_lo, d_hi);
    return hipGetLastError();
}

// Exhaustive check of the acceptance bounds over every 32-bit draw u (the
// acceptance draws of both lattices).  For each u the
// kernel forms the edges as the sweep kernels do; the largest dE they accept
// without the table is lo = floor(elo) and the smallest they reject without
// it is hi + 1, hi = floor(ehi).  It evaluates the exact test of Eq. (3) on
// the FP64 table products at dE = lo, lo - 1 (must accept) and hi + 1,
// hi + 2 (must reject), for those dE in (0, 2^24).
// out[0] counts draws violating the lower bound, out[1] the upper bound,
// out[2] holds the largest |(32 - log2 float(u)) - (32 - log2 u)| as the
// bits of a non-negative double (u > 0), out[3] the widest band hi - lo.
__global__ __launch_bounds__(256) void accept_bounds_check_kernel(const double* __restrict__ tab,
                                                                  unsigned long long* __restrict__ out)
{
    const float c = (float)tab[kTabLn2kT];
    unsigned long long bad_lo = 0, bad_hi = 0;
    double max_err = 0.0;
    int max_band = 0;
    auto thr = [&](int e) {
        return (tab[512 + (e >> 16)] * tab[256 + ((e >> 8) & 255)]) * tab[e & 255];
    };
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < (1ull << 32); v += stride) {
        const uint32_t u = (uint32_t)v;
        float elo, ehi;
        accept_edges(u, c, elo, ehi);
        const int lo = (int)fminf(floorf(elo), 1.0e9f), hi = (int)fminf(floorf(ehi), 1.0e9f);
        max_band = max(max_band, hi - lo);
        if (u == 0u) continue;   // the kernels always consult the table for u = 0
        const double du = (double)u;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int a = lo - k, b = hi + 1 + k;
            if (a > 0 && a < (1 << 24) && !(du < thr(a))) ++bad_lo;
            if (b > 0 && b < (1 << 24) && (du < thr(b))) ++bad_hi;
        }
        const double l = (double)(32.0f - __builtin_amdgcn_logf((float)u));
        max_err = fmax(max_err, fabs(l - (32.0 - log2(du))));
    }
    for (int o = 32; o >= 1; o >>= 1) {
        bad_lo += __shfl_xor(bad_lo, o, kWave);
        bad_hi += __shfl_xor(bad_hi, o, kWave);
        max_err = fmax(max_err, __shfl_xor(max_err, o, kWave));
        max_band = max(max_band, __shfl_xor(max_band, o, kWave));
    }
    if ((threadIdx.x % kWave) == 0) {
        if (bad_lo) atomicAdd(&out[0], bad_lo);
        if (bad_hi) atomicAdd(&out[1], bad_hi);
        atomicMax(&out[2], (unsigned long long)__double_as_longlong(max_err));
        atomicMax(&out[3], (unsigned long long)max_band);
    }
}

hipError_t launch_accept_bounds_check(const double* d_tab, unsigned long long* d_out, hipStream_t stream)
{
    hipLaunchKernelGGL(accept_bounds_check_kernel, dim3(8192), dim3(256), 0, stream, d_tab, d_out);
    return hipGetLastError();
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1, int n,
                              uint32_t* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t c[4] = {ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3]};
    philox4x32_10(c, k0, k1);
    for (int w = 0; w < 4; ++w) out[4 * k + w] = c[w];
}

hipError_t launch_philox(const uint32_t* d_ctr, uint32_t k0, uint32_t k1, int n, uint32_t* d_out,
                         hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, d_ctr, k0, k1, n, d_out);
    return hipGetLastError();
}

}  // namespace smcx
