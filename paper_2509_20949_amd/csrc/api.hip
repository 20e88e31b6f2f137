// api.hip -- C ABI of libsmcx, single-lattice contexts (include/smcx.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "ctx.h"

using namespace smcx;

namespace {
thread_local std::string g_error;
}

namespace smcx {

smcx_status fail_global(smcx_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

smcx_status fail(smcx_ctx* c, smcx_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    g_error = buf;
    return st;
}

smcx_status validate_desc(const smcx_desc* d, int32_t block_out[3], bool for_gpu)
{
    if (!d) return fail_global(SMCX_E_INVALID, "desc is NULL");
    if (d->lattice != SMCX_LATTICE_BCC && d->lattice != SMCX_LATTICE_FCC)
        return fail_global(SMCX_E_INVALID, "lattice = %d is neither BCC (0) nor FCC (1)", d->lattice);
    for (int a = 0; a < 3; ++a) {
        if (d->L[a] < 2) return fail_global(SMCX_E_INVALID, "L[%d] = %d < 2", a, d->L[a]);
        if (for_gpu && d->L[a] < 4)
            return fail_global(SMCX_E_UNSUPPORTED, "L[%d] = %d: the GPU schedule needs >= 4 cells", a, d->L[a]);
        if (d->L[a] > (1 << 28)) return fail_global(SMCX_E_UNSUPPORTED, "L[%d] = %d too large", a, d->L[a]);
        int B = d->block[a] == 0 ? plan_block(d->lattice, d->L[a], d->n_species) : d->block[a];
        if (B < 2) return fail_global(SMCX_E_INVALID, "block[%d] = %d < 2", a, d->block[a]);
        if (B > kMaxBlock) return fail_global(SMCX_E_UNSUPPORTED, "block[%d] = %d > %d", a, B, kMaxBlock);
        block_out[a] = B;
    }
    if (d->n_species < 1 || d->n_species > kMaxK)
        return fail_global(d->n_species < 1 ? SMCX_E_INVALID : SMCX_E_UNSUPPORTED, "n_species = %d outside 1..%d",
                           d->n_species, kMaxK);
    if (d->n_shells < 1 || d->n_shells > kMaxS)
        return fail_global(d->n_shells < 1 ? SMCX_E_INVALID : SMCX_E_UNSUPPORTED, "n_shells = %d outside 1..%d",
                           d->n_shells, kMaxS);
    if (d->lattice == SMCX_LATTICE_FCC && d->n_species > 5)
        return fail_global(SMCX_E_UNSUPPORTED, "FCC lattices support up to 5 species");
    return SMCX_OK;
}

smcx_status validate_epi(const int32_t* epi, int K, int S)
{
    if (!epi) return fail_global(SMCX_E_INVALID, "EPI table is NULL");
    for (int s = 0; s < S; ++s)
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q) {
                const int32_t v = epi[(s * K + p) * K + q];
                if (v != epi[(s * K + q) * K + p])
                    return fail_global(SMCX_E_INVALID, "EPI shell %d not symmetric at (%d, %d)", s + 1, p, q);
                if (v <= -(1 << 22) || v >= (1 << 22))
                    return fail_global(SMCX_E_RANGE, "|EPI| must be < 2^22 micro-eV (shell %d, %d, %d)", s + 1, p, q);
            }
    return SMCX_OK;
}

smcx_status validate_T(double T)
{
    if (!(T >= 1.0 && T <= 5000.0)) return fail_global(SMCX_E_RANGE, "T = %g K outside [1, 5000]", T);
    return SMCX_OK;
}

size_t n_sites(int lattice, const int32_t L[3])
{
    return (size_t)sites_per_cell(lattice) * (size_t)L[0] * L[1] * L[2];
}

// ---- context internals ------------------------------------------------------
smcx_status ctx_hip(smcx_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return SMCX_OK;
    return fail(c, e == hipErrorOutOfMemory ? SMCX_E_NOMEM : SMCX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Fill the geometry part of a DevLattice from a validated desc.
void fill_geometry(DevLattice& L, const smcx_desc* d, const int32_t B[3])
{
    for (int a = 0; a < 3; ++a) {
        L.L[a] = d->L[a];
        L.nb[a] = axis_blocks(d->L[a], B[a]);
    }
    L.key[0] = (uint32_t)d->seed;
    L.key[1] = (uint32_t)(d->seed >> 32);
    L.K = d->n_species;
    L.lattice = d->lattice;
    L.blocks_per_colour = (L.nb[0] / 2) * (L.nb[1] / 2) * (L.nb[2] / 2);
}

bool geometry_ok(const DevLattice& L)
{
    for (int a = 0; a < 3; ++a) {
        if (L.nb[a] < 2 || (L.nb[a] & 1)) return false;
        // every block 2..kMaxBlock cells wide
        for (int k = 0; k < L.nb[a]; ++k) {
            const int64_t w = ((int64_t)(k + 1) * L.L[a]) / L.nb[a] - ((int64_t)k * L.L[a]) / L.nb[a];
            if (w < 2 || w > kMaxBlock) return false;
        }
    }
    return true;
}

smcx_status upload_tables(smcx_ctx* c, const double* T, int n, uint64_t s0)
{
    // The tables are read by enqueued sweeps: wait before replacing them.
    // Two buffers alternate: the new tables go into the one the descriptor
    // does not point at, and the descriptor is repointed only after they are
    // on the device.  A failed call therefore leaves the context sweeping on
    // its previous tables, untouched.
    smcx_status st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    std::vector<double> h((size_t)n * kTab);
    for (int k = 0; k < n; ++k) build_thresholds(T[k], h.data() + (size_t)k * kTab);
    if (n > c->tab_spare_cap) {
        double* buf = nullptr;
        st = ctx_hip(c, hipMalloc(&buf, sizeof(double) * kTab * (size_t)n), "hipMalloc(tables)");
        if (st) return st;
        if (c->d_tabs_spare) (void)hipFree(c->d_tabs_spare);
        c->d_tabs_spare = buf;
        c->tab_spare_cap = n;
    }
    // SMCX_FAULT_TABLES=1 (tests) makes the upload fail here, after the
    // spare buffer has been (re)allocated, as a failed copy would.
    const char* fault = std::getenv("SMCX_FAULT_TABLES");
    if (fault && std::strcmp(fault, "1") == 0)
        return fail(c, SMCX_E_DEVICE, "table upload failure forced by SMCX_FAULT_TABLES");
    st = ctx_hip(c, hipMemcpy(c->d_tabs_spare, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice),
                 "hipMemcpy(tables)");
    if (st) return st;
    DevLattice next = c->h_lat;
    next.tabs = c->d_tabs_spare;
    next.tab_s0 = (uint32_t)s0;
    next.n_tabs = n;
    st = ctx_hip(c, hipMemcpy(c->d_lat, &next, sizeof(DevLattice), hipMemcpyHostToDevice), "hipMemcpy(lattice descriptor)");
    if (st) return st;
    std::swap(c->d_tabs, c->d_tabs_spare);
    std::swap(c->tab_cap, c->tab_spare_cap);
    c->h_lat = next;
    return SMCX_OK;
}

smcx_status read_state(smcx_ctx* c, int64_t* E, uint64_t* accepted)
{
    std::vector<int64_t> h(kStateWords);
    smcx_status st = ctx_hip(c, hipMemcpyAsync(h.data(), c->d_state, sizeof(int64_t) * kStateWords,
                                               hipMemcpyDeviceToHost, c->stream), "hipMemcpyAsync(state)");
    if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    state_sum(h.data(), E, accepted);
    return SMCX_OK;
}

smcx_status write_state(smcx_ctx* c, int64_t E, uint64_t accepted)
{
    std::vector<int64_t> h(kStateWords);
    state_init(h.data(), E, accepted);
    return ctx_hip(c, hipMemcpy(c->d_state, h.data(), sizeof(int64_t) * kStateWords, hipMemcpyHostToDevice),
                   "hipMemcpy(state)");
}

smcx_status recompute_energy(smcx_ctx* c, int64_t* E)
{
    smcx_status st = ctx_hip(c, hipMemsetAsync(c->d_counts, 0, kCountBytes, c->stream), "hipMemsetAsync");
    if (st) return st;
    st = ctx_hip(c, launch_pair_counts(c->h_lat.lattice, c->d_own, c->h_lat.L, c->K, c->S, c->d_counts, c->stream),
                 "pair_counts launch");
    if (st) return st;
    std::vector<unsigned long long> slots((size_t)kCountSlots * kCountWords);
    st = ctx_hip(c, hipMemcpyAsync(slots.data(), c->d_counts, kCountBytes, hipMemcpyDeviceToHost, c->stream),
                 "hipMemcpyAsync");
    if (st) return st;
    st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    unsigned long long h[kCountWords];
    count_sum(slots.data(), h);
    std::memcpy(c->counts, h, sizeof(h));
    int64_t twice = 0;
    for (int s = 0; s < c->S; ++s)
        for (int p = 0; p < c->K; ++p)
            for (int q = 0; q < c->K; ++q)
                twice += (int64_t)h[(s * kMaxK + p) * kMaxK + q] * c->epi[(s * c->K + p) * c->K + q];
    *E = twice / 2;
    return SMCX_OK;
}

static smcx_status ctx_init(smcx_ctx* c, const smcx_desc* d, const int32_t B[3], const int32_t* epi, double T)
{
    c->desc = *d;
    for (int a = 0; a < 3; ++a) c->B[a] = B[a];
    c->K = d->n_species;
    c->S = d->n_shells;
    c->N = n_sites(d->lattice, d->L);
    c->kmax = kmax_for(d->lattice, c->K);
    c->smax = c->S;
    c->epi.assign(epi, epi + (size_t)c->S * c->K * c->K);
    std::memset(&c->h_lat, 0, sizeof(DevLattice));
    fill_geometry(c->h_lat, d, B);
    if (!geometry_ok(c->h_lat)) return fail(c, SMCX_E_UNSUPPORTED, "block geometry outside 2..%d cells", kMaxBlock);

    smcx_status st;
    st = ctx_hip(c, hipMalloc(&c->d_lat, sizeof(DevLattice)), "hipMalloc(descriptor)");
    if (st) return st;
    st = ctx_hip(c, hipMalloc(&c->d_state, sizeof(int64_t) * kStateWords), "hipMalloc(state)");
    if (st) return st;
    st = ctx_hip(c, hipMalloc(&c->d_counts, kCountBytes), "hipMalloc(counts)");
    if (st) return st;
    const int wr = wrow(c->kmax, c->smax);
    std::vector<int32_t> w((size_t)c->kmax * c->kmax * wr);
    const int drop = build_wtab(epi, c->K, c->S, c->kmax, c->smax, wtab_bias(d->lattice, c->kmax), true,
                                w.data());
    st = ctx_hip(c, hipMalloc(&c->d_wtab, sizeof(int32_t) * w.size()), "hipMalloc(weights)");
    if (st) return st;
    st = ctx_hip(c, hipMemcpy(c->d_wtab, w.data(), sizeof(int32_t) * w.size(), hipMemcpyHostToDevice), "hipMemcpy(weights)");
    if (st) return st;
    c->h_lat.wtab = c->d_wtab;
    c->h_lat.drop_last = drop;
    c->h_lat.state = (int64_t*)c->d_state;
    c->h_lat.species = c->d_species;
    if (!c->d_own) c->d_own = c->d_species;
    c->h_lat.sweep0 = 0;   // single lattice: launch step t is the sweep index
    c->h_lat.slab = c->slab ? 1 : 0;
    c->h_lat.z_off = c->z_off;
    c->T_default = T;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 0;
    c->wpg = c->slab ? kWavesPerGroup : plan_waves_per_group(d->lattice, c->h_lat.blocks_per_colour, n_cu);
    st = upload_tables(c, &T, 1, 0);
    if (st) return st;
    int64_t E0 = 0;
    st = recompute_energy(c, &E0);
    if (st) return st;
    return write_state(c, E0, 0);
}

void ctx_release(smcx_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& e : c->events) (void)hipEventDestroy(e);
    c->events.clear();
    if (c->owns_species && c->d_species) (void)hipFree(c->d_species);
    if (c->d_lat) (void)hipFree(c->d_lat);
    if (c->d_state) (void)hipFree(c->d_state);
    if (c->d_counts) (void)hipFree(c->d_counts);
    if (c->d_wtab) (void)hipFree(c->d_wtab);
    if (c->d_tabs) (void)hipFree(c->d_tabs);
    if (c->d_tabs_spare) (void)hipFree(c->d_tabs_spare);
    if (c->owns_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->d_species = nullptr;
    c->d_lat = nullptr;
    c->d_state = nullptr;
    c->d_counts = nullptr;
    c->d_wtab = nullptr;
    c->d_tabs = nullptr;
    c->d_tabs_spare = nullptr;
    c->stream = nullptr;
}

// Temperature of sweep s under the context's schedule.
double temperature_of(const smcx_ctx* c, uint64_t s)
{
    if (c->sched.empty()) return c->T_default;
    if (s < c->sched_s0) return c->sched.front();
    const uint64_t k = s - c->sched_s0;
    return k < c->sched.size() ? c->sched[k] : c->sched.back();
}

// Kernel timing: event pairs are taken from a pool that grows up to
// kEventPairs pairs; when it is full, the elapsed times recorded so far are
// added to the running total (which waits for them) and the pool is reused.
constexpr size_t kEventPairs = 4096;

static smcx_status harvest_events(smcx_ctx* c)
{
    for (size_t k = 0; k < c->ev_used; ++k) {
        float ms = 0.f;
        smcx_status st = ctx_hip(c, hipEventSynchronize(c->events[2 * k + 1]), "hipEventSynchronize");
        if (!st) st = ctx_hip(c, hipEventElapsedTime(&ms, c->events[2 * k], c->events[2 * k + 1]), "hipEventElapsedTime");
        if (st) return st;
        c->ev_total_ms += ms;
        c->ev_launches += 1;
    }
    c->ev_used = 0;
    return SMCX_OK;
}

static smcx_status next_event_pair(smcx_ctx* c, hipEvent_t* e0, hipEvent_t* e1)
{
    if (c->ev_used == kEventPairs) {
        smcx_status st = harvest_events(c);
        if (st) return st;
    }
    while (c->events.size() < 2 * (c->ev_used + 1)) {
        hipEvent_t e;
        smcx_status st = ctx_hip(c, hipEventCreate(&e), "hipEventCreate");
        if (st) return st;
        c->events.push_back(e);
    }
    *e0 = c->events[2 * c->ev_used];
    *e1 = c->events[2 * c->ev_used + 1];
    return SMCX_OK;
}

// One colour phase of sweep s (with kernel timing when enabled).
static smcx_status enqueue_phase(smcx_ctx* c, uint32_t s, int col, int groups)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profiling) {
        smcx_status st = next_event_pair(c, &e0, &e1);
        if (!st) st = ctx_hip(c, hipEventRecord(e0, c->stream), "hipEventRecord");
        if (st) return st;
    }
    hipError_t e = launch_sweep_phase(c->h_lat.lattice, c->d_lat, nullptr, groups, (int)s, col, c->kmax, c->smax,
                                      c->stream, c->slab, c->wpg);
    if (e != hipSuccess) return ctx_hip(c, e, "sweep_phase launch");
    if (c->profiling) {
        smcx_status st = ctx_hip(c, hipEventRecord(e1, c->stream), "hipEventRecord");
        if (st) return st;
        ++c->ev_used;
    }
    return SMCX_OK;
}

// A slab that is the whole z extent of its lattice exchanges halos with
// itself: before a phase its halo planes receive its own wrapped planes;
// after it, the ring plane the phase may have written in a halo goes back
// to the plane it stands for.  Blocks with even z index (the lowest among
// them) run when colour bit 2 is 0 and may write plane -1; blocks with odd
// index (the highest) run otherwise and may write plane Lz.  The two never
// run in one phase, so the plane written back was not changed in place.
// A slab that is the whole lattice exchanges its halo planes with itself
// (plane p of the buffer at b + p P: halos -2, -1 at p = 0, 1, own planes at
// 2 .. Lz+1, halos Lz, Lz+1 at Lz+2, Lz+3).  After a colour phase the one
// halo plane it may have written returns to its owner plane (phase with
// colour bit 2 clear: halo -1 -> plane Lz-1; set: halo Lz -> plane 0);
// before a phase the halos take the current wrapped planes (Lz-2, Lz-1 ->
// halos -2, -1; 0, 1 -> halos Lz, Lz+1).  One kernel does both steps of a
// phase boundary, element by element in that order (the copies touch the
// same offset q of different planes only, so a thread's order is the
// order of the copies).
template <class T>
__global__ void slab_exchange_kernel(T* __restrict__ b, size_t P, size_t Lz, int after, int before)
{
    const size_t n = P;   // elements per plane
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        if (after == 0) b[(Lz + 1) * P + q] = b[P + q];
        else if (after == 1) b[2 * P + q] = b[(Lz + 2) * P + q];
        if (before) {
            b[q] = b[Lz * P + q];
            b[P + q] = b[(Lz + 1) * P + q];
            b[(Lz + 2) * P + q] = b[2 * P + q];
            b[(Lz + 3) * P + q] = b[3 * P + q];
        }
    }
}

// after: -1 (none), or the colour of the phase that just ran; before: the
// next phase follows.
static smcx_status slab_exchange(smcx_ctx* c, int after_col, bool before)
{
    const size_t P = 2 * (size_t)c->h_lat.L[0] * c->h_lat.L[1];   // bytes per plane
    const size_t Lz = (size_t)c->h_lat.L[2];
    uint8_t* b = c->d_species;
    const int after = after_col < 0 ? -1 : ((after_col >> 2) & 1);
    const dim3 block(256);
    if (P % 16 == 0 && (uintptr_t)b % 16 == 0) {
        const size_t n = P / 16;
        const dim3 grid((unsigned)std::min<size_t>((n + 255) / 256, 4096));
        hipLaunchKernelGGL(slab_exchange_kernel<uint4>, grid, block, 0, c->stream, (uint4*)b, n, Lz, after, (int)before);
    } else {
        const dim3 grid((unsigned)std::min<size_t>((P + 255) / 256, 4096));
        hipLaunchKernelGGL(slab_exchange_kernel<uint8_t>, grid, block, 0, c->stream, b, P, Lz, after, (int)before);
    }
    return ctx_hip(c, hipGetLastError(), "slab_exchange_kernel");
}

smcx_status enqueue_sweeps(smcx_ctx* c, int32_t n)
{
    const int groups = (c->h_lat.blocks_per_colour + c->wpg - 1) / c->wpg;
    for (int32_t k = 0; k < n; ++k) {
        const uint32_t s = (uint32_t)(c->sweeps + (uint64_t)k);
        for (int col = 0; col < 8; ++col) {
            smcx_status st = c->slab && k == 0 && col == 0 ? slab_exchange(c, -1, true) : SMCX_OK;
            if (!st) st = enqueue_phase(c, s, col, groups);
            if (!st && c->slab) st = slab_exchange(c, col, !(k == n - 1 && col == 7));
            if (st) return st;
        }
    }
    c->sweeps += (uint64_t)n;
    c->attempted += (uint64_t)n * c->N;
    return SMCX_OK;
}

smcx_status enqueue_phases(smcx_ctx* c, int32_t n)
{
    const int groups = (c->h_lat.blocks_per_colour + c->wpg - 1) / c->wpg;
    for (int32_t k = 0; k < n; ++k) {
        smcx_status st = enqueue_phase(c, (uint32_t)c->sweeps, c->phase, groups);
        if (st) return st;
        if (++c->phase == 8) {
            c->phase = 0;
            c->sweeps += 1;
            c->attempted += c->N;
        }
    }
    return SMCX_OK;
}

}  // namespace smcx

// =============================================================================
extern "C" {

const char* smcx_global_error(void) { return g_error.c_str(); }

const char* smcx_last_error(const smcx_ctx* ctx) { return ctx ? ctx->err.c_str() : g_error.c_str(); }

const char* smcx_status_string(smcx_status s)
{
    switch (s) {
    case SMCX_OK: return "ok";
    case SMCX_E_INVALID: return "invalid argument";
    case SMCX_E_UNSUPPORTED: return "unsupported";
    case SMCX_E_NOMEM: return "out of memory";
    case SMCX_E_DEVICE: return "device error";
    case SMCX_E_RANGE: return "out of range";
    case SMCX_E_STATE: return "invalid state";
    }
    return "unknown status";
}

static smcx_status create_common(const smcx_desc* desc, const uint8_t* species, uint8_t* d_species,
                                 const int32_t* epi, double T, void* stream, smcx_ctx** out, bool slab = false,
                                 uint32_t z_off = 0)
{
    if (!out) return fail_global(SMCX_E_INVALID, "out is NULL");
    *out = nullptr;
    int32_t B[3];
    smcx_status st = validate_desc(desc, B, true);
    if (st) return st;
    st = validate_epi(epi, desc->n_species, desc->n_shells);
    if (st) return st;
    st = validate_T(T);
    if (st) return st;
    const size_t N = n_sites(desc->lattice, desc->L);
    if (species) {
        for (size_t i = 0; i < N; ++i)
            if (species[i] >= desc->n_species)
                return fail_global(SMCX_E_INVALID, "species[%zu] = %d >= K = %d", i, species[i], desc->n_species);
    } else if (!d_species) {
        return fail_global(SMCX_E_INVALID, "species is NULL");
    }
    smcx_ctx* c = new (std::nothrow) smcx_ctx();
    if (!c) return fail_global(SMCX_E_NOMEM, "host allocation failed");
    c->slab = slab;
    c->z_off = z_off;
    // a slab's buffer: 2 halo planes, the slab, 2 halo planes
    const size_t n_buf = slab ? N + 4 * 2 * (size_t)desc->L[0] * desc->L[1] : N;
    if (slab) c->d_own = d_species + 2 * 2 * (size_t)desc->L[0] * desc->L[1];
    if (stream || d_species) {
        c->stream = (hipStream_t)stream;
        c->owns_stream = false;
    } else {
        st = ctx_hip(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
        if (st) { delete c; return st; }
        c->owns_stream = true;
    }
    if (d_species) {
        c->d_species = d_species;
        c->owns_species = false;
    } else {
        st = ctx_hip(c, hipMalloc(&c->d_species, N), "hipMalloc(lattice)");
        if (!st) st = ctx_hip(c, hipMemcpy(c->d_species, species, N, hipMemcpyHostToDevice), "hipMemcpy(lattice)");
        if (st) { ctx_release(c); delete c; return st; }
        c->owns_species = true;
    }
    if (d_species) {
        // validate the borrowed configuration on the device
        unsigned int* d_max = nullptr;
        unsigned int mx = 0;
        st = ctx_hip(c, hipMalloc(&d_max, sizeof(unsigned int)), "hipMalloc");
        if (!st) st = ctx_hip(c, hipMemsetAsync(d_max, 0, sizeof(unsigned int), c->stream), "hipMemsetAsync");
        if (!st) st = ctx_hip(c, launch_species_max(d_species, n_buf, d_max, c->stream), "species_max launch");
        if (!st) st = ctx_hip(c, hipMemcpyAsync(&mx, d_max, sizeof(mx), hipMemcpyDeviceToHost, c->stream), "copy");
        if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        if (d_max) (void)hipFree(d_max);
        if (!st && mx >= (unsigned)desc->n_species)
            st = fail(c, SMCX_E_INVALID, "device species value %u >= K = %d", mx, desc->n_species);
        if (st) { ctx_release(c); delete c; return st; }
    }
    st = ctx_init(c, desc, B, epi, T);
    if (st) {
        g_error = c->err;
        ctx_release(c);
        delete c;
        return st;
    }
    *out = c;
    return SMCX_OK;
}

smcx_status smcx_create(const smcx_desc* desc, const uint8_t* species, const int32_t* epi_ueV, double T_kelvin,
                        smcx_ctx** out)
{
    if (!species) {
        if (out) *out = nullptr;
        return fail_global(SMCX_E_INVALID, "species is NULL");
    }
    return create_common(desc, species, nullptr, epi_ueV, T_kelvin, nullptr, out);
}

smcx_status smcx_create_device(const smcx_desc* desc, uint8_t* d_species, const int32_t* epi_ueV, double T_kelvin,
                               void* hip_stream, smcx_ctx** out)
{
    if (!d_species || ((uintptr_t)d_species & 3u)) {
        if (out) *out = nullptr;
        return fail_global(SMCX_E_INVALID, "d_species is NULL or not 4-byte aligned");
    }
    return create_common(desc, nullptr, d_species, epi_ueV, T_kelvin, hip_stream, out);
}

smcx_status smcx_create_slab(const smcx_desc* desc, uint8_t* d_buffer, uint32_t z_offset, const int32_t* epi_ueV,
                             double T_kelvin, void* hip_stream, smcx_ctx** out)
{
    if (out) *out = nullptr;
    if (!desc) return fail_global(SMCX_E_INVALID, "desc is NULL");
    if (desc->lattice != SMCX_LATTICE_BCC) return fail_global(SMCX_E_UNSUPPORTED, "slabs are BCC only");
    if (!d_buffer || ((uintptr_t)d_buffer & 3u))
        return fail_global(SMCX_E_INVALID, "d_buffer is NULL or not 4-byte aligned");
    return create_common(desc, nullptr, d_buffer, epi_ueV, T_kelvin, hip_stream, out, true, z_offset);
}

smcx_status smcx_slab_phase(smcx_ctx* c, int32_t n)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    if (!c->slab) return fail(c, SMCX_E_STATE, "smcx_slab_phase needs a slab context");
    if (n < 0) return fail(c, SMCX_E_INVALID, "n = %d < 0", n);
    if (c->sweeps + (uint64_t)((c->phase + n + 7) / 8) > 0xffffffffull)
        return fail(c, SMCX_E_RANGE, "sweep counter would pass 2^32");
    return enqueue_phases(c, n);
}

smcx_status smcx_set_temperature(smcx_ctx* c, double T)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    if (c->view) return fail(c, SMCX_E_STATE, "batch views take smcx_batch_set_temperature");
    smcx_status st = validate_T(T);
    if (st) return fail(c, st, "%s", g_error.c_str());
    st = upload_tables(c, &T, 1, c->sweeps);
    if (st) return st;
    c->sched.clear();
    c->T_default = T;
    return SMCX_OK;
}

smcx_status smcx_set_schedule(smcx_ctx* c, const double* T, int32_t n)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    if (c->view) return fail(c, SMCX_E_STATE, "batch views have a fixed temperature");
    if (!T || n < 1) return fail(c, SMCX_E_INVALID, "schedule needs n >= 1 temperatures");
    for (int32_t k = 0; k < n; ++k) {
        smcx_status st = validate_T(T[k]);
        if (st) return fail(c, st, "schedule[%d]: %s", k, g_error.c_str());
    }
    smcx_status st = upload_tables(c, T, n, c->sweeps);
    if (st) return st;
    c->sched.assign(T, T + n);
    c->sched_s0 = c->sweeps;
    c->T_default = T[n - 1];
    return SMCX_OK;
}

smcx_status smcx_sweep(smcx_ctx* c, int32_t n)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    if (c->view) return fail(c, SMCX_E_STATE, "batch views are advanced by smcx_batch_run");
    if (n < 0) return fail(c, SMCX_E_INVALID, "n = %d < 0", n);
    if (c->sweeps + (uint64_t)n > 0xffffffffull) return fail(c, SMCX_E_RANGE, "sweep counter would pass 2^32");
    if (c->phase != 0) return fail(c, SMCX_E_STATE, "a sweep stepped by smcx_slab_phase is unfinished");
    return enqueue_sweeps(c, n);
}

smcx_status smcx_sweep_observed(smcx_ctx* c, int32_t n, int64_t* E, uint64_t* counts)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    if (c->view) return fail(c, SMCX_E_STATE, "batch views are advanced by smcx_batch_run");
    if (n < 0) return fail(c, SMCX_E_INVALID, "n = %d < 0", n);
    if (c->sweeps + (uint64_t)n > 0xffffffffull) return fail(c, SMCX_E_RANGE, "sweep counter would pass 2^32");
    if (c->phase != 0) return fail(c, SMCX_E_STATE, "a sweep stepped by smcx_slab_phase is unfinished");
    if (n == 0) return SMCX_OK;
    // Chunks of up to kChunk sweeps: each sweep's pair counts go to their own
    // copy-slot block of one device buffer (kCountBytes per sweep), read back
    // once per chunk.
    constexpr int32_t kChunk = 256;
    const int32_t chunk = n < kChunk ? n : kChunk;
    unsigned long long* d_buf = nullptr;
    smcx_status st = ctx_hip(c, hipMalloc(&d_buf, kCountBytes * (size_t)chunk), "hipMalloc(observed counts)");
    if (st) return st;
    std::vector<unsigned long long> h((size_t)kCountSlots * kCountWords * chunk);
    const int K = c->K, S = c->S;
    for (int32_t t0 = 0; t0 < n && !st; t0 += chunk) {
        const int32_t m = n - t0 < chunk ? n - t0 : chunk;
        st = ctx_hip(c, hipMemsetAsync(d_buf, 0, kCountBytes * (size_t)m, c->stream), "hipMemsetAsync");
        for (int32_t t = 0; t < m && !st; ++t) {
            st = enqueue_sweeps(c, 1);
            if (!st)
                st = ctx_hip(c, launch_pair_counts(c->h_lat.lattice, c->d_own, c->h_lat.L, K, S,
                                                   d_buf + (size_t)t * kCountSlots * kCountWords, c->stream),
                             "pair_counts launch");
        }
        if (!st)
            st = ctx_hip(c, hipMemcpyAsync(h.data(), d_buf, kCountBytes * (size_t)m, hipMemcpyDeviceToHost, c->stream),
                         "hipMemcpyAsync(observed counts)");
        if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        for (int32_t t = 0; t < m && !st; ++t) {
            unsigned long long sum[kCountWords];
            count_sum(h.data() + (size_t)t * kCountSlots * kCountWords, sum);
            int64_t twice = 0;
            for (int q = 0; q < S; ++q)
                for (int a = 0; a < K; ++a)
                    for (int b = 0; b < K; ++b) {
                        const unsigned long long v = sum[(q * kMaxK + a) * kMaxK + b];
                        twice += (int64_t)v * c->epi[(q * K + a) * K + b];
                        if (counts) counts[(((size_t)(t0 + t) * S + q) * K + a) * K + b] = v;
                    }
            if (E) E[t0 + t] = twice / 2;
            if (t0 + t == n - 1) std::memcpy(c->counts, sum, sizeof(sum));
        }
    }
    (void)hipFree(d_buf);
    return st;
}

smcx_status smcx_energy(smcx_ctx* c, int64_t* E)
{
    if (!c || !E) return fail(c, SMCX_E_INVALID, "NULL argument");
    return read_state(c, E, nullptr);
}

smcx_status smcx_energy_recompute(smcx_ctx* c, int64_t* E)
{
    if (!c || !E) return fail(c, SMCX_E_INVALID, "NULL argument");
    return recompute_energy(c, E);
}

smcx_status smcx_sro(smcx_ctx* c, double* alpha, uint64_t* counts)
{
    if (!c || !alpha) return fail(c, SMCX_E_INVALID, "NULL argument");
    int64_t E;
    smcx_status st = recompute_energy(c, &E);
    if (st) return st;
    const int K = c->K, S = c->S;
    const double N = (double)c->N;
    const int lat = c->h_lat.lattice;
    const int Z[3] = {shell_size(lat, 0), shell_size(lat, 1), shell_size(lat, 2)};
    std::vector<uint64_t> Np(K, 0);
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q) Np[p] += c->counts[(0 * kMaxK + p) * kMaxK + q];
    for (int p = 0; p < K; ++p) Np[p] /= (uint64_t)Z[0];   // every centre has Z_1 first neighbours
    for (int m = 0; m < S; ++m)
        for (int pc = 0; pc < K; ++pc)
            for (int p = 0; p < K; ++p) {
                const uint64_t n = c->counts[(m * kMaxK + pc) * kMaxK + p];
                if (counts) counts[(m * K + pc) * K + p] = n;
                const double P = (double)n / ((double)Z[m] * (double)Np[pc]);
                const double cp = (double)Np[p] / N;
                alpha[(m * K + pc) * K + p] = (Np[p] == 0 || Np[pc] == 0) ? NAN : 1.0 - P / cp;
            }
    return SMCX_OK;
}

smcx_status smcx_get_config(smcx_ctx* c, uint8_t* out, size_t n)
{
    if (!c || !out) return fail(c, SMCX_E_INVALID, "NULL argument");
    if (n < c->N) return fail(c, SMCX_E_INVALID, "buffer of %zu bytes < N = %zu", n, c->N);
    smcx_status st = ctx_hip(c, hipMemcpyAsync(out, c->d_own, c->N, hipMemcpyDeviceToHost, c->stream),
                             "hipMemcpyAsync");
    if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    return st;
}

smcx_status smcx_get_stats(smcx_ctx* c, uint64_t* sweeps, uint64_t* attempted, uint64_t* accepted, int32_t block[3])
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    uint64_t acc = 0;
    smcx_status st = read_state(c, nullptr, &acc);
    if (st) return st;
    if (sweeps) *sweeps = c->sweeps;
    if (attempted) *attempted = c->attempted;
    if (accepted) *accepted = acc;
    if (block)
        for (int a = 0; a < 3; ++a) block[a] = c->B[a];
    return SMCX_OK;
}

smcx_status smcx_set_state(smcx_ctx* c, const uint8_t* species, uint64_t sweep_index)
{
    if (!c || !species) return fail(c, SMCX_E_INVALID, "NULL argument");
    if (c->view) return fail(c, SMCX_E_STATE, "batch views cannot be reset");
    if (sweep_index > 0xffffffffull) return fail(c, SMCX_E_RANGE, "sweep index >= 2^32");
    for (size_t i = 0; i < c->N; ++i)
        if (species[i] >= c->K) return fail(c, SMCX_E_INVALID, "species[%zu] = %d >= K", i, species[i]);
    smcx_status st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (!st) st = ctx_hip(c, hipMemcpy(c->d_own, species, c->N, hipMemcpyHostToDevice), "hipMemcpy");
    if (st) return st;
    c->sweeps = sweep_index;
    c->phase = 0;
    c->attempted = 0;
    int64_t E = 0;
    st = recompute_energy(c, &E);
    if (st) return st;
    return write_state(c, E, 0);
}

smcx_status smcx_synchronize(smcx_ctx* c)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    return ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

smcx_status smcx_profile(smcx_ctx* c, int32_t enable)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    smcx_status st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    c->ev_used = 0;
    c->ev_total_ms = 0.0;
    c->ev_launches = 0;
    c->profiling = enable != 0;
    return SMCX_OK;
}

smcx_status smcx_kernel_time(smcx_ctx* c, double* total_ms, uint64_t* launches)
{
    if (!c) return fail_global(SMCX_E_INVALID, "ctx is NULL");
    smcx_status st = ctx_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (!st) st = harvest_events(c);
    if (st) return st;
    if (total_ms) *total_ms = c->ev_total_ms;
    if (launches) *launches = c->ev_launches;
    return SMCX_OK;
}

void smcx_destroy(smcx_ctx* c)
{
    if (!c || c->view) return;
    ctx_release(c);
    delete c;
}

smcx_status smcx_plan(const smcx_desc* desc, int32_t block[3], int32_t blocks[3])
{
    int32_t B[3];
    smcx_status st = validate_desc(desc, B, true);
    if (st) return st;
    for (int a = 0; a < 3; ++a) {
        if (block) block[a] = B[a];
        if (blocks) blocks[a] = axis_blocks(desc->L[a], B[a]);
    }
    return SMCX_OK;
}

// ---- verification hooks ------------------------------------------------------
smcx_status smcx_threshold_table(double T, double* out)
{
    if (!out) return fail_global(SMCX_E_INVALID, "out is NULL");
    smcx_status st = validate_T(T);
    if (st) return st;
    double tab[kTab];
    build_thresholds(T, tab);
    std::memcpy(out, tab, sizeof(double) * 768);
    return SMCX_OK;
}

smcx_status smcx_weight_rows(int32_t lattice, int32_t K, int32_t S, const int32_t* epi, int32_t* form,
                             int32_t* kmax_out, int32_t* row_len, int32_t* out, size_t n)
{
    if (lattice != 0 && lattice != 1) return fail_global(SMCX_E_INVALID, "lattice must be 0 (BCC) or 1 (FCC)");
    if (K < 1 || K > (lattice == 1 ? 5 : kMaxK)) return fail_global(SMCX_E_INVALID, "K = %d outside the kernels' range", K);
    if (S < 1 || S > kMaxS) return fail_global(SMCX_E_INVALID, "S = %d outside 1..%d", S, kMaxS);
    smcx_status st = validate_epi(epi, K, S);
    if (st) return st;
    const int kmax = kmax_for(lattice, K), wr = wrow(kmax, S);
    const size_t need = (size_t)kmax * kmax * wr;
    if (kmax_out) *kmax_out = kmax;
    if (row_len) *row_len = wr;
    std::vector<int32_t> w(need);
    const int f = build_wtab(epi, K, S, kmax, S, wtab_bias(lattice, kmax), true, w.data());
    if (form) *form = f;
    if (!out) return SMCX_OK;
    if (n < need) return fail_global(SMCX_E_INVALID, "out holds %zu ints < %zu", n, need);
    std::memcpy(out, w.data(), sizeof(int32_t) * need);
    return SMCX_OK;
}

smcx_status smcx_device_thresholds(double T, const int32_t* dE, int32_t n, double* out)
{
    if (!dE || !out || n < 0) return fail_global(SMCX_E_INVALID, "bad argument");
    smcx_status st = validate_T(T);
    if (st) return st;
    if (n == 0) return SMCX_OK;
    double tab[kTab];
    build_thresholds(T, tab);
    double *d_tab = nullptr, *d_out = nullptr;
    int32_t* d_dE = nullptr;
    hipError_t e = hipMalloc(&d_tab, sizeof(tab));
    if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&d_dE, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMemcpy(d_tab, tab, sizeof(tab), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_dE, dE, sizeof(int32_t) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_thresholds(d_tab, d_dE, n, d_out, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d_out, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (d_tab) (void)hipFree(d_tab);
    if (d_out) (void)hipFree(d_out);
    if (d_dE) (void)hipFree(d_dE);
    if (e != hipSuccess) return fail_global(SMCX_E_DEVICE, "device thresholds: %s", hipGetErrorString(e));
    return SMCX_OK;
}

smcx_status smcx_device_accept_bounds(double T, const uint32_t* u, int32_t n, int32_t* lo, int32_t* hi)
{
    if (!u || !lo || !hi || n < 0) return fail_global(SMCX_E_INVALID, "bad argument");
    smcx_status st = validate_T(T);
    if (st) return st;
    if (n == 0) return SMCX_OK;
    double tab[kTab];
    build_thresholds(T, tab);
    double* d_tab = nullptr;
    uint32_t* d_u = nullptr;
    int32_t *d_lo = nullptr, *d_hi = nullptr;
    hipError_t e = hipMalloc(&d_tab, sizeof(tab));
    if (e == hipSuccess) e = hipMalloc(&d_u, sizeof(uint32_t) * n);
    if (e == hipSuccess) e = hipMalloc(&d_lo, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMalloc(&d_hi, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMemcpy(d_tab, tab, sizeof(tab), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_u, u, sizeof(uint32_t) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_accept_bounds(d_tab, d_u, n, d_lo, d_hi, nullptr);
    if (e == hipSuccess) e = hipMemcpy(lo, d_lo, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hi, d_hi, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (d_tab) (void)hipFree(d_tab);
    if (d_u) (void)hipFree(d_u);
    if (d_lo) (void)hipFree(d_lo);
    if (d_hi) (void)hipFree(d_hi);
    if (e != hipSuccess) return fail_global(SMCX_E_DEVICE, "device accept bounds: %s", hipGetErrorString(e));
    return SMCX_OK;
}

smcx_status smcx_device_check_accept_bounds(double T, uint64_t* violations_lo, uint64_t* violations_hi,
                                            double* max_log2_error, int32_t* max_band)
{
    smcx_status st = validate_T(T);
    if (st) return st;
    double tab[kTab];
    build_thresholds(T, tab);
    double* d_tab = nullptr;
    unsigned long long* d_out = nullptr;
    unsigned long long h[4] = {0, 0, 0, 0};
    hipError_t e = hipMalloc(&d_tab, sizeof(tab));
    if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(h));
    if (e == hipSuccess) e = hipMemcpy(d_tab, tab, sizeof(tab), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_out, h, sizeof(h), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_accept_bounds_check(d_tab, d_out, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h, d_out, sizeof(h), hipMemcpyDeviceToHost);
    if (d_tab) (void)hipFree(d_tab);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess) return fail_global(SMCX_E_DEVICE, "accept bounds check: %s", hipGetErrorString(e));
    if (violations_lo) *violations_lo = h[0];
    if (violations_hi) *violations_hi = h[1];
    if (max_log2_error) std::memcpy(max_log2_error, &h[2], sizeof(double));
    if (max_band) *max_band = (int32_t)h[3];
    return SMCX_OK;
}

smcx_status smcx_device_philox(const uint32_t* ctr, const uint32_t key[2], int32_t n, uint32_t* out)
{
    if (!ctr || !key || !out || n < 0) return fail_global(SMCX_E_INVALID, "bad argument");
    if (n == 0) return SMCX_OK;
    uint32_t *d_c = nullptr, *d_o = nullptr;
    hipError_t e = hipMalloc(&d_c, sizeof(uint32_t) * 4 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&d_o, sizeof(uint32_t) * 4 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpy(d_c, ctr, sizeof(uint32_t) * 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_philox(d_c, key[0], key[1], n, d_o, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d_o, sizeof(uint32_t) * 4 * (size_t)n, hipMemcpyDeviceToHost);
    if (d_c) (void)hipFree(d_c);
    if (d_o) (void)hipFree(d_o);
    if (e != hipSuccess) return fail_global(SMCX_E_DEVICE, "device philox: %s", hipGetErrorString(e));
    return SMCX_OK;
}

}  // extern "C"
