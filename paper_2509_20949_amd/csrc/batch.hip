// batch.hip -- many independent lattices advanced together (temperature
// parallelism, paper Section "Distributed SMC-X"), and replica exchange
// between them (equations for P_swap and Delta).
//
// Every replica keeps its own lattice, seed, sweep counter, tables and
// running energy; a phase launch covers the same-colour blocks of every
// replica still running, four blocks of one replica per workgroup.  Which
// workgroup runs which block never enters the arithmetic, so a replica's
// trajectory is exactly that of a single context with the same inputs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "ctx.h"

using namespace smcx;

struct smcx_batch {
    int n = 0;
    int kmax = 2, smax = 1, lattice = 0;
    hipStream_t stream = nullptr;
    uint8_t* d_species = nullptr;               // all lattices, 256-byte aligned slices
    DevLattice* d_lats = nullptr;
    std::vector<DevLattice> h_lats;
    int64_t* d_states = nullptr;                // [n][kStateWords]: running energy, accepted (slots)
    double* d_tabs = nullptr;                   // [n][768]
    int32_t* d_wtabs = nullptr;                 // [n][kmax*kmax*wrow]
    unsigned long long* d_counts = nullptr;     // pair-count scratch shared by the views
    std::vector<double> T;
    std::vector<int32_t> groups;                // workgroups per replica and phase
    std::vector<int32_t> first_static;          // offset of replica r in d_items_static
    WorkItem* d_items_static = nullptr;         // replica order (per-instance launches)
    WorkItem* d_items_run = nullptr;            // running order of the last batched run
    size_t items_total = 0;
    std::vector<smcx_ctx*> views;
    hipGraphExec_t graph = nullptr;
    std::vector<int32_t> graph_key;
    std::string err;
};

namespace {

smcx_status bfail(smcx_batch* b, smcx_status st, const std::string& msg)
{
    if (b) b->err = msg;
    return fail_global(st, "%s", msg.c_str());
}

smcx_status bhip(smcx_batch* b, hipError_t e, const char* what)
{
    if (e == hipSuccess) return SMCX_OK;
    return bfail(b, e == hipErrorOutOfMemory ? SMCX_E_NOMEM : SMCX_E_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void batch_free(smcx_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (smcx_ctx* v : b->views) delete v;
    b->views.clear();
    void* ptrs[] = {b->d_species, b->d_lats, b->d_states, b->d_tabs, b->d_wtabs, b->d_counts, b->d_items_static,
                    b->d_items_run};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

smcx_status upload_table(smcx_batch* b, int r)
{
    double tab[kTab];
    build_thresholds(b->T[r], tab);
    return bhip(b, hipMemcpy(b->d_tabs + (size_t)r * kTab, tab, sizeof(tab), hipMemcpyHostToDevice),
                "hipMemcpy(table)");
}

}  // namespace

extern "C" {

smcx_status smcx_batch_create(int32_t n, const smcx_desc* descs, const uint8_t* const* species,
                              const int32_t* const* epi, const double* T, smcx_batch** out)
{
    if (!out) return fail_global(SMCX_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || !descs || !species || !epi || !T) return fail_global(SMCX_E_INVALID, "bad batch arguments");
    std::vector<int32_t> B(3 * (size_t)n);
    int kmax = 2, smax = 1;
    for (int r = 0; r < n; ++r) {
        smcx_status st = validate_desc(&descs[r], &B[3 * (size_t)r], true);
        if (!st) st = validate_epi(epi[r], descs[r].n_species, descs[r].n_shells);
        if (!st) st = validate_T(T[r]);
        if (!st && !species[r]) st = fail_global(SMCX_E_INVALID, "species is NULL");
        if (st) return fail_global(st, "replica %d: %s", r, smcx_global_error());
        const size_t N = n_sites(descs[r].lattice, descs[r].L);
        for (size_t i = 0; i < N; ++i)
            if (species[r][i] >= descs[r].n_species)
                return fail_global(SMCX_E_INVALID, "replica %d: species[%zu] >= K", r, i);
        if (descs[r].lattice != descs[0].lattice)
            return fail_global(SMCX_E_INVALID, "replica %d: all replicas of a batch share one lattice type", r);
        kmax = std::max(kmax, kmax_for(descs[r].lattice, descs[r].n_species));
        smax = std::max(smax, (int)descs[r].n_shells);
    }
    smcx_batch* b = new (std::nothrow) smcx_batch();
    if (!b) return fail_global(SMCX_E_NOMEM, "host allocation failed");
    b->n = n;
    b->lattice = descs[0].lattice;
    b->kmax = kmax;
    b->smax = smax;
    b->T.assign(T, T + n);
    b->h_lats.assign(n, DevLattice{});
    const int wr = wrow(kmax, smax);
    const size_t wsize = (size_t)kmax * kmax * wr;
    std::vector<size_t> off(n);
    size_t total = 0;
    for (int r = 0; r < n; ++r) {
        off[r] = total;
        total += align256(n_sites(descs[r].lattice, descs[r].L));
    }
    smcx_status st = bhip(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = bhip(b, hipMalloc(&b->d_species, total), "hipMalloc(lattices)");
    if (!st) st = bhip(b, hipMalloc(&b->d_lats, sizeof(DevLattice) * n), "hipMalloc(descriptors)");
    if (!st) st = bhip(b, hipMalloc(&b->d_states, sizeof(int64_t) * kStateWords * n), "hipMalloc(states)");
    if (!st) st = bhip(b, hipMalloc(&b->d_tabs, sizeof(double) * kTab * n), "hipMalloc(tables)");
    if (!st) st = bhip(b, hipMalloc(&b->d_wtabs, sizeof(int32_t) * wsize * n), "hipMalloc(weights)");
    if (!st) st = bhip(b, hipMalloc(&b->d_counts, kCountBytes), "hipMalloc");
    if (st) { batch_free(b); delete b; return st; }

    std::vector<int32_t> w(wsize);
    std::vector<WorkItem> items;
    b->groups.resize(n);
    b->first_static.resize(n);
    for (int r = 0; r < n && !st; ++r) {
        const smcx_desc& d = descs[r];
        const size_t N = n_sites(d.lattice, d.L);
        st = bhip(b, hipMemcpy(b->d_species + off[r], species[r], N, hipMemcpyHostToDevice), "hipMemcpy(lattice)");
        if (st) break;
        const int drop = build_wtab(epi[r], d.n_species, d.n_shells, kmax, smax, wtab_bias(d.lattice, kmax),
                                    true, w.data());
        st = bhip(b, hipMemcpy(b->d_wtabs + wsize * r, w.data(), sizeof(int32_t) * wsize, hipMemcpyHostToDevice),
                  "hipMemcpy(weights)");
        if (!st) st = upload_table(b, r);
        if (st) break;
        DevLattice& L = b->h_lats[r];
        fill_geometry(L, &d, &B[3 * (size_t)r]);
        if (!geometry_ok(L)) { st = bfail(b, SMCX_E_UNSUPPORTED, "block geometry"); break; }
        L.species = b->d_species + off[r];
        L.tabs = b->d_tabs + (size_t)r * kTab;
        L.wtab = b->d_wtabs + wsize * r;
        L.drop_last = drop;
        L.state = b->d_states + (size_t)kStateWords * r;
        L.sweep0 = 0;
        L.tab_s0 = 0;
        L.n_tabs = 1;
        const int wpg = waves_per_group(L.lattice);
        b->groups[r] = (L.blocks_per_colour + wpg - 1) / wpg;
        b->first_static[r] = (int32_t)items.size();
        for (int g = 0; g < b->groups[r]; ++g) items.push_back(WorkItem{r, g * wpg});

        smcx_ctx* v = new (std::nothrow) smcx_ctx();
        if (!v) { st = bfail(b, SMCX_E_NOMEM, "host allocation failed"); break; }
        b->views.push_back(v);
        v->view = true;
        v->desc = d;
        for (int a = 0; a < 3; ++a) v->B[a] = B[3 * (size_t)r + a];
        v->K = d.n_species;
        v->S = d.n_shells;
        v->N = N;
        v->kmax = kmax;
        v->smax = smax;
        v->epi.assign(epi[r], epi[r] + (size_t)d.n_shells * d.n_species * d.n_species);
        v->d_species = L.species;
        v->d_own = L.species;
        v->stream = b->stream;
        v->h_lat = L;
        v->d_lat = b->d_lats + r;
        v->d_state = b->d_states + (size_t)kStateWords * r;
        v->d_counts = b->d_counts;
        v->d_wtab = nullptr;   // owned by the batch
        v->T_default = T[r];
    }
    if (!st) st = bhip(b, hipMemcpy(b->d_lats, b->h_lats.data(), sizeof(DevLattice) * n, hipMemcpyHostToDevice),
                       "hipMemcpy(descriptors)");
    b->items_total = items.size();
    if (!st) st = bhip(b, hipMalloc(&b->d_items_static, sizeof(WorkItem) * std::max<size_t>(1, items.size())),
                       "hipMalloc(items)");
    if (!st) st = bhip(b, hipMalloc(&b->d_items_run, sizeof(WorkItem) * std::max<size_t>(1, items.size())),
                       "hipMalloc(items)");
    if (!st && !items.empty())
        st = bhip(b, hipMemcpy(b->d_items_static, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice),
                  "hipMemcpy(items)");
    // initial energies
    for (int r = 0; r < n && !st; ++r) {
        int64_t E0 = 0;
        st = recompute_energy(b->views[r], &E0);
        if (st) { b->err = b->views[r]->err; break; }
        st = write_state(b->views[r], E0, 0);
        if (st) { b->err = b->views[r]->err; break; }
    }
    if (st) { batch_free(b); delete b; return st; }
    *out = b;
    return SMCX_OK;
}

static smcx_status check_run_args(smcx_batch* b, const int32_t* n_sweeps)
{
    if (!b || !n_sweeps) return bfail(b, SMCX_E_INVALID, "NULL argument");
    for (int r = 0; r < b->n; ++r) {
        if (n_sweeps[r] < 0) return bfail(b, SMCX_E_INVALID, "negative sweep count");
        if (b->views[r]->sweeps + (uint64_t)n_sweeps[r] > 0xffffffffull)
            return bfail(b, SMCX_E_RANGE, "sweep counter would pass 2^32");
    }
    smcx_status st = bhip(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (st) return st;
    for (int r = 0; r < b->n; ++r) b->h_lats[r].sweep0 = (uint32_t)b->views[r]->sweeps;
    return bhip(b, hipMemcpy(b->d_lats, b->h_lats.data(), sizeof(DevLattice) * b->n, hipMemcpyHostToDevice),
                "hipMemcpy(descriptors)");
}

static void finish_run(smcx_batch* b, const int32_t* n_sweeps)
{
    for (int r = 0; r < b->n; ++r) {
        b->views[r]->sweeps += (uint64_t)n_sweeps[r];
        b->views[r]->attempted += (uint64_t)n_sweeps[r] * b->views[r]->N;
    }
}

smcx_status smcx_batch_run(smcx_batch* b, const int32_t* n_sweeps)
{
    smcx_status st = check_run_args(b, n_sweeps);
    if (st) return st;
    // running order: longest runs first, so the replicas still running at
    // step t are a prefix of the work list
    std::vector<int32_t> order(b->n);
    for (int r = 0; r < b->n; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return n_sweeps[x] > n_sweeps[y]; });
    int tmax = b->n ? n_sweeps[order[0]] : 0;
    if (tmax == 0) return SMCX_OK;
    std::vector<int32_t> key(n_sweeps, n_sweeps + b->n);
    if (!b->graph || key != b->graph_key) {
        std::vector<WorkItem> items;
        std::vector<int32_t> prefix_end(b->n);   // items of order[0..k]
        for (int k = 0; k < b->n; ++k) {
            const int r = order[k];
            const int wpg = waves_per_group(b->h_lats[r].lattice);
            for (int g = 0; g < b->groups[r]; ++g) items.push_back(WorkItem{r, g * wpg});
            prefix_end[k] = (int32_t)items.size();
        }
        if (!items.empty()) {
            st = bhip(b, hipMemcpy(b->d_items_run, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice),
                      "hipMemcpy(items)");
            if (st) return st;
        }
        if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
        b->graph_key.clear();
        st = bhip(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (st) return st;
        hipError_t le = hipSuccess;
        int active = b->n;
        for (int t = 0; t < tmax && le == hipSuccess; ++t) {
            while (active > 0 && n_sweeps[order[active - 1]] <= t) --active;
            const int n_groups = prefix_end[active - 1];
            for (int c = 0; c < 8 && le == hipSuccess; ++c)
                le = launch_sweep_phase(b->lattice, b->d_lats, b->d_items_run, n_groups, t, c, b->kmax, b->smax,
                                        b->stream);
        }
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(b->stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bhip(b, le != hipSuccess ? le : ce, "graph capture");
        }
        hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) { b->graph = nullptr; return bhip(b, ie, "hipGraphInstantiate"); }
        b->graph_key = key;
    }
    st = bhip(b, hipGraphLaunch(b->graph, b->stream), "hipGraphLaunch");
    if (st) return st;
    finish_run(b, n_sweeps);
    return SMCX_OK;
}

smcx_status smcx_batch_run_unbatched(smcx_batch* b, const int32_t* n_sweeps)
{
    smcx_status st = check_run_args(b, n_sweeps);
    if (st) return st;
    for (int r = 0; r < b->n; ++r)
        for (int t = 0; t < n_sweeps[r]; ++t)
            for (int c = 0; c < 8; ++c) {
                hipError_t e = launch_sweep_phase(b->lattice, b->d_lats, b->d_items_static + b->first_static[r],
                                                  b->groups[r], t, c, b->kmax, b->smax, b->stream);
                if (e != hipSuccess) return bhip(b, e, "sweep_phase launch");
            }
    finish_run(b, n_sweeps);
    return SMCX_OK;
}

smcx_status smcx_batch_ctx(smcx_batch* b, int32_t r, smcx_ctx** view)
{
    if (!b || !view || r < 0 || r >= b->n) return bfail(b, SMCX_E_INVALID, "bad replica index");
    *view = b->views[r];
    return SMCX_OK;
}

smcx_status smcx_batch_set_temperature(smcx_batch* b, int32_t r, double T)
{
    if (!b || r < 0 || r >= b->n) return bfail(b, SMCX_E_INVALID, "bad replica index");
    smcx_status st = validate_T(T);
    if (st) return bfail(b, st, smcx_global_error());
    st = bhip(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (st) return st;
    b->T[r] = T;
    b->views[r]->T_default = T;
    return upload_table(b, r);
}

// Replica exchange (paper: P_swap = min(1, exp(Delta)),
// Delta = (1/k_B)(1/T_i - 1/T_j)(E_i - E_j)).  Exchanging the temperatures
// of two replicas is the same move as exchanging their configurations.
smcx_status smcx_temperature_ladder(double T0, int32_t n, uint64_t n_atoms, double dT_ref, uint64_t n_ref,
                                    double* out)
{
    if (!out || n < 1 || n_atoms == 0) return fail_global(SMCX_E_INVALID, "ladder needs out, n >= 1, n_atoms >= 1");
    if (!(dT_ref > 0.0) || n_ref == 0) {   // the paper's example: 0.1 K at 10^9 atoms
        dT_ref = 0.1;
        n_ref = 1000000000ull;
    }
    const double dT = dT_ref * std::sqrt((double)n_ref / (double)n_atoms);
    for (int32_t k = 0; k < n; ++k) {
        out[k] = T0 + dT * k;
        smcx_status st = validate_T(out[k]);
        if (st) return fail_global(st, "ladder temperature %d = %g K outside [1, 5000]", k, out[k]);
    }
    return SMCX_OK;
}

smcx_status smcx_batch_exchange(smcx_batch* b, const int32_t* a, const int32_t* bb, int32_t n_pairs, uint64_t seed,
                                uint64_t round, int32_t* accepted)
{
    if (!b || (n_pairs > 0 && (!a || !bb)) || n_pairs < 0) return bfail(b, SMCX_E_INVALID, "bad exchange arguments");
    for (int k = 0; k < n_pairs; ++k) {
        const int x = a[k], y = bb[k];
        if (x < 0 || y < 0 || x >= b->n || y >= b->n || x == y) return bfail(b, SMCX_E_INVALID, "bad replica pair");
        const smcx_ctx *vx = b->views[x], *vy = b->views[y];
        if (std::memcmp(vx->desc.L, vy->desc.L, sizeof(vx->desc.L)) || vx->K != vy->K || vx->S != vy->S ||
            vx->epi != vy->epi)
            return bfail(b, SMCX_E_INVALID, "exchanged replicas must share lattice, species and EPI");
    }
    smcx_status st = bhip(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (st) return st;
    std::vector<int64_t> image((size_t)kStateWords * b->n), states(2 * (size_t)b->n);
    st = bhip(b, hipMemcpy(image.data(), b->d_states, sizeof(int64_t) * image.size(), hipMemcpyDeviceToHost),
              "hipMemcpy(states)");
    if (st) return st;
    for (int r = 0; r < b->n; ++r) {
        uint64_t acc = 0;
        state_sum(image.data() + (size_t)kStateWords * r, &states[2 * (size_t)r], &acc);
    }
    const double kB = 86.17333262;   // micro-eV / K
    for (int k = 0; k < n_pairs; ++k) {
        const int x = a[k], y = bb[k];
        const double Ex = (double)states[2 * (size_t)x], Ey = (double)states[2 * (size_t)y];
        const double delta = (1.0 / kB) * (1.0 / b->T[x] - 1.0 / b->T[y]) * (Ex - Ey);
        uint32_t c[4] = {(uint32_t)k, (uint32_t)round, (uint32_t)(round >> 32), 9u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double p = delta >= 0.0 ? 1.0 : std::exp(delta);
        const int acc = (double)c[0] < std::ldexp(p, 32);
        if (accepted) accepted[k] = acc;
        if (acc) {
            std::swap(b->T[x], b->T[y]);
            b->views[x]->T_default = b->T[x];
            b->views[y]->T_default = b->T[y];
            st = upload_table(b, x);
            if (!st) st = upload_table(b, y);
            if (st) return st;
        }
    }
    return SMCX_OK;
}

smcx_status smcx_batch_synchronize(smcx_batch* b)
{
    if (!b) return fail_global(SMCX_E_INVALID, "batch is NULL");
    return bhip(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
}

void smcx_batch_destroy(smcx_batch* b)
{
    if (!b) return;
    batch_free(b);
    delete b;
}

}  // extern "C"
