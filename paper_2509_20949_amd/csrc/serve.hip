// serve.hip -- continuous batching of sweep requests on one GPU.
//
// Requests wait in arrival order until a slot is free and their device
// footprint fits the budget (first fit: a request that fits may pass one
// that does not).  Admitted lattices stay resident.  Every step advances
// every resident request by up to `sweeps_per_step` sweeps with one launch
// per phase covering all of them, then retires the finished ones, copying
// their configuration to host memory and freeing their device memory, so
// requests that arrive while others run join at the next step.
//
// A request is advanced exactly as a single context would advance it (its
// own seed, sweep counter, tables and energy), so its result does not depend
// on what else is resident.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "ctx.h"

using namespace smcx;

namespace {

enum { WAITING = 0, RESIDENT = 1, FINISHED = 2, FAILED = 3 };

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Request {
    uint64_t id = 0;
    smcx_desc desc{};
    int32_t B[3] = {0, 0, 0};
    std::vector<uint8_t> species;
    std::vector<int32_t> epi;
    double T = 0.0;
    int32_t n_sweeps = 0, done = 0;
    int state = WAITING;
    size_t footprint = 0;
    int kmax = 0, smax = 0, groups = 0, slot = -1;
    bool charged = false;       // footprint counted in the server's budget
    uint8_t* d_mem = nullptr;   // lattice | table | weights
    DevLattice lat{};
    int64_t E = 0;
    uint64_t accepted = 0;
    std::vector<uint8_t> config;
    std::string err;
};

size_t footprint_of(const smcx_desc* d)
{
    const int kmax = kmax_for(d->lattice, d->n_species), smax = d->n_shells;
    return align256(n_sites(d->lattice, d->L)) + align256(sizeof(double) * kTab) +
           align256(sizeof(int32_t) * (size_t)kmax * kmax * wrow(kmax, smax));
}

}  // namespace

struct smcx_server {
    size_t budget = 0, used = 0;
    int max_slots = 0, sweeps_per_step = 1;
    hipStream_t stream = nullptr;
    DevLattice* d_lats = nullptr;            // one entry per slot
    int64_t* d_states = nullptr;             // [slot][kStateWords]
    unsigned long long* d_counts = nullptr;
    WorkItem* d_items = nullptr;
    size_t items_cap = 0;
    std::vector<int> free_slots;
    std::map<uint64_t, Request*> reqs;
    std::deque<uint64_t> waiting;
    std::vector<uint64_t> resident;
    uint64_t next_id = 1;
    uint64_t fault_id = 0;                   // host-forced admission failure (tests)
    std::string err;
};

namespace {

smcx_status sfail(smcx_server* s, smcx_status st, const std::string& msg)
{
    if (s) s->err = msg;
    return fail_global(st, "%s", msg.c_str());
}

smcx_status shipc(smcx_server* s, hipError_t e, const char* what)
{
    if (e == hipSuccess) return SMCX_OK;
    return sfail(s, e == hipErrorOutOfMemory ? SMCX_E_NOMEM : SMCX_E_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

void release_device(smcx_server* s, Request* q)
{
    if (q->d_mem) (void)hipFree(q->d_mem);
    q->d_mem = nullptr;
    if (q->slot >= 0) s->free_slots.push_back(q->slot);
    q->slot = -1;
    if (q->charged) s->used -= q->footprint;
    q->charged = false;
}

// Energy of a freshly admitted lattice from its pair counts.
smcx_status initial_energy(smcx_server* s, Request* q, int64_t* E)
{
    smcx_status st = shipc(s, hipMemsetAsync(s->d_counts, 0, sizeof(unsigned long long) * kMaxS * kMaxK * kMaxK, s->stream),
                           "hipMemsetAsync");
    if (!st) st = shipc(s, launch_pair_counts(q->desc.lattice, q->lat.species, q->lat.L, q->desc.n_species,
                                              q->desc.n_shells, s->d_counts, s->stream), "pair_counts launch");
    unsigned long long h[kMaxS * kMaxK * kMaxK];
    if (!st) st = shipc(s, hipMemcpyAsync(h, s->d_counts, sizeof(h), hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    if (!st) st = shipc(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (st) return st;
    const int K = q->desc.n_species;
    int64_t twice = 0;
    for (int m = 0; m < q->desc.n_shells; ++m)
        for (int p = 0; p < K; ++p)
            for (int r = 0; r < K; ++r) twice += (int64_t)h[(m * kMaxK + p) * kMaxK + r] * q->epi[(m * K + p) * K + r];
    *E = twice / 2;
    return SMCX_OK;
}

smcx_status admit(smcx_server* s, Request* q)
{
    if (q->id == s->fault_id) return sfail(s, SMCX_E_NOMEM, "admission failure forced by SMCX_FAULT_REQUEST");
    const size_t N = n_sites(q->desc.lattice, q->desc.L);
    const size_t off_tab = align256(N);
    const size_t off_w = off_tab + align256(sizeof(double) * kTab);
    smcx_status st = shipc(s, hipMalloc(&q->d_mem, q->footprint), "hipMalloc(request)");
    if (st) return st;
    q->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->used += q->footprint;
    q->charged = true;
    double tab[kTab];
    build_thresholds(q->T, tab);
    std::vector<int32_t> w((size_t)q->kmax * q->kmax * wrow(q->kmax, q->smax));
    const int drop = build_wtab(q->epi.data(), q->desc.n_species, q->desc.n_shells, q->kmax, q->smax,
                                wtab_bias(q->desc.lattice, q->kmax), true, w.data());
    st = shipc(s, hipMemcpy(q->d_mem, q->species.data(), N, hipMemcpyHostToDevice), "hipMemcpy(lattice)");
    if (!st) st = shipc(s, hipMemcpy(q->d_mem + off_tab, tab, sizeof(tab), hipMemcpyHostToDevice), "hipMemcpy(table)");
    if (!st) st = shipc(s, hipMemcpy(q->d_mem + off_w, w.data(), sizeof(int32_t) * w.size(), hipMemcpyHostToDevice),
                        "hipMemcpy(weights)");
    if (st) return st;
    DevLattice& L = q->lat;
    std::memset(&L, 0, sizeof(L));
    fill_geometry(L, &q->desc, q->B);
    L.species = q->d_mem;
    L.tabs = (const double*)(q->d_mem + off_tab);
    L.wtab = (const int32_t*)(q->d_mem + off_w);
    L.drop_last = drop;
    L.state = s->d_states + (size_t)kStateWords * q->slot;
    L.n_tabs = 1;
    const int wpg = waves_per_group(L.lattice);
    q->groups = (L.blocks_per_colour + wpg - 1) / wpg;
    int64_t E0 = 0;
    st = initial_energy(s, q, &E0);
    if (st) return st;
    std::vector<int64_t> init(kStateWords);
    state_init(init.data(), E0, 0);
    st = shipc(s, hipMemcpy(s->d_states + (size_t)kStateWords * q->slot, init.data(), sizeof(int64_t) * kStateWords,
                            hipMemcpyHostToDevice), "hipMemcpy(state)");
    if (st) return st;
    q->species.clear();
    q->species.shrink_to_fit();
    return SMCX_OK;
}

}  // namespace

extern "C" {

size_t smcx_server_footprint(const smcx_desc* d)
{
    int32_t B[3];
    if (validate_desc(d, B, true) != SMCX_OK) return 0;
    return footprint_of(d);
}

smcx_status smcx_server_create(size_t budget, int32_t max_slots, int32_t sweeps_per_step, smcx_server** out)
{
    if (!out) return fail_global(SMCX_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || sweeps_per_step < 1 || budget == 0)
        return fail_global(SMCX_E_INVALID, "server needs budget > 0, max_slots >= 1, sweeps_per_step >= 1");
    smcx_server* s = new (std::nothrow) smcx_server();
    if (!s) return fail_global(SMCX_E_NOMEM, "host allocation failed");
    s->budget = budget;
    s->max_slots = max_slots;
    s->sweeps_per_step = sweeps_per_step;
    for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
    if (const char* f = std::getenv("SMCX_FAULT_REQUEST")) s->fault_id = std::strtoull(f, nullptr, 10);
    smcx_status st = shipc(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = shipc(s, hipMalloc(&s->d_lats, sizeof(DevLattice) * max_slots), "hipMalloc(descriptors)");
    if (!st) st = shipc(s, hipMalloc(&s->d_states, sizeof(int64_t) * kStateWords * max_slots), "hipMalloc(states)");
    if (!st) st = shipc(s, hipMalloc(&s->d_counts, sizeof(unsigned long long) * kMaxS * kMaxK * kMaxK), "hipMalloc");
    if (st) {
        smcx_server_destroy(s);
        return st;
    }
    *out = s;
    return SMCX_OK;
}

smcx_status smcx_server_submit(smcx_server* s, const smcx_desc* desc, const uint8_t* species, const int32_t* epi,
                               double T, int32_t n_sweeps, uint64_t* request_id)
{
    if (!s || !request_id) return sfail(s, SMCX_E_INVALID, "NULL argument");
    int32_t B[3];
    smcx_status st = validate_desc(desc, B, true);
    if (!st) st = validate_epi(epi, desc->n_species, desc->n_shells);
    if (!st) st = validate_T(T);
    if (st) return sfail(s, st, smcx_global_error());
    if (!species || n_sweeps < 0) return sfail(s, SMCX_E_INVALID, "species NULL or negative sweep count");
    const size_t N = n_sites(desc->lattice, desc->L);
    for (size_t i = 0; i < N; ++i)
        if (species[i] >= desc->n_species) return sfail(s, SMCX_E_INVALID, "species value >= K");
    Request* q = new (std::nothrow) Request();
    if (!q) return sfail(s, SMCX_E_NOMEM, "host allocation failed");
    q->id = s->next_id++;
    q->desc = *desc;
    std::memcpy(q->B, B, sizeof(B));
    q->species.assign(species, species + N);
    q->epi.assign(epi, epi + (size_t)desc->n_shells * desc->n_species * desc->n_species);
    q->T = T;
    q->n_sweeps = n_sweeps;
    q->kmax = kmax_for(desc->lattice, desc->n_species);
    q->smax = desc->n_shells;
    q->footprint = footprint_of(desc);
    if (q->footprint > s->budget) {
        delete q;
        return sfail(s, SMCX_E_NOMEM, "request footprint exceeds the server budget");
    }
    s->reqs[q->id] = q;
    s->waiting.push_back(q->id);
    *request_id = q->id;
    return SMCX_OK;
}

smcx_status smcx_server_step(smcx_server* s, int32_t* n_resident, int32_t* n_waiting, int32_t* n_finished)
{
    if (!s) return fail_global(SMCX_E_INVALID, "server is NULL");
    int finished_now = 0;
    // 1) admission, first fit in arrival order
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
        Request* q = s->reqs[*it];
        if ((int)s->resident.size() >= s->max_slots) break;
        if (s->used + q->footprint > s->budget) { ++it; continue; }
        smcx_status st = admit(s, q);
        if (st) {
            q->err = s->err;
            q->state = FAILED;
            release_device(s, q);
            it = s->waiting.erase(it);
            continue;
        }
        q->state = RESIDENT;
        s->resident.push_back(q->id);
        it = s->waiting.erase(it);
    }
    // 2) one batched step over the resident requests, grouped by kernel variant
    std::vector<Request*> run;
    for (uint64_t id : s->resident) {
        Request* q = s->reqs[id];
        if (q->n_sweeps - q->done > 0) run.push_back(q);
    }
    if (!run.empty()) {
        std::vector<DevLattice> lats(s->max_slots);
        for (Request* q : run) {
            q->lat.sweep0 = (uint32_t)q->done;
            lats[q->slot] = q->lat;
        }
        smcx_status st = shipc(s, hipMemcpy(s->d_lats, lats.data(), sizeof(DevLattice) * s->max_slots,
                                            hipMemcpyHostToDevice), "hipMemcpy(descriptors)");
        if (st) return st;
        auto steps_of = [&](Request* q) { return std::min(s->sweeps_per_step, q->n_sweeps - q->done); };
        std::stable_sort(run.begin(), run.end(), [&](Request* x, Request* y) {
            if (x->desc.lattice != y->desc.lattice) return x->desc.lattice < y->desc.lattice;
            if (x->kmax != y->kmax) return x->kmax < y->kmax;
            if (x->smax != y->smax) return x->smax < y->smax;
            return steps_of(x) > steps_of(y);
        });
        std::vector<WorkItem> items;
        struct Group { int lattice, kmax, smax; size_t begin; std::vector<std::pair<int, size_t>> ends; };
        std::vector<Group> groups;
        for (Request* q : run) {
            if (groups.empty() || groups.back().lattice != q->desc.lattice || groups.back().kmax != q->kmax ||
                groups.back().smax != q->smax)
                groups.push_back(Group{q->desc.lattice, q->kmax, q->smax, items.size(), {}});
            for (int g = 0; g < q->groups; ++g) items.push_back(WorkItem{q->slot, g * waves_per_group(q->desc.lattice)});
            groups.back().ends.push_back({steps_of(q), items.size()});
        }
        if (items.size() > s->items_cap) {
            if (s->d_items) (void)hipFree(s->d_items);
            s->d_items = nullptr;
            s->items_cap = 0;
            st = shipc(s, hipMalloc(&s->d_items, sizeof(WorkItem) * items.size()), "hipMalloc(items)");
            if (st) return st;
            s->items_cap = items.size();
        }
        st = shipc(s, hipMemcpy(s->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice),
                   "hipMemcpy(items)");
        if (st) return st;
        for (const Group& G : groups) {
            const int tmax = G.ends.front().first;
            for (int t = 0; t < tmax; ++t) {
                // requests with more than t steps this round form a prefix
                size_t end = G.begin;
                for (const auto& e : G.ends)
                    if (e.first > t) end = e.second;
                for (int c = 0; c < 8; ++c) {
                    hipError_t e = launch_sweep_phase(G.lattice, s->d_lats, s->d_items + G.begin, (int)(end - G.begin),
                                                      t, c, G.kmax, G.smax, s->stream);
                    if (e != hipSuccess) return shipc(s, e, "sweep_phase launch");
                }
            }
        }
        st = shipc(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        if (st) return st;
        for (Request* q : run) q->done += steps_of(q);
    }
    // 3) retire finished requests
    for (auto it = s->resident.begin(); it != s->resident.end();) {
        Request* q = s->reqs[*it];
        if (q->done < q->n_sweeps) { ++it; continue; }
        const size_t N = n_sites(q->desc.lattice, q->desc.L);
        q->config.resize(N);
        std::vector<int64_t> st2(kStateWords);
        smcx_status st = shipc(s, hipMemcpy(q->config.data(), q->lat.species, N, hipMemcpyDeviceToHost), "hipMemcpy");
        if (!st) st = shipc(s, hipMemcpy(st2.data(), s->d_states + (size_t)kStateWords * q->slot,
                                         sizeof(int64_t) * kStateWords, hipMemcpyDeviceToHost), "hipMemcpy");
        if (st) {
            q->state = FAILED;
            q->err = s->err;
        } else {
            state_sum(st2.data(), &q->E, &q->accepted);
            q->state = FINISHED;
            ++finished_now;
        }
        release_device(s, q);
        it = s->resident.erase(it);
    }
    if (n_resident) *n_resident = (int32_t)s->resident.size();
    if (n_waiting) *n_waiting = (int32_t)s->waiting.size();
    if (n_finished) *n_finished = finished_now;
    return SMCX_OK;
}

smcx_status smcx_server_poll(smcx_server* s, uint64_t id, int32_t* state)
{
    if (!s || !state) return fail_global(SMCX_E_INVALID, "NULL argument");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, SMCX_E_INVALID, "unknown request id");
    *state = it->second->state;
    return SMCX_OK;
}

smcx_status smcx_server_result(smcx_server* s, uint64_t id, int64_t* E, uint64_t* accepted, uint8_t* config, size_t n)
{
    if (!s) return fail_global(SMCX_E_INVALID, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, SMCX_E_INVALID, "unknown request id");
    Request* q = it->second;
    if (q->state == FAILED) {
        const std::string msg = "request failed: " + q->err;
        s->reqs.erase(it);
        delete q;
        return sfail(s, SMCX_E_STATE, msg);
    }
    if (q->state != FINISHED) return sfail(s, SMCX_E_STATE, "request not finished");
    if (config && n < q->config.size()) return sfail(s, SMCX_E_INVALID, "config buffer too small");
    if (E) *E = q->E;
    if (accepted) *accepted = q->accepted;
    if (config) std::memcpy(config, q->config.data(), q->config.size());
    s->reqs.erase(it);
    delete q;
    return SMCX_OK;
}

void smcx_server_destroy(smcx_server* s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->reqs) {
        if (kv.second->d_mem) (void)hipFree(kv.second->d_mem);
        delete kv.second;
    }
    void* ptrs[] = {s->d_lats, s->d_states, s->d_counts, s->d_items};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char* smcx_server_last_error(const smcx_server* s) { return s ? s->err.c_str() : smcx_global_error(); }

}  // extern "C"
