// serve.hip -- continuous batching of sweep requests on one GPU.
//
// Requests wait in arrival order until a slot is free and their device
// footprint fits (first fit: a request that fits may pass one that does
// not).  Admitted lattices stay resident in one device arena of the
// server's HBM budget, allocated once when the server is created, so
// admission and retirement never allocate or free device memory.  Every
// step advances every resident request by up to `sweeps_per_step` sweeps
// with one launch per phase covering all of them.
//
// The step is pipelined.  A call waits for the previous call's kernels,
// retires what they finished (results copied to host memory on a second
// stream while this call's kernels run), launches this call's kernels and
// returns without waiting for them; admissions upload their lattice and
// tables and compute their initial pair counts on the second stream, also
// while the kernels run, and join the next step.  Requests that arrive
// while others run therefore join at the next step, and host work overlaps
// device work.
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
    std::vector<uint8_t> species;   // host sources of the asynchronous uploads, kept until retirement
    std::vector<uint8_t> upload;    // table | weight rows | zero pair counts
    std::vector<int64_t> zero_state;
    std::vector<int32_t> epi;
    double T = 0.0;
    int32_t n_sweeps = 0, done = 0, running = 0;   // running: sweeps of the step in flight
    int state = WAITING;
    size_t footprint = 0;
    int kmax = 0, smax = 0, groups = 0, slot = -1;
    size_t off = 0;                 // arena offset: lattice | table | weights | pair counts
    bool placed = false;            // holds an arena range and a slot
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
           align256(sizeof(int32_t) * (size_t)kmax * kmax * wrow(kmax, smax)) + align256(kCountBytes);
}

// First-fit allocator of arena ranges (offsets), free ranges coalesced.
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n) { free_.clear(); free_[0] = n; }
    bool take(size_t n, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void give(size_t off, size_t n)
    {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

}  // namespace

struct smcx_server {
    size_t budget = 0, used = 0;
    int max_slots = 0, sweeps_per_step = 1;
    hipStream_t stream = nullptr;            // sweep kernels
    hipStream_t ustream = nullptr;           // uploads, initial pair counts, result copies
    hipEvent_t step_done = nullptr;          // the kernels of the step in flight
    hipEvent_t uploads_done = nullptr;       // the admissions of the last call
    bool in_flight = false;
    uint8_t* d_arena = nullptr;              // `budget` bytes
    Arena arena;
    DevLattice* d_lats = nullptr;            // one entry per slot
    int64_t* d_states = nullptr;             // [slot][kStateWords]
    WorkItem* d_items = nullptr;
    size_t items_cap = 0;
    std::vector<DevLattice> h_lats;          // sources of the asynchronous descriptor and item copies
    std::vector<WorkItem> h_items;
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
    if (!q->placed) return;
    s->arena.give(q->off, q->footprint);
    s->free_slots.push_back(q->slot);
    s->used -= q->footprint;
    q->slot = -1;
    q->placed = false;
}

// Admission of a request that holds an arena range and a slot: on the
// upload stream, its lattice, table, weight rows, zeroed state slots and
// the pair counts of the initial configuration (read back at retirement:
// E = E0 + sum dE).
smcx_status admit(smcx_server* s, Request* q)
{
    if (q->id == s->fault_id) return sfail(s, SMCX_E_NOMEM, "admission failure forced by SMCX_FAULT_REQUEST");
    const size_t N = n_sites(q->desc.lattice, q->desc.L);
    const size_t off_tab = align256(N);
    const size_t off_w = off_tab + align256(sizeof(double) * kTab);
    const size_t wbytes = sizeof(int32_t) * (size_t)q->kmax * q->kmax * wrow(q->kmax, q->smax);
    const size_t off_c = off_w + align256(wbytes);
    uint8_t* m = s->d_arena + q->off;
    // host image of table | weights | zero counts, and a zero state image
    // (members of the request: the copies from them are asynchronous)
    std::vector<uint8_t>& img = q->upload;
    img.assign(off_c + kCountBytes - off_tab, 0);
    build_thresholds(q->T, (double*)img.data());
    const int drop = build_wtab(q->epi.data(), q->desc.n_species, q->desc.n_shells, q->kmax, q->smax,
                                wtab_bias(q->desc.lattice, q->kmax), true, (int32_t*)(img.data() + (off_w - off_tab)));
    std::vector<int64_t>& zero = q->zero_state;
    zero.assign(kStateWords, 0);
    smcx_status st = shipc(s, hipMemcpyAsync(m, q->species.data(), N, hipMemcpyHostToDevice, s->ustream),
                           "hipMemcpyAsync(lattice)");
    if (!st) st = shipc(s, hipMemcpyAsync(m + off_tab, img.data(), img.size(), hipMemcpyHostToDevice, s->ustream),
                        "hipMemcpyAsync(tables)");
    if (!st) st = shipc(s, hipMemcpyAsync(s->d_states + (size_t)kStateWords * q->slot, zero.data(),
                                          sizeof(int64_t) * kStateWords, hipMemcpyHostToDevice, s->ustream),
                        "hipMemcpyAsync(state)");
    if (st) return st;
    DevLattice& L = q->lat;
    std::memset(&L, 0, sizeof(L));
    fill_geometry(L, &q->desc, q->B);
    L.species = m;
    L.tabs = (const double*)(m + off_tab);
    L.wtab = (const int32_t*)(m + off_w);
    L.drop_last = drop;
    L.state = s->d_states + (size_t)kStateWords * q->slot;
    L.n_tabs = 1;
    const int wpg = waves_per_group(L.lattice);
    q->groups = (L.blocks_per_colour + wpg - 1) / wpg;
    return shipc(s, launch_pair_counts(q->desc.lattice, m, q->desc.L, q->desc.n_species, q->desc.n_shells,
                                       (unsigned long long*)(m + off_c), s->ustream),
                 "pair_counts launch");
}

// Retirement of a request whose sweeps are done (its kernels have
// completed): configuration, state slots and initial pair counts to host
// memory on the upload stream.  Returns after the copies are enqueued; the
// caller synchronises the stream before reading them.
smcx_status retire_copies(smcx_server* s, Request* q, std::vector<int64_t>& st2, std::vector<unsigned long long>& cnt)
{
    const size_t N = n_sites(q->desc.lattice, q->desc.L);
    const size_t off_c = (size_t)((const uint8_t*)q->lat.wtab - s->d_arena - q->off) +
                         align256(sizeof(int32_t) * (size_t)q->kmax * q->kmax * wrow(q->kmax, q->smax));
    q->config.resize(N);
    smcx_status st = shipc(s, hipMemcpyAsync(q->config.data(), q->lat.species, N, hipMemcpyDeviceToHost, s->ustream),
                           "hipMemcpyAsync(config)");
    if (!st) st = shipc(s, hipMemcpyAsync(st2.data(), q->lat.state, sizeof(int64_t) * kStateWords,
                                          hipMemcpyDeviceToHost, s->ustream), "hipMemcpyAsync(state)");
    if (!st) st = shipc(s, hipMemcpyAsync(cnt.data(), s->d_arena + q->off + off_c, kCountBytes,
                                          hipMemcpyDeviceToHost, s->ustream), "hipMemcpyAsync(counts)");
    return st;
}

int64_t energy_from_counts(const Request* q, const unsigned long long* h)
{
    const int K = q->desc.n_species;
    int64_t twice = 0;
    for (int m = 0; m < q->desc.n_shells; ++m)
        for (int p = 0; p < K; ++p)
            for (int r = 0; r < K; ++r) twice += (int64_t)h[(m * kMaxK + p) * kMaxK + r] * q->epi[(m * K + p) * K + r];
    return twice / 2;
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
    s->budget = align256(budget);
    s->max_slots = max_slots;
    s->sweeps_per_step = sweeps_per_step;
    for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->arena.init(s->budget);
    s->h_lats.assign(max_slots, DevLattice{});
    if (const char* f = std::getenv("SMCX_FAULT_REQUEST")) s->fault_id = std::strtoull(f, nullptr, 10);
    smcx_status st = shipc(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = shipc(s, hipStreamCreateWithFlags(&s->ustream, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = shipc(s, hipEventCreateWithFlags(&s->step_done, hipEventDisableTiming), "hipEventCreate");
    if (!st) st = shipc(s, hipEventCreateWithFlags(&s->uploads_done, hipEventDisableTiming), "hipEventCreate");
    if (!st) st = shipc(s, hipMalloc(&s->d_arena, s->budget), "hipMalloc(arena)");
    if (!st) st = shipc(s, hipMalloc(&s->d_lats, sizeof(DevLattice) * max_slots), "hipMalloc(descriptors)");
    if (!st) st = shipc(s, hipMalloc(&s->d_states, sizeof(int64_t) * kStateWords * max_slots), "hipMalloc(states)");
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
    // 1) the previous call's kernels: wait for them and count their sweeps
    smcx_status st = SMCX_OK;
    if (s->in_flight) {
        st = shipc(s, hipEventSynchronize(s->step_done), "hipEventSynchronize");
        if (st) return st;
        s->in_flight = false;
        for (uint64_t id : s->resident) {
            Request* q = s->reqs[id];
            q->done += q->running;
            q->running = 0;
        }
    }
    // 2) the sweeps of this call, launched before any host-side bookkeeping
    std::vector<Request*> run;
    for (uint64_t id : s->resident) {
        Request* q = s->reqs[id];
        if (q->n_sweeps - q->done > 0) run.push_back(q);
    }
    if (!run.empty()) {
        auto steps_of = [&](Request* q) { return std::min(s->sweeps_per_step, q->n_sweeps - q->done); };
        for (Request* q : run) {
            q->lat.sweep0 = (uint32_t)q->done;
            s->h_lats[q->slot] = q->lat;
        }
        std::stable_sort(run.begin(), run.end(), [&](Request* x, Request* y) {
            if (x->desc.lattice != y->desc.lattice) return x->desc.lattice < y->desc.lattice;
            if (x->kmax != y->kmax) return x->kmax < y->kmax;
            if (x->smax != y->smax) return x->smax < y->smax;
            return steps_of(x) > steps_of(y);
        });
        s->h_items.clear();
        struct Group { int lattice, kmax, smax; size_t begin; std::vector<std::pair<int, size_t>> ends; };
        std::vector<Group> groups;
        for (Request* q : run) {
            if (groups.empty() || groups.back().lattice != q->desc.lattice || groups.back().kmax != q->kmax ||
                groups.back().smax != q->smax)
                groups.push_back(Group{q->desc.lattice, q->kmax, q->smax, s->h_items.size(), {}});
            for (int g = 0; g < q->groups; ++g)
                s->h_items.push_back(WorkItem{q->slot, g * waves_per_group(q->desc.lattice)});
            groups.back().ends.push_back({steps_of(q), s->h_items.size()});
        }
        if (s->h_items.size() > s->items_cap) {
            // grows rarely (the work list of a larger mix): the previous
            // kernels are done, so the old list can go
            if (s->d_items) (void)hipFree(s->d_items);
            s->d_items = nullptr;
            s->items_cap = 0;
            st = shipc(s, hipMalloc(&s->d_items, sizeof(WorkItem) * s->h_items.size() * 2), "hipMalloc(items)");
            if (st) return st;
            s->items_cap = s->h_items.size() * 2;
        }
        // the admissions of the previous call must be on the device first
        st = shipc(s, hipStreamWaitEvent(s->stream, s->uploads_done, 0), "hipStreamWaitEvent");
        if (!st) st = shipc(s, hipMemcpyAsync(s->d_lats, s->h_lats.data(), sizeof(DevLattice) * s->max_slots,
                                              hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync(descriptors)");
        if (!st) st = shipc(s, hipMemcpyAsync(s->d_items, s->h_items.data(), sizeof(WorkItem) * s->h_items.size(),
                                              hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync(items)");
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
        st = shipc(s, hipEventRecord(s->step_done, s->stream), "hipEventRecord");
        if (st) return st;
        s->in_flight = true;
        for (Request* q : run) q->running = steps_of(q);
    }
    // 3) retire the requests the previous kernels finished (copies on the
    //    upload stream, while this call's kernels run)
    std::vector<Request*> leaving;
    for (uint64_t id : s->resident) {
        Request* q = s->reqs[id];
        if (q->done >= q->n_sweeps && q->running == 0) leaving.push_back(q);
    }
    if (!leaving.empty()) {
        std::vector<std::vector<int64_t>> sts(leaving.size(), std::vector<int64_t>(kStateWords));
        std::vector<std::vector<unsigned long long>> cnts(leaving.size(),
                                                          std::vector<unsigned long long>((size_t)kCountSlots * kCountWords));
        std::vector<smcx_status> rst(leaving.size());
        for (size_t k = 0; k < leaving.size(); ++k) rst[k] = retire_copies(s, leaving[k], sts[k], cnts[k]);
        st = shipc(s, hipStreamSynchronize(s->ustream), "hipStreamSynchronize");
        if (st) return st;
        for (size_t k = 0; k < leaving.size(); ++k) {
            Request* q = leaving[k];
            if (rst[k]) {
                q->state = FAILED;
                q->err = s->err;
            } else {
                int64_t dE = 0;
                state_sum(sts[k].data(), &dE, &q->accepted);
                unsigned long long counts[kCountWords];
                count_sum(cnts[k].data(), counts);
                q->E = energy_from_counts(q, counts) + dE;
                q->state = FINISHED;
                ++finished_now;
            }
            q->species = std::vector<uint8_t>();
            q->upload = std::vector<uint8_t>();
            q->zero_state = std::vector<int64_t>();
            release_device(s, q);
            s->resident.erase(std::find(s->resident.begin(), s->resident.end(), q->id));
        }
    }
    // 4) admissions, first fit in arrival order: uploads on the upload
    //    stream, joining the next call's step
    bool uploaded = false;
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
        Request* q = s->reqs[*it];
        if ((int)s->resident.size() >= s->max_slots) break;
        size_t off = 0;
        if (!s->arena.take(q->footprint, &off)) { ++it; continue; }
        q->off = off;
        q->slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->used += q->footprint;
        q->placed = true;
        st = admit(s, q);
        if (st) {
            q->err = s->err;
            q->state = FAILED;
            release_device(s, q);
            it = s->waiting.erase(it);
            continue;
        }
        uploaded = true;
        q->state = RESIDENT;
        s->resident.push_back(q->id);
        it = s->waiting.erase(it);
    }
    if (uploaded) {
        st = shipc(s, hipEventRecord(s->uploads_done, s->ustream), "hipEventRecord");
        if (st) return st;
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
    if (s->ustream) (void)hipStreamSynchronize(s->ustream);
    for (auto& kv : s->reqs) delete kv.second;
    void* ptrs[] = {s->d_arena, s->d_lats, s->d_states, s->d_items};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->step_done) (void)hipEventDestroy(s->step_done);
    if (s->uploads_done) (void)hipEventDestroy(s->uploads_done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->ustream) (void)hipStreamDestroy(s->ustream);
    delete s;
}

const char* smcx_server_last_error(const smcx_server* s) { return s ? s->err.c_str() : smcx_global_error(); }

}  // extern "C"
