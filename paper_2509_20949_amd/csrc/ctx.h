// ctx.h -- library-internal definition of the opaque handles of smcx.h.
#pragma once

#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "smcx_internal.h"

struct smcx_ctx {
    smcx_desc desc{};
    int32_t B[3] = {0, 0, 0};
    int K = 0, S = 0;
    size_t N = 0;
    int kmax = 0, smax = 0;
    std::vector<int32_t> epi;
    uint8_t* d_species = nullptr;
    bool owns_species = false;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    smcx::DevLattice h_lat{};
    smcx::DevLattice* d_lat = nullptr;
    void* d_state = nullptr;                 // int64 running energy, uint64 accepted
    unsigned long long* d_counts = nullptr;  // pair-count scratch [kMaxS][kMaxK][kMaxK]
    int32_t* d_wtab = nullptr;
    double* d_tabs = nullptr;                // tables the descriptor points at
    int tab_cap = 0;
    double* d_tabs_spare = nullptr;          // the other buffer of the pair (upload_tables)
    int tab_spare_cap = 0;
    uint64_t sweeps = 0, attempted = 0;
    double T_default = 0.0;
    std::vector<double> sched;
    uint64_t sched_s0 = 0;
    uint64_t counts[smcx::kMaxS * smcx::kMaxK * smcx::kMaxK] = {};
    bool profiling = false;
    std::vector<hipEvent_t> events;          // pool of (start, end) pairs, reused
    size_t ev_used = 0;                      // pairs recorded since the last harvest
    double ev_total_ms = 0.0;                // harvested kernel time since profiling was enabled
    uint64_t ev_launches = 0;
    bool view = false;                       // replica view owned by a batch
    // z-slab (smcx_create_slab): the caller's buffer holds 2 halo planes, the
    // slab's Lz planes and 2 more halo planes; d_own = its first own plane
    bool slab = false;
    uint32_t z_off = 0;                      // global z of the slab's first own plane
    uint8_t* d_own = nullptr;                // the lattice's own sites (= d_species unless a slab)
    int phase = 0;                           // colour phases of the current sweep already enqueued
    int wpg = 0;                             // blocks per workgroup of the colour launches (plan_waves_per_group)
    std::string err;
};

namespace smcx {
smcx_status fail_global(smcx_status st, const char* fmt, ...);
smcx_status fail(smcx_ctx* c, smcx_status st, const char* fmt, ...);
smcx_status validate_desc(const smcx_desc* d, int32_t block_out[3], bool for_gpu);
smcx_status validate_epi(const int32_t* epi, int K, int S);
smcx_status validate_T(double T);
size_t n_sites(int lattice, const int32_t L[3]);
smcx_status ctx_hip(smcx_ctx* c, hipError_t e, const char* what);
void fill_geometry(DevLattice& L, const smcx_desc* d, const int32_t B[3]);
bool geometry_ok(const DevLattice& L);
smcx_status recompute_energy(smcx_ctx* c, int64_t* E);
// Running energy / accepted count of a context (sums over the state slots).
smcx_status read_state(smcx_ctx* c, int64_t* E, uint64_t* accepted);
smcx_status write_state(smcx_ctx* c, int64_t E, uint64_t accepted);
smcx_status enqueue_sweeps(smcx_ctx* c, int32_t n);
smcx_status enqueue_phases(smcx_ctx* c, int32_t n);
void ctx_release(smcx_ctx* c);
}  // namespace smcx
