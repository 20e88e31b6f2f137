/*
 * smcx.h -- C ABI of libsmcx: canonical-ensemble Metropolis swap sweeps on a
 * multicomponent BCC lattice with an effective-pair-interaction (EPI)
 * energy, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Liu, Yang, Zhou, Xu, "SMC-X: A Distributed Scalable Monte Carlo
 * Simulation Method for Chemically Complex Alloys", arXiv:2509.20949.
 *   - canonical (NVT) target distribution: Section "Monte Carlo
 *     simulation", Eq. (1); observables as ensemble averages, Eq. (2);
 *   - Metropolis acceptance min(1, exp(-beta dE)): Eq. (3);
 *   - one sweep (MC step) = one trial per lattice site: text after Eq. (3);
 *   - link cells visited so that every site is tried once per step and
 *     concurrently updated sites do not interact: Section "Distributed
 *     SMC-X", equation for P_LC;
 *   - EPI model (pair interactions only): Section "Results and discussion";
 *   - Warren-Cowley SRO: Section "Evolution of chemical defects",
 *     Eq. (SRO);
 *   - independent temperatures run side by side (temperature
 *     parallelism) and replica exchange: Section "Distributed SMC-X",
 *     equations for P_swap and Delta.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice.  Cells (x, y, z), 0 <= x < L[0] etc., periodic on every axis,
 *   n_sub sites per cell at offsets (in units of a/2) BCC: b = 0 (0,0,0),
 *   b = 1 (1,1,1); FCC: (0,0,0), (1,1,0), (1,0,1), (0,1,1).  Canonical site
 *   id i = ((z*L[1] + y)*L[0] + x)*n_sub + b.  Species arrays hold one
 *   uint8 per site in canonical order, values 0..K-1.
 * Energy.  E = 1/2 sum_i sum_{delta in shells 1..S} V_s(sigma_i,
 *   sigma_{i+delta}).  BCC shells: 8 at (+-a/2, +-a/2, +-a/2), 6 at
 *   (+-a, 0, 0), 12 at (+-a, +-a, 0); FCC shells: 12 at (+-a/2, +-a/2, 0),
 *   6 at (+-a, 0, 0), 24 at (+-a, +-a/2, +-a/2) (and permutations).  The EPI table
 *   is int32 micro-eV, layout epi[s][p][q] (S*K*K entries), symmetric in
 *   (p, q), |V| < 2^22.  Energies are exact int64 micro-eV.
 * Trial.  Sweep s, colour phase c; key = (seed & 0xffffffff, seed >> 32).
 *   BCC: a site (cell, b) with local cell l in its block and residue class
 *   m = ((l_z%3)*3 + l_y%3)*3 + l_x%3 (sub-colour q = 2m + b) takes the
 *   32-bit word w = word 2*(m & 1) + b of Philox4x32-10(key, (g & 0xffffffff,
 *   g >> 32, s, c + 256*(m >> 1))), g = the cell at local coordinates
 *   3*floor(l/3) of the same block, as its acceptance draw u.  The partner
 *   of every trial of one (sweep, colour, sub-colour q) set is the first
 *   neighbour with +a/2 along x iff bit q of X is set, along y iff bit 2q
 *   and along z iff bit 2q+1 of R is set (-a/2 otherwise), X and R the 128
 *   bits of Philox4x32-10(key, (0, 0, s, 40 + c)) and of
 *   Philox4x32-10(key, (0, 0, s, 32 + c)) (bit t = bit t%32 of word t/32).
 *   FCC: site b of a cell takes u = word b of Philox4x32-10(key, (cell &
 *   0xffffffff, cell >> 32, s, c)) as its acceptance draw.  The partner of
 *   every trial of one (sweep, colour, sub-colour q) set is drawn once from
 *   r = Philox4x32-10(key, (q, 0, s, c + 64)): its sublattice b' = the k-th
 *   sublattice other than b, k = (r0 * 3) >> 32, and bits 30 and 31 of r1
 *   give the signs (+a/2 when set) on the two axes where b and b' differ.
 *   Both lattices accept an uphill swap iff dE < 2^24 and
 *   (double)u < (T2[dE>>16] * T1[(dE>>8)&255]) * T0[dE&255], with
 *   beta = 1 / (86.17333262 * T) per micro-eV and
 *   T0[l] = exp(-l beta), T1[m] = exp(-256 m beta),
 *   T2[h] = 2^32 exp(-65536 h beta), built in FP64 on the host.
 *   dE <= 0 always accepts.  Swaps of equal species are no-ops.
 * Schedule.  Per axis n = max(2, min(2*ceil(L/(2B)), 2*floor(L/4))) blocks
 *   with bounds floor(k L / n); sweep s shifts the block grid by
 *   o_a = (r_a * L_a) >> 32 with r = Philox4x32-10(key, (0, 0, s, 8)).
 *   A site's colour is the parity pattern of its block indices, its
 *   sub-colour (((l_z%3)*3 + l_y%3)*3 + l_x%3)*n_sub + b from its local cell
 *   coordinates; phases run c = 0..7, rounds q = 0..27*n_sub-1.  Trials of one
 *   (c, q) set never interact, nor do blocks of one colour, so the result is
 *   that of the sequential order (c, q, site id) bit for bit.
 *
 * Memory and threads.  Every call that takes host pointers copies what it
 *   needs; the caller keeps ownership.  smcx_create_device borrows a device
 *   buffer that must outlive the context.  smcx_sweep and smcx_batch_run
 *   only enqueue work on the context's HIP stream; every query synchronises
 *   that stream.  One context must not be used from two threads at once;
 *   distinct contexts may.  No C++ exception crosses this interface.
 * Errors.  Every status-returning call returns SMCX_OK or a negative code;
 *   smcx_last_error(ctx) (or smcx_global_error() where no context exists)
 *   returns a message for the last failing call on that thread/context.
 */
#ifndef SMCX_H
#define SMCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smcx_ctx smcx_ctx;
typedef struct smcx_batch smcx_batch;
typedef struct smcx_server smcx_server;

typedef enum {
    SMCX_OK = 0,
    SMCX_E_INVALID = -1,      /* bad pointer, size, species >= K, asymmetric EPI */
    SMCX_E_UNSUPPORTED = -2,  /* valid for the method, not for this library (L < 4, B > 12, K > 8, S > 3,
                                 FCC with K > 5) */
    SMCX_E_NOMEM = -3,        /* device or host allocation failed, or over budget */
    SMCX_E_DEVICE = -4,       /* a HIP runtime call failed */
    SMCX_E_RANGE = -5,        /* |V| >= 2^22, T outside [1, 5000] K, sweep counter overflow */
    SMCX_E_STATE = -6         /* call not valid in the object's current state */
} smcx_status;

enum { SMCX_LATTICE_BCC = 0, SMCX_LATTICE_FCC = 1 };
enum { SMCX_MAX_SPECIES = 8, SMCX_MAX_SHELLS = 3, SMCX_MAX_BLOCK = 12 };

typedef struct {
    int32_t lattice;    /* SMCX_LATTICE_BCC (2 sites per cubic cell) or
                           SMCX_LATTICE_FCC (4 sites per cell, K <= 5) */
    int32_t L[3];       /* cells per axis, each >= 4 */
    int32_t n_species;  /* K, 2..8 */
    int32_t n_shells;   /* S, 1..3 */
    int32_t block[3];   /* schedule block-width parameter B per axis, 2..12;
                           0 lets the library choose (smcx_plan reports the
                           choice).  B changes the schedule, hence the
                           trajectory; the oracle must use the same B. */
    uint64_t seed;      /* Philox key */
} smcx_desc;

/* ---- single lattice ----------------------------------------------------
 * smcx_create: copies N = n_sub*L0*L1*L2 species bytes and the S*K*K EPI table,
 * allocates the lattice on the current HIP device and creates a stream.
 * T is the temperature of every sweep until changed.  The sweep counter
 * starts at 0.  Errors: INVALID, UNSUPPORTED, RANGE, NOMEM, DEVICE. */
smcx_status smcx_create(const smcx_desc* desc, const uint8_t* species, const int32_t* epi_ueV,
                        double T_kelvin, smcx_ctx** out);

/* smcx_create_device: as smcx_create, but the lattice lives in the caller's
 * device buffer d_species (N bytes, canonical order, 4-byte aligned, already
 * holding the configuration; borrowed, updated in place), and work is enqueued on
 * hip_stream (a hipStream_t, or NULL for the null stream).  The species are
 * validated on the device. */
smcx_status smcx_create_device(const smcx_desc* desc, uint8_t* d_species, const int32_t* epi_ueV,
                               double T_kelvin, void* hip_stream, smcx_ctx** out);

/* smcx_plan: the schedule the library runs for desc, computed on the host
 * (no device): block receives the block-width parameter B per axis (the
 * desc's, or the library's choice where the desc gives 0: a fixed function
 * of the lattice type, the axis length and K, so a trajectory is
 * reproducible), blocks the number of blocks per axis of the shifted grid,
 * n = max(2, min(2*ceil(L/(2B)), 2*floor(L/4))).  Both nullable.  Errors as
 * smcx_create's checks of desc. */
smcx_status smcx_plan(const smcx_desc* desc, int32_t block[3], int32_t blocks[3]);

/* ---- one z-slab of a larger lattice (lattice parallelism with ghost
 * layers, Section "Distributed SMC-X") --------------------------------------
 * smcx_create_slab: a BCC context for cells 0..L[2]-1 along z of a slab
 * whose first plane is plane z_offset of the whole lattice (its cells keep
 * their global ids in the random-number counters; L[0], L[1] are the whole
 * lattice's).  d_buffer (borrowed, 4-byte aligned, updated in place) holds
 * L[2] + 4 planes of 2*L[0]*L[1] bytes: planes z_offset-2, z_offset-1 of the
 * lattice (the halo below), the slab's own L[2] planes, then planes
 * z_offset+L[2], z_offset+L[2]+1 (the halo above); all hold valid species.
 * The block grid of a slab is not shifted along z, so its blocks stay
 * aligned to the slab boundaries (x and y shift as usual); with an even
 * number of blocks per slab the global colouring is the one of a single
 * lattice of all slabs stacked.  A phase reads the halo planes and may
 * write the first plane of either halo (the first-neighbour ring of its
 * edge blocks): z-blocks of even index, including the lowest, run when
 * colour bit 2 is 0 and may write plane z_offset-1; odd ones, including the
 * highest, run otherwise and may write plane z_offset+L[2].
 *   smcx_sweep on a slab context treats the slab as the whole lattice,
 * periodic along z: before every phase it copies its own wrapped planes
 * into the halos and afterwards copies a written halo plane back (the
 * exchange with itself).  smcx_slab_phase enqueues the next n colour phases
 * without any exchange: the caller brings the halos up to date between
 * phases (e.g. with the neighbouring slabs' planes) and returns written
 * halo planes to their owners.  Energy queries, smcx_sro and smcx_get_config
 * cover the slab's own planes, taken as periodic along z (exact when the
 * slab is the whole lattice).  Errors: as smcx_create_device; UNSUPPORTED
 * for FCC. */
smcx_status smcx_create_slab(const smcx_desc* desc, uint8_t* d_buffer, uint32_t z_offset, const int32_t* epi_ueV,
                             double T_kelvin, void* hip_stream, smcx_ctx** out);
smcx_status smcx_slab_phase(smcx_ctx* ctx, int32_t n);

/* Temperature of every following sweep (kelvin, 1..5000). */
smcx_status smcx_set_temperature(smcx_ctx* ctx, double T_kelvin);

/* Temperatures of the next n sweeps (an anneal); later sweeps keep the
 * last value.  T_per_sweep is copied. */
smcx_status smcx_set_schedule(smcx_ctx* ctx, const double* T_per_sweep, int32_t n);

/* Enqueue n >= 0 sweeps (Section "Monte Carlo simulation": one trial per
 * site each).  Asynchronous.  RANGE if the sweep counter would pass 2^32. */
smcx_status smcx_sweep(smcx_ctx* ctx, int32_t n);

/* n sweeps as smcx_sweep(n), recording after every sweep t (0-based) the
 * pair counts N_m[p'][p] of the configuration (Eq. (SRO): the numerators of
 * the Warren-Cowley parameters) in counts[((t*S + m)*K + p')*K + p] and its
 * energy, E = 1/2 sum_m sum_{p',p} N_m[p'][p] V_m(p', p) (micro-eV, equal to
 * the running energy), in E_ueV[t].  Either output may be NULL.  The counts
 * stay on the device between sweeps (a device buffer of 24 KiB per sweep,
 * at most 256 sweeps at a time, allocated and freed by the call) and are
 * read back once per 256 sweeps: no host synchronisation per sweep.
 * Returns when all n sweeps are done.  Errors: as smcx_sweep; NOMEM if the
 * buffer cannot be allocated, DEVICE if a HIP call fails (sweeps already
 * enqueued by the call stay done). */
smcx_status smcx_sweep_observed(smcx_ctx* ctx, int32_t n, int64_t* E_ueV, uint64_t* counts);

/* Running energy: the initial energy plus every accepted dE (micro-eV). */
smcx_status smcx_energy(smcx_ctx* ctx, int64_t* E_ueV);

/* Energy recomputed from the current configuration by a full pass. */
smcx_status smcx_energy_recompute(smcx_ctx* ctx, int64_t* E_ueV);

/* Warren-Cowley SRO, Eq. (SRO): alpha[(m*K + p')*K + p] = 1 - P_m^{p|p'}/c_p,
 * p' the centre species; NaN when species p or p' is absent.  counts
 * (nullable) receives the pair counts N_m[p'][p] (S*K*K uint64). */
smcx_status smcx_sro(smcx_ctx* ctx, double* alpha, uint64_t* counts);

/* Copy the configuration (canonical order) into out (n >= N bytes). */
smcx_status smcx_get_config(smcx_ctx* ctx, uint8_t* out, size_t n);

/* Counters: sweeps done, attempted trials (N per sweep), accepted swaps
 * that changed the configuration; block receives the schedule parameter B. */
smcx_status smcx_get_stats(smcx_ctx* ctx, uint64_t* sweeps, uint64_t* attempted,
                           uint64_t* accepted, int32_t block[3]);

/* Resume: replace the configuration (N bytes, copied) and set the sweep
 * counter, recomputing the energy.  With the same seed, B and temperatures
 * the continuation is bit-identical to an uninterrupted run. */
smcx_status smcx_set_state(smcx_ctx* ctx, const uint8_t* species, uint64_t sweep_index);

/* Wait for all enqueued work. */
smcx_status smcx_synchronize(smcx_ctx* ctx);

/* Kernel timing of the sweep kernel: when enabled, every colour-phase
 * launch is bracketed by HIP events on the context's stream.
 * smcx_kernel_time returns the summed duration (ms) and launch count since
 * enabling (synchronises). */
smcx_status smcx_profile(smcx_ctx* ctx, int32_t enable);
smcx_status smcx_kernel_time(smcx_ctx* ctx, double* total_ms, uint64_t* launches);

void smcx_destroy(smcx_ctx* ctx);
const char* smcx_last_error(const smcx_ctx* ctx);
const char* smcx_global_error(void);
const char* smcx_status_string(smcx_status s);

/* ---- many lattices in one launch (temperature parallelism) --------------
 * n independent replicas, each with its own desc (L, K, S, B, seed), species
 * and EPI table (pointers may repeat) and temperature.  All are resident on
 * the device.  A replica's trajectory is exactly that of a single context
 * with the same inputs: work placement never enters the arithmetic. */
smcx_status smcx_batch_create(int32_t n, const smcx_desc* descs, const uint8_t* const* species,
                              const int32_t* const* epi_ueV, const double* T_kelvin,
                              smcx_batch** out);
/* Advance replica r by n_sweeps[r] >= 0 sweeps.  All phases of all replicas
 * are captured once into a HIP graph and launched as one graph; each phase
 * kernel covers the blocks of every replica still running. */
smcx_status smcx_batch_run(smcx_batch* batch, const int32_t* n_sweeps);
/* Same work, one launch per replica and phase (the per-instance baseline). */
smcx_status smcx_batch_run_unbatched(smcx_batch* batch, const int32_t* n_sweeps);
/* Per-replica view: a context usable with smcx_energy, smcx_energy_recompute,
 * smcx_sro, smcx_get_config, smcx_get_stats.  Owned by the batch. */
smcx_status smcx_batch_ctx(smcx_batch* batch, int32_t r, smcx_ctx** view);
smcx_status smcx_batch_set_temperature(smcx_batch* batch, int32_t r, double T_kelvin);
/* Replica exchange (equations for P_swap and Delta): for each listed pair
 * (a[k], b[k]) in order, exchange the temperatures of replicas a and b with
 * probability min(1, exp((1/kB)(1/T_a - 1/T_b)(E_a - E_b))), deciding with
 * Philox4x32-10(key = (seed lo, seed hi), counter = (k, round lo, round hi, 9))
 * word 0
 * as u: accept iff (double)u < 2^32 * min(1, exp(Delta)).  Replicas must
 * share L and K.  accepted[k] (nullable) receives the decisions. */
smcx_status smcx_batch_exchange(smcx_batch* batch, const int32_t* a, const int32_t* b, int32_t n_pairs,
                                uint64_t seed, uint64_t round, int32_t* accepted);
/* Temperature ladder for replica exchange sized to the system (equation for
 * Delta T: the spacing of neighbouring temperatures scales as
 * 1/sqrt(N_atom), so that neighbouring energy distributions keep
 * overlapping as the system grows).  out[k] = T0 + k dT, k < n, with
 * dT = dT_ref sqrt(n_ref / n_atoms); dT_ref <= 0 or n_ref = 0 take the
 * paper's example, 0.1 K at 10^9 atoms.  Host only.  RANGE if a
 * temperature leaves [1, 5000] K. */
smcx_status smcx_temperature_ladder(double T0, int32_t n, uint64_t n_atoms, double dT_ref, uint64_t n_ref,
                                    double* out);
smcx_status smcx_batch_synchronize(smcx_batch* batch);
void smcx_batch_destroy(smcx_batch* batch);

/* ---- serving: continuous batching of sweep requests ---------------------
 * A server owns a number of slots and a device arena of hbm_budget_bytes,
 * allocated once by smcx_server_create: admitting and retiring requests
 * never allocates or frees device memory.  Submitted requests wait, in
 * arrival order, until a slot is free and a range of the arena holds their
 * footprint (first fit; a request that fits may pass one that does not).
 * Admitted lattices stay resident; each step advances every resident
 * request by up to `sweeps_per_step` sweeps in one batched launch per
 * phase.  A request's result equals that of a single context with the same
 * inputs. */
smcx_status smcx_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t sweeps_per_step,
                               smcx_server** out);
smcx_status smcx_server_submit(smcx_server* srv, const smcx_desc* desc, const uint8_t* species,
                               const int32_t* epi_ueV, double T_kelvin, int32_t n_sweeps,
                               uint64_t* request_id);
/* One scheduling step, pipelined with the device: wait for the previous
 * step's kernels, launch this step's (asynchronously, on the server's
 * stream), retire the requests the previous step finished (their results
 * are copied to host memory on a second stream while this step runs) and
 * admit waiting requests (uploads and initial pair counts on the second
 * stream; they join the next step).  A request therefore finishes one call
 * after its last sweeps were launched.  Reports counts after the call. */
smcx_status smcx_server_step(smcx_server* srv, int32_t* n_resident, int32_t* n_waiting,
                             int32_t* n_finished_this_step);
/* Status of a request: 0 waiting, 1 resident, 2 finished, 3 failed. */
smcx_status smcx_server_poll(smcx_server* srv, uint64_t request_id, int32_t* state);
/* Result of a finished request; config (nullable, n >= N bytes).  Frees it. */
smcx_status smcx_server_result(smcx_server* srv, uint64_t request_id, int64_t* E_ueV,
                               uint64_t* accepted, uint8_t* config, size_t n);
/* Device bytes a request of this shape holds while resident. */
size_t smcx_server_footprint(const smcx_desc* desc);
void smcx_server_destroy(smcx_server* srv);
const char* smcx_server_last_error(const smcx_server* srv);

/* ---- sweeps without device allocation -----------------------------------
 * For callers that cannot allocate device memory: code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * smcx_sweep_noalloc runs sweeps sweep0 .. sweep0+n-1 of the lattice in the
 * caller's device buffer d_species (N bytes, canonical order, 4-byte
 * aligned; updated in place) on hip_stream (NULL: the null stream) of the
 * current device, with desc, EPI and T as for smcx_create_device and a fixed
 * temperature.  The trajectory is that of a context created on the same
 * inputs, set to sweep index sweep0 (smcx_set_state) and advanced by
 * smcx_sweep(n), bit for bit.  dE_ueV and accepted (nullable) receive the
 * energy change and the number of accepted swaps of these n sweeps.
 * It calls no hipMalloc or hipFree: the lattice descriptor, the
 * running-state slots, the threshold table and the pair-weight rows live in
 * a library-owned device array of 32 KiB per device (held until the process
 * ends; every valid desc fits, K <= 8 and S <= 3 need at most 22,784 bytes,
 * and a larger need is rejected with SMCX_E_UNSUPPORTED).  All calls on one
 * device share that array: calls that overlap in time on one device (from
 * several threads, or on several streams) race and must not be made.  The
 * call validates the species on the device and synchronises hip_stream
 * before returning.  Errors: as smcx_create_device, RANGE if sweep0 + n
 * passes 2^32, DEVICE. */
smcx_status smcx_sweep_noalloc(const smcx_desc* desc, uint8_t* d_species, const int32_t* epi_ueV,
                               double T_kelvin, uint64_t sweep0, int32_t n, void* hip_stream,
                               int64_t* dE_ueV, uint64_t* accepted);

/* ---- verification hooks ---------------------------------------------------
 * smcx_threshold_table: the host table the library builds for T (768 doubles:
 * T0, T1, T2).  smcx_device_thresholds: the threshold products computed by
 * the device's FP64 unit for n energy changes (host arrays; synchronous).
 * smcx_device_accept_bounds: for n acceptance draws u (host array), the
 * bounds the sweep kernels use to skip the table test of Eq. (3): they
 * accept an uphill change dE <= lo[k] and reject dE > hi[k] without the
 * table, and evaluate the table only in between (and for u = 0); the
 * library claims that these decisions equal the table test's (host arrays;
 * synchronous).
 * smcx_device_philox: Philox4x32-10 evaluated on the device for n counters
 * (host arrays of 4n words; synchronous). */
smcx_status smcx_threshold_table(double T_kelvin, double* out768);
/* smcx_weight_rows: the pair-weight rows the library builds for a lattice
 * type (0 BCC, 1 FCC), K species, S shells and an EPI table [S][K][K]
 * (host memory; no device).  *form: 0 full fields, 1 the last species
 * folded in, 2 byte-dot digits; the table has kmax*kmax rows of *row_len
 * int32 entries, row (a, b) at a*kmax + b (layouts in the library's
 * tables.cpp).  out may be NULL to query kmax and row_len; otherwise it
 * must hold n >= kmax*kmax*row_len ints.  Errors as smcx_create's EPI checks. */
smcx_status smcx_weight_rows(int32_t lattice, int32_t K, int32_t S, const int32_t* epi, int32_t* form,
                             int32_t* kmax, int32_t* row_len, int32_t* out, size_t n);
smcx_status smcx_device_thresholds(double T_kelvin, const int32_t* dE, int32_t n, double* out);
smcx_status smcx_device_accept_bounds(double T_kelvin, const uint32_t* u, int32_t n, int32_t* lo, int32_t* hi);
smcx_status smcx_device_philox(const uint32_t* ctr, const uint32_t key[2], int32_t n, uint32_t* out);
/* smcx_device_check_accept_bounds: the claim above, checked on the device
 * for every 32-bit draw u at temperature T (the acceptance draws of both
 * lattices are whole 32-bit words): violations_lo counts draws whose bound lo or
 * lo - 1 (where in (0, 2^24)) fails the table test, violations_hi those
 * whose hi + 1 or hi + 2 passes it; max_log2_error receives the largest
 * |(32 - log2 float(u)) - (32 - log2 u)| of the device's FP32 logarithm over
 * u > 0, max_band the widest hi - lo.  Every output is nullable; synchronous. */
smcx_status smcx_device_check_accept_bounds(double T_kelvin, uint64_t* violations_lo, uint64_t* violations_hi,
                                            double* max_log2_error, int32_t* max_band);

#ifdef __cplusplus
}
#endif
#endif /* SMCX_H */
