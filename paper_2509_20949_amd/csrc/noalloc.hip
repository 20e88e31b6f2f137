// noalloc.hip -- smcx_sweep_noalloc: sweeps of a lattice in the caller's
// device buffer that allocate no device memory.
//
// smcx_sweep needs a context, whose creation allocates the per-lattice
// device state the sweep kernels read and write besides the lattice itself:
// the lattice descriptor, the running-state slots the waves add their
// energy changes and accept counts into, the threshold table and the
// pair-weight rows.  Here that state lives in one file-scope device array,
// `scratch`, of fixed size; the caller passes the lattice (input and
// output) and receives the energy change and accept count.  The kernels are
// the context path's own, so the trajectory is the same bit for bit.
#include <cstring>
#include <mutex>

#include "../../include/smcx.h"
#include "ctx.h"

using namespace smcx;

namespace {

// Scratch layout (byte offsets; every part 256-byte aligned).  The largest
// weight table (K = 8, S = 3: 64 rows of 28 ints) ends at 22,784 bytes.
constexpr size_t kScratchBytes = 32768;
constexpr size_t kOffLat = 0;                                            // DevLattice
constexpr size_t kOffMax = 128;                                          // species-maximum word
constexpr size_t kOffState = 256;                                        // kStateWords int64
constexpr size_t kOffTab = kOffState + sizeof(int64_t) * kStateWords;    // kTab doubles
constexpr size_t kOffW = (kOffTab + sizeof(double) * kTab + 255) & ~(size_t)255;   // weight rows
static_assert(sizeof(DevLattice) <= kOffMax, "descriptor overlaps the maximum word");
static_assert(kOffW + sizeof(int32_t) * 64 * wrow(8, 3) <= kScratchBytes, "scratch too small for K = 8, S = 3");

// The array itself.  In host code its name is only a host-side stand-in:
// the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
smcx_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_global(SMCX_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_global(SMCX_E_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail_global(SMCX_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SMCX_OK;
}

smcx_status hip_ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return SMCX_OK;
    return fail_global(SMCX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" smcx_status smcx_sweep_noalloc(const smcx_desc* desc, uint8_t* d_species, const int32_t* epi_ueV,
                                          double T_kelvin, uint64_t sweep0, int32_t n, void* hip_stream,
                                          int64_t* dE_ueV, uint64_t* accepted)
{
    int32_t B[3];
    smcx_status st = validate_desc(desc, B, true);
    if (st) return st;
    st = validate_epi(epi_ueV, desc->n_species, desc->n_shells);
    if (st) return st;
    st = validate_T(T_kelvin);
    if (st) return st;
    if (!d_species || ((uintptr_t)d_species & 3u))
        return fail_global(SMCX_E_INVALID, "d_species is NULL or not 4-byte aligned");
    if (n < 0) return fail_global(SMCX_E_INVALID, "n = %d < 0", n);
    if (sweep0 + (uint64_t)n > 0xffffffffull) return fail_global(SMCX_E_RANGE, "sweep counter would pass 2^32");

    const int lattice = desc->lattice, K = desc->n_species, S = desc->n_shells;
    const int kmax = kmax_for(lattice, K);
    const size_t wbytes = sizeof(int32_t) * (size_t)kmax * kmax * wrow(kmax, S);
    const size_t need = kOffW + wbytes;
    if (need > kScratchBytes)
        return fail_global(SMCX_E_UNSUPPORTED, "K = %d, S = %d need %zu bytes of scratch > the maximum %zu", K, S,
                           need, kScratchBytes);

    DevLattice h;
    std::memset(&h, 0, sizeof(h));
    fill_geometry(h, desc, B);
    if (!geometry_ok(h)) return fail_global(SMCX_E_UNSUPPORTED, "block geometry outside 2..%d cells", kMaxBlock);

    void* base = nullptr;
    st = scratch_address(&base);
    if (st) return st;
    unsigned char* d = (unsigned char*)base;

    // Host image of the scratch contents: descriptor, zero maximum word,
    // zero running-state slots (the sums count this call only), the
    // threshold table of T and the weight rows.  Stack memory only.
    alignas(16) unsigned char img[kScratchBytes];
    std::memset(img, 0, need);
    h.species = d_species;
    h.tabs = (const double*)(d + kOffTab);
    h.wtab = (const int32_t*)(d + kOffW);
    h.state = (int64_t*)(d + kOffState);
    h.sweep0 = (uint32_t)sweep0;
    h.tab_s0 = (uint32_t)sweep0;
    h.n_tabs = 1;
    h.drop_last = build_wtab(epi_ueV, K, S, kmax, S, wtab_bias(lattice, kmax), true, (int32_t*)(img + kOffW));
    build_thresholds(T_kelvin, (double*)(img + kOffTab));
    std::memcpy(img + kOffLat, &h, sizeof(h));

    hipStream_t stream = (hipStream_t)hip_stream;
    st = hip_ok(hipMemcpyAsync(d, img, need, hipMemcpyHostToDevice, stream), "hipMemcpyAsync(scratch)");
    if (st) return st;

    // The kernels trust species < K: check the borrowed lattice first.
    const size_t N = n_sites(lattice, desc->L);
    unsigned int mx = 0;
    st = hip_ok(launch_species_max(d_species, N, (unsigned int*)(d + kOffMax), stream), "species_max launch");
    if (!st) st = hip_ok(hipMemcpyAsync(&mx, d + kOffMax, sizeof(mx), hipMemcpyDeviceToHost, stream), "copy");
    if (!st) st = hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st) return st;
    if (mx >= (unsigned)K) return fail_global(SMCX_E_INVALID, "device species value %u >= K = %d", mx, K);

    const int wpg = waves_per_group(lattice);
    const int groups = (h.blocks_per_colour + wpg - 1) / wpg;
    for (int32_t k = 0; k < n; ++k)
        for (int col = 0; col < 8; ++col) {
            st = hip_ok(launch_sweep_phase(lattice, (const DevLattice*)(d + kOffLat), nullptr, groups, k, col, kmax,
                                           S, stream),
                        "sweep_phase launch");
            if (st) return st;
        }

    int64_t slots[kStateWords];
    st = hip_ok(hipMemcpyAsync(slots, d + kOffState, sizeof(slots), hipMemcpyDeviceToHost, stream),
                "hipMemcpyAsync(state)");
    if (!st) st = hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st) return st;
    int64_t e = 0;
    uint64_t a = 0;
    state_sum(slots, &e, &a);
    if (dE_ueV) *dE_ueV = e;
    if (accepted) *accepted = a;
    return SMCX_OK;
}
