// Earliest arrival without any allocation, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid it).  The query's state -- arrival words, claim words, the two
// frontier queues, arrival codes, counters and the chunk list -- lives in one
// fixed device array, `scratch`, that every call on a device shares.
//
// In host code `scratch` names a host-side stand-in, not a device address:
// its device address is taken once per device with hipGetSymbolAddress (on
// the first call on that device, with the device current) and only that
// address is ever passed to kernels or copies.  Each process holds one copy
// of the array per device it runs on, until it exits.
//
// Calls on one device would race on the shared array; the library serialises
// them with a per-device lock, so overlapping calls from several host
// threads wait for each other.  The array keeps the previous call's contents:
// every word a query reads before writing is cleared by a fill kernel at the
// start of the call (arrival and claim words, arrival codes, counters).
#include "internal.h"
#include "stage.h"

#include <algorithm>
#include <mutex>

namespace kairos {

namespace {

constexpr uint64_t SCRATCH_BYTES = KAIROS_NOALLOC_SCRATCH_BYTES;
constexpr uint64_t CHUNK_CAP = 1ull << 20;        // chunk-list entries; longer rounds walk the excess in place
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct DeviceScratch {
    std::mutex mu;
    unsigned char *ptr = nullptr;  // device address of `scratch` on this device
    bool looked_up = false;
    hipError_t lookup_error = hipSuccess;
};
DeviceScratch g_dev[MAX_DEVICES];

__global__ void zero_words_kernel(uint32_t *p, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

}  // namespace

}  // namespace kairos

using namespace kairos;

extern "C" int kairos_earliest_arrival_noalloc(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                                               uint32_t *out)
{
    if (!g || !out) return KAIROS_ERR_INVALID;
    (void)hipGetLastError();
    if (src >= g->n || t_alpha > t_omega || t_omega > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return KAIROS_ERR_DEVICE;
    if (dev != g->device) return KAIROS_ERR_INVALID;  // the graph lives on another device
    const uint64_t chunk_cap = std::min<uint64_t>(CHUNK_CAP, g->m / 64 + 1);
    if (slot_layout(g, chunk_cap, nullptr, 0, nullptr, nullptr) > SCRATCH_BYTES) return KAIROS_ERR_SCRATCH;
    DeviceScratch &d = g_dev[dev];
    std::lock_guard<std::mutex> lk(d.mu);
    if (!d.looked_up) {
        void *p = nullptr;
        d.lookup_error = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        d.ptr = d.lookup_error == hipSuccess ? (unsigned char *)p : nullptr;
        d.looked_up = true;
    }
    if (d.lookup_error != hipSuccess || !d.ptr) {
        note_hip_error(d.lookup_error, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        return KAIROS_ERR_DEVICE;
    }
    uint32_t host_words[256];  // counter read-back: ordinary host memory
    Slot s;
    slot_layout(g, chunk_cap, d.ptr, SCRATCH_BYTES, host_words, &s);
    // counters and work statistics start at zero (the arrival and claim
    // words, codes and queues are filled by the query itself)
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, s.stream, s.cnt, (uint32_t)CNT_WORDS);
    hipLaunchKernelGGL(zero_words_kernel, dim3(64), dim3(256), 0, s.stream, (uint32_t *)s.stats,
                       (uint32_t)(ST_TOTAL_WORDS * 2));
    if (hipGetLastError() != hipSuccess) return KAIROS_ERR_DEVICE;
    set_unprofiled(true);
    int rc = run_earliest_arrival(g, &s, src, t_alpha, t_omega, out, false);
    set_unprofiled(false);
    if (hipStreamSynchronize(s.stream) != hipSuccess && rc == KAIROS_OK) rc = KAIROS_ERR_DEVICE;
    return rc;
}
