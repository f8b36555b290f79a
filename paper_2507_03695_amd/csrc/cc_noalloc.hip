// cc_noalloc.hip — the whole single-graph path without any allocation, for
// callers that cannot allocate (code under stream capture, tight serving loops,
// harnesses that forbid it).
//
// Every kernel of cc_solve_async's path that needs memory beyond the caller's
// edges and labels (the status word and zero-root state, the sampled-degree hash
// table, the per-block minima of compress, the zero-root membership bitmap) takes
// it from one fixed array in the library's device image, `scratch` below. Each
// device holds its own copy of the array until the process ends. Host code never
// passes the array's name to a kernel: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and only
// that address is used. The regrouped hooks (whose buffers grow with the entry
// count) and the exact-degree zero root (a count per vertex) are not available
// here; the direct hooks handle every size.
#include <mutex>

#include "cc_internal.h"

namespace ccm {

constexpr uint64_t kNoAllocBytes = CC_NOALLOC_SCRATCH_BYTES;
constexpr uint32_t kNoAllocSamples = 16384;          // zero-root sample: K entries
constexpr uint32_t kNoAllocTable = 4 * kNoAllocSamples;   // hash slots (a power of two)
constexpr uint64_t kOffState = 0;                    // DevState (64 bytes) in 256
constexpr uint64_t kOffKeys = 256;
constexpr uint64_t kOffCounts = kOffKeys + 4ull * kNoAllocTable;
constexpr uint64_t kOffMin = kOffCounts + 4ull * kNoAllocTable;
constexpr uint64_t kOffBits = (kOffMin + 4ull * kGridCap + 255) & ~255ull;
constexpr uint64_t kBitsWords = (kNoAllocBytes - kOffBits) / 4;
static_assert(kOffBits < kNoAllocBytes, "scratch too small for its fixed part");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_na_mu;
static char* g_na_ptr[kMaxDevices] = {};

// Device address of this device's scratch (set up once per device).
static int scratch_of(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        CCM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CC_EDEVICE, "no device address for the scratch array");
        g_na_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_na_ptr[dev];
    return CC_OK;
}

// The status word and the zero-root relabelling state start at zero for each
// call (a kernel, not a memset, so the call can be captured into a graph).
__global__ void k_na_reset(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st_agent(&st->status, 0u);
        st_agent(&st->minz, kEmpty);
        st_agent(&st->zroot, 0u);
        st_agent64(&st->zsel, 0ull);
    }
}

// The call's outcome: CC_ERANGE if an endpoint was out of range, else CC_OK.
__global__ void k_na_status(DevState* st, int32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t w = ld_agent(&st->status);
        __hip_atomic_store(out, (w & kStatusRange) ? (int32_t)CC_ERANGE : (int32_t)CC_OK,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace ccm

using namespace ccm;

extern "C" int cc_solve_noalloc(uint64_t n, uint64_t m, const uint32_t* edge_list, uint32_t* L,
                                uint32_t flags, uint32_t zroot_hint, int32_t* status,
                                void* stream) {
    if (n > 0xFFFFFFFFull) return fail(CC_EINVAL, "n must be < 2^32");
    if (m && !edge_list) return fail(CC_EINVAL, "edge_list is NULL with m > 0");
    if (n && !L) return fail(CC_EINVAL, "L is NULL with n > 0");
    if (n == 0 && m) return fail(CC_ERANGE, "entries given for an empty vertex set");
    if (m > (1ull << 40)) return fail(CC_EINVAL, "m above 2^40");
    const uint32_t allowed = CC_F_ZROOT | CC_F_ZROOT_HINT | CC_F_NO_SPLIT | CC_F_NO_TILE |
                             CC_F_SYMMETRIC;
    if (flags & ~allowed)
        return fail(CC_EINVAL, "flag not available without allocation (CC_F_ZROOT_EXACT, unknown)");
    if ((flags & CC_F_ZROOT_HINT) && n && zroot_hint >= n)
        return fail(CC_EINVAL, "zroot_hint must be < n");
    if ((flags & CC_F_ZROOT) && (n + 31) / 32 > kBitsWords)
        return fail(CC_ENOMEM, "n exceeds the zero-root bitmap of the fixed scratch (" +
                                   std::to_string(kBitsWords * 32) + " vertices)");
    int dev = 0;
    CCM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CC_EINVAL, "device ordinal out of range");
    char* base = nullptr;
    int rc = scratch_of(dev, &base);
    if (rc) return rc;
    hipStream_t hs = (hipStream_t)stream;
    // A slot whose every buffer lies in the scratch array; nothing in it is ever
    // grown (the bitmap's capacity is the array's rest, the regrouped hooks are
    // off, the exact-degree count is refused above).
    Slot s{};
    s.device = dev;
    s.st = reinterpret_cast<DevState*>(base + kOffState);
    s.hkeys = reinterpret_cast<uint32_t*>(base + kOffKeys);
    s.hcounts = reinterpret_cast<uint32_t*>(base + kOffCounts);
    s.bmin = reinterpret_cast<uint32_t*>(base + kOffMin);
    s.table = kNoAllocTable;
    s.samples = kNoAllocSamples;
    s.zbits = reinterpret_cast<uint32_t*>(base + kOffBits);
    s.zbits_cap = kBitsWords;
    s.no_grow = true;
    s.no_tiled = true;
    k_na_reset<<<1, 64, 0, hs>>>(s.st);
    CCM_HIP(hipGetLastError());
    if ((rc = run_solve(&s, n, m, edge_list, L, flags, zroot_hint, hs))) return rc;
    if (status) {
        k_na_status<<<1, 64, 0, hs>>>(s.st, status);
        CCM_HIP(hipGetLastError());
    }
    return CC_OK;
}
