// cc_internal.h — declarations shared by the library's own translation units.
// Not installed; the public interface is include/cc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cc.h"

namespace ccm {

// Device-resident state of one solve slot (a context has one; the server one per
// slot). Lives in device memory; kernels read and update it, the host reads it
// only through explicit copies.
struct DevState {
    uint32_t status;    // kStatus* bits, reported and cleared by slot_sync
    uint32_t minz;      // smallest member of the zero root's component (compress, k_minz)
    uint32_t zroot;     // the zero root chosen for the current solve
    uint32_t pad0;
    uint64_t zsel;      // packed argmax (count << 32) | (0xFFFFFFFF - id); 0 = none
    uint64_t log_count; // messages of a drained update log (cc_hook_log_drain)
    uint64_t pad1[4];
};
static_assert(sizeof(DevState) == 64, "DevState is one 64-byte block");

constexpr uint32_t kStatusRange = 1u;
constexpr uint32_t kStatusInternal = 2u;   // a scratch bound check failed (a bug)
constexpr uint32_t kStatusLogFull = 4u;    // an update log ran out of capacity
constexpr uint32_t kStatusBadOffsets = 8u; // CSR offsets not a valid row index
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Path splitting in the direct hooks' walks pays only where the parent array
// outgrows one XCD's L2 (4 MB): below that every walk step is an L2 hit and the
// splitting stores, which go to memory, cost more than the steps they save
// (ER n = 2^16, 2^20 entries: 0.82 ms with splitting, 0.14 ms without; R-MAT
// n = 2^22 direct hook: 4.9 ms with, 7.2 ms without). CC_F_NO_SPLIT turns it
// off everywhere.
constexpr uint64_t kSplitMinBytes = 4ull << 20;
__host__ __device__ inline bool split_walks(uint32_t flags, uint64_t n, uint64_t entry_bytes = 4) {
    return !(flags & CC_F_NO_SPLIT) && n * entry_bytes > kSplitMinBytes;
}
// Hooking in two parts: without path splitting the walks of one pass grow long
// while the forest forms (link by index makes chains that nothing shortens),
// and every later entry walks them. Where that applies to enough entries per
// vertex, the first quarter of the entries is hooked, the forest pointer-jumped
// (a flat forest with the same components, from which Algorithm 1 continues)
// and the rest hooked over it.
__host__ __device__ inline bool hook_in_two_parts(uint64_t n, uint64_t m, bool split) {
    return !split && m >= (1ull << 18) && m >= 4 * n;
}
constexpr uint32_t kGridCap = 256 * 32;   // blocks of a grid-stride launch over n

// One graph of a batched launch: where its entries and labels live.
struct GraphDesc {
    const int32_t* edges;   // 2*m int32, local IDs
    int32_t* L;             // n int32 labels (also the parent array when it is not in LDS)
    int32_t* status;        // where the graph's status code goes
    uint32_t n;
    uint32_t pad;
    int64_t m;
};
static_assert(sizeof(GraphDesc) == 40, "GraphDesc layout");

// Scratch of the batched path: the work tickets, the work lists, the chunk
// tables of the whole-device graphs and the descriptors, uploaded in one copy
// per launch (layout in cc_batch.hip).
struct BatchScratch {
    char* dev = nullptr;       // device
    char* host = nullptr;      // pinned host staging of the same layout
    uint64_t cap = 0;          // graphs
};

// A batch schedule (cc_batch_sched): which graphs run on the whole device, which
// on one wavefront, the rest on one workgroup each.
typedef cc_batch_sched BatchSched;

// Scratch of the tiled zero-root hook (one block, grown on demand).
struct TiledScratch {
    char* buf = nullptr;
    uint64_t cap = 0;
};

// Scratch owned by one slot.
struct Slot {
    int device = 0;
    DevState* st = nullptr;        // device
    uint32_t* hkeys = nullptr;     // device, zroot hash table keys   [table]
    uint32_t* hcounts = nullptr;   // device, zroot hash table counts [table]
    uint32_t* bmin = nullptr;      // device, per-block minima of compress [kGridCap]
    uint32_t* xs = nullptr;        // device, export counts and offsets [4 * kGridCap + 2]
    uint32_t table = 0;            // power of two >= 4 * samples
    uint32_t samples = 0;          // K
    uint32_t* deg = nullptr;       // device, exact-degree counts (grown on demand)
    uint64_t deg_cap = 0;
    uint32_t* host_status = nullptr;  // pinned host block of 64 bytes (status word, read-backs)
    BatchScratch batch;
    // Zero-root membership bitmap: bit x set => x is in the zero root's tree.
    uint32_t* zbits = nullptr;     // device, ceil(n/32) words (grown on demand)
    uint64_t zbits_cap = 0;        // words
    // Host-side order of the steps: a CC_F_ZROOT hook needs cc_zroot after the
    // latest cc_init on the same n (the bitmap describes that solve).
    uint64_t cur_n = 0;
    bool zr_ready = false;
    TiledScratch tiled;
    uint32_t* csr_tiles = nullptr; // device, first row of every CSR tile (grown on demand)
    uint64_t csr_tiles_cap = 0;
    // Nothing is grown: a solve that would need a larger buffer than the slot
    // holds fails with CC_ENOMEM (a server's lent block, the allocation-free
    // entry point).
    bool no_grow = false;
    // The regrouped hooks (buffers per entry) are not taken (the allocation-free
    // entry point, whose fixed scratch cannot hold them).
    bool no_tiled = false;
};

int slot_create(Slot* s, int device, uint32_t samples);
void slot_destroy(Slot* s);

// Enqueue steps (arguments already validated by the caller).
int run_init(Slot* s, uint64_t n, uint32_t* P, hipStream_t stream);
int run_zroot(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t flags,
              uint32_t hint, hipStream_t stream);
int run_push(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
             hipStream_t stream);
// How the direct zero-root hooks settle an entry with exactly one endpoint in
// the membership bitmap. Linking the other endpoint's tree under z costs a walk,
// a coherent read and a CAS on P, but every vertex of that tree then walks to z
// and is marked when an entry reaches it, so the bitmap grows faster; marking
// the endpoint alone (compress passes the mark on to its tree) touches no P.
// Once P outgrows the MALL (256 MB) each of those P accesses goes to HBM and
// marking wins: R-MAT-30 1/16 share (4 GiB P), 46.9 -> 40.8 ms (37.6 with the
// second endpoint's word read coherently, so that its mark is one atomic);
// R-MAT-26 + extras direct, 21.7 -> 21.1 ms. Below it linking wins: R-MAT-22 direct 2.2
// against 2.8 ms, R-MAT-24 5.5 against 5.8, R-MAT-26 1/16 share 2.8 against
// 3.2. kHookLinkZ, an internal flag of run_hook (beside the public CC_F_*,
// never accepted from a caller), asks for linking at any size: the regrouped
// hook's warm-up seeds its filter's bitmap (10.1 against 10.4 ms on R-MAT-26 +
// extras).
constexpr uint32_t kHookLinkZ = 0x80000000u;
constexpr uint64_t kMallBytes = 256ull << 20;
inline bool hook_links_z(uint32_t flags, uint64_t n) {
    return (flags & kHookLinkZ) || n * 4 <= kMallBytes;
}
int run_hook(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
             uint32_t flags, hipStream_t stream);
// final_labels (zero root): z's component ends labelled with its smallest ID
// directly, as run_canon would make it; otherwise it keeps the label z.
int run_compress(Slot* s, uint64_t n, uint32_t* P, uint32_t flags, hipStream_t stream,
                 bool final_labels = false);
// Plain-path hook that appends its links to a caller-owned log (cc_hook_log).
int run_hook_log(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                 uint32_t flags, uint32_t* log, uint64_t log_cap, uint64_t* log_count,
                 hipStream_t stream);
// The log counter of the slot's DevState set to 0 (a kernel: capturable).
int log_count_reset(Slot* s, hipStream_t stream);
// The counter's value written to a pinned host word (a kernel, ordered on stream).
int log_count_snap(Slot* s, uint64_t* host_word, hipStream_t stream);
int run_canon(Slot* s, uint64_t n, uint32_t* L, hipStream_t stream);
int run_hook_ids(Slot* s, uint64_t n, uint64_t count, const uint32_t* ids, uint32_t target,
                 uint32_t* P, uint32_t flags, hipStream_t stream);

// Exchange (cc_exchange.hip): synchronous export of a share's parent array.
int run_export(Slot* s, uint64_t n, const uint32_t* P, uint32_t zroot, uint32_t* pairs,
               uint64_t pairs_cap, uint32_t* zero_ids, uint64_t zero_cap, uint64_t* n_pairs,
               uint64_t* n_zero, hipStream_t stream);
// Compact IDs of the exchange (cc_exchange.hip); k in 1..4, buffers 4-byte aligned.
int run_pack_ids(Slot* s, uint64_t count, const uint32_t* ids, uint32_t k, uint8_t* out,
                 hipStream_t stream);
int run_unpack_ids(Slot* s, uint64_t count, const uint8_t* in, uint32_t k, uint32_t* ids,
                   hipStream_t stream);
int run_solve(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* L,
              uint32_t flags, uint32_t hint, hipStream_t stream);
// Whole path on CSR input (m = off[n], read by the caller).
int run_solve_csr(Slot* s, uint64_t n, uint64_t m, const uint64_t* off, const uint32_t* adj,
                  uint32_t* L, uint32_t flags, uint32_t hint, hipStream_t stream);
// Plain path with 64-bit IDs (cc_wide.hip).
int run_solve_w(Slot* s, uint64_t n, uint64_t m, const uint64_t* edges, uint64_t* L,
                uint32_t flags, hipStream_t stream);
// Size the zero-root membership bitmap for n and clear it (only z set).
int zbits_reset(Slot* s, uint64_t n, hipStream_t stream);
// Copy the status word to the host, clear it, wait for the stream; CC_OK,
// CC_ERANGE, CC_ENOMEM (a full update log) or CC_EINVAL (bad CSR offsets).
int slot_sync(Slot* s, hipStream_t stream);

// Tiled zero-root hook (cc_tiled.hip): both membership tests in LDS.
bool tiled_eligible(uint64_t n, uint64_t m, bool zr);
// Bytes of the regrouped hook's buffers for n vertices and m COO entries.
uint64_t tiled_scratch_bytes(uint64_t n, uint64_t m, bool plain);
// Device bytes a whole-path solve (run_solve) grows in its slot for these
// arguments: the bitmap, exact degrees, the regrouped hook's buffers.
uint64_t solve_scratch_bytes(uint64_t n, uint64_t m, uint32_t flags);
// Lend a block of device memory (at least solve_scratch_bytes(n, m, flags)) to
// a slot for one run_solve: its grown buffers point into the block and nothing
// is allocated; slot_return_scratch gives the slot its own buffers back.
struct LentScratch {
    uint32_t* zbits; uint64_t zbits_cap;
    uint32_t* deg; uint64_t deg_cap;
    TiledScratch tiled;
};
void slot_lend_scratch(Slot* s, char* block, uint64_t n, uint64_t m, uint32_t flags, LentScratch* saved);
void slot_return_scratch(Slot* s, const LentScratch* saved);
// plain = true: the plain path (key = ID) hooks the first-endpoint buckets in
// order instead (better locality for the first endpoints' parent reads).
// sym: the list holds every pair in both orders; only u < v is hooked.
int run_hook_tiled(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                   hipStream_t stream, bool plain = false, bool sym = false);
void tiled_free(TiledScratch* t);
// The same on CSR input, where the rows already are the first-endpoint buckets.
int run_hook_tiled_csr(Slot* s, uint64_t n, uint64_t m, const uint64_t* off, const uint32_t* adj,
                       uint32_t* P, hipStream_t stream, bool sym = false);

// Batched path (cc_batch.hip).
// The schedule taken when nothing else is known about a batch.
BatchSched batch_default_sched();
// Largest n of a wave-role graph on this device (its LDS per wavefront).
int batch_wave_cap(int device, uint32_t* cap);
// Role of one graph under a schedule: kRoleTile, kRoleWave or kRoleMulti.
constexpr int kRoleTile = 0, kRoleWave = 1, kRoleMulti = 2;
int batch_role(const GraphDesc& d, const BatchSched& sc, uint32_t wave_cap);
// Enqueue one batch (the whole-device launches of its multi graphs, then the
// persistent launch) over G graphs described on the host.
int launch_batch(Slot* s, uint32_t G, const GraphDesc* descs, const BatchSched& sc,
                 hipStream_t stream);
// Size the slot's batch scratch for G graphs now (so later launches of at most
// G graphs allocate nothing).
int batch_reserve(Slot* s, uint32_t G);
// Offsets read back and checked, descriptors built (cc_batch's arguments).
int batch_descs(uint32_t G, const int64_t* vtx_off, const int64_t* edge_off, const int32_t* edges,
                int32_t* L, int32_t* status, hipStream_t stream, std::vector<GraphDesc>* out);
void batch_scratch_free(BatchScratch* b);
// A captured cc_batch (opaque handle): creation takes descriptors built by
// batch_descs and captures the upload and the launches into a graph.
int batch_graph_create(Slot* s, uint32_t G, const GraphDesc* descs, const BatchSched& sc,
                       void** out);
int batch_graph_launch(void* g, hipStream_t stream);
void batch_graph_destroy(void* g);

// Error reporting.
int fail(int code, const std::string& detail);
int hip_fail(hipError_t e, const char* what);
#define CCM_HIP(call)                                             \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::ccm::hip_fail(e_, #call);  \
    } while (0)

int device_cu_count(int device);

// Coherence point between dependent kernels on one stream. Each XCD of the
// device has its own L2; a clean line cached on one XCD is not invalidated when
// another XCD (or an atomic performed beyond the L2) changes the data, and the
// kernel boundary alone has been observed not to drop such lines. This launch
// runs workgroups on every XCD, each writing back and invalidating its L2
// (agent-scope acquire-release fence), so the next kernel on the stream reads
// what the previous ones wrote.
int cohere(hipStream_t stream);

// Coherent (agent-scope) accesses to the small shared words of DevState.
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Race-testing builds (compiled with CCM_STRESS_DELAYS, a separate library):
// before each link CAS and each path-splitting store a wave pauses for 0 to 7
// short sleeps, drawn from the clock, the lane and `salt`. The pause widens the
// windows in which other waves change the same entries. The ordinary build
// compiles this to nothing.
__device__ __forceinline__ void stress_delay(uint32_t salt) {
#ifdef CCM_STRESS_DELAYS
    uint32_t h = (salt ^ (threadIdx.x * 0x9E3779B9u) ^ (uint32_t)clock64()) * 0x85EBCA6Bu;
    h ^= h >> 13;
    for (uint32_t i = 0; i < (h & 7u); ++i) __builtin_amdgcn_s_sleep(2);
#else
    (void)salt;
#endif
}

// Device, memory budget and zero-root sample count of a context.
int ctx_info(cc_ctx* ctx, int* device, uint64_t* budget, uint32_t* samples);

// Batch schedule tuner (cc_tune.hip): picks stored per device and shape, in
// memory and optionally in a file.
struct Tuner {
    std::mutex mu;
    std::string path;                          // the cache file ("" = none)
    std::map<std::string, BatchSched> picks;   // key: device | signature
    bool forced = false;
    BatchSched force{};
    bool autotune = false;
};
// Read the cache file (if any) into the tuner.
void tuner_open(Tuner* t, const char* path_opt, bool autotune);
// The schedule cc_batch takes for these graphs, and its source (CC_SCHED_*).
// With autotune and no stored pick, tunes first (runs the batch).
int tuner_choose(Tuner* t, Slot* s, uint32_t G, const GraphDesc* descs, hipStream_t stream,
                 BatchSched* out, uint32_t* source);
int tuner_tune(Tuner* t, Slot* s, uint32_t G, const GraphDesc* descs, uint32_t reps,
               hipStream_t stream, cc_batch_tune_result* out);
// Stored pick or default for these graphs (no forcing, no tuning): the server's.
BatchSched tuner_lookup(Tuner* t, int device, uint32_t G, const GraphDesc* descs);
Tuner* ctx_tuner(cc_ctx* ctx);

}  // namespace ccm
