/*
 * cc.h — connected-components labelling on AMD Instinct MI355X (gfx950).
 *
 * The library labels the connected components of an undirected graph given as
 * a COO list of unordered vertex pairs. It follows the Jayanti-Tarjan
 * disjoint-set-union method of Sec. II (Algorithm 1): one pass over the edges
 * in which every worker finds the roots of both endpoints in one shared parent
 * array P and links the root of greater key under the other with a
 * compare-and-swap, then pointer jumping. The root-function generalisation of
 * Sec. IV (Algorithm 3 with RobinCC's R, Formulas 1-2) is the CC_F_ZROOT
 * variant: the vertex of largest (sampled) degree takes the smallest key, its
 * sampled neighbours are attached to it first (Initial Push), and edges whose
 * endpoints both already hang from it are dropped.
 *
 * Output labelling. Sec. II defines the output as an array L with L_u == L_v
 * iff u and v are connected. Every entry point here returns the canonical such
 * array: L_v is the smallest vertex ID of v's component (the identity JT with
 * link by index reaches, Sec. II text after Algorithm 1). The CC_F_ZROOT
 * variant reaches the same array after a final relabelling of the zero root's
 * component, so results never depend on thread schedule, edge order, the zero
 * root chosen, or the batch a graph was solved in.
 *
 * Conventions.
 *  - Device pointers are HIP device memory owned by the caller (for instance
 *    torch tensors). The library never frees or retains them past the call
 *    (synchronous entry points) or past completion of the stream (async
 *    entry points).
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *  - Edge lists are 2*m uint32 (or int32) values: entry i is the unordered
 *    pair (edge[2i], edge[2i+1]). Self-loops and repeated pairs are allowed
 *    and change nothing. The input need not be symmetric (Sec. II: processing
 *    (u,v) makes (v,u) a no-op).
 *  - Vertex IDs are 32-bit (Sec. V uses 4-byte IDs below 2^32 vertices), so
 *    n <= 2^32 - 1, except in cc_solve_u64, which takes 8-byte IDs.
 *  - Every function returns a status code; on failure a thread-local
 *    description is available from cc_last_error_detail().
 */
#ifndef CCMI_CC_H
#define CCMI_CC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CC_OK         0
#define CC_EINVAL   (-1)  /* bad argument: n >= 2^32, NULL with nonzero size, bad offsets */
#define CC_ERANGE   (-2)  /* some endpoint >= n; labels are then unspecified */
#define CC_ENOMEM   (-3)  /* device memory or the configured HBM budget is exhausted */
#define CC_EDEVICE  (-4)  /* a HIP call failed; the detail string names it */
#define CC_EAGAIN   (-5)  /* server queue full; submit again later */
#define CC_ECANCELED (-6) /* server closed before the request ran */
#define CC_ETIMEDOUT (-7) /* wait timed out; the request is still pending */

/* Human-readable name of a status code (static storage). */
const char* cc_strerror(int code);
/* Detail of the last failure on the calling thread (thread-local storage). */
const char* cc_last_error_detail(void);
/* Library version as 10000*major + 100*minor + patch. */
int cc_version(void);

/* ---- solve flags ------------------------------------------------------ */
/* Zero planting (Sec. IV, Formula 1): the sampled max-degree vertex is the
   root of smallest key; Initial Push from it; giant-component edge skip.   */
#define CC_F_ZROOT        0x1u
/* With CC_F_ZROOT: take the exact maximum-degree vertex (a full counting
   pass over all entries) instead of the sampled estimate.                  */
#define CC_F_ZROOT_EXACT  0x2u
/* With CC_F_ZROOT: the zero root is `zroot_hint` (must be < n).            */
#define CC_F_ZROOT_HINT   0x4u
/* Plain root walks without path splitting (Algorithm 1's finds as printed)
   everywhere, and no pointer jumping inside a hook. Without the flag the
   regrouped hooks and the batch's workgroup role split paths, and the direct
   hooks split them where the parent array exceeds 4 MB (one XCD's L2; below
   that the walks are L2 hits and the splitting stores cost more than they
   save). Below that size the direct hook, given at least 2^18 entries and 4
   per vertex, instead runs one pointer-jumping pass (with CC_F_ZROOT, the
   compress pass) after the first quarter of the entries, so that the rest
   walk a flat forest.                                                      */
#define CC_F_NO_SPLIT     0x8u
/* Keep the direct hook, which takes the entries in their given order, where
   the regrouped hooks would apply (4 <= ceil(n / 2^19) <= 256, or 8 <= with
   CC_F_ZROOT, and 2^24 <= m < 2^32, without CC_F_NO_SPLIT). With CC_F_ZROOT the regrouped hook
   sorts the entries by the vertex ranges of both endpoints so that both
   membership tests read LDS; without it, the plain hook takes the entries
   grouped by their first endpoint's range, so that those parent reads stay in
   L2. Labels are identical either way. Pass it for lists in which a vertex
   recurs in many entries at once, such as a Reducer's messages from several
   shares: grouped, their links contend for the same roots (R-MAT-26's 165 M
   SiskinCC messages: 4.6 ms in the given order, 13 ms grouped). */
#define CC_F_NO_TILE      0x10u
/* cc_compress with CC_F_ZROOT: give the zero root's component its smallest ID
   in the same pass (what cc_canon writes), so that no cc_canon is needed.
   Ignored elsewhere; the whole-path entry points always do this. */
#define CC_F_CANON        0x20u
/* The list holds every pair in both orders (a symmetrised COO list, or a
   symmetric CSR graph): only the entries with u < v are hooked, so each edge
   is processed once (Sec. II: once (u,v) has been processed, (v,u) changes
   nothing; a symmetric graph needs one direction of each edge). The other
   entries are still read (and range-checked), not hooked. On a list that is
   not symmetric the labels are those of its u < v entries alone. Accepted by
   the whole-path calls (also cc_solve_u64), cc_hook and cc_hook_log. */
#define CC_F_SYMMETRIC    0x40u
/* Every other bit is reserved: each call that takes flags returns CC_EINVAL
   when one is set. */

/* ---- context ----------------------------------------------------------- */
typedef struct cc_ctx cc_ctx;

typedef struct cc_ctx_opts {
    int      device;          /* HIP device ordinal; -1 = the current device   */
    uint32_t zroot_samples;   /* entries sampled for the zero root; 0 = 65536  */
    uint64_t hbm_budget;      /* bytes the server may hold resident; 0 = 3/4 of
                                 free memory at creation                        */
    const char* tune_cache;   /* file of tuned batch schedules: read at
                                 creation, appended by cc_batch_tune. NULL =
                                 the CCMI_TUNE_CACHE environment variable (if
                                 set), "" = no file (memory only)              */
    uint32_t batch_autotune;  /* 1: cc_batch tunes (cc_batch_tune, 3 timed runs
                                 per candidate) a batch whose shape has no
                                 stored pick before it runs it; 0: such a batch
                                 takes the default schedule                     */
    uint32_t reserved;        /* 0 */
} cc_ctx_opts;

/* Create a context on a device: it owns scratch memory (status word, zero
   root selection state, a sampled-degree hash table, per-block minima) and
   pinned host staging, and grows on demand what larger solves need: the
   zero-root membership bitmap (n/8 bytes), the buffers of the regrouped hooks
   (about 14 bytes per entry), the CSR tile tables and the batch work list.
   opts may be NULL (defaults). */
int cc_create(cc_ctx** out, const cc_ctx_opts* opts);
/* Release a context and everything it owns. Waits for its work to finish. */
void cc_destroy(cc_ctx* ctx);

/* ---- single graph --------------------------------------------------------- */

/*
 * Label the components of one graph (plain path, Algorithm 1 with path
 * splitting), synchronously, on the current device's default context and the
 * null stream.
 *   n          vertex count (IDs are 0..n-1), n <= 2^32-1; n == 0 is a no-op
 *   m          number of entries (unordered pairs)
 *   edge_list  device, 2*m uint32, read only; may be NULL iff m == 0
 *   L          device, n uint32, written: L_v = min ID of v's component;
 *              may be NULL iff n == 0. L doubles as the parent array.
 * Returns CC_OK, CC_EINVAL, CC_ERANGE (an endpoint >= n), CC_EDEVICE.
 */
int cc_solve(uint64_t n, uint64_t m, const uint32_t* edge_list, uint32_t* L);

/* ---- per-call status -------------------------------------------------------
 * The outcome of one asynchronous whole-path call (cc_solve_async,
 * cc_solve_csr, cc_solve_u64) that was given a cc_status_t. The caller owns
 * the struct; the library fills it when the call is enqueued (its fields are
 * the library's), and cc_status_wait resolves it. Each such call ends its
 * stream work by moving the context's status word into one record of a ring
 * of CC_STATUS_RING records kept by the context (pinned host memory), so the
 * outcome belongs to that call alone even when several calls are queued on
 * one stream before anyone waits. */
#define CC_STATUS_RING 256
typedef struct cc_status_t {
    cc_ctx*  ctx;     /* the context of the call                                */
    uint64_t seq;     /* the call's number on its context (from 1; 0 = unset)  */
    uint32_t slot;    /* its record in the context's ring                      */
    uint32_t pad;
} cc_status_t;

/* Wait until the stream work of the call that filled *st has completed and
   return that call's outcome: CC_OK, CC_ERANGE (an endpoint >= n; its labels
   are unspecified) or CC_EINVAL (CSR offsets that are not a valid row index).
   The outcome covers what the call enqueued plus any step calls queued on the
   same context since the previous outcome was taken (by another such call or
   by cc_sync). timeout_us < 0 waits without limit; CC_ETIMEDOUT when the work
   has not completed in time (wait again later). A status may be waited for
   any number of times until CC_STATUS_RING later calls with a status on the
   same context have reused its record (then CC_EINVAL). The context must
   outlive the wait. */
int cc_status_wait(cc_status_t* st, int64_t timeout_us);

/*
 * Enqueue the whole path on `stream` and return without waiting:
 * init (Algorithm 1 / 3 initialisation), [zero root + Initial Push when
 * CC_F_ZROOT], hook (one pass over the entries), compress (pointer jumping)
 * and, with CC_F_ZROOT, the min-ID relabelling of the zero root's component.
 * Argument errors are returned at once. Out-of-range endpoints are reported
 * through `st` when it is not NULL (cc_status_wait), otherwise they stay in
 * the context's status word for the next cc_sync.
 * Buffers must stay valid until the stream reaches the end of this work.
 * Solves queued on one context share its scratch and zero-root state: queue
 * them on one stream, or use one context per concurrent stream.
 */
int cc_solve_async(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edge_list,
                   uint32_t* L, uint32_t flags, uint32_t zroot_hint, void* stream,
                   cc_status_t* st);

/* The whole path on CSR input: row u of the graph holds the entries
   (u, adj[j]) for j in [offsets[u], offsets[u+1]), unordered pairs as in the
   COO form (a symmetric CSR lists each edge twice, which is allowed; no
   symmetry is needed, Sec. II). With CC_F_ZROOT the zero root is the vertex
   with the longest row, ties to the lowest ID (Algorithm 4 reads degrees from
   CSR; CC_F_ZROOT_HINT uses zroot_hint instead), and the Initial Push covers
   its whole row. Rows are hooked in order, so runs of entries share their
   first endpoint's parent reads; within the limits of CC_F_NO_TILE's
   regrouped hooks, the zero-root solve instead takes the regrouped hook with
   the rows of each vertex range as its first-endpoint buckets (CC_F_NO_TILE
   keeps the direct one).
     n        vertices, < 2^32
     offsets  device, n+1 uint64, non-decreasing, offsets[0] = 0; m =
              offsets[n] is read back (the call waits for `stream` once, before
              enqueueing)
     adj      device, m uint32 (each < n; others set CC_ERANGE at cc_sync)
     L        device, n uint32, written: L_v = smallest vertex ID of v's
              component
   Offsets that are not a valid row index make the next cc_sync return
   CC_EINVAL (labels unspecified; no access leaves the arrays). Asynchronous
   after the read-back; status through `st` (cc_status_wait) when it is not
   NULL, else through cc_sync. */
int cc_solve_csr(cc_ctx* ctx, uint64_t n, const uint64_t* offsets, const uint32_t* adj, uint32_t* L,
                 uint32_t flags, uint32_t zroot_hint, void* stream, cc_status_t* st);

/* The plain path (Algorithm 1: init, hook with path splitting, pointer
   jumping) with 8-byte vertex IDs, for vertex counts at and beyond 2^32
   (Sec. V switches to 8-byte IDs there).
     n      vertices, < 2^62 (P takes 8n bytes of device memory)
     edges  device, 2*m uint64 as (u_i, v_i) pairs, each < n (others set
            CC_ERANGE at cc_sync and are skipped)
     L      device, n uint64, written: L_v = smallest ID of v's component
     flags  CC_F_NO_SPLIT and CC_F_SYMMETRIC (anything else: CC_EINVAL)
   Asynchronous on `stream`; status through `st` (cc_status_wait) when it is
   not NULL, else through cc_sync. */
int cc_solve_u64(cc_ctx* ctx, uint64_t n, uint64_t m, const uint64_t* edges, uint64_t* L,
                 uint32_t flags, void* stream, cc_status_t* st);

/* Wait for `stream`, then return (and clear) the status accumulated by the
   context's work since the previous cc_sync (or since the last call whose
   outcome went to a cc_status_t): CC_OK, CC_ERANGE, CC_ENOMEM
   (an update log of cc_hook_log ran out of capacity) or CC_EINVAL (CSR
   offsets of cc_solve_csr were not a valid row index). */
int cc_sync(cc_ctx* ctx, void* stream);

/* ---- the steps, one entry point each (asynchronous on `stream`) ----------
 * Precondition of cc_push, cc_hook and cc_compress: P holds a parent forest
 * made by the preceding steps on the same n (every entry < n). Any other
 * content of P is undefined behaviour (the walks follow whatever P holds).  */

/* Algorithm 1 / 3 initialisation: P_v = v for v < n (P holds vertex IDs; a
   vertex is a root iff P_v == v). Also resets the zero-root relabelling
   state. P: device, n uint32, written. */
int cc_init(cc_ctx* ctx, uint64_t n, uint32_t* P, void* stream);

/* Zero root selection (Algorithm 4 max_degree; Sec. IV Zero Planting).
   Sampled (default): entries i_j = floor(j*m/K), j < K (all entries when
   m <= K, K = zroot_samples); exact (CC_F_ZROOT_EXACT): all entries. The
   root is the vertex with the most endpoint occurrences among those entries
   that are not self-loops, ties to the lowest ID; vertex 0 when nothing is
   counted. CC_F_ZROOT_HINT stores zroot_hint instead. The choice stays in
   the context (read it with cc_get_zroot). edges: device, 2*m uint32. */
int cc_zroot(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t flags,
             uint32_t zroot_hint, void* stream);

/* Initial Push (Algorithm 4 initial-push loop): for every entry of the
   zero-root sample with exactly one endpoint equal to the zero root z, the
   other endpoint x gets P_x = z. Run after cc_init and cc_zroot, before
   cc_hook. P: device, n uint32, updated in place. */
int cc_push(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
            void* stream);

/* Hooking (Algorithm 1 / 3 hooking loop): one pass over the m entries; per
   entry both roots are found (with path splitting unless CC_F_NO_SPLIT) and
   the root of greater key is linked under the other by compare-and-swap,
   retrying from the value the failed CAS returns. key(x) = x, or with
   CC_F_ZROOT key(z) = 0 and key(x) = x + 1 (R of Formula 1). With
   CC_F_ZROOT the context also keeps a membership bitmap of the vertices
   known to be connected to z: an entry with both endpoints in it is skipped,
   and an entry with exactly one endpoint in it only adds the other endpoint
   (that bit is the entry's link to z). After a CC_F_ZROOT
   hook the components are therefore given by P and the bitmap together;
   cc_compress with CC_F_ZROOT resolves both. Requires cc_init then cc_zroot
   on the same n (else CC_EINVAL). Out-of-range endpoints set the status word
   and are skipped. */
int cc_hook(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
            uint32_t flags, void* stream);

/* Hooking with SiskinCC's update log (Sec. III, Algorithm 2): the plain-path
   hook of cc_hook (key = ID; CC_F_ZROOT is rejected with CC_EINVAL), which
   also appends a message (r, p) each time a root r is linked under p. A
   vertex's parent is set by a link at most once (non-roots are never linked),
   so after cc_init and any sequence of cc_hook_log calls the log holds each
   vertex other than its component's lowest ID at most once, n minus the
   number of components in all; taken as edges, the messages connect exactly
   what the processed entries connect. The order is that of the links on the
   device (schedule-dependent).
     log        device, 2*log_cap uint32, owned by the caller; message i is
                log[2i] (the linked root), log[2i+1] (its new parent)
     log_count  device, one uint64, owned by the caller: the number of
                messages already in the log. The call appends at that index
                and adds its own count (set it to 0 before the first call).
                Messages past log_cap are counted but not written, and the
                next cc_sync returns CC_ENOMEM.
   log and log_count are complete when the stream reaches the end of the
   call. Other arguments and errors as for cc_hook. */
int cc_hook_log(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                uint32_t flags, uint32_t* log, uint64_t log_cap, uint64_t* log_count,
                void* stream);

/* cc_hook_log with the messages sent on while the pass runs (Sec. III:
   SiskinCC sends its updates as it makes them, not after its pass). The entries
   are hooked in `chunks` consecutive launches on `stream` (entries
   [k*ceil(m/chunks), ...) in launch k), all enqueued at once; after each, the
   messages that launch appended are copied, on the context's own copy stream,
   from `log` into host_log while the later launches run (R-MAT-26, 8 launches:
   the 265 MB of messages arrive 0.3 ms after the last launch ends, against
   5 ms for one copy after a single logged launch).
     log, log_cap    device, the messages as they are made (as cc_hook_log;
                     log_cap >= n - 1 holds every message a solve can make)
     host_log        host, 2*host_cap uint32, owned by the caller: message i is
                     host_log[2i], host_log[2i+1] once the call returns. Pinned
                     memory (hipHostMalloc, torch pin_memory) lets the copies
                     overlap the launches; pageable memory works but does not
     chunks          1..CC_DRAIN_MAX_CHUNKS
     n_messages      host, out: the messages of this call (the context's own
                     counter starts at 0)
   Synchronous: returns when every message is in host_log. CC_ENOMEM when the
   messages exceed min(log_cap, host_cap) (the first that many are delivered).
   Other arguments and errors as for cc_hook_log (an endpoint >= n: the next
   cc_sync returns CC_ERANGE). */
#define CC_DRAIN_MAX_CHUNKS 1024
int cc_hook_log_drain(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                      uint32_t flags, uint32_t* log, uint64_t log_cap, uint32_t* host_log,
                      uint64_t host_cap, uint32_t chunks, uint64_t* n_messages, void* stream);

/* Pointer jumping (Algorithm 1 / 3 final loop): P_v <- root of v for every
   v. On the plain path the result is the min-ID labelling. With CC_F_ZROOT
   (requires cc_init then cc_zroot on the same n, else CC_EINVAL) a tree that
   holds a vertex of the membership bitmap is z's component: its members get
   P_v = z, and the smallest member of z's component is recorded for
   cc_canon; with CC_F_CANON as well they get that smallest ID at once. */
int cc_compress(cc_ctx* ctx, uint64_t n, uint32_t* P, uint32_t flags, void* stream);

/* Relabelling of the zero root's component (CC_F_ZROOT only): L_v == z is
   replaced by the smallest ID of z's component recorded by cc_compress. */
int cc_canon(cc_ctx* ctx, uint64_t n, uint32_t* L, void* stream);

/* Synchronously read the context's current zero root (after cc_zroot). */
int cc_get_zroot(cc_ctx* ctx, void* stream, uint32_t* zroot_out);

/* ---- exchange between edge shares (Reducer emulation on one device) --------
 * Sec. III (SiskinCC, high-level algorithm): every machine processes its share
 * of the edges into its own global-size P, then sends the pairs (v, P_v) with
 * P_v != v to a Reducer, which processes them like edges and ends with pointer
 * jumping. Sec. IV (RobinCC): vertices whose parent is the zero root are sent
 * as the ID alone (zero-converged vertices). Sec. V bounds the volume by
 * min(|E|, (g-1)|V|) pairs for g machines.                                    */

/* Export of one share's parent array after cc_compress (so P_v is v's root,
   or the zero root z for its component when the share was solved with
   CC_F_ZROOT). For every v < n with P_v != v: if P_v == zroot, v goes to
   zero_ids; otherwise the pair (v, P_v) goes to pairs. zroot = 0xFFFFFFFF sends
   every non-root as a pair. Both lists are written in increasing v.
     P        device, n uint32, read
     pairs    device, 2*pairs_cap uint32, written (may be NULL if pairs_cap == 0)
     zero_ids device, zero_cap uint32, written (may be NULL if zero_cap == 0)
     n_pairs, n_zero  host, the counts (always set on CC_OK and on CC_ENOMEM)
   Synchronous on `stream`. CC_ENOMEM (nothing written) when a count exceeds its
   capacity: call again with larger buffers. */
int cc_export(cc_ctx* ctx, uint64_t n, const uint32_t* P, uint32_t zroot, uint32_t* pairs,
              uint64_t pairs_cap, uint32_t* zero_ids, uint64_t zero_cap, uint64_t* n_pairs,
              uint64_t* n_zero, void* stream);

/* The Reducer side of zero-converged messages (Algorithm 4's received
   (v, max_degree_vID) pairs): every ids[i] is connected to `target`.
   Without CC_F_ZROOT: the pairs (ids[i], target) are hooked (Algorithm 1,
   key = ID). With CC_F_ZROOT and target equal to the context's zero root
   (cc_init then cc_zroot on the same n): each ids[i] is added to the membership
   bitmap, which is the link to z that cc_compress resolves. With CC_F_ZROOT
   and another target: hooked with the keys of Formula 1.
     ids  device, count uint32 (each < n; out-of-range IDs set CC_ERANGE at
          cc_sync and are skipped)
     P    device, n uint32, updated in place */
int cc_hook_ids(cc_ctx* ctx, uint64_t n, uint64_t count, const uint32_t* ids, uint32_t target,
                uint32_t* P, uint32_t flags, void* stream);

/* Compact vertex IDs of the exchange (Sec. V): an ID below n travels in
   cc_id_bytes(n) = ceil(log2(n) / 8) bytes (1 for n <= 256; at least 1).
   Host-only arithmetic; valid for any n >= 0. */
uint32_t cc_id_bytes(uint64_t n);

/* Encode count IDs as count * id_bytes bytes: ID i occupies bytes
   [i*id_bytes, (i+1)*id_bytes) of out, least significant byte first. Pairs
   are encoded as their 2*count IDs.
     ids       device, count uint32, 4-byte aligned
     id_bytes  1..4 (else CC_EINVAL)
     out       device, count * id_bytes bytes, 4-byte aligned, owned by the
               caller
   An ID >= 2^(8*id_bytes) has only its low bytes written and sets CC_ERANGE
   at the next cc_sync. Asynchronous on `stream`. */
int cc_pack_ids(cc_ctx* ctx, uint64_t count, const uint32_t* ids, uint32_t id_bytes, uint8_t* out,
                void* stream);

/* Decode count IDs written by cc_pack_ids with the same id_bytes.
     in   device, count * id_bytes bytes, 4-byte aligned (nothing past
          count * id_bytes is read)
     ids  device, count uint32, 4-byte aligned, owned by the caller
   Asynchronous on `stream`. */
int cc_unpack_ids(cc_ctx* ctx, uint64_t count, const uint8_t* in, uint32_t id_bytes, uint32_t* ids,
                  void* stream);

/* ---- allocation-free whole path ------------------------------------------- */

/* Bytes of the fixed scratch array behind cc_solve_noalloc (one per device). */
#define CC_NOALLOC_SCRATCH_BYTES (16u << 20)

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops that must not allocate, harnesses that forbid it): the whole
 * path of cc_solve_async (init, [zero root + Initial Push], hook, compress,
 * relabelling), with no allocation at all. Its scratch (status word, zero-root
 * state, a 16,384-entry sampled-degree table, per-block minima, the zero-root
 * membership bitmap) is a fixed array of CC_NOALLOC_SCRATCH_BYTES in the
 * library's device image; each device holds its own copy until the process
 * ends, located at the first call on that device. Every call on a device
 * shares that device's array, so calls that overlap on one device race: queue
 * them on one stream. The hooks are the direct ones (the regrouped hooks'
 * buffers grow with m).
 *   n, m, edge_list, L, zroot_hint, stream   as for cc_solve_async
 *   flags   CC_F_ZROOT, CC_F_ZROOT_HINT, CC_F_NO_SPLIT, CC_F_NO_TILE,
 *           CC_F_SYMMETRIC (CC_F_ZROOT_EXACT or others: CC_EINVAL)
 *   status  device, one int32, owned by the caller (may be NULL): written at
 *           the end of the call's stream work with CC_OK or CC_ERANGE (an
 *           endpoint >= n; labels unspecified)
 * Limits: with CC_F_ZROOT, n <= 8 * (CC_NOALLOC_SCRATCH_BYTES - 557,312)
 * (about 129 M vertices; more: CC_ENOMEM, nothing enqueued); plain: n < 2^32.
 * Asynchronous on `stream`; argument errors are returned at once.
 */
int cc_solve_noalloc(uint64_t n, uint64_t m, const uint32_t* edge_list, uint32_t* L,
                     uint32_t flags, uint32_t zroot_hint, int32_t* status, void* stream);

/* ---- many graphs in one launch ------------------------------------------- */

/*
 * Label G independent graphs with local int32 IDs in one persistent launch.
 *   vtx_off, edge_off  device, G+1 int64 each, non-decreasing, starting at 0
 *   edges              device, 2*edge_off[G] int32: graph g's entries are
 *                      edges[2*edge_off[g] .. 2*edge_off[g+1]) with IDs in
 *                      [0, n_g), n_g = vtx_off[g+1] - vtx_off[g] < 2^31
 *   L                  device, vtx_off[G] int32, written: L[vtx_off[g] + v]
 *                      = smallest local ID of v's component in graph g
 *   status             device, G int32, written: CC_OK or CC_ERANGE per graph
 * The schedule (cc_batch_sched) is the context's choice: the one forced with
 * cc_batch_sched_force if any, else the pick stored for the batch's shape by
 * cc_batch_tune (in this context or in the tune_cache file), else (with
 * batch_autotune) a pick tuned now, else the default schedule.
 * Synchronous: returns after the labels are written.
 * Returns CC_OK when the launch ran (per-graph outcomes are in `status`).
 */
int cc_batch(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
             const int32_t* edges, int32_t* L, int32_t* status, void* stream);

/* The same batch captured once and replayed. Creation does everything of
   cc_batch that needs the host (reads and checks the offsets, builds the
   largest-first work list in its own pinned and device buffers, with the
   schedule cc_batch would take at creation) and captures the rest (the upload
   of the work list, which also resets the work tickets, the whole-device
   launches of multi graphs and the persistent launch) into a hipGraph; each cc_batch_graph_launch
   replays it on `stream` asynchronously, with no host work. The graph keeps
   the pointers it was created with: edges, L and status must stay allocated
   (their contents may change between launches: a replay labels whatever the
   edges hold then) until cc_batch_graph_destroy. Launches of one graph must
   not overlap (they share its work ticket). Errors: as cc_batch at creation;
   CC_EDEVICE if capture or instantiation fails. */
typedef struct cc_batch_graph cc_batch_graph;
int cc_batch_graph_create(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                          const int32_t* edges, int32_t* L, int32_t* status, void* stream,
                          cc_batch_graph** out);
int cc_batch_graph_launch(cc_batch_graph* graph, void* stream);
void cc_batch_graph_destroy(cc_batch_graph* graph);

/* ---- batch schedules and their tuner -------------------------------------- */
/*
 * Where each graph of a batch runs. The method is the same in every role
 * (Algorithm 1 with path splitting, then pointer jumping; labels identical):
 *   multi  multi_min_n > 0 and n >= multi_min_n: the whole device solves the
 *          graph before the persistent launch. Its vertices and its entries
 *          are split into chunks dealt to all workgroups (one launch per step
 *          for all such graphs: init, hook, compress); its parent array is its
 *          label slice in HBM.
 *   wave   n <= min(wave_max_n, CC_BATCH_WAVE_MAX_N) and m <= CC_BATCH_WAVE_MAX_M:
 *          one 64-lane wavefront solves the graph with its parent array in an
 *          8 KB partition of LDS (16-bit entries); a workgroup runs 16 such
 *          graphs at once.
 *   tile   otherwise: one 1,024-thread workgroup solves the graph, its parent
 *          array in LDS (16-bit entries) when n <= 2^16, else in HBM.
 * The persistent launch deals the tile graphs first (largest first), then the
 * wave graphs (largest first); a workgroup out of tile graphs turns to waves.
 */
typedef struct cc_batch_sched {
    uint32_t wave_max_n;      /* 0 = no wave role                               */
    uint32_t multi_min_n;     /* 0 = no multi role                              */
} cc_batch_sched;
#define CC_BATCH_WAVE_MAX_N 4096u
#define CC_BATCH_WAVE_MAX_M 65536u

/* cc_batch with an explicit schedule (NULL: the context's choice, as cc_batch). */
int cc_batch_ex(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                const int32_t* edges, int32_t* L, int32_t* status,
                const cc_batch_sched* sched, void* stream);

/* Force the schedule of the context's later cc_batch calls, captured batches
   and nothing else (a server keeps its own choice); NULL returns the choice to
   the stored picks and the default. */
int cc_batch_sched_force(cc_ctx* ctx, const cc_batch_sched* sched);

#define CC_TUNE_MAX_CAND 16
#define CC_SCHED_DEFAULT 0u   /* no pick stored for the shape                   */
#define CC_SCHED_TUNED   1u   /* timed by this call                             */
#define CC_SCHED_STORED  2u   /* a pick stored earlier (this context or the file) */
#define CC_SCHED_FORCED  3u   /* cc_batch_sched_force                           */
typedef struct cc_batch_tune_result {
    cc_batch_sched pick;                    /* the schedule cc_batch now takes   */
    uint32_t source;                        /* CC_SCHED_*                        */
    uint32_t n_cand;                        /* candidates timed (0 if reps == 0) */
    cc_batch_sched cand[CC_TUNE_MAX_CAND];
    float cand_ms[CC_TUNE_MAX_CAND];        /* best of reps, milliseconds        */
    char signature[320];                    /* the shape key, NUL-terminated     */
} cc_batch_tune_result;

/*
 * Tune the schedule for this batch's shape. The shape key is the device (its
 * architecture name and compute-unit count) and the batch's size histogram:
 * for each power-of-two range of n, the bit length of the graph count and of
 * the mean entries per vertex (times 2) in that range. With reps > 0 every
 * candidate (wave_max_n in {0, 256, 1024, 4096} x multi_min_n in {0, 2^14,
 * 2^16 + 1, 2^18}, those that place the graphs differently for this batch)
 * runs once untimed and reps times timed (HIP events on `stream`, from the
 * upload of the work list to the end of the launch); the fastest becomes the
 * stored pick for the shape, in the context and appended to the tune_cache
 * file if there is one. Every run writes L and status as cc_batch would.
 * With reps == 0 nothing runs: `out` reports the schedule cc_batch would take
 * and its source. Synchronous. Errors: as cc_batch; CC_EDEVICE if the cache
 * file cannot be appended (the pick is still stored in the context).
 */
int cc_batch_tune(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                  const int32_t* edges, int32_t* L, int32_t* status, uint32_t reps,
                  cc_batch_tune_result* out, void* stream);

/* ---- continuous-batching server ------------------------------------------- */
typedef struct cc_server cc_server;

typedef struct cc_serve_opts {
    uint32_t max_inflight;     /* requests resident on the device at once; 0 = 64   */
    uint32_t queue_capacity;   /* submitted but not yet admitted; 0 = 4096           */
    uint32_t streams;          /* HIP streams used for overlap; 0 = 4                */
    uint32_t small_n;          /* requests with n <= small_n go to batched launches;
                                  0 = 65536                                          */
    uint64_t hbm_budget;       /* bytes of device memory the server may hold; 0 =
                                  the context's budget                              */
    uint32_t coalesce_us;      /* coalescing window: small ready requests wait until
                                  the oldest of them has been ready this long (or
                                  half a staging buffer has gathered) so that later
                                  arrivals join the same batched launch; 0 = none   */
    uint32_t reserved;         /* 0 */
} cc_serve_opts;

typedef struct cc_req_stats {
    int32_t  status;          /* the request's outcome (CC_OK, CC_ERANGE, ...)       */
    uint32_t batched;         /* 1 if it ran inside a batched launch                 */
    uint64_t t_submit_ns;     /* CLOCK_MONOTONIC timestamps: submitted,               */
    uint64_t t_admit_ns;      /* admitted (memory or a batch place granted),          */
    uint64_t t_start_ns;      /* its device work started (a worker took it),          */
    uint64_t t_done_ns;       /* labels in host memory                                */
} cc_req_stats;

/* Start a server thread on ctx's device. */
int cc_serve_open(cc_ctx* ctx, const cc_serve_opts* opts, cc_server** out);

/*
 * Submit one request (non-blocking). edges_host: 2*m uint32 in host memory,
 * L_host: n uint32 in host memory; both stay owned by the caller and must
 * remain valid until cc_serve_wait returns for this ticket. Admission waits
 * until the request's device footprint fits the budget: 8m + 4n bytes (edges,
 * labels) plus the scratch its solve needs (the zero-root bitmap, the
 * regrouped hook's buffers), all taken from the server's arena, so serving
 * allocates nothing per request. Small requests (n <= small_n) go to batched
 * launches through per-worker staging instead. flags: CC_F_ZROOT,
 * CC_F_ZROOT_EXACT, CC_F_NO_SPLIT, CC_F_NO_TILE, CC_F_SYMMETRIC (applied on the
 * single-graph path; batched requests take the plain path, same labels).
 * Returns CC_EAGAIN when the queue is full, CC_ENOMEM when the request alone
 * exceeds the budget, CC_EINVAL for bad arguments.
 */
int cc_serve_submit(cc_server* srv, uint64_t n, uint64_t m, const uint32_t* edges_host,
                    uint32_t* L_host, uint32_t flags, uint64_t* ticket);

/* Wait up to timeout_us (< 0: forever) for a ticket; fills stats if non-NULL
   and returns the request's status, or CC_ETIMEDOUT. A ticket can be waited
   for once. */
int cc_serve_wait(cc_server* srv, uint64_t ticket, int64_t timeout_us, cc_req_stats* stats);

/* Stop accepting requests, finish everything admitted, cancel what is still
   queued (their wait returns CC_ECANCELED), join the thread, free. */
int cc_serve_close(cc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* CCMI_CC_H */
