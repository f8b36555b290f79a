// cc_tune.hip — the batch schedule tuner.
//
// A schedule (cc_batch_sched) assigns each graph of a batch a role: whole
// device, one wavefront, or one workgroup (cc_batch.hip). Which assignment is
// fastest depends on the size mix and on the device, so the tuner measures it:
// every candidate that places the graphs differently runs on the batch itself,
// timed with HIP events, and the fastest is stored under a key made of the
// device (architecture name, compute-unit count) and the batch's shape (a
// coarse size histogram). Later batches of the same key take the stored pick.
// Picks live in the context and, if a cache file is configured, in that file:
// one text line per pick, appended, read back when a context is created (a
// later line for the same key wins).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "cc_internal.h"

namespace ccm {

static const char kFileTag[] = "ccmi-batch-tune-v1";
static const uint32_t kWaveCand[] = {0u, 256u, 1024u, CC_BATCH_WAVE_MAX_N};
static const uint32_t kMultiCand[] = {0u, 1u << 14, (1u << 16) + 1, 1u << 18};

static int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// "<arch>/<CUs>cu" of a device, read once per device.
static std::string device_key(int device) {
    static std::mutex mu;
    static std::map<int, std::string> keys;
    std::lock_guard<std::mutex> lk(mu);
    auto it = keys.find(device);
    if (it != keys.end()) return it->second;
    hipDeviceProp_t p;
    std::string key = "unknown";
    if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        std::string arch(p.gcnArchName);
        arch = arch.substr(0, arch.find(':'));
        key = arch + "/" + std::to_string(p.multiProcessorCount) + "cu";
    } else {
        (void)hipGetLastError();
    }
    keys[device] = key;
    return key;
}

// The batch's shape: for each bit length b of n present, "b.q.r" with q the bit
// length of the number of such graphs and r that of twice their mean entries
// per vertex. Batches with the same shape differ at most by factors of two in
// each range's count and density.
static std::string signature(uint32_t G, const GraphDesc* d) {
    uint64_t cnt[33] = {}, sn[33] = {}, sm[33] = {};
    for (uint32_t g = 0; g < G; ++g) {
        const int b = bitlen(d[g].n);
        ++cnt[b];
        sn[b] += d[g].n;
        sm[b] += (uint64_t)d[g].m;
    }
    std::string s;
    for (int b = 0; b <= 32; ++b) {
        if (!cnt[b]) continue;
        const uint64_t dens = 2 * sm[b] / std::max<uint64_t>(sn[b], 1);
        if (!s.empty()) s += ',';
        s += std::to_string(b) + "." + std::to_string(bitlen(cnt[b])) + "." +
             std::to_string(bitlen(dens));
    }
    return s.empty() ? std::string("empty") : s;
}

void tuner_open(Tuner* t, const char* path_opt, bool autotune) {
    std::lock_guard<std::mutex> lk(t->mu);
    t->autotune = autotune;
    const char* p = path_opt ? path_opt : std::getenv("CCMI_TUNE_CACHE");
    t->path = p ? p : "";
    if (t->path.empty()) return;
    std::ifstream in(t->path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string tag, dev, sig;
        uint64_t w = 0, mm = 0;
        if (!(ls >> tag >> dev >> sig >> w >> mm) || tag != kFileTag) continue;
        if (w > CC_BATCH_WAVE_MAX_N || mm > 0xFFFFFFFFull) continue;
        BatchSched sc;
        sc.wave_max_n = (uint32_t)w;
        sc.multi_min_n = (uint32_t)mm;
        t->picks[dev + "|" + sig] = sc;
    }
}

// Forced, stored or default schedule (no tuning); caller holds t->mu.
static BatchSched lookup_locked(Tuner* t, const std::string& key, uint32_t* source) {
    if (t->forced) {
        *source = CC_SCHED_FORCED;
        return t->force;
    }
    auto it = t->picks.find(key);
    if (it != t->picks.end()) {
        *source = CC_SCHED_STORED;
        return it->second;
    }
    *source = CC_SCHED_DEFAULT;
    return batch_default_sched();
}

BatchSched tuner_lookup(Tuner* t, int device, uint32_t G, const GraphDesc* descs) {
    const std::string key = device_key(device) + "|" + signature(G, descs);
    std::lock_guard<std::mutex> lk(t->mu);
    auto it = t->picks.find(key);
    return it != t->picks.end() ? it->second : batch_default_sched();
}

int tuner_choose(Tuner* t, Slot* s, uint32_t G, const GraphDesc* descs, hipStream_t stream,
                 BatchSched* out, uint32_t* source) {
    const std::string key = device_key(s->device) + "|" + signature(G, descs);
    bool tune = false;
    {
        std::lock_guard<std::mutex> lk(t->mu);
        *out = lookup_locked(t, key, source);
        tune = *source == CC_SCHED_DEFAULT && t->autotune;
    }
    if (!tune) return CC_OK;
    cc_batch_tune_result r;
    int rc = tuner_tune(t, s, G, descs, 3, stream, &r);
    if (rc) return rc;
    *out = r.pick;
    *source = CC_SCHED_TUNED;
    return CC_OK;
}

int tuner_tune(Tuner* t, Slot* s, uint32_t G, const GraphDesc* descs, uint32_t reps,
               hipStream_t stream, cc_batch_tune_result* out) {
    std::memset(out, 0, sizeof(*out));
    const std::string sig = signature(G, descs);
    const std::string key = device_key(s->device) + "|" + sig;
    std::snprintf(out->signature, sizeof(out->signature), "%s", key.c_str());
    if (reps == 0) {
        std::lock_guard<std::mutex> lk(t->mu);
        out->pick = lookup_locked(t, key, &out->source);
        return CC_OK;
    }
    uint32_t wave_cap = 0;
    int rc = batch_wave_cap(s->device, &wave_cap);
    if (rc) return rc;
    // candidates that place the graphs differently
    std::vector<BatchSched> cands;
    std::vector<std::vector<uint8_t>> placed;
    for (uint32_t mm : kMultiCand) {
        for (uint32_t w : kWaveCand) {
            BatchSched c;
            c.wave_max_n = w;
            c.multi_min_n = mm;
            std::vector<uint8_t> roles(G);
            for (uint32_t g = 0; g < G; ++g) roles[g] = (uint8_t)batch_role(descs[g], c, wave_cap);
            bool dup = false;
            for (const auto& p : placed) dup |= p == roles;
            if (dup) continue;
            placed.push_back(std::move(roles));
            cands.push_back(c);
        }
    }
    hipEvent_t a = nullptr, b = nullptr;
    CCM_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(CC_EDEVICE, "hipEventCreate failed");
    }
    size_t best = 0;
    float best_ms = 0.f;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        // one untimed run (first-use costs), then reps timed ones
        rc = launch_batch(s, G, descs, cands[i], stream);
        if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = fail(CC_EDEVICE, "tuning run failed");
        float ms_best = 0.f;
        for (uint32_t r = 0; r < reps && !rc; ++r) {
            float ms = 0.f;
            if (hipEventRecord(a, stream) != hipSuccess) rc = fail(CC_EDEVICE, "hipEventRecord failed");
            if (!rc) rc = launch_batch(s, G, descs, cands[i], stream);
            if (!rc && (hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&ms, a, b) != hipSuccess))
                rc = fail(CC_EDEVICE, "tuning run timing failed");
            if (!rc && (r == 0 || ms < ms_best)) ms_best = ms;
        }
        if (rc) break;
        if (i < CC_TUNE_MAX_CAND) {
            out->cand[i] = cands[i];
            out->cand_ms[i] = ms_best;
            out->n_cand = (uint32_t)i + 1;
        }
        if (i == 0 || ms_best < best_ms) {
            best = i;
            best_ms = ms_best;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) {
        (void)hipGetLastError();
        return rc;
    }
    const BatchSched pick = cands[best];
    std::lock_guard<std::mutex> lk(t->mu);
    t->picks[key] = pick;
    out->pick = lookup_locked(t, key, &out->source);
    if (out->source == CC_SCHED_STORED) out->source = CC_SCHED_TUNED;
    if (!t->path.empty()) {
        std::FILE* f = std::fopen(t->path.c_str(), "a");
        if (!f) return fail(CC_EDEVICE, "cannot append to the tune cache file " + t->path);
        std::fprintf(f, "%s %s %s %u %u %.4f\n", kFileTag, device_key(s->device).c_str(), sig.c_str(),
                     pick.wave_max_n, pick.multi_min_n, (double)best_ms);
        const bool ok = std::fclose(f) == 0;
        if (!ok) return fail(CC_EDEVICE, "cannot write the tune cache file " + t->path);
    }
    return CC_OK;
}

}  // namespace ccm
