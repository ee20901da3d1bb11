// Tuning of the persistent batched solve.
//
// The launch configuration (threads per workgroup, edges per thread and
// load round, dynamic LDS per workgroup) is picked per batch shape by
// timing every candidate on a sample of the batch.  The choice is cached
// per (architecture, log2 of the mean vertex count, log2 of the mean stored
// entries per vertex, weight type), in memory for the process and, when
// MSF_TUNE_CACHE names a file, in that file across processes (one line per
// shape: arch nb db wt candidate).  MSF_BATCH_CONFIG=<index> forces a
// candidate.  Every candidate computes the same forests (the result does
// not depend on the schedule); only the time differs.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "msf_internal.hpp"
#include "persist.hpp"

namespace msf {

namespace {

using Key = std::tuple<std::string, int, int, int>;

std::mutex g_mu;
std::map<Key, int> g_cache;
bool g_loaded = false;

const char *cache_path() { return getenv("MSF_TUNE_CACHE"); }

void load_cache()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char arch[64];
    int nb, db, wt, idx;
    while (fscanf(f, "%63s %d %d %d %d", arch, &nb, &db, &wt, &idx) == 5)
        g_cache[Key(arch, nb, db, wt)] = idx;
    fclose(f);
}

void store_cache(const Key &k, int idx)
{
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), idx);
    fclose(f);
}

// The device's architecture name, queried once per device (the full
// property query costs far more than a batch's host-side set-up).
std::string arch_of(int device)
{
    static std::mutex mu;
    static std::map<int, std::string> known;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(device);
    if (it != known.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    a = colon == std::string::npos ? a : a.substr(0, colon);
    known[device] = a;
    return a;
}

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

}  // namespace

bool persist_cfg_fits(int device, const PersistCfg &cfg)
{
    int maxlds = 0;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
        hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    // room for the kernel's own static LDS (under 2 KB)
    return (int)cfg.lds + 4096 <= maxlds;
}

msf_status persist_pick(Ctx *c, const BatchShape &shape, int wt, const PersistTuneRun &run,
                        int *chosen)
{
    int ncand = 0;
    const PersistCfg *cand = persist_candidates(&ncand);
    if (const char *f = getenv("MSF_BATCH_CONFIG")) {
        const int i = atoi(f);
        if (i < 0 || i >= ncand || !persist_cfg_fits(c->device, cand[i])) {
            set_error("MSF_BATCH_CONFIG=%d: no such candidate on this device", i);
            return MSF_EINVAL;
        }
        *chosen = i;
        return MSF_OK;
    }
    const Key key(arch_of(c->device), ilog2(shape.mean_n), ilog2(shape.mean_deg), wt);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache();
        auto it = g_cache.find(key);
        if (it != g_cache.end() && it->second >= 0 && it->second < ncand &&
            persist_cfg_fits(c->device, cand[it->second])) {
            *chosen = it->second;
            return MSF_OK;
        }
    }
    // time every candidate that fits this device on the sample, twice each
    // (the first run also warms the sample's data), and keep the fastest
    int best = -1;
    float best_ms = 0.f;
    for (int i = 0; i < ncand; ++i) {
        if (!persist_cfg_fits(c->device, cand[i])) continue;
        float ms = 0.f;
        MSF_TRY(run(i, nullptr));
        MSF_TRY(run(i, &ms));
        if (best < 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    if (best < 0) {
        set_error("no persistent configuration fits this device");
        return MSF_EDEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_cache.find(key) == g_cache.end()) {
            g_cache[key] = best;
            store_cache(key, best);
        }
    }
    *chosen = best;
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

extern "C" int msf_batch_configs(int32_t *nt, int32_t *ept, int32_t *lds_bytes, int32_t cap)
{
    int ncand = 0;
    const PersistCfg *cand = persist_candidates(&ncand);
    for (int i = 0; i < ncand && i < cap; ++i) {
        if (nt) nt[i] = cand[i].nt;
        if (ept) ept[i] = cand[i].ept;
        if (lds_bytes) lds_bytes[i] = (int32_t)cand[i].lds;
    }
    return ncand;
}
