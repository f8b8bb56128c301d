// Autotuner entry points of the multi-RHS kernels: timing of every candidate
// launch configuration on the matrix itself, with an optional on-disk cache
// (a JSON object, one entry per line) keyed by the matrix signature and R.
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>

#include "rad_internal.h"

namespace rad {
namespace {

struct CacheEntry {
    MmConfig c;
    double ms = 0.0;
};

std::map<std::string, CacheEntry> read_cache(const std::string &path) {
    std::map<std::string, CacheEntry> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"'), q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        CacheEntry e;
        int tn = 0, pe = 0, bpc = 0;
        double ms = 0;
        if (std::sscanf(line.c_str() + q1 + 1, ": {\"tn\": %d, \"persistent\": %d, \"blocks_per_cu\": %d, \"ms\": %lf",
                        &tn, &pe, &bpc, &ms) == 4 &&
            (tn == 64 || tn == 128 || tn == 256) && (pe == 0 || pe == 1) && bpc >= 0 && bpc <= 64) {
            e.c = MmConfig{tn, pe, bpc};
            e.ms = ms;
            out[line.substr(q0 + 1, q1 - q0 - 1)] = e;
        }
    }
    return out;
}

void write_cache(const std::string &path, const std::map<std::string, CacheEntry> &m) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        RAD_REQUIRE(f.good(), "cannot write the autotuner cache " + path);
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : m) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "{\"tn\": %d, \"persistent\": %d, \"blocks_per_cu\": %d, \"ms\": %.6f}",
                          kv.second.c.tn, kv.second.c.persistent, kv.second.c.blocks_per_cu, kv.second.ms);
            f << "\"" << kv.first << "\": " << buf << (++i < m.size() ? ",\n" : "\n");
        }
        f << "}\n";
    }
    RAD_REQUIRE(std::rename(tmp.c_str(), path.c_str()) == 0, "cannot replace the autotuner cache " + path);
}

// cached iteration graphs hold the launches of the previous configuration
void clear_graphs(rad_hmat *H) {
    for (auto &g : H->graphs) {
        (void)hipGraphExecDestroy(g.ex);
        (void)hipGraphDestroy(g.g);
    }
    H->graphs.clear();
}

void set_tuned(rad_hmat *H, int64_t R, const MmConfig &c) {
    clear_graphs(H);
    for (auto &e : H->tuned)
        if (e.first == R) {
            e.second = c;
            return;
        }
    H->tuned.push_back({R, c});
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" {

rad_status rad_hmat_autotune(rad_hmat *H, int64_t R, int32_t nrep, const char *cache_path, int32_t *config,
                             double *ms, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(H != nullptr, "null matrix handle");
        RAD_REQUIRE(R >= kMfmaMinRhs && R <= H->max_rhs, "R must be in [16, max_rhs]");
        RAD_REQUIRE(nrep >= 1, "nrep must be >= 1");
        RAD_HIP(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const std::string key = H->sched_sig + "_R" + std::to_string(R);
        std::map<std::string, CacheEntry> cache;
        if (cache_path) cache = read_cache(cache_path);
        auto it = cache.find(key);
        MmConfig best;
        double best_ms = 0.0;
        if (it != cache.end()) {
            best = it->second.c;
            set_tuned(H, R, best);
        } else {
            const size_t bytes = (size_t)H->N * (size_t)mm_ldr(R) * (H->dtype == RAD_F64 ? 8 : 4);
            RAD_HIP(hipMemsetAsync(H->w_x.p, 0, bytes, s));
            RAD_HIP(hipMemsetAsync(H->w_e.p, 0, bytes, s));
            auto res = mm_autotune(H, R, nrep, s);
            clear_graphs(H);
            best = mm_config(H, R);
            for (const auto &r : res)
                if (r.first.tn == best.tn && r.first.persistent == best.persistent &&
                    r.first.blocks_per_cu == best.blocks_per_cu)
                    best_ms = r.second;
            if (cache_path) {
                cache[key] = CacheEntry{best, best_ms};
                write_cache(cache_path, cache);
            }
        }
        if (config) {
            config[0] = best.tn;
            config[1] = best.persistent;
            config[2] = best.blocks_per_cu;
        }
        if (ms) *ms = best_ms;
    });
}

rad_status rad_hmat_set_config(rad_hmat *H, int64_t R, const int32_t *config) {
    return guard([&] {
        RAD_REQUIRE(H != nullptr && config != nullptr, "null matrix handle or config");
        RAD_REQUIRE(R >= kMfmaMinRhs && R <= H->max_rhs, "R must be in [16, max_rhs]");
        RAD_REQUIRE(config[0] == 64 || config[0] == 128 || (config[0] == 256 && H->dtype == RAD_F32),
                    "tn must be 64 or 128 (or 256 for FP32)");
        RAD_REQUIRE(config[1] == 0 || config[1] == 1, "persistent must be 0 or 1");
        RAD_REQUIRE(config[2] >= 1 && config[2] <= 64, "blocks_per_cu must be in [1, 64]");
        set_tuned(H, R, MmConfig{config[0], config[1], config[2]});
    });
}

rad_status rad_hmat_get_config(const rad_hmat *H, int64_t R, int32_t *config) {
    return guard([&] {
        RAD_REQUIRE(H != nullptr && config != nullptr, "null matrix handle or config");
        const MmConfig c = mm_config(H, R);
        config[0] = c.tn;
        config[1] = c.persistent;
        config[2] = c.blocks_per_cu;
    });
}

}  // extern "C"
