// Host-side check of the autotuner's on-disk cache (librad's autotune.cpp):
// "write PATH" stores three fixed entries; "read PATH" prints every entry it
// accepts as "key tn persistent blocks_per_cu ms".  No HIP call is made.
#include "autotune.cpp"

#include <cstdio>
#include <cstring>

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    const std::string path = argv[2];
    if (!std::strcmp(argv[1], "write")) {
        std::map<std::string, rad::CacheEntry> m;
        m["sigA|R=1024"] = rad::CacheEntry{rad::MmConfig{64, 1, 4}, 0.123456};
        m["sigA|R=256"] = rad::CacheEntry{rad::MmConfig{128, 0, 0}, 1.5};
        m["sigB|R=64"] = rad::CacheEntry{rad::MmConfig{256, 1, 2}, 26.308218};
        rad::write_cache(path, m);
        return 0;
    }
    for (const auto &kv : rad::read_cache(path))
        std::printf("%s %d %d %d %.6f\n", kv.first.c_str(), kv.second.c.tn, kv.second.c.persistent,
                    kv.second.c.blocks_per_cu, kv.second.ms);
    return 0;
}
