// Autotuning cache (host code): shapes found by timing, keyed by device
// architecture and workload signature, kept in a plain text file.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "mm_host.h"

namespace mmh {

namespace {
std::mutex g_cache_mu;

const char* cache_path() {
    const char* p = std::getenv("MM_TUNE_CACHE");
    return p && *p ? p : nullptr;
}
}  // namespace

bool tune_cache_lookup(const std::string& key, uint32_t out[kTuneValues]) {
    const char* path = cache_path();
    if (!path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string k;
        uint32_t v[kTuneValues];
        if (!(ss >> k)) continue;
        bool ok = true;
        for (int j = 0; j < kTuneValues && ok; ++j) ok = static_cast<bool>(ss >> v[j]);
        if (!ok) continue;
        if (k == key) {
            for (int j = 0; j < kTuneValues; ++j) out[j] = v[j];
            found = true;  // keep reading: the last entry wins
        }
    }
    return found;
}

void tune_cache_store(const std::string& key, const uint32_t v[kTuneValues]) {
    const char* path = cache_path();
    if (!path) return;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::ofstream out(path, std::ios::app);
    if (!out) return;
    out << key;
    for (int j = 0; j < kTuneValues; ++j) out << ' ' << v[j];
    out << '\n';
}

std::string device_arch(int device) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "";
    std::string a = p.gcnArchName;
    for (char& c : a)
        if (c == ' ') c = '_';
    return a;
}

}  // namespace mmh
