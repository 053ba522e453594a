// tune_cache.cpp -- persistent tuning choices.
//
// The paper chooses its block depths by experiment on the target machine.
// Here the tuners measure on the device they run on; this file keeps what
// they find in a text file, so that later processes start from it.  One
// entry per line, fields separated by single spaces:
//
//   mgemm-tune v1 single <arch> <cus> <version> <precision> <trans> <M> <N> <K> <config>
//   mgemm-tune v1 grouped <arch> <cus> <version> <precision> <batch> <c0>,<c1>,<c2>,<c3>
//
// <arch> is the device's architecture name (e.g. gfx950) and <cus> its
// compute-unit count ("nodevice" and 0 when no device is visible), <version>
// is mgemm_version(), <trans> two letters (NN, NT, TN, TT), <batch> a 16-hex-
// digit FNV-1a hash of a grouped batch's count and its problems' trans
// flags and sizes, in order.  Only entries whose arch, cus and version match
// the current device and library are used; of several for one key the last
// wins.  Lines are appended, each with one write, so processes may share a
// file; unreadable lines are skipped.
#include <hip/hip_runtime.h>

#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <string>

#include "host_common.hpp"
#include "mgemm.h"

namespace mgemm {

static const char* TAG = "mgemm-tune v1";

void device_key(std::string& arch, int& cus) {
    arch = "nodevice";
    cus = 0;
    int count = 0, dev = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    arch.assign(prop.gcnArchName, strcspn(prop.gcnArchName, ": "));
    cus = prop.multiProcessorCount;
}

uint64_t batch_key(const mgemm_problem* probs, int64_t count) {
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ULL;
        }
    };
    mix((uint64_t)count);
    for (int64_t i = 0; i < count; ++i) {
        mix((uint64_t)(trans_code(probs[i].transA) & 3) | ((uint64_t)(trans_code(probs[i].transB) & 3) << 2));
        mix((uint64_t)probs[i].M);
        mix((uint64_t)probs[i].N);
        mix((uint64_t)probs[i].K);
    }
    return h;
}

static bool append_line(const char* path, const std::string& line) {
    std::FILE* f = std::fopen(path, "a");
    if (!f) return false;
    const bool ok = std::fwrite(line.data(), 1, line.size(), f) == line.size();
    return std::fclose(f) == 0 && ok;
}

// Calls fn(kind, fields after the device key) for every line whose device
// key matches.  Returns false when the file cannot be opened.
template <class Fn>
static bool scan(const char* path, const std::string& arch, int cus, Fn&& fn) {
    std::FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    const std::string head = std::string(TAG) + " ";
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, head.c_str(), head.size()) != 0) continue;
        char kind[16], a[64];
        int c = 0, ver = 0, used = 0;
        if (std::sscanf(line + head.size(), "%15s %63s %d %d %n", kind, a, &c, &ver, &used) < 4)
            continue;
        if (arch != a || cus != c || ver != mgemm_version()) continue;
        fn(std::string(kind), line + head.size() + used);
    }
    std::fclose(f);
    return true;
}

bool grouped_cache_lookup(const char* path, int precision, uint64_t key, int* configs) {
    std::string arch;
    int cus = 0;
    device_key(arch, cus);
    bool found = false;
    scan(path, arch, cus, [&](const std::string& kind, const char* rest) {
        if (kind != "grouped") return;
        int prec = -1, c[4];
        uint64_t k = 0;
        if (std::sscanf(rest, "%d %" SCNx64 " %d,%d,%d,%d", &prec, &k, &c[0], &c[1], &c[2],
                        &c[3]) != 6)
            return;
        if (prec != precision || k != key) return;
        for (int b = 0; b < 4; ++b) configs[b] = c[b];
        found = true;
    });
    return found;
}

bool grouped_cache_store(const char* path, int precision, uint64_t key, const int* configs) {
    std::string arch;
    int cus = 0;
    device_key(arch, cus);
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s grouped %s %d %d %d %016" PRIx64 " %d,%d,%d,%d\n", TAG,
                  arch.c_str(), cus, mgemm_version(), precision, key, configs[0], configs[1],
                  configs[2], configs[3]);
    return append_line(path, buf);
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int mgemm_save_choices(const char* path) {
    if (!path) return fail(MGEMM_ERR_UNSUPPORTED, "path is NULL");
    std::string arch;
    int cus = 0;
    device_key(arch, cus);
    std::string out;
    for_each_choice([&](int precision, int ta, int tb, int64_t M, int64_t N, int64_t K, int cfg) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "%s single %s %d %d %d %c%c %" PRId64 " %" PRId64 " %" PRId64 " %d\n", TAG,
                      arch.c_str(), cus, mgemm_version(), precision, ta ? 'T' : 'N',
                      tb ? 'T' : 'N', M, N, K, cfg);
        out += buf;
    });
    if (out.empty()) return MGEMM_OK;
    if (!append_line(path, out)) return fail(MGEMM_ERR_UNSUPPORTED, std::string("cannot write ") + path);
    return MGEMM_OK;
}

int mgemm_load_choices(const char* path, int64_t* loaded) {
    if (loaded) *loaded = 0;
    if (!path) return fail(MGEMM_ERR_UNSUPPORTED, "path is NULL");
    std::string arch;
    int cus = 0;
    device_key(arch, cus);
    int64_t n = 0;
    const bool opened = scan(path, arch, cus, [&](const std::string& kind, const char* rest) {
        if (kind != "single") return;
        int prec = -1, cfg = -1;
        char tr[3] = {0, 0, 0};
        int64_t M = 0, N = 0, K = 0;
        if (std::sscanf(rest, "%d %2s %" SCNd64 " %" SCNd64 " %" SCNd64 " %d", &prec, tr, &M, &N,
                        &K, &cfg) != 6)
            return;
        if (mgemm_record_choice(prec, tr[0], tr[1], M, N, K, cfg) == MGEMM_OK) ++n;
    });
    if (!opened) return fail(MGEMM_ERR_UNSUPPORTED, std::string("cannot read ") + path);
    if (loaded) *loaded = n;
    return MGEMM_OK;
}

}  // extern "C"
