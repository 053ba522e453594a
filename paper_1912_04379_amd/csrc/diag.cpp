// diag.cpp -- diagnostics switched on from the environment.  Both variables
// are read at every call, so a process can turn them on and off:
//
//   MGEMM_FAULT=alloc  every workspace, packed-operand or plan allocation
//                      reports failure before anything is launched, so that
//                      callers can exercise their MGEMM_ERR_ALLOC paths;
//   MGEMM_LOG=1        one line per call on stderr: the entry point, its
//                      arguments, the configuration and path taken (or the
//                      status of a rejected call); any other value except
//                      "0" is the path of a file the lines are appended to.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "host_common.hpp"

namespace mgemm {

bool fault_injected() {
    const char* v = std::getenv("MGEMM_FAULT");
    return v && std::strcmp(v, "alloc") == 0;
}

bool log_enabled() {
    const char* v = std::getenv("MGEMM_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
}

static std::mutex g_log_mu;

void log_line(const char* fmt, ...) {
    const char* v = std::getenv("MGEMM_LOG");
    if (!v || !*v || std::strcmp(v, "0") == 0) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(g_log_mu);
    const bool to_stderr = std::strcmp(v, "1") == 0;
    std::FILE* f = to_stderr ? stderr : std::fopen(v, "a");
    if (!f) return;
    std::fprintf(f, "mgemm: %s\n", buf);
    if (to_stderr) std::fflush(f);
    else std::fclose(f);
}

}  // namespace mgemm
