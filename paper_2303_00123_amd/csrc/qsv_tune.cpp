// Autotuner cache for batch tile shapes: an in-context map from batch shape
// key to (tile_bits, low_bits), optionally persisted as one JSON object per
// line in the file named by QSV_TUNE_CACHE, keyed by GPU architecture.
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "qsv_internal.h"

namespace qsv {

bool log_enabled() {
    static const int on = [] {
        const char* v = std::getenv("QSV_LOG");
        return (v && *v && std::strcmp(v, "0") != 0) ? 1 : 0;
    }();
    return on != 0;
}

void logf(const char* fmt, ...) {
    if (!log_enabled()) return;
    std::va_list ap;
    va_start(ap, fmt);
    std::fputs("[qsv] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

static std::string arch_name(qsv_ctx ctx) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, ctx->device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static uint64_t full_key(uint64_t key, int dtype) { return key ^ (uint64_t(dtype) << 60); }

static void load_cache(qsv_ctx ctx) {
    ctx->tune_loaded = true;
    const char* path = std::getenv("QSV_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = arch_name(ctx);
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char a[64] = {0};
        unsigned long long key = 0;
        int dtype = 0, tb = 0, lb = 0;
        if (std::sscanf(line, " {\"arch\": \"%63[^\"]\", \"key\": \"%llx\", \"dtype\": %d, \"tile_bits\": %d, \"low_bits\": %d",
                        a, &key, &dtype, &tb, &lb) == 5 &&
            arch == a && tb >= kMinTileBits && tb <= kMaxTileBits && lb >= 0 && lb <= tb - 2)
            ctx->tuned[full_key(key, dtype)] = std::make_pair(tb, lb);
    }
    std::fclose(f);
}

bool tune_lookup(qsv_ctx ctx, uint64_t key, int dtype, int* tile_bits, int* low_bits) {
    if (!ctx->tune_loaded) load_cache(ctx);
    auto it = ctx->tuned.find(full_key(key, dtype));
    if (it == ctx->tuned.end()) return false;
    *tile_bits = it->second.first;
    *low_bits = it->second.second;
    return true;
}

void tune_store(qsv_ctx ctx, uint64_t key, int dtype, int tile_bits, int low_bits, double ms) {
    ctx->tuned[full_key(key, dtype)] = std::make_pair(tile_bits, low_bits);
    const char* path = std::getenv("QSV_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"key\": \"%016llx\", \"dtype\": %d, \"tile_bits\": %d, "
                 "\"low_bits\": %d, \"ms\": %.4f}\n",
                 arch_name(ctx).c_str(), static_cast<unsigned long long>(key), dtype, tile_bits,
                 low_bits, ms);
    std::fclose(f);
}

}  // namespace qsv
