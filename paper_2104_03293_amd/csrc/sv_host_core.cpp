// libsv host: error reporting, plan knobs and launch profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "sv_host.h"

// ============================================================================ errors
static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char* sv_last_error(void) { return g_err.c_str(); }

extern "C" const char* sv_version(void) { return "libsv 0.1.0 (gfx950)"; }


// ============================================================================ knobs
namespace {
std::mutex g_knob_mu;
std::map<std::string, int> g_knobs = {
    {"fuse", 1},      // 1: snake-ordered fused passes; 0: one op per pass
    {"cmin64", 4},    // minimum carrier bits (contiguous run 2^c amplitudes) for complex64
    {"cmin128", 3},   // ... for complex128
    {"ntmin", 4},     // passes whose contiguous runs hold >= 2^ntmin amplitudes stream with nontemporal hints
    {"persist", 0},   // tile passes: workgroups per CU of a persistent grid (0: one workgroup per tile)
    {"stagger", 0},   // persistent grids: start delay of the second half (units of 64*127 clocks)
    {"snake", 1},     // group order of a layer: 1 = B, A, C, ... (the contiguous group A in a middle slot);
                      // 2 = last group first (C, A, B, ...); 0 = A, B, C, ...
    {"dpp", 1},       // 1: one active bit may be butterflied across lanes to save a layout
    {"ldsswz", 4},    // LDS slot swizzle width of the tile passes (3..5)
    {"batchwide", 2}, // complex64 batch scan: 2 = 2^13 LDS states, four waves, two workgroups
                      // per CU; 1 = 2^14 LDS states, eight waves; 0 = 2^14, four waves
    {"batch128", 1},  // complex128 batch scan (2^13 LDS states, one workgroup per CU): 1 = eight
                      // waves, 0 = four
    {"c64t13", 0},    // complex64 one-vector programs: 1 = 13-bit tiles (four waves), 0 = 14-bit tiles
    {"c64occ", 1},    // complex64 14-bit tiles: 1 = no lane position 4, two workgroups per CU
    {"c64g4", 1},     // complex64 two-vector passes: 1 = four waves per SIMD (two workgroups per CU)
    {"kc34", 1},      // two-vector passes with 3 or 4 layouts: 1 = straight-line kernels, 0 = layout loop
    {"c64g14", 2},    // complex64 adjoint programs on 14-bit tiles: 1 always, 2 when fewer groups, 0 never
    {"batchslab", 256},  // batch scan, states above the LDS tile: MiB of the cache-resident slab of one
                         // sliced launch (0: per-workgroup slots in device memory)
    {"genunit", 1},   // general single-qubit layers: 1 = unit-diagonal form where the matrices allow it
    {"ntinit", 1},    // write-only first passes: 1 = nontemporal stores
    {"split", 0},     // bits above the contiguous tile: 0 = near-equal groups, 1 = largest groups first
    {"xcd", -1},      // x > 0: XCD-aware tile order, 8 * 2^(x-1) interleaved streams of contiguous tiles;
                      // 0: tile = workgroup index; -1: 8 streams for states up to 64 GiB, 32 above
                      // (n = 32 complex128: 241 -> 226 ms per p = 4 evaluation; n = 33: 589 -> 461 ms);
                      // -2: per tile group, 32 streams for groups from bit 20 up (and above 64 GiB)
    {"adjzeta", -1},  // adjoint: 1 = two one-vector reverse sweeps of psi +- i t lambda; 0 = one sweep of
                      // both vectors (two-vector passes); -1 = 1 for complex128 (n = 32, p = 4: 731 vs
                      // 767 ms), 0 for complex64 (449 vs 432 ms, and the f32 rounding of the two
                      // sweeps does not cancel in their difference)
    {"c128t14", 0},   // complex128 one-vector programs (not the adjoint): 1 = 14-bit tiles (512 threads,
                      // one workgroup per CU), 0 = 13-bit tiles (256 threads, two workgroups per CU)
    {"fail_next_launch", 0},  // 1: the next tile-pass launch reports a launch failure (error-path tests)
};
// Accepted range of every knob.
const std::map<std::string, std::pair<int, int>> g_knob_range = {
    {"fuse", {0, 1}},    {"cmin64", {0, 8}},   {"cmin128", {0, 8}},  {"ntmin", {0, 64}},   {"persist", {0, 8}},
    {"stagger", {0, 64}}, {"snake", {0, 2}},   {"dpp", {0, 1}},      {"ldsswz", {3, 5}},   {"batchwide", {0, 2}},
    {"batch128", {0, 1}}, {"c64t13", {0, 1}},  {"c64occ", {0, 1}},   {"c64g4", {0, 1}},    {"kc34", {0, 1}},
    {"c64g14", {0, 2}},  {"ntinit", {0, 1}},   {"batchslab", {0, 4096}}, {"genunit", {0, 1}},   {"split", {0, 1}},    {"xcd", {-2, 5}},      {"c128t14", {0, 1}}, {"adjzeta", {-1, 1}},
    {"fail_next_launch", {0, 1}},
};
}  // namespace

int knob(const char* k) {
    std::lock_guard<std::mutex> g(g_knob_mu);
    return g_knobs[k];
}

std::vector<std::string> knob_names() {
    std::lock_guard<std::mutex> g(g_knob_mu);
    std::vector<std::string> names;
    for (auto& kv : g_knobs) names.push_back(kv.first);
    return names;
}

namespace {
// Tuned per-(dtype, n) overrides: text lines "c128 32 cmin128 4" (from the
// autotuner), loaded from $SV_TUNE_CACHE on first use or by sv_tune_load.
std::map<std::tuple<int, int, std::string>, int> g_tuned;
bool g_tuned_loaded = false;

int load_tuned_locked(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return -1;
    char dt[16], name[64];
    int n, v;
    int cnt = 0;
    while (fscanf(f, "%15s %d %63s %d", dt, &n, name, &v) == 4) {
        const int d = std::string(dt) == "c128" ? 2 : (std::string(dt) == "c64" ? 1 : 0);
        if (d && g_knobs.count(name)) {
            g_tuned[std::make_tuple(d, n, std::string(name))] = v;
            cnt++;
        }
    }
    fclose(f);
    return cnt;
}
}  // namespace

// Knob value for a plan: tuned override for (dtype, n) if present, else the global value.
int knob_for(const char* k, int dtype, int n) {
    std::lock_guard<std::mutex> g(g_knob_mu);
    if (!g_tuned_loaded) {
        g_tuned_loaded = true;
        const char* p = getenv("SV_TUNE_CACHE");
        if (p && *p) (void)load_tuned_locked(p);
    }
    auto it = g_tuned.find(std::make_tuple(dtype, n, std::string(k)));
    if (it != g_tuned.end()) return it->second;
    return g_knobs[k];
}
// Error-path tests: knob fail_next_launch = 1 makes the next tile-pass launch
// report hipErrorLaunchFailure (nothing is launched), then clears itself.
bool take_injected_failure() {
    std::lock_guard<std::mutex> g(g_knob_mu);
    int& v = g_knobs["fail_next_launch"];
    if (v == 0) return false;
    v = 0;
    return true;
}

extern "C" int sv_tune_load(const char* path) {
    if (!path) {
        std::lock_guard<std::mutex> g(g_knob_mu);
        g_tuned.clear();
        g_tuned_loaded = true;
        return SV_OK;
    }
    std::lock_guard<std::mutex> g(g_knob_mu);
    g_tuned.clear();
    g_tuned_loaded = true;
    const int cnt = load_tuned_locked(path);
    if (cnt < 0) return fail(SV_ERR_ARG, "sv_tune_load: cannot read '%s'", path);
    return SV_OK;
}

extern "C" int sv_tune_set(const char* name, int value) {
    if (!name) return fail(SV_ERR_ARG, "sv_tune_set: name is NULL");
    std::lock_guard<std::mutex> g(g_knob_mu);
    auto it = g_knobs.find(name);
    if (it == g_knobs.end()) return fail(SV_ERR_ARG, "sv_tune_set: unknown knob '%s'", name);
    const auto& rg = g_knob_range.at(name);
    if (value < rg.first || value > rg.second)
        return fail(SV_ERR_ARG, "%s must be in [%d, %d]", name, rg.first, rg.second);
    it->second = value;
    return SV_OK;
}

extern "C" int sv_tune_get(const char* name, int* value) {
    if (!name || !value) return fail(SV_ERR_ARG, "sv_tune_get: NULL argument");
    std::lock_guard<std::mutex> g(g_knob_mu);
    auto it = g_knobs.find(name);
    if (it == g_knobs.end()) return fail(SV_ERR_ARG, "sv_tune_get: unknown knob '%s'", name);
    *value = it->second;
    return SV_OK;
}

// ============================================================================ profiling
// Optional per-launch timing with HIP events recorded on the launch stream,
// plus the algorithmic bytes of each pass (vectors read + vectors written).
namespace {
struct ProfRec {
    hipEvent_t a, b;
    std::string kind;
    double bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
}  // namespace

static void prof_clear_locked() {
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
}

extern "C" int sv_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_clear_locked();
    g_prof_on = on != 0;
    return SV_OK;
}

extern "C" int sv_profile_report(char* buf, size_t len) {
    if (!buf || len == 0) return fail(SV_ERR_ARG, "sv_profile_report: empty buffer");
    std::lock_guard<std::mutex> g(g_prof_mu);
    std::map<std::string, std::tuple<long, double, double>> agg;  // launches, ms, bytes
    for (auto& r : g_prof) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return fail(SV_ERR_HIP, "profile: %s", hipGetErrorString(e));
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return fail(SV_ERR_HIP, "profile: %s", hipGetErrorString(e));
        // "kind/detail" records count under the kind and under the full name
        const size_t slash = r.kind.find('/');
        for (const std::string& key : {r.kind.substr(0, slash), r.kind}) {
            auto& t = agg[key];
            std::get<0>(t) += 1;
            std::get<1>(t) += ms;
            std::get<2>(t) += r.bytes;
            if (slash == std::string::npos) break;
        }
    }
    std::string js = "{";
    bool first = true;
    for (auto& kv : agg) {
        char tmp[256];
        snprintf(tmp, sizeof(tmp), "%s\"%s\":{\"launches\":%ld,\"ms\":%.6f,\"bytes\":%.1f}", first ? "" : ",",
                 kv.first.c_str(), std::get<0>(kv.second), std::get<1>(kv.second), std::get<2>(kv.second));
        js += tmp;
        first = false;
    }
    js += "}";
    prof_clear_locked();
    snprintf(buf, len, "%s", js.c_str());
    return SV_OK;
}

bool prof_begin(hipStream_t st, hipEvent_t* a) {
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on) return false;
    }
    if (hipEventCreate(a) != hipSuccess) return false;
    (void)hipEventRecord(*a, st);
    return true;
}

void prof_end(hipStream_t st, hipEvent_t a, const std::string& kind, double bytes) {
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(ProfRec{a, b, kind, bytes});
}

int device_cu_count(int dev) {
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
    return cus;
}


