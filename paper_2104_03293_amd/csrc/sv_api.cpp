// Host side of libsv: argument checking, tile planning, pass programs and
// launch sequencing behind the C ABI of include/sv.h.
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

#include "../../include/sv.h"
#include "sv_internal.h"

using namespace svk;

// ============================================================================ errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
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

#define HIPCHECK(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

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
    {"ntinit", 1},    // write-only first passes: 1 = nontemporal stores
    {"split", 0},     // bits above the contiguous tile: 0 = near-equal groups, 1 = largest groups first
    {"xcd", -1},      // x > 0: XCD-aware tile order, 8 * 2^(x-1) interleaved streams of contiguous tiles;
                      // 0: tile = workgroup index; -1: 8 streams for states up to 64 GiB, 32 above
                      // (n = 32 complex128: 241 -> 226 ms per p = 4 evaluation; n = 33: 589 -> 461 ms)
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
    {"c64g14", {0, 2}},  {"ntinit", {0, 1}},   {"batchslab", {0, 4096}},   {"split", {0, 1}},    {"xcd", {-1, 5}},      {"c128t14", {0, 1}}, {"adjzeta", {-1, 1}},
    {"fail_next_launch", {0, 1}},
};
int knob(const char* k) {
    std::lock_guard<std::mutex> g(g_knob_mu);
    return g_knobs[k];
}
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
}  // namespace

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

static bool prof_begin(hipStream_t st, hipEvent_t* a) {
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on) return false;
    }
    if (hipEventCreate(a) != hipSuccess) return false;
    (void)hipEventRecord(*a, st);
    return true;
}

static void prof_end(hipStream_t st, hipEvent_t a, const std::string& kind, double bytes) {
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(ProfRec{a, b, kind, bytes});
}

// ============================================================================ objects
struct Work {
    double2* d_tab = nullptr;
    size_t tab_cap = 0;  // double2
    double* d_part = nullptr;
    size_t part_cap = 0;  // doubles
    double* d_res = nullptr;
    double* h_res = nullptr;
    size_t res_cap = 0;  // doubles
    double* d_spin = nullptr;  // per-tile spin partials [ntiles][kTF]
    size_t spin_cap = 0;       // doubles
    double* d_gmat = nullptr;  // general single-qubit layers, kGenBlock doubles per MIX op
    double* h_gmat = nullptr;  // pinned staging copy
    size_t gmat_cap = 0;       // doubles
};

struct sv_state_s {
    int n = 0;
    sv_dtype dt = SV_C128;
    void* ptr = nullptr;
    size_t bytes = 0;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    bool failed = false;
    Work w;
};

// The amplitude type is part of the key: it sets the LDS swizzle width and
// the byte strides stored in the table.
struct GeoKey {
    int T, R, c, lo, g, n, dt;
    uint64_t layouts;  // signature of the register blocks and lane butterflies (plan knobs change them)
    bool operator<(const GeoKey& o) const {
        return std::tie(T, R, c, lo, g, n, dt, layouts) < std::tie(o.T, o.R, o.c, o.lo, o.g, o.n, o.dt, o.layouts);
    }
};

struct sv_ising_s {
    int n = 0, m = 0;
    std::vector<double> h, J;
    std::vector<int32_t> ei, ej;
    bool integer = true;  // h, J integral
    int qden = 0;         // smallest q in {1, 2, 4} with q h, q J integral (0: none): E on the grid Z / q
    double scale = 0.0;
    int lut_half = -1;    // q * max(sum|h|+sum|J|, 2 max_k(|h_k| + sum_j |J_kj|)) when qden > 0
    // device tables
    double* d_h = nullptr;
    int32_t* d_adj_ptr = nullptr;
    int32_t* d_adj_nbr = nullptr;
    double* d_adj_J = nullptr;
    int32_t* d_ei = nullptr;
    int32_t* d_ej = nullptr;
    double* d_J = nullptr;
    // ground cache
    bool has_ground = false;
    double emin = 0.0;
    uint64_t deg = 0, argmin = 0;
    std::map<GeoKey, GeoBuf*> geos;
    std::map<std::tuple<int, int, int, int, int>, double*> tfs;  // (T, c, lo, g, n) -> per-tile field table
    std::mutex mu;
};

static size_t elem_size(sv_dtype d) { return d == SV_C128 ? 16 : 8; }

// Compute units of a device (cached per device; 256 on MI355X).
static int device_cu_count(int dev) {
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
static int max_n(sv_dtype d) { return d == SV_C128 ? 33 : 34; }
static bool dtype_ok(int d) { return d == SV_C64 || d == SV_C128; }

// ============================================================================ geometry
// One tile geometry: carriers [0, c), group bits [lo, lo + g), phantom bits >= n.
struct Geometry {
    int T, R, c, lo, g, n;
    uint32_t phantom;
    uint64_t ntiles;
    std::vector<std::vector<int>> blocks;  // register bit blocks per layout
    std::vector<uint32_t> act_fwd, act_bwd;
    std::vector<uint32_t> dpp;  // per layout: lane positions butterflied across lanes (bit 3 or 4)
    bool pivot = true;          // layouts share tile bit T-1 in register slot R-1 (half-tile exchanges)
};

static uint32_t swizzle(uint32_t u, int G) {
    uint32_t x = u >> G, f = 0;
    for (int i = 0; i < 6; i++) {
        f ^= x;
        x >>= G;
    }
    return u ^ (f & ((1u << G) - 1u));
}

static int swz_bits(sv_dtype d) { return d == SV_C128 ? 3 : 4; }  // planning: lowest lane bits of a 128-B run
// LDS slot swizzle width of the tile passes: the high tile bits are folded into
// the low 4 slot bits.  With 16 lanes served per LDS cycle for 16-B elements
// this keeps every complex128 exchange of every plan conflict-free (checked by
// replaying the plans); 3 bits left the contiguous group's second layout
// two-way conflicted (measured as LDS bank-conflict cycles).
static int lds_swz_bits(sv_dtype d, int n) { return knob_for("ldsswz", (int)d, n); }

// Register-bit blocks for a geometry.  Every block keeps the pivot (tile bit
// T-1) in register slot R-1 so that an LDS exchange runs in two halves.  The
// first layout holds the top R tile bits, leaving tile bits 0..5 to the lanes
// (coalesced loads); for group A the low block [0, R-1) comes second; the
// remaining active bits are covered from the top with blocks that start at or
// above the swizzle width G, so the last layout again has the carriers as its
// lowest lane bits (coalesced stores).
// pivot: every layout keeps tile bit T - 1 in register slot R - 1, so that an
// LDS exchange moves half a tile at a time (one-vector kernels, two
// workgroups per CU); without it (two-vector kernels, one workgroup per CU
// with a full-tile LDS buffer) all R register slots are free.
static Geometry make_geometry(int n, int T, int R, int c, int lo, int g, int G, uint32_t lane_pos_mask, bool pivot) {
    Geometry geo{};
    geo.pivot = pivot;
    geo.T = T;
    geo.R = R;
    geo.c = c;
    geo.lo = lo;
    geo.g = g;
    geo.n = n;
    geo.phantom = 0;
    for (int l = 0; l < T; l++)
        if (l >= n) geo.phantom |= 1u << l;
    geo.ntiles = n > T ? (1ull << (n - T)) : 1ull;
    const bool groupA = (g == 0);
    uint32_t active = 0;
    if (groupA) {
        for (int l = 0; l < std::min(n, T); l++) active |= 1u << l;
    } else {
        for (int l = c; l < T; l++) active |= 1u << l;
    }
    const int F = pivot ? R - 1 : R;  // free register slots of a block
    std::vector<std::vector<int>> blk;
    {
        std::vector<int> b0;
        for (int l = T - R; l < T; l++) b0.push_back(l);
        blk.push_back(b0);
    }
    auto add = [&](int a) {
        std::vector<int> b;
        for (int l = a; l < a + F; l++) b.push_back(l);
        if (pivot) b.push_back(T - 1);
        blk.push_back(b);
    };
    if (groupA) {
        add(0);
        // cover [F, T - R) from the top; the last block starts at or above the
        // swizzle width when it can
        int hi = T - R;
        while (hi > F) {
            const int a = (hi - F <= F) ? std::max(hi - F, std::min(G, F)) : hi - F;
            add(a);
            hi = a;
        }
    } else {
        int hi = T - R;
        while (hi > c) {
            int a = std::max(hi - F, c);
            add(a);
            hi = a;
        }
    }
    // keep blocks that touch active bits
    std::vector<std::vector<int>> keep;
    for (auto& b : blk) {
        uint32_t m = 0;
        for (int l : b) m |= 1u << l;
        if (m & active) keep.push_back(b);
    }
    if (keep.empty()) keep.push_back(blk[0]);
    // One layout fewer: if every active bit but one (x) fits in K - 1 register
    // blocks and x then sits at an allowed lane position of the last layout
    // (lane_pos_mask: 3 = DPP row_ror:8, 4 = ds_swizzle xor 16), x is
    // butterflied across lanes there instead of through another LDS exchange.
    // The last layout keeps the lowest tile bits as its lowest lanes
    // (coalesced stores).
    std::vector<uint32_t> dpp(keep.size(), 0u);
    if (lane_pos_mask != 0 && (keep.size() >= 3 || (keep.size() == 2 && !groupA))) {
        const int K0 = (int)keep.size();
        uint32_t b0 = 0;
        for (int l : keep[0]) b0 |= 1u << l;
        std::vector<int> U;
        for (int l = 0; l < T; l++)
            if ((active >> l & 1u) && !(b0 >> l & 1u)) U.push_back(l);
        const int nlow = groupA ? std::min(G, F) : c;  // tile bits that stay the lowest lanes at the end
        auto in = [](const std::vector<int>& v, int l) { return std::find(v.begin(), v.end(), l) != v.end(); };
        // pad a block to F free bits with bits that need no butterfly here
        auto pad = [&](std::vector<int>& b, int x, bool last) {
            for (int l = pivot ? T - 2 : T - 1; l >= 0 && (int)b.size() < F; l--) {
                if (in(b, l) || l == x || (last && l < nlow)) continue;
                if ((active >> l & 1u) && !(b0 >> l & 1u)) continue;  // only inactive or first-layout bits
                b.push_back(l);
            }
            return (int)b.size() == F;
        };
        bool found = false;
        for (size_t xi = 0; xi < U.size() && !found; xi++) {
            const int x = U[xi];
            std::vector<int> V;
            for (int l : U)
                if (l != x) V.push_back(l);
            const int nv = (int)V.size();
            const int m = (nv + F - 1) / F;  // register blocks after the first
            if (m + 1 >= K0 || nv > 20) continue;
            for (uint32_t sub = 0; sub < (1u << nv) && !found; sub++) {
                if (__builtin_popcount(sub) != std::min(F, nv)) continue;
                std::vector<int> last, mid;
                for (int q = 0; q < nv; q++) (sub >> q & 1u ? last : mid).push_back(V[q]);
                if ((int)mid.size() > (m - 1) * F) continue;
                if (!pad(last, x, true)) continue;
                uint32_t lm = pivot ? 1u << (T - 1) : 0u;
                for (int l : last) lm |= 1u << l;
                std::vector<int> tbits;
                for (int l = 0; l < T; l++)
                    if (!(lm >> l & 1u)) tbits.push_back(l);
                bool ok = (int)tbits.size() >= 6;
                for (int q = 0; q < nlow && ok; q++) ok = tbits[q] == q;
                int pos = -1;
                for (int q = 0; q < 6 && ok; q++)
                    if (tbits[q] == x) pos = q;
                if (!ok || pos < 0 || !(lane_pos_mask >> pos & 1u)) continue;
                std::vector<std::vector<int>> nb{keep[0]};
                bool good = true;
                for (size_t q = 0; q < mid.size() && good; q += F) {
                    std::vector<int> b(mid.begin() + q, mid.begin() + std::min(mid.size(), q + F));
                    good = pad(b, x, false);
                    if (pivot) b.push_back(T - 1);
                    nb.push_back(b);
                }
                if (!good) continue;
                if (pivot) last.push_back(T - 1);
                nb.push_back(last);
                keep = nb;
                dpp.assign(keep.size(), 0u);
                dpp.back() = 1u << pos;
                found = true;
            }
        }
    }
    const int K = (int)keep.size();
    geo.blocks = keep;
    geo.dpp = dpp;
    geo.act_fwd.assign(K, 0);
    geo.act_bwd.assign(K, 0);
    uint32_t done = 0;
    for (int j = 0; j < K; j++) {
        for (int k = 0; k < R; k++) {
            int l = geo.blocks[j][k];
            if ((active >> l & 1u) && !(done >> l & 1u)) geo.act_fwd[j] |= 1u << k;
        }
        for (int l : geo.blocks[j]) done |= 1u << l;
    }
    done = 0;
    for (int j = K - 1; j >= 0; j--) {
        for (int k = 0; k < R; k++) {
            int l = geo.blocks[j][k];
            if ((active >> l & 1u) && !(done >> l & 1u)) geo.act_bwd[j] |= 1u << k;
        }
        for (int l : geo.blocks[j]) done |= 1u << l;
    }
    return geo;
}

// Tile groups covering all qubits: group A = tile bits 0..T-1 (contiguous),
// then the bits above T split into near-equal groups of at most T - cmin bits,
// each tile carrying 2^c contiguous amplitudes (c = T - g >= cmin).
static std::vector<Geometry> plan_groups(int n, sv_dtype dt, int nv, bool grad = false, bool general = false) {
    Shape sh = shape_for((int)dt, nv, grad);
    // complex64 adjoint family on 14-bit tiles: the forward tiles, and 1024-thread two-vector
    // tiles of 4 register bits.  Knob c64g14: 1 always, 2 (default) when that needs fewer tile
    // groups than the 13-bit family (e.g. three instead of four at n = 32), 0 never.
    if (dt == SV_C64 && grad) {
        const int mode = knob_for("c64g14", (int)dt, n);
        const int cm = std::max(swz_bits(dt), knob_for("cmin64", (int)dt, n));
        auto ngroups = [&](int T) { return n <= T ? 1 : 1 + (n - T + (T - cm) - 1) / (T - cm); };
        if (mode == 1 || (mode == 2 && ngroups(14) < ngroups(13))) sh = nv == 1 ? Shape{14, 5} : Shape{14, 4};
    }
    // complex128 one-vector programs on 14-bit tiles (general single-qubit layers keep 13-bit tiles)
    if (dt == SV_C128 && nv == 1 && !grad && !general && knob_for("c128t14", (int)dt, n) != 0) sh = Shape{14, 5};
    const int T = sh.T, R = sh.R, G = swz_bits(dt);
    // lane positions the one-vector kernels butterfly across lanes: 3, and 4 for
    // 14-bit complex64 tiles.  Two-vector passes keep every qubit in registers:
    // their lane butterflies would cost six cross-lane moves per amplitude
    // (both vectors and the gradient pair term), more than the exchange saved.
    const bool pos4 = dt == SV_C64 && T == 14 && knob_for("c64occ", (int)dt, n) == 0;
    const uint32_t dpp = (knob_for("dpp", (int)dt, n) == 0 || nv == 2) ? 0u : (pos4 ? 0x18u : 0x8u);
    std::vector<Geometry> out;
    if (n <= T) {
        out.push_back(make_geometry(n, T, R, n, n, 0, G, dpp, nv == 1));
        return out;
    }
    out.push_back(make_geometry(n, T, R, T, T, 0, G, dpp, nv == 1));
    const int cmin = std::max(G, knob_for(dt == SV_C128 ? "cmin128" : "cmin64", (int)dt, n));
    const int rest = n - T, gmax = T - cmin;
    const int ng = (rest + gmax - 1) / gmax;
    const bool largest_first = knob_for("split", (int)dt, n) != 0;
    int lo = T;
    for (int i = 0; i < ng; i++) {
        int g = largest_first ? std::min(gmax, n - lo) : rest / ng + (i < rest % ng ? 1 : 0);
        out.push_back(make_geometry(n, T, R, T - g, lo, g, G, dpp, nv == 1));
        lo += g;
    }
    return out;
}

static int global_bit(const Geometry& geo, int l) {
    if (l >= geo.n) return -1;
    if (l < geo.c) return l;
    return geo.lo + (l - geo.c);
}

// Build the device table for a geometry and (optionally) an instance.
static int build_geobuf(const Geometry& geo, const sv_ising_s* H, sv_dtype dt, GeoBuf** out) {
    GeoBuf hb;
    memset(&hb, 0, sizeof(hb));
    const int T = geo.T, R = geo.R, G = lds_swz_bits(dt, geo.n);
    const int NTB = T - R, NT = 1 << NTB;
    if (T >= kTF) return fail(SV_ERR_UNSUPPORTED, "internal: tile of %d bits exceeds the field table", T);
    std::vector<int> inv(64, -1);  // global bit -> tile bit
    for (int l = 0; l < kMaxT; l++) {
        hb.P[l] = l < T ? global_bit(geo, l) : -1;
        if (l < T && hb.P[l] >= 0) inv[hb.P[l]] = l;
    }
    auto gmap = [&](uint32_t u) -> uint64_t {
        return (uint64_t)(u & ((1u << geo.c) - 1u)) | ((uint64_t)(u >> geo.c) << geo.lo);
    };
    const int K = (int)geo.blocks.size();
    if (K > kMaxLayouts) return fail(SV_ERR_UNSUPPORTED, "internal: too many layouts (%d)", K);
    // per-thread coupling tables follow the header (instance geometries only)
    const size_t head = (sizeof(GeoBuf) + 7) / 8;  // in doubles
    const size_t per_layout = (size_t)(R + 1) * NT;
    std::vector<double> tabs(H ? (size_t)K * per_layout : 0, 0.0);
    for (int j = 0; j < K; j++) {
        GeoLayout& L = hb.L[j];
        const std::vector<int>& rb = geo.blocks[j];
        uint32_t rmask = 0;
        L.rbpack = 0;
        for (int k = 0; k < R; k++) {
            rmask |= 1u << rb[k];
            L.rbpack |= (uint32_t)rb[k] << (4 * k);
        }
        L.tmask = ((1u << T) - 1u) & ~rmask;
        std::vector<int> tb;  // thread-id bit j -> tile bit tb[j]
        for (int l = 0; l < T; l++)
            if (L.tmask >> l & 1u) tb.push_back(l);
        L.act_fwd = (int32_t)geo.act_fwd[j];
        L.act_bwd = (int32_t)geo.act_bwd[j];
        L.dpp = (int32_t)geo.dpp[j];
        for (int r = 0; r < (1 << R); r++) {
            uint32_t u = 0;
            for (int k = 0; k < R; k++)
                if (r >> k & 1) u |= 1u << rb[k];
            L.reg_u[r] = u;
            const uint32_t um = geo.pivot ? (u & ((1u << (T - 1)) - 1u)) : u;  // half-tile slots drop the pivot
            L.reg_lds[r] = swizzle(um, G) * (uint32_t)elem_size(dt);
            L.reg_goff[r] = (u & geo.phantom) ? 0 : gmap(u);
        }
        L.thr_off = 0;
        if (H) {
            L.thr_off = (uint32_t)(head + (size_t)j * per_layout);
            double* tab = tabs.data() + (size_t)j * per_layout;
            std::vector<int> slot_of(T, -1);
            for (int k = 0; k < R; k++) slot_of[rb[k]] = k;
            auto spin_t = [&](int t, int l) {  // spin of tile bit l (a thread bit) for thread t
                for (int q = 0; q < NTB; q++)
                    if (tb[q] == l) return ((t >> q) & 1) ? 1.0 : -1.0;
                return 0.0;
            };
            for (int e = 0; e < H->m; e++) {
                const int la = inv[H->ei[e]], lb = inv[H->ej[e]];
                if (la < 0 || lb < 0) continue;  // not an intra-tile coupling
                const double Jv = H->J[e];
                const int ka = slot_of[la], kb = slot_of[lb];
                if (ka < 0 && kb < 0) {
                    for (int t = 0; t < NT; t++) tab[t] += Jv * spin_t(t, la) * spin_t(t, lb);
                } else if (ka >= 0 && kb >= 0) {
                    for (int r = 0; r < (1 << R); r++) {
                        const double sa = (r >> ka & 1) ? 1.0 : -1.0, sb = (r >> kb & 1) ? 1.0 : -1.0;
                        L.Q[r] += Jv * sa * sb;
                    }
                } else {
                    const int k = ka >= 0 ? ka : kb;
                    const int lt = ka >= 0 ? lb : la;
                    for (int t = 0; t < NT; t++) tab[(size_t)(1 + k) * NT + t] += Jv * spin_t(t, lt);
                }
            }
        }
    }
    const size_t bytes = head * 8 + tabs.size() * 8;
    std::vector<double> img(bytes / 8, 0.0);
    memcpy(img.data(), &hb, sizeof(GeoBuf));
    if (!tabs.empty()) memcpy(img.data() + head, tabs.data(), tabs.size() * 8);
    GeoBuf* d = nullptr;
    HIPCHECK(hipMalloc(&d, bytes));
    hipError_t e = hipMemcpy(d, img.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(SV_ERR_HIP, "hipMemcpy(geo) failed: %s", hipGetErrorString(e));
    }
    *out = d;
    return SV_OK;
}

static std::mutex g_geo_mu;
static std::map<GeoKey, GeoBuf*> g_plain_geos;  // instance-free tables (mixer-only passes)

// lookup_only: return the cached table or fail (calls that may not allocate).
static int get_geobuf(const Geometry& geo, sv_ising_s* H, sv_dtype dt, GeoBuf** out, bool lookup_only = false) {
    uint64_t sig = 1469598103934665603ull;  // FNV-1a over the layout description
    auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
    for (size_t j = 0; j < geo.blocks.size(); j++) {
        for (int l : geo.blocks[j]) mix((uint64_t)l);
        mix(1000u + geo.dpp[j]);
    }
    mix(geo.pivot ? 7u : 9u);
    mix(100u + (uint64_t)lds_swz_bits(dt, geo.n));
    GeoKey key{geo.T, geo.R, geo.c, geo.lo, geo.g, geo.n, (int)dt, sig};
    if (H) {
        std::lock_guard<std::mutex> g(H->mu);
        auto it = H->geos.find(key);
        if (it != H->geos.end()) {
            *out = it->second;
            return SV_OK;
        }
        if (lookup_only)
            return fail(SV_ERR_UNSUPPORTED,
                        "the instance has no device tables for this n, dtype and plan yet (run sv_qaoa_energy "
                        "once with a state of the same n and dtype to build them)");
        int rc = build_geobuf(geo, H, dt, out);
        if (rc) return rc;
        H->geos[key] = *out;
        return SV_OK;
    }
    std::lock_guard<std::mutex> g(g_geo_mu);
    auto it = g_plain_geos.find(key);
    if (it != g_plain_geos.end()) {
        *out = it->second;
        return SV_OK;
    }
    if (lookup_only) return fail(SV_ERR_UNSUPPORTED, "no geometry table for this n, dtype and plan yet");
    int rc = build_geobuf(geo, nullptr, dt, out);
    if (rc) return rc;
    g_plain_geos[key] = *out;
    return SV_OK;
}

// ============================================================================ programs
// Events of a circuit, in application order.
enum EvKind { EV_INIT, EV_PHASE, EV_MIX, EV_REDUCE, EV_LAMINIT, EV_GGAMMA, EV_SPINZ, EV_E2, EV_ZETA, EV_EFORM };
struct Event {
    EvKind kind;
    int group = 0;      // EV_MIX
    double angle = 0;   // EV_PHASE gamma / EV_MIX beta / EV_ZETA t
    int vec = 1;        // vectors touched (bit0 psi, bit1 lam)
    int res = -1;       // result index (REDUCE: 3 consecutive; GGAMMA, E2, EFORM; MIX grad-beta)
    int gm = -1;        // EV_MIX: index of a general single-qubit layer (Program::layers), -1: exp(-i angle X)
};

struct Pass {
    int group = 0;
    int nv = 1;
    bool has_mix = false;
    bool init = false;
    int load = 1, store = 1;
    std::vector<Op> ops;
    std::vector<int> slot_dst;                  // result index of each slot
    std::vector<std::pair<int, double>> phase;  // (layout, gamma) per phase table
    int spin_res = -1;                          // PT_SPINZ: first result index of the n spin expectations
    bool gen = false;                           // its MIX ops are general single-qubit layers
};

struct Program {
    std::vector<Pass> passes;
    int nres = 0;
    const double* layers = nullptr;  // general layers, host [layer][qubit][8] (complex 2x2, row-major)
    int nq = 0;                      // qubits per layer
};

static int point_rank(int flags) {
    // position of a POINT part in the kernel's fixed execution order
    if (flags & (PT_PHASE_PSI | PT_PHASE_LAM)) return 3;
    if (flags & (PT_GGAMMA | PT_EFORM)) return 2;
    if (flags & (PT_LAM_INIT | PT_ZETA)) return 1;
    return 0;
}

// Partition events into passes (greedy).  A pass has one tile group and the
// fixed shape  MIX{0,2} POINT{0,1} MIX{0,2}  (kernel slots 0-1, 2, 3-4).
// Consecutive POINT events merge into one POINT when the kernel's fixed order
// (reduce, lambda init, grad-gamma, phase) agrees with the event order.
static Program build_program(const std::vector<Event>& evs, int nres, bool fuse) {
    Program prog;
    prog.nres = nres;
    Pass cur;
    bool open = false;
    bool lam_live = false;  // two-vector passes carry at most 4 reduction slots
    int nmix_pre = 0, nmix_post = 0;
    bool has_point = false;
    auto limit = [&](const Event& e) {
        return (lam_live || e.kind == EV_LAMINIT || (e.vec & 2)) ? 4 : kMaxSlots;
    };
    auto close = [&]() {
        if (open) prog.passes.push_back(cur);
        cur = Pass();
        open = false;
    };
    auto start = [&](int group) {
        cur = Pass();
        cur.group = group;
        cur.ops.assign(kMaxOps, Op{});
        for (Op& o : cur.ops) {
            o.kind = 0;
            o.slot = o.slot2 = o.slot3 = o.qidx = -1;
        }
        nmix_pre = nmix_post = 0;
        has_point = false;
        open = true;
    };
    for (const Event& e : evs) {
        if (e.kind == EV_INIT) {
            close();
            start(0);
            cur.init = true;
            continue;
        }
        if (e.kind == EV_MIX && e.gm >= 0) {
            // general single-qubit layer: one op; a pass without a POINT takes up
            // to four of them (the empty point slot is skipped)
            bool can = open && (!cur.has_mix || (cur.group == e.group && fuse && cur.gen));
            if (can) can = has_point ? nmix_post < 2 : (nmix_pre < 2 || nmix_post < 2);
            if (!can) {
                close();
                start(e.group);
            }
            cur.group = e.group;
            cur.gen = true;
            Op op{};
            op.kind = OP_MIX;
            op.flags = MIX_PSI | MIX_GEN;
            op.slot = -1;
            op.slot2 = -1;
            op.qidx = e.gm;
            op.a = 0.0;
            op.b = 1.0;
            if (!has_point && nmix_pre < 2) {
                cur.ops[nmix_pre++] = op;
            } else {
                has_point = true;  // later POINT events start a new pass
                cur.ops[3 + nmix_post++] = op;
            }
            cur.has_mix = true;
            continue;
        }
        if (e.kind == EV_MIX) {
            // exp(-i beta X) = (-1)^k exp(-i beta' X), beta' = beta - k pi in [-pi/2, pi/2];
            // |beta'| > pi/4 is applied as two halves so that |tan| <= 1.
            const double kpi = std::nearbyint(e.angle / M_PI);
            const double bred = e.angle - kpi * M_PI;
            const double sign = (std::fmod(std::fabs(kpi), 2.0) == 1.0) ? -1.0 : 1.0;
            const int nhalf = std::fabs(bred) > M_PI / 4 ? 2 : 1;
            const double bh = bred / nhalf;
            const int slots = e.res >= 0 ? 1 : 0;
            bool can = open && (!cur.has_mix || (cur.group == e.group && fuse && !cur.gen)) &&
                       (int)cur.slot_dst.size() + slots <= limit(e);
            if (can) {
                if (!has_point) can = nmix_pre + nhalf <= 2;
                else can = nmix_post + nhalf <= 2;
            }
            if (!can) {
                close();
                start(e.group);
            }
            cur.group = e.group;  // a POINT-only prefix runs in layout 0 of any group
            for (int h = 0; h < nhalf; h++) {
                Op op{};
                op.kind = OP_MIX;
                op.flags = (e.vec & 1 ? MIX_PSI : 0) | (e.vec & 2 ? MIX_LAM : 0);
                op.slot = -1;
                op.slot2 = -1;
                op.qidx = -1;
                if (e.res >= 0 && h == 0) {
                    op.flags |= MIX_GBETA;
                    op.slot = (int)cur.slot_dst.size();
                    cur.slot_dst.push_back(e.res);
                }
                op.a = std::tan(bh);
                op.b = (h == 0 ? sign : 1.0) * std::cos(bh);
                if (!has_point) cur.ops[nmix_pre++] = op;
                else cur.ops[3 + nmix_post++] = op;
            }
            cur.has_mix = true;
            continue;
        }
        int flag = 0;
        if (e.kind == EV_PHASE) flag = (e.vec & 1 ? PT_PHASE_PSI : 0) | (e.vec & 2 ? PT_PHASE_LAM : 0);
        if (e.kind == EV_REDUCE) flag = PT_REDUCE;
        if (e.kind == EV_LAMINIT) flag = PT_LAM_INIT;
        if (e.kind == EV_GGAMMA) flag = PT_GGAMMA;
        if (e.kind == EV_SPINZ) flag = PT_SPINZ;
        if (e.kind == EV_E2) flag = PT_E2;
        if (e.kind == EV_ZETA) flag = PT_ZETA;
        if (e.kind == EV_EFORM) flag = PT_EFORM;
        const int slots =
            e.kind == EV_REDUCE ? 3 : ((e.kind == EV_GGAMMA || e.kind == EV_E2 || e.kind == EV_EFORM) ? 1 : 0);
        bool merge = false;
        if (open && has_point && nmix_post == 0) {
            const Op& last = cur.ops[2];
            merge = !(last.flags & flag);
            if (merge) {
                // a reduction reads only |psi|^2 and E, which a phase leaves alone
                const int mine = point_rank(flag);
                const int lastmax = point_rank(last.flags);
                // (spin sums, like the reduction, read only |psi|^2)
                merge = mine > lastmax ||
                        ((flag == PT_REDUCE || flag == PT_SPINZ || flag == PT_E2) &&
                         !(last.flags & (PT_LAM_INIT | PT_GGAMMA | PT_ZETA)));
            }
        }
        bool fits = open && (!fuse ? !cur.has_mix : true) && (int)cur.slot_dst.size() + slots <= limit(e);
        if (fits && !merge) fits = !has_point;  // a new POINT needs the (single) point slot
        if (fits && has_point && !merge) fits = false;
        if (!fits) {
            const int g = (open && cur.has_mix && nmix_post == 0 && !has_point) ? cur.group : 0;
            close();
            start(g);
            merge = false;
        }
        if (!merge) {
            Op op{};
            op.kind = OP_POINT;
            op.slot = -1;
            op.slot2 = -1;
            op.slot3 = -1;
            op.qidx = -1;
            cur.ops[2] = op;
            has_point = true;
        }
        Op& op = cur.ops[2];
        op.flags |= flag;
        if (e.kind == EV_REDUCE) {
            op.slot = (int)cur.slot_dst.size();
            for (int q = 0; q < 3; q++) cur.slot_dst.push_back(e.res + q);
        } else if (e.kind == EV_GGAMMA || e.kind == EV_EFORM) {
            op.slot2 = (int)cur.slot_dst.size();
            cur.slot_dst.push_back(e.res);
        } else if (e.kind == EV_E2) {
            op.slot3 = (int)cur.slot_dst.size();
            cur.slot_dst.push_back(e.res);
        } else if (e.kind == EV_ZETA) {
            op.b = e.angle;
        } else if (e.kind == EV_PHASE) {
            op.a = e.angle;
            op.qidx = (int)cur.phase.size();
            cur.phase.push_back({-1, e.angle});
        } else if (e.kind == EV_LAMINIT) {
            lam_live = true;
        } else if (e.kind == EV_SPINZ) {
            cur.spin_res = e.res;
        }
    }
    close();
    // vector liveness: load what holds data before a pass, store what holds data after
    int live = 1;
    for (Pass& p : prog.passes) {
        if (p.init) live = 1;
        p.load = p.init ? 4 : live;
        bool touches_lam = (live & 2) != 0;
        for (const Op& op : p.ops) {
            if (op.kind == OP_POINT && (op.flags & PT_LAM_INIT)) live |= 2;
            if (op.kind == OP_MIX && (op.flags & MIX_LAM)) touches_lam = true;
            if (op.kind == OP_POINT && (op.flags & (PT_LAM_INIT | PT_GGAMMA | PT_PHASE_LAM))) touches_lam = true;
        }
        p.store = live;
        p.nv = touches_lam ? 2 : 1;
    }
    return prog;
}

// Assign each phase table the layout its POINT op runs in: a MIX walks the
// layouts from whichever end it is at to the other end.
static void finalize_program(Program& prog, const std::vector<Geometry>* groups_by_nv) {
    for (Pass& p : prog.passes) {
        const int K = (int)groups_by_nv[p.nv][p.group].blocks.size();
        int cur = 0;
        for (Op& op : p.ops) {
            if (op.kind == OP_MIX) {
                if (K > 1) cur = (cur == 0) ? K - 1 : 0;
            } else if (op.kind == OP_POINT && (op.flags & (PT_PHASE_PSI | PT_PHASE_LAM))) {
                p.phase[op.qidx].first = cur;
            }
        }
    }
}

// ============================================================================ execution
static int ensure_work(sv_state_s* s, size_t part_doubles, size_t res_doubles) {
    Work& w = s->w;
    if (part_doubles > w.part_cap) {
        if (w.d_part) (void)hipFree(w.d_part);
        w.d_part = nullptr;
        w.part_cap = 0;
        HIPCHECK(hipMalloc(&w.d_part, part_doubles * sizeof(double)));
        w.part_cap = part_doubles;
    }
    if (res_doubles > w.res_cap) {
        if (w.d_res) (void)hipFree(w.d_res);
        if (w.h_res) (void)hipHostFree(w.h_res);
        w.d_res = nullptr;
        w.h_res = nullptr;
        w.res_cap = 0;
        HIPCHECK(hipMalloc(&w.d_res, res_doubles * sizeof(double)));
        HIPCHECK(hipHostMalloc(&w.h_res, res_doubles * sizeof(double), hipHostMallocDefault));
        w.res_cap = res_doubles;
    }
    return SV_OK;
}

static IsingDev ising_dev(const sv_ising_s* H) {
    IsingDev d{};
    if (!H) return d;
    d.h = H->d_h;
    d.adj_ptr = H->d_adj_ptr;
    d.adj_nbr = H->d_adj_nbr;
    d.adj_J = H->d_adj_J;
    d.ei = H->d_ei;
    d.ej = H->d_ej;
    d.J = H->d_J;
    d.n = H->n;
    d.m = H->m;
    return d;
}

// Per-tile field table of an instance for a tile geometry, built once (on the
// caller's stream, which is synchronized so that later passes on any stream
// may use it) and kept until the instance is freed.
static int get_tf(sv_ising_s* H, const Geometry& geo, const GeoBuf* gb, hipStream_t stream, const double** out,
                  bool lookup_only = false) {
    const auto key = std::make_tuple(geo.T, geo.c, geo.lo, geo.g, geo.n);
    std::lock_guard<std::mutex> g(H->mu);
    auto it = H->tfs.find(key);
    if (it != H->tfs.end()) {
        *out = it->second;
        return SV_OK;
    }
    if (lookup_only)
        return fail(SV_ERR_UNSUPPORTED,
                    "the instance has no field table for this n, dtype and plan yet (run sv_qaoa_energy once with "
                    "a state of the same n and dtype to build it)");
    double* d = nullptr;
    HIPCHECK(hipMalloc(&d, geo.ntiles * (size_t)kTF * sizeof(double)));
    TfArgs a;
    memset(&a, 0, sizeof(a));
    a.is = ising_dev(H);
    a.geo = gb;
    a.tf = d;
    a.ntiles = geo.ntiles;
    a.T = geo.T;
    a.c = geo.c;
    a.lo = geo.lo;
    a.g = geo.g;
    int e = launch_tile_fields(a, stream);
    if (e == 0) e = (int)hipStreamSynchronize(stream);
    if (e != 0) {
        (void)hipFree(d);
        return fail(SV_ERR_HIP, "field table build failed: %s", hipGetErrorString((hipError_t)e));
    }
    H->tfs[key] = d;
    *out = d;
    return SV_OK;
}

// Energies on a grid Z / q are computed exactly in FP64, so the ground set compares exactly.
static double ground_tol(const sv_ising_s* H) { return H->qden > 0 ? 0.0 : 1e-9 * std::max(1.0, H->scale); }

static int run_ground(sv_ising_s* H, hipStream_t stream);

// Run a program on state s (and lam for two-vector programs).
struct Plan {
    std::vector<Geometry> by_nv[3];  // [1]: one-vector tile shape, [2]: two-vector shape
};

// grad: the adjoint family, whose one- and two-vector tiles share T.
static Plan make_plan(int n, sv_dtype dt, bool grad = false, bool general = false) {
    Plan pl;
    // complex64 one-vector programs may use the 13-bit tiles of the adjoint family
    // (not programs with general single-qubit layers, whose kernels exist for 14-bit tiles)
    if (dt == SV_C64 && !general && knob_for("c64t13", (int)dt, n) != 0) grad = true;
    pl.by_nv[1] = plan_groups(n, dt, 1, grad, general);
    pl.by_nv[2] = plan_groups(n, dt, 2, grad, general);
    return pl;
}

// fx != nullptr: the call may not allocate.  Partials and phase tables go to the
// fixed device region fx describes, every result is written once, straight to
// fx->out (no clearing), and the instance's tables and ground-state cache must
// already exist; programs that need more (spin sums, general layers) are refused.
// first_src: the first pass loads psi from this buffer instead of s (out of place).
static int run_program(sv_state_s* s, sv_state_s* lam, sv_ising_s* H, Program& prog, const Plan& plan,
                       bool need_ground, const FixedScratch* fx = nullptr, const void* first_src = nullptr) {
    finalize_program(prog, plan.by_nv);
    if (s->failed) return fail(SV_ERR_HIP, "state is in a failed state after an earlier HIP error");
    double emin = 0.0, etol = 0.0;
    if (need_ground && H) {
        if (fx) {
            std::lock_guard<std::mutex> g(H->mu);
            if (!H->has_ground)
                return fail(SV_ERR_UNSUPPORTED, "the instance has no ground-state cache yet (call sv_ground once)");
        } else {
            int rc = run_ground(H, s->stream);
            if (rc) return rc;
        }
        emin = H->emin;
        etol = ground_tol(H);
    }
    size_t part_need = 1;
    for (const Pass& p : prog.passes)
        part_need = std::max(part_need, (size_t)plan.by_nv[p.nv][p.group].ntiles * std::max<size_t>(1, p.slot_dst.size()));
    int rc = SV_OK;
    // the slot reduction's first stage follows the partials
    const size_t stage_off = part_need;
    part_need += (size_t)kReduceBlocks * kMaxSlots;
    if (fx) {
        if (part_need > fx->part_doubles)
            return fail(SV_ERR_UNSUPPORTED, "reduction partials need %zu doubles, the fixed scratch holds %zu",
                        part_need, fx->part_doubles);
        std::vector<int> writers(std::max(prog.nres, 0), 0);
        for (const Pass& p : prog.passes) {
            if (p.spin_res >= 0) return fail(SV_ERR_UNSUPPORTED, "spin sums need allocated scratch");
            for (int d : p.slot_dst)
                if (d >= 0 && d < prog.nres) writers[d]++;
        }
        for (int w : writers)
            if (w != 1) return fail(SV_ERR_UNSUPPORTED, "internal: a result without exactly one writer");
    } else {
        rc = ensure_work(s, part_need, std::max(prog.nres, 1));
        if (rc) return rc;
    }
    double* const d_part = fx ? fx->part : s->w.d_part;
    size_t spin_need = 0;
    for (const Pass& p : prog.passes)
        if (p.spin_res >= 0) spin_need = std::max(spin_need, (size_t)plan.by_nv[p.nv][p.group].ntiles * kTF);
    if (spin_need > s->w.spin_cap) {
        if (s->w.d_spin) (void)hipFree(s->w.d_spin);
        s->w.d_spin = nullptr;
        s->w.spin_cap = 0;
        HIPCHECK(hipMalloc(&s->w.d_spin, spin_need * sizeof(double)));
        s->w.spin_cap = spin_need;
    }
    if (prog.nres > 0 && !fx) {
        hipError_t e = hipMemsetAsync(s->w.d_res, 0, prog.nres * sizeof(double), s->stream);
        if (e != hipSuccess) {
            s->failed = true;
            return fail(SV_ERR_HIP, "hipMemsetAsync: %s", hipGetErrorString(e));
        }
    }
    const double amp0 = std::pow(2.0, -0.5 * s->n);
    // phase tables of every pass, built by one setup launch
    const int lut_half = H ? H->lut_half : -1;
    std::vector<TableJob> jobs;
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> offs(prog.passes.size());
    size_t tab_need = 0;
    for (size_t pi = 0; pi < prog.passes.size(); pi++) {
        const Pass& p = prog.passes[pi];
        if (p.phase.empty()) continue;
        const Geometry& geo = plan.by_nv[p.nv][p.group];
        GeoBuf* gb = nullptr;
        rc = get_geobuf(geo, H, s->dt, &gb, fx != nullptr);
        if (rc) return rc;
        for (const auto& ph : p.phase) {
            TableJob j{};
            j.gamma = ph.second;
            j.Q = gb->L[ph.first].Q;  // device address inside the geometry table
            j.nr = 1 << geo.R;
            j.L = lut_half;
            j.qinv = H && H->qden > 0 ? 1.0 / H->qden : 1.0;
            j.qph_off = (uint32_t)tab_need;
            tab_need += j.nr;
            j.lut_off = (uint32_t)tab_need;
            if (lut_half >= 0) tab_need += 2 * lut_half + 1;
            offs[pi].push_back({j.qph_off, j.lut_off});
            jobs.push_back(j);
        }
    }
    if (fx && tab_need > fx->tab_entries)
        return fail(SV_ERR_UNSUPPORTED, "phase tables need %zu entries, the fixed scratch holds %zu", tab_need,
                    fx->tab_entries);
    if (!fx && tab_need > s->w.tab_cap) {
        if (s->w.d_tab) (void)hipFree(s->w.d_tab);
        s->w.d_tab = nullptr;
        s->w.tab_cap = 0;
        HIPCHECK(hipMalloc(&s->w.d_tab, tab_need * sizeof(double2)));
        s->w.tab_cap = tab_need;
    }
    double2* const d_tab = fx ? fx->tab : s->w.d_tab;
    if (!jobs.empty()) {
        int e = launch_tables(jobs.data(), (int)jobs.size(), d_tab, s->stream);
        if (e != 0) {
            s->failed = true;
            return fail(SV_ERR_HIP, "table launch failed: %s", hipGetErrorString((hipError_t)e));
        }
    }
    // general single-qubit layers: one block of kGenBlock doubles per MIX op
    // (matrix of tile bit l at 8 l; identity for phantom bits)
    std::vector<std::array<int, kMaxOps>> genblk(prog.passes.size());
    std::vector<std::array<bool, kMaxOps>> genreal(prog.passes.size());  // every matrix of the op is real
    size_t nblk = 0;
    for (size_t pi = 0; pi < prog.passes.size(); pi++) {
        genblk[pi].fill(-1);
        for (int i = 0; i < kMaxOps; i++) {
            const Op& op = prog.passes[pi].ops[i];
            if (op.kind == OP_MIX && (op.flags & MIX_GEN)) genblk[pi][i] = (int)nblk++;
        }
    }
    if (nblk > 0) {
        if (fx) return fail(SV_ERR_UNSUPPORTED, "general layers need allocated scratch");
        if (!prog.layers || prog.nq != s->n) return fail(SV_ERR_ARG, "internal: general layers without matrices");
        const size_t need = nblk * (size_t)kGenBlock;
        // the staging buffer may still feed the previous call's copy
        HIPCHECK(hipStreamSynchronize(s->stream));
        if (need > s->w.gmat_cap) {
            if (s->w.d_gmat) (void)hipFree(s->w.d_gmat);
            if (s->w.h_gmat) (void)hipHostFree(s->w.h_gmat);
            s->w.d_gmat = nullptr;
            s->w.h_gmat = nullptr;
            s->w.gmat_cap = 0;
            HIPCHECK(hipMalloc(&s->w.d_gmat, need * sizeof(double)));
            HIPCHECK(hipHostMalloc(&s->w.h_gmat, need * sizeof(double), hipHostMallocDefault));
            s->w.gmat_cap = need;
        }
        for (size_t pi = 0; pi < prog.passes.size(); pi++) {
            const Geometry& geo = plan.by_nv[prog.passes[pi].nv][prog.passes[pi].group];
            for (int i = 0; i < kMaxOps; i++) {
                if (genblk[pi][i] < 0) continue;
                double* blk = s->w.h_gmat + (size_t)genblk[pi][i] * kGenBlock;
                const int layer = prog.passes[pi].ops[i].qidx;
                bool real = true;
                for (int l = 0; l < kGenBlock / 8; l++) {
                    const int q = l < geo.T ? global_bit(geo, l) : -1;
                    if (q < 0) {
                        const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
                        memcpy(blk + 8 * l, id, sizeof(id));
                    } else {
                        memcpy(blk + 8 * l, prog.layers + ((size_t)layer * s->n + q) * 8, 8 * sizeof(double));
                    }
                    for (int c = 1; c < 8; c += 2) real = real && blk[8 * l + c] == 0.0;
                }
                genreal[pi][i] = real;
            }
        }
        hipError_t e = hipMemcpyAsync(s->w.d_gmat, s->w.h_gmat, need * sizeof(double), hipMemcpyHostToDevice,
                                      s->stream);
        if (e != hipSuccess) {
            s->failed = true;
            return fail(SV_ERR_HIP, "hipMemcpyAsync (layer matrices): %s", hipGetErrorString(e));
        }
    }
    const int ntmin = knob_for("ntmin", (int)s->dt, s->n);
    const int persist = knob_for("persist", (int)s->dt, s->n);
    const int stagger = knob_for("stagger", (int)s->dt, s->n);
    const int ncu = persist > 0 ? device_cu_count(s->device) : 0;
    for (size_t pi = 0; pi < prog.passes.size(); pi++) {
        const Pass& p = prog.passes[pi];
        const Geometry& geo = plan.by_nv[p.nv][p.group];
        if (p.nv == 2 && !lam) return fail(SV_ERR_ARG, "internal: two-vector pass without lam");
        GeoBuf* gb = nullptr;
        rc = get_geobuf(geo, H, s->dt, &gb, fx != nullptr);
        if (rc) return rc;
        PassArgs a;
        memset(&a, 0, sizeof(a));
        a.psi = s->ptr;
        a.src = (pi == 0) ? first_src : nullptr;
        a.lam = lam ? lam->ptr : nullptr;
        a.partials = d_part;
        a.geo = gb;
        a.ntiles = geo.ntiles;
        a.n = s->n;
        a.c = geo.c;
        a.lo = geo.lo;
        a.g = geo.g;
        a.phantom = geo.phantom;
        a.nlayouts = (int)geo.blocks.size();
        a.load = p.load;
        a.store = p.store;
        a.nslots = (int)p.slot_dst.size();
        a.nops = 0;
        a.need_e = 0;
        a.nt = (geo.phantom == 0 && geo.c >= ntmin) ? 3 : 0;
        if (geo.phantom == 0 && (p.load & 4) && knob_for("ntinit", (int)s->dt, s->n) != 0) a.nt = 3;
        a.swz = lds_swz_bits(s->dt, s->n);
        a.grid = persist * ncu;
        a.stagger = stagger;
        a.xcd = knob_for("xcd", (int)s->dt, s->n);
        if (a.xcd < 0) a.xcd = ((size_t(1) << s->n) * elem_size(s->dt)) > (size_t(64) << 30) ? 3 : 1;
        for (const Op& op : p.ops) {
            a.nops += op.kind != 0;
            if (op.kind == OP_POINT && H) a.need_e = 1;
        }
        a.tf = nullptr;
        if (a.need_e) {
            rc = get_tf(H, geo, gb, s->stream, &a.tf, fx != nullptr);
            if (rc) return rc;
        }
        a.nphase = (int)p.phase.size();
        a.ptab = d_tab;
        a.lut_half = lut_half;
        a.lut_q = H && H->qden > 0 ? (double)H->qden : 1.0;
        a.spin_part = p.spin_res >= 0 ? s->w.d_spin : nullptr;
        for (int q = 0; q < a.nphase; q++) {
            a.qph_off[q] = offs[pi][q].first;
            a.lut_off[q] = offs[pi][q].second;
        }
        a.emin = emin;
        a.etol = etol;
        a.amp0 = amp0;
        for (int i = 0; i < kMaxOps; i++) {
            a.ops[i] = p.ops[i];
            if (genblk[pi][i] >= 0) a.ops[i].qidx = genblk[pi][i];
        }
        a.gmat = p.gen ? s->w.d_gmat : nullptr;
        // one-vector passes of the adjoint sweeps: 1 = quadratic forms only, 2 = also zeta / E form
        a.qf = 0;
        if (p.nv == 1)
            for (const Op& op : p.ops) {
                if (op.kind == OP_MIX && (op.flags & MIX_GBETA)) a.qf = std::max(a.qf, 1);
                if (op.kind == OP_POINT && (op.flags & (PT_ZETA | PT_EFORM))) a.qf = std::max(a.qf, 2);
                if (op.kind == OP_POINT && (op.flags & PT_ZETA) && (op.flags & PT_REDUCE)) a.qf = 3;
            }
        a.kc34 = knob_for("kc34", (int)s->dt, s->n);
        a.occ4 = (s->dt == SV_C64 && p.nv == 2 && knob_for("c64g4", (int)s->dt, s->n) != 0) ? 1 : 0;
        if (s->dt == SV_C64 && geo.T == 14) {
            a.occ4 = 1;
            for (uint32_t m : geo.dpp)
                if (m & 16u) a.occ4 = 0;
        }
        a.gen_real = 1;
        for (int i = 0; i < kMaxOps; i++)
            if (genblk[pi][i] >= 0 && !genreal[pi][i]) a.gen_real = 0;
        hipEvent_t ev0;
        const bool prof = !fx && prof_begin(s->stream, &ev0);
        int e = take_injected_failure() ? (int)hipErrorLaunchFailure : launch_pass((int)s->dt, p.nv, geo.T, a, s->stream);
        if (prof) {
            const int nrd = (p.load & 4) ? 0 : __builtin_popcount(p.load & 3);
            const int nwr = __builtin_popcount(p.store & 3);
            // kind/geometry: aggregated under the kind, and per tile shape, carrier bits and layouts
            const std::string kind = std::string("pass_") + (s->dt == SV_C128 ? "c128" : "c64") + "_nv" +
                                     std::to_string(p.nv) + "/T" + std::to_string(geo.T) + "c" +
                                     std::to_string(geo.c) + (geo.g > 0 ? "o" + std::to_string(geo.lo) : "") +
                                     "L" + std::to_string(a.nlayouts) +
                                     ((p.load & 4) ? "w" : "");
            prof_end(s->stream, ev0, kind, (double)(nrd + nwr) * (double)s->bytes);
        }
        if (e != 0) {
            s->failed = true;
            return fail(SV_ERR_HIP, "pass launch failed: %s", hipGetErrorString((hipError_t)e));
        }
        if (p.spin_res >= 0) {
            SpinArgs sa;
            memset(&sa, 0, sizeof(sa));
            sa.part = s->w.d_spin;
            sa.ntiles = geo.ntiles;
            sa.c = geo.c;
            sa.lo = geo.lo;
            sa.g = geo.g;
            sa.T = geo.T;
            sa.n = s->n;
            for (int l = 0; l < 16; l++) sa.qubit[l] = l < geo.T ? global_bit(geo, l) : -1;
            sa.out = s->w.d_res + p.spin_res;
            e = launch_spin_reduce(sa, s->stream);
            if (e != 0) {
                s->failed = true;
                return fail(SV_ERR_HIP, "spin reduce launch failed: %s", hipGetErrorString((hipError_t)e));
            }
        }
        if (a.nslots > 0) {
            e = launch_reduce_slots(d_part, geo.ntiles, a.nslots, p.slot_dst.data(), fx ? 0 : 1,
                                    fx ? fx->out : s->w.d_res, d_part + stage_off, s->stream);
            if (e != 0) {
                s->failed = true;
                return fail(SV_ERR_HIP, "reduce launch failed: %s", hipGetErrorString((hipError_t)e));
            }
        }
    }
    return SV_OK;
}

static int fetch_results(sv_state_s* s, int nres) {
    if (nres <= 0) return SV_OK;
    hipError_t e = hipMemcpyAsync(s->w.h_res, s->w.d_res, nres * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->failed = true;
        return fail(SV_ERR_HIP, "result copy failed: %s", hipGetErrorString(e));
    }
    return SV_OK;
}

// ============================================================================ states
extern "C" int sv_alloc(int n, sv_dtype dtype, void* stream, sv_state* out) {
    if (!out) return fail(SV_ERR_ARG, "sv_alloc: out is NULL");
    if (!dtype_ok(dtype)) return fail(SV_ERR_ARG, "sv_alloc: bad dtype %d", (int)dtype);
    if (n < 1 || n > max_n(dtype)) return fail(SV_ERR_ARG, "sv_alloc: n=%d outside [1, %d]", n, max_n(dtype));
    const size_t bytes = (size_t(1) << n) * elem_size(dtype);
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) return fail(SV_ERR_HIP, "hipMemGetInfo: %s", hipGetErrorString(e));
    if (bytes > fr) return fail(SV_ERR_OOM, "sv_alloc: need %zu bytes, %zu free", bytes, fr);
    void* p = nullptr;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ERR_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    auto* s = new sv_state_s();
    s->n = n;
    s->dt = dtype;
    s->ptr = p;
    s->bytes = bytes;
    s->owned = true;
    s->stream = (hipStream_t)stream;
    (void)hipGetDevice(&s->device);
    *out = s;
    return SV_OK;
}

extern "C" int sv_wrap(int n, sv_dtype dtype, void* ptr, size_t bytes, void* stream, sv_state* out) {
    if (!out) return fail(SV_ERR_ARG, "sv_wrap: out is NULL");
    if (!dtype_ok(dtype)) return fail(SV_ERR_ARG, "sv_wrap: bad dtype %d", (int)dtype);
    if (n < 1 || n > max_n(dtype)) return fail(SV_ERR_ARG, "sv_wrap: n=%d outside [1, %d]", n, max_n(dtype));
    if (!ptr) return fail(SV_ERR_ARG, "sv_wrap: NULL device pointer");
    if ((uintptr_t)ptr % 16) return fail(SV_ERR_ARG, "sv_wrap: pointer not 16-byte aligned");
    const size_t need = (size_t(1) << n) * elem_size(dtype);
    if (bytes < need) return fail(SV_ERR_ARG, "sv_wrap: %zu bytes given, %zu needed", bytes, need);
    auto* s = new sv_state_s();
    s->n = n;
    s->dt = dtype;
    s->ptr = ptr;
    s->bytes = need;
    s->owned = false;
    s->stream = (hipStream_t)stream;
    (void)hipGetDevice(&s->device);
    *out = s;
    return SV_OK;
}

extern "C" int sv_free(sv_state s) {
    if (!s) return SV_OK;
    if (s->owned && s->ptr) (void)hipFree(s->ptr);
    if (s->w.d_part) (void)hipFree(s->w.d_part);
    if (s->w.d_spin) (void)hipFree(s->w.d_spin);
    if (s->w.d_gmat) (void)hipFree(s->w.d_gmat);
    if (s->w.h_gmat) (void)hipHostFree(s->w.h_gmat);
    if (s->w.d_tab) (void)hipFree(s->w.d_tab);
    if (s->w.d_res) (void)hipFree(s->w.d_res);
    if (s->w.h_res) (void)hipHostFree(s->w.h_res);
    delete s;
    return SV_OK;
}

extern "C" int sv_set_stream(sv_state s, void* stream) {
    if (!s) return fail(SV_ERR_ARG, "sv_set_stream: NULL state");
    s->stream = (hipStream_t)stream;
    return SV_OK;
}

extern "C" int sv_copy_to_host(sv_state s, void* host, size_t bytes) {
    if (!s || !host) return fail(SV_ERR_ARG, "sv_copy_to_host: NULL argument");
    if (bytes != s->bytes) return fail(SV_ERR_ARG, "sv_copy_to_host: %zu bytes, state has %zu", bytes, s->bytes);
    if (s->failed) return fail(SV_ERR_HIP, "state is in a failed state");
    hipError_t e = hipMemcpyAsync(host, s->ptr, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->failed = true;
        return fail(SV_ERR_HIP, "copy to host: %s", hipGetErrorString(e));
    }
    return SV_OK;
}

extern "C" int sv_copy_from_host(sv_state s, const void* host, size_t bytes) {
    if (!s || !host) return fail(SV_ERR_ARG, "sv_copy_from_host: NULL argument");
    if (bytes != s->bytes) return fail(SV_ERR_ARG, "sv_copy_from_host: %zu bytes, state has %zu", bytes, s->bytes);
    if (s->failed) return fail(SV_ERR_HIP, "state is in a failed state");
    hipError_t e = hipMemcpyAsync(s->ptr, host, bytes, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->failed = true;
        return fail(SV_ERR_HIP, "copy from host: %s", hipGetErrorString(e));
    }
    return SV_OK;
}

// ============================================================================ instances
extern "C" int sv_ising_create(int n, const double* h, int m, const int32_t* ei, const int32_t* ej,
                               const double* J, sv_ising* out) {
    if (!out) return fail(SV_ERR_ARG, "sv_ising_create: out is NULL");
    if (n < 1 || n > 34) return fail(SV_ERR_ARG, "sv_ising_create: n=%d outside [1, 34]", n);
    if (m < 0) return fail(SV_ERR_ARG, "sv_ising_create: m=%d < 0", m);
    if (!h) return fail(SV_ERR_ARG, "sv_ising_create: h is NULL");
    if (m > 0 && (!ei || !ej || !J)) return fail(SV_ERR_ARG, "sv_ising_create: coupling arrays are NULL");
    std::set<std::pair<int, int>> seen;
    for (int i = 0; i < n; i++)
        if (!std::isfinite(h[i])) return fail(SV_ERR_NUMERIC, "sv_ising_create: h[%d] is not finite", i);
    for (int k = 0; k < m; k++) {
        const int a = ei[k], b = ej[k];
        if (a < 0 || a >= n || b < 0 || b >= n)
            return fail(SV_ERR_ARG, "sv_ising_create: coupling %d has endpoint outside [0, %d)", k, n);
        if (a == b) return fail(SV_ERR_ARG, "sv_ising_create: coupling %d is a self-coupling (%d, %d)", k, a, b);
        if (!std::isfinite(J[k])) return fail(SV_ERR_NUMERIC, "sv_ising_create: J[%d] is not finite", k);
        auto key = std::make_pair(std::min(a, b), std::max(a, b));
        if (!seen.insert(key).second)
            return fail(SV_ERR_ARG, "sv_ising_create: pair (%d, %d) listed twice", key.first, key.second);
    }
    auto* H = new sv_ising_s();
    H->n = n;
    H->m = m;
    H->h.assign(h, h + n);
    if (m > 0) {
        H->ei.assign(ei, ei + m);
        H->ej.assign(ej, ej + m);
        H->J.assign(J, J + m);
    }
    for (double v : H->h) H->scale += std::fabs(v);
    for (double v : H->J) H->scale += std::fabs(v);
    // Coefficients on a grid Z / q (integers, or the half-integers of exact
    // cover instances, Eqs. HChi-HCJij) give energies on that grid: the phase
    // factors then come from a table of exp(-i gamma m / q).
    for (int q : {1, 2, 4}) {
        bool ok = true;
        for (double v : H->h) ok = ok && q * v == std::round(q * v);
        for (double v : H->J) ok = ok && q * v == std::round(q * v);
        if (ok) {
            H->qden = q;
            break;
        }
    }
    H->integer = H->qden == 1;
    if (H->qden > 0) {
        std::vector<double> loc(n, 0.0);
        for (int i = 0; i < n; i++) loc[i] = std::fabs(H->h[i]);
        for (int k = 0; k < m; k++) {
            loc[H->ei[k]] += std::fabs(H->J[k]);
            loc[H->ej[k]] += std::fabs(H->J[k]);
        }
        double L = H->scale;
        for (double v : loc) L = std::max(L, 2.0 * v);
        L *= H->qden;
        if (L <= 65536.0) H->lut_half = (int)std::ceil(L);
    }
    // CSR adjacency over both endpoints
    std::vector<int32_t> ptr(n + 1, 0), nbr(2 * m);
    std::vector<double> aj(2 * m);
    for (int k = 0; k < m; k++) {
        ptr[H->ei[k] + 1]++;
        ptr[H->ej[k] + 1]++;
    }
    for (int i = 0; i < n; i++) ptr[i + 1] += ptr[i];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int k = 0; k < m; k++) {
        nbr[fill[H->ei[k]]] = H->ej[k];
        aj[fill[H->ei[k]]++] = H->J[k];
        nbr[fill[H->ej[k]]] = H->ei[k];
        aj[fill[H->ej[k]]++] = H->J[k];
    }
    auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 8));
        if (e != hipSuccess) return e;
        if (bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        return e;
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up((void**)&H->d_h, H->h.data(), n * sizeof(double));
    if (e == hipSuccess) e = up((void**)&H->d_adj_ptr, ptr.data(), (n + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = up((void**)&H->d_adj_nbr, nbr.data(), 2 * m * sizeof(int32_t));
    if (e == hipSuccess) e = up((void**)&H->d_adj_J, aj.data(), 2 * m * sizeof(double));
    if (e == hipSuccess) e = up((void**)&H->d_ei, H->ei.data(), m * sizeof(int32_t));
    if (e == hipSuccess) e = up((void**)&H->d_ej, H->ej.data(), m * sizeof(int32_t));
    if (e == hipSuccess) e = up((void**)&H->d_J, H->J.data(), m * sizeof(double));
    if (e != hipSuccess) {
        sv_ising_free(H);
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SV_ERR_OOM : SV_ERR_HIP, "sv_ising_create: %s", hipGetErrorString(e));
    }
    *out = H;
    return SV_OK;
}

extern "C" int sv_ising_exact_cover(int nrows, int ncols, const uint8_t* a, double* constant, sv_ising* out) {
    if (!a || !out) return fail(SV_ERR_ARG, "sv_ising_exact_cover: NULL argument");
    if (nrows < 1 || nrows > 34) return fail(SV_ERR_ARG, "sv_ising_exact_cover: nrows = %d outside [1, 34]", nrows);
    if (ncols < 1) return fail(SV_ERR_ARG, "sv_ising_exact_cover: ncols = %d", ncols);
    for (size_t k = 0; k < (size_t)nrows * ncols; k++)
        if (a[k] > 1) return fail(SV_ERR_ARG, "sv_ising_exact_cover: entry %zu is %d, not 0/1", k, (int)a[k]);
    // overlaps (a a^T)_ij and row counts (a b)_i
    std::vector<int64_t> ov((size_t)nrows * nrows, 0), cnt(nrows, 0);
    for (int i = 0; i < nrows; i++)
        for (int f = 0; f < ncols; f++) cnt[i] += a[(size_t)i * ncols + f];
    for (int i = 0; i < nrows; i++)
        for (int j = i; j < nrows; j++) {
            int64_t o = 0;
            for (int f = 0; f < ncols; f++) o += a[(size_t)i * ncols + f] & a[(size_t)j * ncols + f];
            ov[(size_t)i * nrows + j] = ov[(size_t)j * nrows + i] = o;
        }
    std::vector<double> h(nrows), J;
    std::vector<int32_t> ei, ej;
    int64_t off = 0, diag = 0, cnt_sum = 0;
    for (int i = 0; i < nrows; i++) {
        int64_t row = 0;
        for (int j = 0; j < nrows; j++) row += ov[(size_t)i * nrows + j];
        h[i] = 0.5 * (double)row - (double)cnt[i];  // Eq. HChi
        diag += ov[(size_t)i * nrows + i];
        cnt_sum += cnt[i];
        for (int j = i + 1; j < nrows; j++) {
            const int64_t o = ov[(size_t)i * nrows + j];
            off += o;
            if (o == 0) continue;
            ei.push_back(i);
            ej.push_back(j);
            J.push_back(0.5 * (double)o);  // Eq. HCJij
        }
    }
    // Eq. HCC: C = b^T b + sum_{i<j} (aa^T)_ij / 2 + sum_i ((aa^T)_ii - 2 (ab)_i) / 2
    if (constant) *constant = (double)ncols + 0.5 * (double)off + 0.5 * (double)(diag - 2 * cnt_sum);
    return sv_ising_create(nrows, h.data(), (int)J.size(), ei.data(), ej.data(), J.data(), out);
}

extern "C" int sv_rescale_factor(sv_ising H, double* r) {
    if (!H || !r) return fail(SV_ERR_ARG, "sv_rescale_factor: NULL argument");
    double v = 0.0;
    for (double x : H->h) v = std::max({v, x / 2.0, x / -2.0});
    for (double x : H->J) v = std::max({v, x / 1.0, x / -1.0});
    *r = v;
    return SV_OK;
}

extern "C" int sv_ising_free(sv_ising H) {
    if (!H) return SV_OK;
    for (void* p : {(void*)H->d_h, (void*)H->d_adj_ptr, (void*)H->d_adj_nbr, (void*)H->d_adj_J, (void*)H->d_ei,
                    (void*)H->d_ej, (void*)H->d_J})
        if (p) (void)hipFree(p);
    for (auto& kv : H->geos) (void)hipFree(kv.second);
    for (auto& kv : H->tfs) (void)hipFree(kv.second);
    delete H;
    return SV_OK;
}

// ============================================================================ ground
static int run_ground(sv_ising_s* H, hipStream_t stream) {
    {
        std::lock_guard<std::mutex> g(H->mu);
        if (H->has_ground) return SV_OK;
    }
    const sv_dtype dt = SV_C64;  // enumeration tiles use the complex64 tile shape
    const Shape sh = shape_for((int)dt, 1, false);
    std::vector<Geometry> groups = plan_groups(H->n, dt, 1);
    const Geometry& geo = groups[0];
    GeoBuf* gb = nullptr;
    int rc = get_geobuf(geo, H, dt, &gb);
    if (rc) return rc;
    const double* tf = nullptr;
    rc = get_tf(H, geo, gb, stream, &tf);
    if (rc) return rc;
    (void)sh;
    double* d_e = nullptr;
    uint64_t *d_c = nullptr, *d_a = nullptr;
    double* d_out = nullptr;
    const size_t nt = geo.ntiles;
    HIPCHECK(hipMalloc(&d_e, nt * sizeof(double)));
    HIPCHECK(hipMalloc(&d_c, nt * sizeof(uint64_t)));
    HIPCHECK(hipMalloc(&d_a, nt * sizeof(uint64_t)));
    HIPCHECK(hipMalloc(&d_out, 3 * sizeof(double)));
    GroundArgs a;
    memset(&a, 0, sizeof(a));
    a.geo = gb;
    a.tf = tf;
    a.ntiles = geo.ntiles;
    a.n = H->n;
    a.c = geo.c;
    a.lo = geo.lo;
    a.g = geo.g;
    a.phantom = geo.phantom;
    a.part_e = d_e;
    a.part_cnt = d_c;
    a.part_arg = d_a;
    a.mode = 0;
    int e = launch_ground((int)dt, a, stream);
    if (!e) e = launch_ground_finish(a, d_out, nullptr, nullptr, stream);
    double emin = 0;
    if (!e) e = (int)hipMemcpyAsync(&emin, d_out, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (!e) e = (int)hipStreamSynchronize(stream);
    uint64_t cnt = 0, arg = 0;
    if (!e) {
        a.mode = 1;
        a.emin = emin;
        a.etol = ground_tol(H);
        e = launch_ground((int)dt, a, stream);
        if (!e) e = launch_ground_finish(a, nullptr, (uint64_t*)(d_out + 1), (uint64_t*)(d_out + 2), stream);
        uint64_t tmp[2];
        if (!e) e = (int)hipMemcpyAsync(tmp, d_out + 1, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
        if (!e) e = (int)hipStreamSynchronize(stream);
        cnt = tmp[0];
        arg = tmp[1];
    }
    (void)hipFree(d_e);
    (void)hipFree(d_c);
    (void)hipFree(d_a);
    (void)hipFree(d_out);
    if (e) return fail(SV_ERR_HIP, "ground enumeration failed: %s", hipGetErrorString((hipError_t)e));
    std::lock_guard<std::mutex> g(H->mu);
    H->emin = emin;
    H->deg = cnt;
    H->argmin = arg;
    H->has_ground = true;
    return SV_OK;
}

extern "C" int sv_ground(sv_ising H, double* e_min, uint64_t* degeneracy, uint64_t* argmin) {
    if (!H) return fail(SV_ERR_ARG, "sv_ground: NULL instance");
    int rc = run_ground(H, nullptr);
    if (rc) return rc;
    if (e_min) *e_min = H->emin;
    if (degeneracy) *degeneracy = H->deg;
    if (argmin) *argmin = H->argmin;
    return SV_OK;
}

// ============================================================================ drivers
static int check_pair(sv_state s, sv_ising H, const char* who) {
    if (!s) return fail(SV_ERR_ARG, "%s: NULL state", who);
    if (!H) return fail(SV_ERR_ARG, "%s: NULL instance", who);
    if (s->n != H->n) return fail(SV_ERR_ARG, "%s: state has n=%d, instance n=%d", who, s->n, H->n);
    return SV_OK;
}

static int check_angles(int p, const double* a, const double* b, const char* who) {
    if (p < 1) return fail(SV_ERR_ARG, "%s: p=%d < 1", who, p);
    if (!a || !b) return fail(SV_ERR_ARG, "%s: NULL angle array", who);
    for (int k = 0; k < p; k++)
        if (!std::isfinite(a[k]) || !std::isfinite(b[k]))
            return fail(SV_ERR_NUMERIC, "%s: non-finite angle at layer %d", who, k + 1);
    return SV_OK;
}

extern "C" int sv_init_plus(sv_state s) {
    if (!s) return fail(SV_ERR_ARG, "sv_init_plus: NULL state");
    Plan plan = make_plan(s->n, s->dt);
    Program prog = build_program({Event{EV_INIT}}, 0, true);
    return run_program(s, nullptr, nullptr, prog, plan, false);
}

extern "C" int sv_cost_phase(sv_state s, sv_ising H, double gamma) {
    int rc = check_pair(s, H, "sv_cost_phase");
    if (rc) return rc;
    if (!std::isfinite(gamma)) return fail(SV_ERR_NUMERIC, "sv_cost_phase: gamma is not finite");
    Plan plan = make_plan(s->n, s->dt);
    Event e{EV_PHASE};
    e.angle = gamma;
    Program prog = build_program({e}, 0, true);
    return run_program(s, nullptr, H, prog, plan, false);
}

// Order in which a layer visits the tile groups.  Odd layers walk it forward
// and even layers backward (snake), so the end groups of consecutive layers
// share a pass while every middle group costs one pass per layer.  The
// contiguous group A streams fastest, so it takes a middle position.
static std::vector<int> group_order(int ngroups, int dt, int n) {
    std::vector<int> o;
    const int mode = knob_for("snake", dt, n);
    if (ngroups <= 2 || mode == 0) {
        for (int i = 0; i < ngroups; i++) o.push_back(i);
        return o;
    }
    if (mode == 2) {  // the last (shortest-carrier-free) group first: C, A, B, ...
        o.push_back(ngroups - 1);
        for (int i = 0; i < ngroups - 1; i++) o.push_back(i);
        return o;
    }
    o.push_back(1);
    o.push_back(0);
    for (int i = 2; i < ngroups; i++) o.push_back(i);
    return o;
}

static void push_mixer(std::vector<Event>& ev, const std::vector<int>& order, double beta, bool reversed, int vec,
                       int res) {
    const int ng = (int)order.size();
    for (int i = 0; i < ng; i++) {
        Event e{EV_MIX};
        e.group = order[reversed ? ng - 1 - i : i];
        e.angle = beta;
        e.vec = vec;
        e.res = res;
        ev.push_back(e);
    }
}

extern "C" int sv_mixer(sv_state s, double beta) {
    if (!s) return fail(SV_ERR_ARG, "sv_mixer: NULL state");
    if (!std::isfinite(beta)) return fail(SV_ERR_NUMERIC, "sv_mixer: beta is not finite");
    Plan plan = make_plan(s->n, s->dt);
    std::vector<Event> ev;
    push_mixer(ev, group_order((int)plan.by_nv[1].size(), 0, s->n), beta, false, 1, -1);
    Program prog = build_program(ev, 0, true);
    return run_program(s, nullptr, nullptr, prog, plan, false);
}

// Forward circuit events: layer k applies the phase then the mixer groups in
// snake order (odd layers ascending, even layers descending), so consecutive
// layers meet on the same tile group and share a pass.
static void forward_events(std::vector<Event>& ev, const std::vector<int>& order, int p, const double* gamma,
                           const double* beta, bool from_plus, int reduce_every_step_base) {
    if (from_plus) ev.push_back(Event{EV_INIT});
    for (int k = 0; k < p; k++) {
        Event ph{EV_PHASE};
        ph.angle = gamma[k];
        ev.push_back(ph);
        push_mixer(ev, order, beta[k], (k % 2) == 1, 1, -1);
        if (reduce_every_step_base >= 0) {
            Event r{EV_REDUCE};
            r.res = reduce_every_step_base + 3 * k;
            ev.push_back(r);
        }
    }
}

extern "C" int sv_qaoa_forward(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                               int from_plus) {
    int rc = check_pair(s, H, "sv_qaoa_forward");
    if (rc) return rc;
    rc = check_angles(p, gamma, beta, "sv_qaoa_forward");
    if (rc) return rc;
    Plan plan = make_plan(s->n, s->dt);
    std::vector<Event> ev;
    forward_events(ev, group_order((int)plan.by_nv[1].size(), (int)s->dt, s->n), p, gamma, beta, from_plus != 0, -1);
    Program prog = build_program(ev, 0, knob_for("fuse", (int)s->dt, s->n) != 0);
    return run_program(s, nullptr, H, prog, plan, false);
}

// Program of one energy evaluation: the forward circuit with the reduction
// (results 0..2: norm, energy, p_gs) merged into its last mixer pass.
static Program energy_program(const sv_state_s* s, const Plan& plan, int p, const double* gamma, const double* beta,
                              int from_plus) {
    std::vector<Event> ev;
    forward_events(ev, group_order((int)plan.by_nv[1].size(), (int)s->dt, s->n), p, gamma, beta, from_plus != 0, -1);
    Event r{EV_REDUCE};
    r.res = 0;
    ev.push_back(r);  // merges into the last mixer pass as its point op
    return build_program(ev, 3, knob_for("fuse", (int)s->dt, s->n) != 0);
}

int sv_internal_set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int sv_internal_qaoa_energy_fixed(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                                  int from_plus, int device, const FixedScratch& fx) {
    int rc = check_pair(s, H, "sv_qaoa_energy_noalloc");
    if (rc) return rc;
    rc = check_angles(p, gamma, beta, "sv_qaoa_energy_noalloc");
    if (rc) return rc;
    if (s->device != device)
        return fail(SV_ERR_ARG, "sv_qaoa_energy_noalloc: the state lives on device %d, device %d is current", s->device,
                    device);
    Plan plan = make_plan(s->n, s->dt);
    Program prog = energy_program(s, plan, p, gamma, beta, from_plus);
    return run_program(s, nullptr, H, prog, plan, true, &fx);
}

extern "C" int sv_qaoa_energy(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                              int from_plus, double* energy, double* p_gs, double* norm) {
    int rc = check_pair(s, H, "sv_qaoa_energy");
    if (rc) return rc;
    rc = check_angles(p, gamma, beta, "sv_qaoa_energy");
    if (rc) return rc;
    Plan plan = make_plan(s->n, s->dt);
    Program prog = energy_program(s, plan, p, gamma, beta, from_plus);
    rc = run_program(s, nullptr, H, prog, plan, true);
    if (rc) return rc;
    rc = fetch_results(s, 3);
    if (rc) return rc;
    if (norm) *norm = s->w.h_res[0];
    if (energy) *energy = s->w.h_res[1];
    if (p_gs) *p_gs = s->w.h_res[2];
    return SV_OK;
}

extern "C" int sv_aqa_run_observe(sv_state s, sv_ising H, int steps, const double* gamma, const double* beta,
                                  double* pgs_per_step, double* energy_per_step, double* spinz_per_step) {
    int rc = check_pair(s, H, "sv_aqa_run");
    if (rc) return rc;
    rc = check_angles(steps, gamma, beta, "sv_aqa_run");
    if (rc) return rc;
    const bool want = pgs_per_step || energy_per_step;
    const bool spins = spinz_per_step != nullptr;
    Plan plan = make_plan(s->n, s->dt);
    std::vector<Event> ev;
    forward_events(ev, group_order((int)plan.by_nv[1].size(), (int)s->dt, s->n), steps, gamma, beta, true,
                   want ? 0 : -1);
    // per-step spin sums ride in the pass that ends each step (after its reduction, if any)
    const int nres = (want ? 3 * steps : 0) + (spins ? steps * s->n : 0);
    if (spins) {
        std::vector<Event> with;
        int k = 0;
        for (size_t i = 0; i < ev.size(); i++) {
            with.push_back(ev[i]);
            const bool step_end = (i + 1 == ev.size()) || ev[i + 1].kind == EV_PHASE;
            if (step_end && ev[i].kind != EV_INIT && ev[i].kind != EV_PHASE) {
                Event sz{EV_SPINZ};
                sz.res = (want ? 3 * steps : 0) + k * s->n;
                with.push_back(sz);
                k++;
            }
        }
        ev.swap(with);
    }
    Program prog = build_program(ev, nres, knob_for("fuse", (int)s->dt, s->n) != 0);
    rc = run_program(s, nullptr, H, prog, plan, want);
    if (rc || nres == 0) return rc;
    rc = fetch_results(s, nres);
    if (rc) return rc;
    for (int k = 0; k < steps; k++) {
        if (pgs_per_step) pgs_per_step[k] = s->w.h_res[3 * k + 2];
        if (energy_per_step) energy_per_step[k] = s->w.h_res[3 * k + 1];
    }
    if (spins) {
        const double* sp = s->w.h_res + (want ? 3 * steps : 0);
        for (int k = 0; k < steps * s->n; k++) spinz_per_step[k] = sp[k];
    }
    return SV_OK;
}

extern "C" int sv_aqa_run(sv_state s, sv_ising H, int steps, const double* gamma, const double* beta,
                          double* pgs_per_step, double* energy_per_step) {
    return sv_aqa_run_observe(s, H, steps, gamma, beta, pgs_per_step, energy_per_step, nullptr);
}

extern "C" int sv_spin_z(sv_state s, double* out) {
    if (!s || !out) return fail(SV_ERR_ARG, "sv_spin_z: NULL argument");
    Plan plan = make_plan(s->n, s->dt);
    Event sz{EV_SPINZ};
    sz.res = 0;
    Program prog = build_program({sz}, s->n, true);
    prog.passes[0].store = 0;
    int rc = run_program(s, nullptr, nullptr, prog, plan, false);
    if (rc) return rc;
    rc = fetch_results(s, s->n);
    if (rc) return rc;
    for (int i = 0; i < s->n; i++) out[i] = s->w.h_res[i];
    return SV_OK;
}

// ============================================================================ general layers
// Events of one general single-qubit layer: every tile group once, in snake order.
static void push_layer(std::vector<Event>& ev, const std::vector<int>& order, int layer, bool reversed) {
    const int ng = (int)order.size();
    for (int i = 0; i < ng; i++) {
        Event e{EV_MIX};
        e.group = order[reversed ? ng - 1 - i : i];
        e.gm = layer;
        ev.push_back(e);
    }
}

extern "C" int sv_gate_layers(sv_state s, int nlayers, const double* U) {
    if (!s) return fail(SV_ERR_ARG, "sv_gate_layers: NULL state");
    if (nlayers < 0) return fail(SV_ERR_ARG, "sv_gate_layers: nlayers=%d < 0", nlayers);
    if (nlayers == 0) return SV_OK;
    if (!U) return fail(SV_ERR_ARG, "sv_gate_layers: NULL matrices");
    const size_t cnt = (size_t)nlayers * s->n * 8;
    for (size_t i = 0; i < cnt; i++)
        if (!std::isfinite(U[i]))
            return fail(SV_ERR_NUMERIC, "sv_gate_layers: non-finite entry in layer %d, qubit %d", (int)(i / 8 / s->n),
                        (int)(i / 8 % s->n));
    Plan plan = make_plan(s->n, s->dt, false, true);
    const std::vector<int> order = group_order((int)plan.by_nv[1].size(), (int)s->dt, s->n);
    const int ng = (int)order.size();
    // Gates on different qubits commute, so each tile group takes up to four
    // consecutive layers in one pass (the pass shape has four mixer slots).
    std::vector<Event> ev;
    for (int c0 = 0; c0 < nlayers; c0 += 4) {
        const int c1 = std::min(nlayers, c0 + 4);
        for (int gi = 0; gi < ng; gi++) {
            for (int l = c0; l < c1; l++) {
                Event e{EV_MIX};
                e.group = order[gi];
                e.gm = l;
                ev.push_back(e);
            }
        }
    }
    Program prog = build_program(ev, 0, true);
    prog.layers = U;
    prog.nq = s->n;
    return run_program(s, nullptr, nullptr, prog, plan, false);
}

// exp(i theta (a X + c Z)) with Z = diag(-1, +1) (the paper's |0> is the -1
// eigenstate): cos(theta r) I + i sin(theta r) / r (a X + c Z), r = |(a, c)|.
static void spin_exp(double theta, double a, double c, double m[8]) {
    const double r = std::hypot(a, c);
    const double cs = std::cos(theta * r);
    const double sr = r > 0.0 ? std::sin(theta * r) / r : theta;
    const double v[8] = {cs, -sr * c, 0.0, sr * a, 0.0, sr * a, cs, sr * c};
    memcpy(m, v, sizeof(v));
}

// 2x2 complex product out = x y (row-major, interleaved re/im).
static void mat_mul(const double* x, const double* y, double* out) {
    double o[8];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 2; k++) {
                const double ar = x[(2 * i + k) * 2], ai = x[(2 * i + k) * 2 + 1];
                const double br = y[(2 * k + j) * 2], bi = y[(2 * k + j) * 2 + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            o[(2 * i + j) * 2] = re;
            o[(2 * i + j) * 2 + 1] = im;
        }
    memcpy(out, o, sizeof(o));
}

// Second-order product-formula time stepping of Eq. AQA4 for the annealing
// Hamiltonian of Eqs. AQA0-AQA3 (x fields A, z fields -B h_i, zz couplings -B J_ij):
// step l applies M_l P_J(tau B_l) M_l with M_l = prod_i exp(i tau/2 (A_l X_i - B_l h_i Z_i))
// and P_J(gamma) = exp(-i gamma sum_{i<j} J_ij s_i s_j).  On the device P_J is the cost
// phase exp(-i gamma E) times the diagonal exp(+i gamma sum_i h_i s_i), which is folded
// into the single-qubit matrix beside it: N_l = D_l M_l.  Without per-step observables the
// outer halves of consecutive steps merge, so a step costs one general layer and one phase.
extern "C" int sv_qsds_run(sv_state s, sv_ising H, int steps, double tau, const double* A, const double* B,
                           int from_plus, double* energy_per_step, double* pgs_per_step, double* spinz_per_step) {
    int rc = check_pair(s, H, "sv_qsds_run");
    if (rc) return rc;
    if (steps < 1) return fail(SV_ERR_ARG, "sv_qsds_run: steps=%d < 1", steps);
    if (!A || !B) return fail(SV_ERR_ARG, "sv_qsds_run: NULL schedule array");
    if (!std::isfinite(tau)) return fail(SV_ERR_NUMERIC, "sv_qsds_run: tau is not finite");
    for (int l = 0; l < steps; l++)
        if (!std::isfinite(A[l]) || !std::isfinite(B[l]))
            return fail(SV_ERR_NUMERIC, "sv_qsds_run: non-finite schedule value at step %d", l);
    const int n = s->n;
    const bool want = energy_per_step || pgs_per_step;
    const bool spins = spinz_per_step != nullptr;
    const bool observe = want || spins;
    std::vector<double> Mh((size_t)steps * n * 8), Nh((size_t)steps * n * 8);
    for (int l = 0; l < steps; l++) {
        const double gam = tau * B[l];
        for (int i = 0; i < n; i++) {
            double* m = &Mh[((size_t)l * n + i) * 8];
            double* nn = &Nh[((size_t)l * n + i) * 8];
            spin_exp(0.5 * tau, A[l], -B[l] * H->h[i], m);
            // D = diag(exp(-i gam h_i), exp(+i gam h_i)) times M: scale the rows
            const double c = std::cos(gam * H->h[i]), sn = std::sin(gam * H->h[i]);
            for (int row = 0; row < 2; row++) {
                const double dr = c, di = row == 0 ? -sn : sn;
                for (int col = 0; col < 2; col++) {
                    const double xr = m[(2 * row + col) * 2], xi = m[(2 * row + col) * 2 + 1];
                    nn[(2 * row + col) * 2] = dr * xr - di * xi;
                    nn[(2 * row + col) * 2 + 1] = dr * xi + di * xr;
                }
            }
        }
    }
    // layer list and events
    std::vector<double> layers;
    auto add_layer = [&](const double* src) { layers.insert(layers.end(), src, src + (size_t)n * 8); };
    Plan plan = make_plan(n, s->dt, false, true);
    const std::vector<int> order = group_order((int)plan.by_nv[1].size(), (int)s->dt, n);
    std::vector<Event> ev;
    if (from_plus) ev.push_back(Event{EV_INIT});
    int nl = 0;
    auto layer_events = [&]() {
        push_layer(ev, order, nl, (nl % 2) == 1);
        nl++;
    };
    auto phase = [&](int l) {
        Event ph{EV_PHASE};
        ph.angle = tau * B[l];
        ev.push_back(ph);
    };
    const int nres = (want ? 3 * steps : 0) + (spins ? steps * n : 0);
    if (!observe) {
        add_layer(&Nh[0]);
        layer_events();
        std::vector<double> prod((size_t)n * 8);
        for (int l = 0; l < steps; l++) {
            phase(l);
            if (l + 1 < steps) {
                for (int i = 0; i < n; i++)
                    mat_mul(&Nh[((size_t)(l + 1) * n + i) * 8], &Mh[((size_t)l * n + i) * 8], &prod[(size_t)i * 8]);
                add_layer(prod.data());
            } else {
                add_layer(&Mh[(size_t)l * n * 8]);
            }
            layer_events();
        }
    } else {
        for (int l = 0; l < steps; l++) {
            add_layer(&Nh[(size_t)l * n * 8]);
            layer_events();
            phase(l);
            add_layer(&Mh[(size_t)l * n * 8]);
            layer_events();
            if (want) {
                Event r{EV_REDUCE};
                r.res = 3 * l;
                ev.push_back(r);
            }
            if (spins) {
                Event sz{EV_SPINZ};
                sz.res = (want ? 3 * steps : 0) + l * n;
                ev.push_back(sz);
            }
        }
    }
    Program prog = build_program(ev, nres, knob_for("fuse", (int)s->dt, n) != 0);
    prog.layers = layers.data();
    prog.nq = n;
    rc = run_program(s, nullptr, H, prog, plan, want);
    if (rc || nres == 0) return rc;
    rc = fetch_results(s, nres);
    if (rc) return rc;
    for (int l = 0; l < steps; l++) {
        if (energy_per_step) energy_per_step[l] = s->w.h_res[3 * l + 1];
        if (pgs_per_step) pgs_per_step[l] = s->w.h_res[3 * l + 2];
    }
    if (spins) {
        const double* sp = s->w.h_res + (want ? 3 * steps : 0);
        for (int k = 0; k < steps * n; k++) spinz_per_step[k] = sp[k];
    }
    return SV_OK;
}

extern "C" int sv_expect(sv_state s, sv_ising H, double* energy, double* p_gs, double* norm) {
    int rc = check_pair(s, H, "sv_expect");
    if (rc) return rc;
    Plan plan = make_plan(s->n, s->dt);
    Event r{EV_REDUCE};
    r.res = 0;
    Program prog = build_program({r}, 3, true);
    prog.passes[0].store = 0;
    rc = run_program(s, nullptr, H, prog, plan, true);
    if (rc) return rc;
    rc = fetch_results(s, 3);
    if (rc) return rc;
    if (norm) *norm = s->w.h_res[0];
    if (energy) *energy = s->w.h_res[1];
    if (p_gs) *p_gs = s->w.h_res[2];
    return SV_OK;
}

// Adjoint by two one-vector reverse sweeps.  psi_k and lambda_k = U_{k+1}^+ ... U_p^+ H psi_p
// are carried back by the same unitaries, so zeta_s = psi + i s t lambda (s = +1, -1) is too,
// and for a Hermitian A (sum of sigma^x_q, or H_C) expanding the quadratic form gives
//   <zeta_+|A|zeta_+> - <zeta_-|A|zeta_-> = 4 t Im <lambda|A|psi>,
// the quantity of the two-vector sweep (df/dbeta_k: A = H_D inside layer k's mixer;
// df/dgamma_k: A = H_C between the phase and the mixer of layer k).  Each sweep is a chain of
// one-vector passes (two workgroups per CU) that undoes the layers and accumulates the forms:
// 2 Re(conj(a) b) per butterfly pair and E |zeta|^2 at the phase.  The forward circuit stops
// before the last mixer group of layer p; each sweep's first pass applies that group, forms
// zeta = psi_p (1 + i s t E) pointwise (the zeta_+ pass also reduces norm, <H_C> and P_gs of
// psi_p) and undoes the group again, so psi_p itself is never stored.  t is fixed before the
// circuit runs: 1 / sqrt(sum h^2 + sum J^2), the spread of H_C in |+>, which keeps |psi| and
// t |lambda| of one order.  zeta_+ goes to lam's buffer (its first pass reads psi's), zeta_-
// then overwrites psi; everything runs on psi's stream.
static int grad_zeta(sv_state_s* psi, sv_state_s* lam, sv_ising_s* H, int p, const double* gamma,
                     const double* beta, int psi_is_forward, double* energy, double* p_gs, double* dgamma,
                     double* dbeta) {
    Plan plan = make_plan(psi->n, psi->dt);
    const std::vector<int> order = group_order((int)plan.by_nv[1].size(), (int)psi->dt, psi->n);
    const bool fuse = knob_for("fuse", (int)psi->dt, psi->n) != 0;
    double s2 = 0.0;
    for (double v : H->h) s2 += v * v;
    for (double v : H->J) s2 += v * v;
    const double t = s2 > 0.0 ? 1.0 / std::sqrt(s2) : 1.0;
    // forward circuit without the last mixer group of layer p
    std::vector<Event> ev;
    Event last{EV_MIX};
    if (!psi_is_forward) {
        forward_events(ev, order, p, gamma, beta, true, -1);
        last = ev.back();
        ev.pop_back();
        if (last.kind != EV_MIX) return fail(SV_ERR_ARG, "internal: forward circuit does not end in a mixer");
        Program fwd = build_program(ev, 0, fuse);
        int rc = run_program(psi, nullptr, H, fwd, plan, false);
        if (rc) return rc;
    }
    // the reverse sweep of one zeta: (last group) reductions, zeta, undo layer p .. 1 with the forms
    auto sweep = [&](double ts, bool reduce) {
        std::vector<Event> rev;
        if (!psi_is_forward) rev.push_back(last);
        if (reduce) {
            Event r{EV_REDUCE};
            r.res = 2 * p;
            rev.push_back(r);
        }
        Event z{EV_ZETA};
        z.angle = ts;
        rev.push_back(z);
        for (int k = p - 1; k >= 0; k--) {
            push_mixer(rev, order, -beta[k], (k % 2) == 0, 1, p + k);
            Event ef{EV_EFORM};
            ef.res = k;
            rev.push_back(ef);
            if (k > 0) {
                Event ph{EV_PHASE};
                ph.angle = -gamma[k];
                rev.push_back(ph);
            }
        }
        Program prog = build_program(rev, 2 * p + (reduce ? 3 : 0), fuse);
        prog.passes.back().store = 0;
        return prog;
    };
    Program plus = sweep(t, true);
    Program minus = sweep(-t, false);
    const hipStream_t lam_stream = lam->stream;
    lam->stream = psi->stream;
    int rc = run_program(lam, nullptr, H, plus, plan, true, nullptr, psi->ptr);
    lam->stream = lam_stream;
    if (rc) return rc;
    rc = run_program(psi, nullptr, H, minus, plan, false);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(psi->stream);
    if (e != hipSuccess) {
        psi->failed = true;
        return fail(SV_ERR_HIP, "sv_grad: %s", hipGetErrorString(e));
    }
    rc = fetch_results(lam, 2 * p + 3);
    if (rc) return rc;
    rc = fetch_results(psi, 2 * p);
    if (rc) return rc;
    if (energy) *energy = lam->w.h_res[2 * p + 1];
    if (p_gs) *p_gs = lam->w.h_res[2 * p + 2];
    for (int k = 0; k < p; k++) {
        dgamma[k] = (lam->w.h_res[k] - psi->w.h_res[k]) / (2.0 * t);
        dbeta[k] = (lam->w.h_res[p + k] - psi->w.h_res[p + k]) / (2.0 * t);
    }
    return SV_OK;
}

// Reverse sweep of the adjoint method.  Result layout: [0..2] norm, energy,
// pgs; [3 + k] = sum E Im(conj lam psi) for gamma_k; [3 + p + k] = pair sums
// for beta_k.  df/dgamma_k = 2 * res[3+k], df/dbeta_k = 2 * res[3+p+k].
extern "C" int sv_grad(sv_state psi, sv_state lam, sv_ising H, int p, const double* gamma, const double* beta,
                       int psi_is_forward, double* energy, double* p_gs, double* dgamma, double* dbeta) {
    int rc = check_pair(psi, H, "sv_grad");
    if (rc) return rc;
    if (!lam) return fail(SV_ERR_ARG, "sv_grad: NULL lam state");
    if (lam == psi) return fail(SV_ERR_ARG, "sv_grad: psi and lam must be different states");
    if (lam->n != psi->n || lam->dt != psi->dt)
        return fail(SV_ERR_ARG, "sv_grad: lam (n=%d, dtype=%d) does not match psi (n=%d, dtype=%d)", lam->n,
                    (int)lam->dt, psi->n, (int)psi->dt);
    if (!dgamma || !dbeta) return fail(SV_ERR_ARG, "sv_grad: NULL gradient output");
    rc = check_angles(p, gamma, beta, "sv_grad");
    if (rc) return rc;
    if (lam->failed) return fail(SV_ERR_HIP, "lam state is in a failed state");
    // the one-vector sweeps run on the default one-vector tiles (13-bit complex128, 14-bit
    // complex64 with four waves per SIMD)
    const int dt = (int)psi->dt, nq = psi->n;
    const bool zeta_tiles = psi->dt == SV_C128 ? knob_for("c128t14", dt, nq) == 0
                                               : (knob_for("c64t13", dt, nq) == 0 && knob_for("c64occ", dt, nq) != 0);
    const int zeta = knob_for("adjzeta", dt, nq);
    if ((zeta > 0 || (zeta < 0 && psi->dt == SV_C128)) && zeta_tiles)
        return grad_zeta(psi, lam, H, p, gamma, beta, psi_is_forward, energy, p_gs, dgamma, dbeta);
    // both vectors share one tile geometry: plan with the two-vector shape
    Plan plan = make_plan(psi->n, psi->dt, true);
    const std::vector<int> order = group_order((int)plan.by_nv[1].size(), (int)psi->dt, psi->n);
    std::vector<Event> ev;
    if (!psi_is_forward) forward_events(ev, order, p, gamma, beta, true, -1);
    Event r{EV_REDUCE};
    r.res = 0;
    ev.push_back(r);
    ev.push_back(Event{EV_LAMINIT});
    for (int k = p - 1; k >= 0; k--) {
        // undo the mixer of layer k (groups in the reverse of their forward order)
        push_mixer(ev, order, -beta[k], (k % 2) == 0, 3, 3 + p + k);
        Event gg{EV_GGAMMA};
        gg.res = 3 + k;
        ev.push_back(gg);
        if (k > 0) {
            Event ph{EV_PHASE};
            ph.angle = -gamma[k];
            ph.vec = 3;
            ev.push_back(ph);
        }
    }
    Program prog = build_program(ev, 3 + 2 * p, knob_for("fuse", (int)psi->dt, psi->n) != 0);
    // Trims.  In the pass where lam = E psi is formed, psi is mixed forward by
    // one group and then undone by the same group: the loaded values are already
    // that result, so psi is not written back.  The final pass writes nothing.
    if (!psi_is_forward) {
        for (Pass& ps : prog.passes) {
            std::vector<const Op*> fw, un;
            int laminit = -1, phased = 0;
            for (int i = 0; i < (int)ps.ops.size(); i++) {
                const Op& op = ps.ops[i];
                if (op.kind == OP_POINT && (op.flags & PT_LAM_INIT)) laminit = i;
                if (op.kind == OP_POINT && (op.flags & PT_PHASE_PSI)) phased++;
                if (op.kind == OP_MIX && (op.flags & MIX_PSI)) (laminit < 0 ? fw : un).push_back(&op);
            }
            bool inverse = laminit >= 0 && !fw.empty() && fw.size() == un.size() && phased == 0 && !ps.init;
            for (size_t i = 0; inverse && i < fw.size(); i++) {
                const Op* f = fw[fw.size() - 1 - i];
                const Op* u = un[i];
                inverse = (u->a == -f->a) && (std::fabs(u->b) == std::fabs(f->b));
            }
            if (inverse) ps.store &= ~1;
        }
    }
    prog.passes.back().store = 0;
    rc = run_program(psi, lam, H, prog, plan, p_gs != nullptr);
    if (rc) return rc;
    rc = fetch_results(psi, 3 + 2 * p);
    if (rc) return rc;
    if (energy) *energy = psi->w.h_res[1];
    if (p_gs) *p_gs = psi->w.h_res[2];
    for (int k = 0; k < p; k++) {
        dgamma[k] = 2.0 * psi->w.h_res[3 + k];
        dbeta[k] = 2.0 * psi->w.h_res[3 + p + k];
    }
    return SV_OK;
}

// ============================================================================ streaming ceiling
extern "C" int sv_stream_ceiling(sv_state s, int c, int lo, double* ms) {
    if (!s || !ms) return fail(SV_ERR_ARG, "sv_stream_ceiling: NULL argument");
    if (s->failed) return fail(SV_ERR_HIP, "state is in a failed state after an earlier HIP error");
    const int T = s->dt == SV_C128 ? 13 : 14;
    const int g = T - c;
    if (s->n < T || c < 0 || c > T || (g > 0 && (lo < c || lo + g > s->n)))
        return fail(SV_ERR_ARG, "sv_stream_ceiling: geometry c=%d lo=%d does not fit n=%d with %d-bit tiles", c, lo,
                    s->n, T);
    StreamArgs a;
    memset(&a, 0, sizeof(a));
    a.ntiles = 1ull << (s->n - T);
    a.c = c;
    a.lo = g > 0 ? lo : T;
    a.g = g;
    a.xcd = knob_for("xcd", (int)s->dt, s->n);
    if (a.xcd < 0) a.xcd = ((size_t(1) << s->n) * elem_size(s->dt)) > (size_t(64) << 30) ? 3 : 1;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SV_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    e = hipEventRecord(e0, s->stream);
    if (e == hipSuccess) e = (hipError_t)launch_stream((int)s->dt, s->ptr, a, s->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        s->failed = true;
        return fail(SV_ERR_HIP, "sv_stream_ceiling: %s", hipGetErrorString(e));
    }
    *ms = t;
    return SV_OK;
}

// ============================================================================ schedules
extern "C" int sv_schedule_linear(int steps, double tau, int paper_sign, double* gamma, double* beta) {
    if (steps < 1) return fail(SV_ERR_ARG, "sv_schedule_linear: steps=%d < 1", steps);
    if (!gamma || !beta) return fail(SV_ERR_ARG, "sv_schedule_linear: NULL output");
    if (!std::isfinite(tau)) return fail(SV_ERR_NUMERIC, "sv_schedule_linear: tau is not finite");
    for (int k = 1; k <= steps; k++) {
        const double s = (double)k / steps;
        gamma[k - 1] = tau * s;                                    // tau B(s_k), B(s) = s
        beta[k - 1] = (paper_sign ? -1.0 : 1.0) * tau * (1.0 - s);  // tau A(s_k) with H_I = -H_D
    }
    return SV_OK;
}

extern "C" int sv_schedule_second_order(int p, double tau, const double* A, const double* B, double* gamma,
                                        double* beta) {
    if (p < 2) return fail(SV_ERR_ARG, "sv_schedule_second_order: p=%d < 2 (grid (k-1)/(p-1) undefined)", p);
    if (!gamma || !beta) return fail(SV_ERR_ARG, "sv_schedule_second_order: NULL output");
    if (!std::isfinite(tau)) return fail(SV_ERR_NUMERIC, "sv_schedule_second_order: tau is not finite");
    std::vector<double> a(p), b(p);
    for (int k = 0; k < p; k++) {
        const double s = (double)k / (p - 1);
        a[k] = A ? A[k] : 1.0 - s;
        b[k] = B ? B[k] : s;
        if (!std::isfinite(a[k]) || !std::isfinite(b[k]))
            return fail(SV_ERR_NUMERIC, "sv_schedule_second_order: schedule value %d is not finite", k);
    }
    for (int k = 0; k < p; k++) {
        gamma[k] = tau * b[k];
        beta[k] = (k + 1 < p) ? -tau * (a[k + 1] + a[k]) / 2.0 : -tau * a[k] / 2.0;
    }
    return SV_OK;
}

// ============================================================================ describe
extern "C" int sv_tune_describe(int n, sv_dtype dtype, char* buf, size_t len) {
    if (!buf || len == 0) return fail(SV_ERR_ARG, "sv_tune_describe: empty buffer");
    if (!dtype_ok(dtype)) return fail(SV_ERR_ARG, "sv_tune_describe: bad dtype");
    if (n < 1 || n > max_n(dtype)) return fail(SV_ERR_ARG, "sv_tune_describe: bad n");
    std::string js = "{\"knobs\":{";
    {
        std::lock_guard<std::mutex> g(g_knob_mu);
        bool first = true;
        for (auto& kv : g_knobs) {
            js += (first ? "" : ",") + std::string("\"") + kv.first + "\":" + std::to_string(kv.second);
            first = false;
        }
    }
    js += "},\"knobs_for_size\":{";
    {
        std::vector<std::string> names;
        {
            std::lock_guard<std::mutex> g(g_knob_mu);
            for (auto& kv : g_knobs) names.push_back(kv.first);
        }
        bool first = true;
        for (const std::string& k : names) {
            // the values a plan for this (dtype, n) uses: tuned overrides over the global knobs
            const int nsz = (k == "batchwide" || k == "batch128" || k == "batchslab") ? 0 : n;
            js += (first ? "" : ",") + std::string("\"") + k + "\":" + std::to_string(knob_for(k.c_str(), (int)dtype, nsz));
            first = false;
        }
    }
    js += "},\"plans\":{";
    for (int fam = 0; fam < 3; fam++) {
        const int nv = fam == 2 ? 2 : 1;
        // the one-vector family is what make_plan gives the forward programs
        const bool grad = fam >= 1 || (dtype == SV_C64 && knob_for("c64t13", (int)dtype, n) != 0);
        std::vector<Geometry> groups = plan_groups(n, dtype, nv, grad);
        const char* key = fam == 0 ? "nv1" : (fam == 1 ? "grad_nv1" : "grad_nv2");
        js += std::string(fam == 0 ? "" : ",") + "\"" + key + "\":[";
        for (size_t i = 0; i < groups.size(); i++) {
            const Geometry& g = groups[i];
            js += (i ? "," : "") + std::string("{\"T\":") + std::to_string(g.T) + ",\"R\":" + std::to_string(g.R) +
                  ",\"c\":" + std::to_string(g.c) + ",\"lo\":" + std::to_string(g.lo) + ",\"g\":" +
                  std::to_string(g.g) + ",\"ntiles\":" + std::to_string(g.ntiles) + ",\"phantom\":" +
                  std::to_string(g.phantom) + ",\"blocks\":[";
            for (size_t j = 0; j < g.blocks.size(); j++) {
                js += (j ? "," : "") + std::string("{\"bits\":[");
                for (size_t k = 0; k < g.blocks[j].size(); k++)
                    js += (k ? "," : "") + std::to_string(g.blocks[j][k]);
                js += "],\"fwd\":" + std::to_string(g.act_fwd[j]) + ",\"bwd\":" + std::to_string(g.act_bwd[j]) +
                      ",\"dpp\":" + std::to_string(g.dpp[j]) + "}";
            }
            js += "]}";
        }
        js += "]";
    }
    js += "}}";
    snprintf(buf, len, "%s", js.c_str());
    return SV_OK;
}

// ============================================================================ batch scan
extern "C" int sv_batch_p1_scan(int n_inst, const sv_ising* insts, int n_gamma, const double* gammas, int n_beta,
                                const double* betas, sv_dtype dtype, void* stream, double* energy_out,
                                double* pgs_out) {
    if (n_inst < 1 || !insts) return fail(SV_ERR_ARG, "sv_batch_p1_scan: no instances");
    if (n_gamma < 1 || n_beta < 1 || !gammas || !betas) return fail(SV_ERR_ARG, "sv_batch_p1_scan: empty grid");
    if (!energy_out || !pgs_out) return fail(SV_ERR_ARG, "sv_batch_p1_scan: NULL output");
    if (!dtype_ok(dtype)) return fail(SV_ERR_ARG, "sv_batch_p1_scan: bad dtype");
    if ((int64_t)n_gamma * n_beta > (1 << 24)) return fail(SV_ERR_ARG, "sv_batch_p1_scan: grid too large");
    for (int a = 0; a < n_gamma; a++)
        if (!std::isfinite(gammas[a])) return fail(SV_ERR_NUMERIC, "sv_batch_p1_scan: gamma %d not finite", a);
    for (int b = 0; b < n_beta; b++)
        if (!std::isfinite(betas[b])) return fail(SV_ERR_NUMERIC, "sv_batch_p1_scan: beta %d not finite", b);
    const int wide = dtype == SV_C64 ? knob_for("batchwide", (int)dtype, 0) : knob_for("batch128", (int)dtype, 0);
    const int lut_cap = batch_lut_cap((int)dtype, wide);
    const int S = batch_lds_bits((int)dtype, wide);
    const int nmax_batch = S + 5;  // the high bits of a state fit one thread's 32 registers
    std::vector<BatchInst> bi(n_inst);
    std::vector<double> hh, JJ;
    std::vector<int32_t> ii, jj;
    uint64_t etot = 0;
    int max_n = 1;
    for (int i = 0; i < n_inst; i++) {
        const sv_ising_s* H = insts[i];
        if (!H) return fail(SV_ERR_ARG, "sv_batch_p1_scan: instance %d is NULL", i);
        if (H->n > nmax_batch)
            return fail(SV_ERR_UNSUPPORTED, "sv_batch_p1_scan: instance %d has n=%d > %d", i, H->n, nmax_batch);
        BatchInst& b = bi[i];
        b.n = H->n;
        b.m = H->m;
        b.hoff = (int32_t)hh.size();
        b.coff = (int32_t)JJ.size();
        b.eoff = etot;
        etot += 1ull << H->n;
        max_n = std::max(max_n, H->n);
        hh.insert(hh.end(), H->h.begin(), H->h.end());
        JJ.insert(JJ.end(), H->J.begin(), H->J.end());
        ii.insert(ii.end(), H->ei.begin(), H->ei.end());
        jj.insert(jj.end(), H->ej.begin(), H->ej.end());
        b.emin = 0.0;  // filled on the device
        b.etol = ground_tol(H);
        const int L = (int)std::ceil(H->scale);
        if (H->integer && 2 * L + 1 <= lut_cap) {
            b.lut_lo = -L;
            b.lut_n = 2 * L + 1;
        } else {
            b.lut_lo = 0;
            b.lut_n = 0;
        }
    }
    // work units (instance, gamma), largest state first
    std::vector<int32_t> uinst, ugam;
    std::vector<int> order(n_inst);
    for (int i = 0; i < n_inst; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bi[x].n > bi[y].n; });
    for (int i : order)
        for (int a = 0; a < n_gamma; a++) {
            uinst.push_back(i);
            ugam.push_back(a);
        }
    const size_t elem = elem_size(dtype);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const int grid = device_cu_count(dev) * (wide == 2 ? 2 : 1);
    // states above the LDS tile: the sliced path (slab launches) where the variant has
    // 13-bit LDS states, else per-workgroup slots of the persistent kernel
    const int slab_mb = knob_for("batchslab", (int)dtype, 0);
    const bool sliced = slab_mb > 0 && S == 13 && max_n > S;
    const uint64_t slot = (max_n > S && !sliced) ? (1ull << max_n) : 0;
    const size_t slab_bytes = sliced ? std::max((size_t)slab_mb << 20, (size_t(1) << max_n) * elem_size(dtype)) : 0;
    auto states_per_launch = [&](int n) -> int64_t {
        return std::max<int64_t>(1, (int64_t)(slab_bytes / ((size_t(1) << n) * elem_size(dtype))));
    };
    size_t part_doubles = 0;
    if (sliced)
        for (int n = S + 1; n <= max_n; n++)
            part_doubles = std::max(part_doubles, (size_t)states_per_launch(n) * 2 << (n - S));
    const size_t nout = (size_t)n_inst * n_gamma * n_beta;
    hipStream_t st = (hipStream_t)stream;
    // device buffers
    std::vector<void*> bufs;
    bool oom = false;
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            oom = true;
            return nullptr;
        }
        bufs.push_back(p);
        return p;
    };
    auto cleanup = [&]() {
        for (void* p : bufs) (void)hipFree(p);
        bufs.clear();
    };
    BatchArgs ba;
    memset(&ba, 0, sizeof(ba));
    BatchInst* d_inst = (BatchInst*)dalloc(bi.size() * sizeof(BatchInst));
    double* d_h = (double*)dalloc(hh.size() * sizeof(double));
    double* d_J = (double*)dalloc(JJ.size() * sizeof(double));
    int32_t* d_ei = (int32_t*)dalloc(ii.size() * sizeof(int32_t));
    int32_t* d_ej = (int32_t*)dalloc(jj.size() * sizeof(int32_t));
    double* d_e = (double*)dalloc(etot * sizeof(double));
    uint16_t* d_x = (uint16_t*)dalloc(etot * sizeof(uint16_t));
    int32_t* d_ui = (int32_t*)dalloc(uinst.size() * sizeof(int32_t));
    int32_t* d_ug = (int32_t*)dalloc(ugam.size() * sizeof(int32_t));
    double* d_g = (double*)dalloc(n_gamma * sizeof(double));
    double* d_b = (double*)dalloc(n_beta * sizeof(double));
    double* d_oe = (double*)dalloc(nout * sizeof(double));
    double* d_op = (double*)dalloc(nout * sizeof(double));
    unsigned* d_cnt = (unsigned*)dalloc(sizeof(unsigned));
    void* d_scr = dalloc(slot * grid * elem);
    void* d_slab = sliced ? dalloc(slab_bytes) : nullptr;
    // partial sums, two buffers: a launch's columns fill one while its slice kernel
    // finishes the previous launch's states from the other
    double* d_part = sliced ? (double*)dalloc(2 * part_doubles * sizeof(double)) : nullptr;
    if (oom) {
        cleanup();
        return fail(SV_ERR_OOM, "sv_batch_p1_scan: device allocation failed");
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* d, const void* h, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st);
    };
    up(d_inst, bi.data(), bi.size() * sizeof(BatchInst));
    up(d_h, hh.data(), hh.size() * sizeof(double));
    up(d_J, JJ.data(), JJ.size() * sizeof(double));
    up(d_ei, ii.data(), ii.size() * sizeof(int32_t));
    up(d_ej, jj.data(), jj.size() * sizeof(int32_t));
    up(d_ui, uinst.data(), uinst.size() * sizeof(int32_t));
    up(d_ug, ugam.data(), ugam.size() * sizeof(int32_t));
    up(d_g, gammas, n_gamma * sizeof(double));
    up(d_b, betas, n_beta * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(d_cnt, 0, sizeof(unsigned), st);
    ba.inst = d_inst;
    ba.ninst = n_inst;
    ba.h = d_h;
    ba.ei = d_ei;
    ba.ej = d_ej;
    ba.J = d_J;
    ba.etab = d_e;
    ba.eidx = d_x;
    ba.unit_inst = d_ui;
    ba.unit_gam = d_ug;
    ba.nunits = (int32_t)uinst.size();
    ba.gammas = d_g;
    ba.ng = n_gamma;
    ba.betas = d_b;
    ba.nb = n_beta;
    ba.out_e = d_oe;
    ba.out_p = d_op;
    ba.counter = d_cnt;
    ba.scratch = d_scr;
    ba.scratch_elems = slot;
    int ke = 0;
    if (e == hipSuccess) ke = launch_batch_energy(ba, max_n, st);
    if (e == hipSuccess && !ke) {
        hipEvent_t ev0;
        const bool prof = prof_begin(st, &ev0);
        if (!sliced) {
            ke = launch_batch_scan((int)dtype, ba, grid, wide, st);
        } else {
            // units are sorted by n, largest first: those with n <= S take the persistent
            // kernel, the others go through slab launches of one n each
            size_t first_small = 0;
            while (first_small < uinst.size() && bi[uinst[first_small]].n > S) first_small++;
            if (first_small < uinst.size()) {
                BatchArgs bs = ba;
                bs.unit_inst = d_ui + first_small;
                bs.unit_gam = d_ug + first_small;
                bs.nunits = (int32_t)(uinst.size() - first_small);
                ke = launch_batch_scan((int)dtype, bs, grid, wide, st);
            }
            BatchArgs prev = ba;  // the launch whose states are still to be finished
            prev.s_count = 0;
            int nlaunch = 0;
            auto finish_of = [&](BatchArgs& bs) {
                bs.f_n = prev.s_n;
                bs.f_u0 = prev.s_u0;
                bs.f_base = prev.s_base;
                bs.f_count = prev.s_count;
                bs.f_part = prev.part;
            };
            for (size_t u0 = 0; u0 < first_small && !ke;) {
                const int n = bi[uinst[u0]].n;
                size_t u1 = u0;
                while (u1 < first_small && bi[uinst[u1]].n == n) u1++;
                const int64_t states = (int64_t)(u1 - u0) * n_beta;
                const int64_t per = states_per_launch(n);
                for (int64_t s0 = 0; s0 < states && !ke; s0 += per) {
                    BatchArgs bs = ba;
                    bs.s_n = n;
                    bs.s_u0 = (int32_t)u0;
                    bs.s_base = s0;
                    bs.s_count = (int32_t)std::min(per, states - s0);
                    bs.slab = d_slab;
                    bs.part = d_part + (nlaunch & 1) * part_doubles;
                    finish_of(bs);
                    ke = launch_batch_sliced((int)dtype, bs, wide, st);
                    prev = bs;
                    nlaunch++;
                }
                u0 = u1;
            }
            if (!ke && prev.s_count > 0) {
                BatchArgs bs = ba;
                finish_of(bs);
                ke = launch_batch_finish(bs, st);
            }
        }
        if (prof) prof_end(st, ev0, std::string("batch_") + (dtype == SV_C128 ? "c128" : "c64"), 0.0);
    }
    if (e == hipSuccess && !ke) e = hipMemcpyAsync(energy_out, d_oe, nout * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && !ke) e = hipMemcpyAsync(pgs_out, d_op, nout * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && !ke) e = hipStreamSynchronize(st);
    cleanup();
    if (ke) return fail(SV_ERR_HIP, "batch launch failed: %s", hipGetErrorString((hipError_t)ke));
    if (e != hipSuccess) return fail(SV_ERR_HIP, "sv_batch_p1_scan: %s", hipGetErrorString(e));
    return SV_OK;
}
