// libsv host: tile geometries and their device tables, pass programs, program
// execution (launch sequencing, reductions, results) and ground states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <complex>
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

// ============================================================================ geometry

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
std::vector<Geometry> plan_groups(int n, sv_dtype dt, int nv, bool grad, bool general) {
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

// General single-qubit layers in unit-diagonal form (kernel side: MIX_GUNIT).
// A matrix M = [[a, b], [c, d]] with |a|, |d| >= 1/4 and |d| = |a| (to 1e-9, as
// for every unitary) is written M = |a| D N with
// D = diag(a, d) / |a| and N = [[1, b/a], [c/d, 1]]: the kernel applies N at
// half the arithmetic of a general 2x2 matrix and multiplies the pass's
// pending scale by |a|.  D is carried to the right of the later layers of its
// qubit (N' D = D (D^-1 N' D), and D^-1 N' D again has a unit diagonal) and
// of the diagonal phase ops (which commute with it), until the next layer in
// the general form applies M D; the last layer always takes the general form,
// so the state leaves the program exact.  Observables of |psi|^2 (energy,
// P_gs, spins) do not see D, whose entries have modulus one.  Layers are
// applied in index order, each once per qubit (both callers build them so).
// pass_ops: the general ops of each pass as (layer, qubits of its tile group).
// A pass runs one kernel, so its ops all take the same form: the unit form
// where every matrix of every op of the pass allows it.  An op (a layer on one
// tile group) occurs in one pass only, so the choice is settled pass by pass.
static GenLayers unit_diagonal_layers(const double* L, int nl, int n, bool enable,
                                      const std::vector<std::vector<std::pair<int, std::vector<int>>>>& pass_ops) {
    using cd = std::complex<double>;
    GenLayers gl;
    gl.m.assign(L, L + (size_t)nl * n * 8);
    gl.unit.assign((size_t)nl * n, 0);
    gl.mod.assign((size_t)nl * n, 1.0);
    if (!enable) return gl;
    auto eligible = [&](int ly, int q) {
        if (ly + 1 >= nl) return false;  // the last layer applies what is still pending
        const double* m = L + ((size_t)ly * n + q) * 8;
        const double aa = std::abs(cd(m[0], m[1])), ad = std::abs(cd(m[6], m[7]));
        return aa >= 0.25 && ad >= 0.25 && std::abs(ad / aa - 1.0) <= 1e-9;
    };
    for (const auto& ops : pass_ops) {
        bool all = true;
        for (const auto& op : ops)
            for (int q : op.second) all = all && eligible(op.first, q);
        if (!all) continue;
        for (const auto& op : ops)
            for (int q : op.second) gl.unit[(size_t)op.first * n + q] = 1;
    }
    std::vector<cd> d0(n, cd(1.0)), d1(n, cd(1.0));  // pending diagonal of each qubit
    for (int ly = 0; ly < nl; ly++) {
        const double* M = L + (size_t)ly * n * 8;
        for (int q = 0; q < n; q++) {
            const bool unit = gl.unit[(size_t)ly * n + q] != 0;
            const double* m = M + 8 * q;
            const cd a(m[0], m[1]), b(m[2], m[3]), c(m[4], m[5]), d(m[6], m[7]);
            double* o = gl.m.data() + ((size_t)ly * n + q) * 8;
            if (unit) {
                // D^-1 N D with D = diag(d0, d1): off-diagonals times d1/d0 and d0/d1
                const double aa = std::abs(a);
                const cd x = b / a * (d1[q] / d0[q]), y = c / d * (d0[q] / d1[q]);
                const double v[8] = {1.0, 0.0, x.real(), x.imag(), y.real(), y.imag(), 1.0, 0.0};
                memcpy(o, v, sizeof(v));
                gl.mod[(size_t)ly * n + q] = aa;
                d0[q] *= a / aa;
                d1[q] *= d / aa;
            } else {
                // M D applies the pending diagonal
                const cd p = a * d0[q], r = b * d1[q], t = c * d0[q], w = d * d1[q];
                const double v[8] = {p.real(), p.imag(), r.real(), r.imag(), t.real(), t.imag(), w.real(), w.imag()};
                memcpy(o, v, sizeof(v));
                d0[q] = d1[q] = cd(1.0);
            }
        }
    }
    return gl;
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

void release_plain_geos() {
    std::lock_guard<std::mutex> g(g_geo_mu);
    if (g_plain_geos.empty()) return;
    (void)hipDeviceSynchronize();  // launches that may still read them
    for (auto& kv : g_plain_geos) (void)hipFree(kv.second);
    g_plain_geos.clear();
}

// Tile order of a pass (PassArgs::xcd) for knob value x: x >= 0 as given; -1: 8
// interleaved streams (x = 1) up to 64 GiB states, 32 (x = 3) above; -2: by tile
// group, 32 streams for a group whose bits start at 20 or above (runs megabytes
// apart) and for every group of a state above 64 GiB, 8 for the others.
int xcd_order(int x, const Geometry& geo, int n, sv_dtype dt) {
    const bool big = ((size_t(1) << n) * elem_size(dt)) > (size_t(64) << 30);
    if (x == -1) return big ? 3 : 1;
    if (x == -2) return (big || (geo.g > 0 && geo.lo >= 20)) ? 3 : 1;
    return x;
}

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
Program build_program(const std::vector<Event>& evs, int nres, bool fuse) {
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
double ground_tol(const sv_ising_s* H) { return H->qden > 0 ? 0.0 : 1e-9 * std::max(1.0, H->scale); }



// grad: the adjoint family, whose one- and two-vector tiles share T.
Plan make_plan(int n, sv_dtype dt, bool grad, bool general) {
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
int run_program(sv_state_s* s, sv_state_s* lam, sv_ising_s* H, Program& prog, const Plan& plan,
                       bool need_ground, const FixedScratch* fx, const void* first_src) {
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
    // (matrix of tile bit l at 8 l; identity for phantom bits), in the unit-diagonal
    // form where the layer allows it
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
        // qubits a general op of a pass acts on: the active tile bits of its group
        auto op_qubits = [&](const Geometry& geo) {
            std::vector<int> qs;
            for (int l = geo.g == 0 ? 0 : geo.c; l < std::min(geo.T, geo.n); l++) {
                const int q = global_bit(geo, l);
                if (q >= 0) qs.push_back(q);
            }
            return qs;
        };
        int nl = 0;
        std::vector<std::vector<std::pair<int, std::vector<int>>>> pass_ops;
        for (const Pass& ps : prog.passes) {
            const std::vector<int> qs = op_qubits(plan.by_nv[ps.nv][ps.group]);
            std::vector<std::pair<int, std::vector<int>>> ops;
            for (const Op& op : ps.ops)
                if (op.kind == OP_MIX && (op.flags & MIX_GEN)) {
                    nl = std::max(nl, op.qidx + 1);
                    ops.emplace_back(op.qidx, qs);
                }
            if (!ops.empty()) pass_ops.push_back(ops);
        }
        const GenLayers gl = unit_diagonal_layers(prog.layers, nl, s->n, knob_for("genunit", (int)s->dt, s->n) != 0,
                                                  pass_ops);
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
                Op& op = prog.passes[pi].ops[i];
                const int layer = op.qidx;
                bool real = true;
                for (int l = 0; l < kGenBlock / 8; l++) {
                    const int q = l < geo.T ? global_bit(geo, l) : -1;
                    if (q < 0) {
                        const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
                        memcpy(blk + 8 * l, id, sizeof(id));
                    } else {
                        memcpy(blk + 8 * l, gl.m.data() + ((size_t)layer * s->n + q) * 8, 8 * sizeof(double));
                    }
                    for (int c = 1; c < 8; c += 2) real = real && blk[8 * l + c] == 0.0;
                }
                genreal[pi][i] = real;
                const std::vector<int> qs = op_qubits(geo);
                if (!qs.empty() && gl.unit[(size_t)layer * s->n + qs[0]]) {  // all or none of the op's qubits
                    // the moduli of the op's qubits join the pending scale
                    double sc = 1.0;
                    for (int q : qs) sc *= gl.mod[(size_t)layer * s->n + q];
                    op.flags |= MIX_GUNIT;
                    op.b = sc;
                }
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
        a.xcd = xcd_order(knob_for("xcd", (int)s->dt, s->n), geo, s->n, s->dt);
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
        a.gen_unit = 0;
        for (int i = 0; i < kMaxOps; i++) {
            if (genblk[pi][i] < 0) continue;
            if (!genreal[pi][i]) a.gen_real = 0;
            if (p.ops[i].flags & MIX_GUNIT) a.gen_unit = 1;  // every general op of the pass, by construction
        }
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

int fetch_results(sv_state_s* s, int nres) {
    if (nres <= 0) return SV_OK;
    hipError_t e = hipMemcpyAsync(s->w.h_res, s->w.d_res, nres * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->failed = true;
        return fail(SV_ERR_HIP, "result copy failed: %s", hipGetErrorString(e));
    }
    return SV_OK;
}


// ============================================================================ ground
int run_ground(sv_ising_s* H, hipStream_t stream) {
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

