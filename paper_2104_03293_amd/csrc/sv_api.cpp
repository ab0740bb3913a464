// libsv host: states, instances and the circuit entry points of the C ABI
// (include/sv.h): argument checks, event lists and their programs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
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

// ============================================================================ states
static std::atomic<int> g_live_states{0};  // states not yet freed (sv_alloc, sv_wrap)

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
    g_live_states++;
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
    g_live_states++;
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
    if (--g_live_states == 0) release_plain_geos();
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
    {
        Geometry geo{};
        geo.c = c;
        geo.lo = a.lo;
        geo.g = g;
        a.xcd = xcd_order(knob_for("xcd", (int)s->dt, s->n), geo, s->n, s->dt);
    }
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
    const std::vector<std::string> names = knob_names();
    std::string js = "{\"knobs\":{";
    {
        bool first = true;
        for (const std::string& k : names) {
            js += (first ? "" : ",") + std::string("\"") + k + "\":" + std::to_string(knob(k.c_str()));
            first = false;
        }
    }
    js += "},\"knobs_for_size\":{";
    {
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

