// Host-side internals of libsv shared by its translation units: the objects
// behind the C handles, tile geometries, pass programs, plan knobs, error
// reporting and launch profiling.
//   sv_host_core.cpp  errors, plan knobs, launch profiling
//   sv_plan.cpp       tile geometries, pass programs, program execution, ground states
//   sv_api.cpp        states, instances and the circuit entry points
//   sv_batch.cpp      the batched p = 1 landscape scan
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sv.h"
#include "sv_internal.h"

using namespace svk;

#define HIPCHECK(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// ---------------------------------------------------------------- errors
// Sets the calling thread's last error message (sv_last_error) and returns code.
int fail(int code, const char* fmt, ...);

// ---------------------------------------------------------------- knobs
int knob(const char* k);                              // global value
int knob_for(const char* k, int dtype, int n);        // tuned override for (dtype, n), else global
bool take_injected_failure();                         // knob fail_next_launch (error-path tests)
std::vector<std::string> knob_names();

// ---------------------------------------------------------------- profiling
bool prof_begin(hipStream_t st, hipEvent_t* a);
void prof_end(hipStream_t st, hipEvent_t a, const std::string& kind, double bytes);

// ---------------------------------------------------------------- objects
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

// Matrices of general single-qubit layers as the kernels apply them.
struct GenLayers {
    std::vector<double> m;       // [layer][qubit][8]
    std::vector<uint8_t> unit;   // [layer][qubit]: unit-diagonal form (MIX_GUNIT)
    std::vector<double> mod;     // [layer][qubit]: diagonal modulus of a unit layer, else 1
};

// Tile shapes of a program: [1] one-vector, [2] two-vector.
struct Plan {
    std::vector<Geometry> by_nv[3];  // [1]: one-vector tile shape, [2]: two-vector shape
};

inline size_t elem_size(sv_dtype d) { return d == SV_C128 ? 16 : 8; }
inline int max_n(sv_dtype d) { return d == SV_C128 ? 33 : 34; }
inline bool dtype_ok(int d) { return d == SV_C64 || d == SV_C128; }
int device_cu_count(int dev);  // compute units of a device (cached; 256 on MI355X)

// ---------------------------------------------------------------- planning and execution
std::vector<Geometry> plan_groups(int n, sv_dtype dt, int nv, bool grad = false, bool general = false);
Plan make_plan(int n, sv_dtype dt, bool grad = false, bool general = false);
Program build_program(const std::vector<Event>& evs, int nres, bool fuse);
// fx != nullptr: the call may not allocate (see run_program in sv_plan.cpp).
int run_program(sv_state_s* s, sv_state_s* lam, sv_ising_s* H, Program& prog, const Plan& plan, bool need_ground,
                const FixedScratch* fx = nullptr, const void* first_src = nullptr);
int fetch_results(sv_state_s* s, int nres);
// Frees the instance-free geometry tables (mixer-only programs); called when the
// last state is freed, so they live no longer than the states that use them.
void release_plain_geos();
double ground_tol(const sv_ising_s* H);
int xcd_order(int x, const Geometry& geo, int n, sv_dtype dt);  // PassArgs::xcd for knob value x
int run_ground(sv_ising_s* H, hipStream_t stream);
