// Internal structures shared by the host planner (sv_api.cpp) and the gfx950
// kernels (sv_kernels.hip).  Not part of the public ABI.
//
// Vocabulary
//   tile      : 2^T amplitudes handled by one workgroup in one pass.  Tile-local
//               bit l maps to global bit P[l]: carriers l < c map to global bits
//               0..c-1 (contiguous runs of 2^c amplitudes), group bits l >= c map
//               to global bits lo .. lo+g-1.  Tile-local bits >= n (only when
//               n < T) are phantom: they address nothing.
//   layout    : which R tile bits a thread holds in registers (2^R amplitudes per
//               thread); the other T-R tile bits are the thread index.  A pass
//               moves the tile through a few layouts via LDS exchanges so that
//               every active qubit is register-local once.  Register slot R-1
//               is tile bit T-1 in every layout (the pivot), so an exchange
//               runs in two halves of 2^(T-1) amplitudes each.
//   op        : MIX (one butterfly per active qubit, Eq. twocomponentupdates) or
//               POINT (work on E(z) in the current layout: phase exp(-i gamma E),
//               reductions, lambda = E psi, gradient terms).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sv.h"

namespace svk {

constexpr int kMaxT = 16;
constexpr int kMaxR = 6;
constexpr int kMaxLayouts = 4;
constexpr int kMaxOps = 5;  // fixed pass shape: MIX MIX POINT MIX MIX
constexpr int kMaxSlots = 8;
constexpr int kMaxPhase = 4;
constexpr int kMaxTT = 128;
constexpr int kMaxTR = 16;

enum OpKind : int32_t { OP_MIX = 1, OP_POINT = 2 };

// MIX flags: which vectors get the butterflies; accumulate grad-beta terms
// (two-vector passes: pair sums Im(conj(lam_a) psi_b + conj(lam_b) psi_a);
// one-vector passes: the quadratic form 2 Re(conj(psi_a) psi_b) of the pair).
// Every MIX applies (u, v) <- (u - i a v, v - i a u) per active qubit, with
// a = tan(beta') for |beta'| <= pi/4, and multiplies the vector's uniform
// pending scale by b = +-cos(beta') per qubit (the host reduces beta modulo pi
// and splits larger angles into two halves).
enum MixFlags : int32_t { MIX_PSI = 1, MIX_LAM = 2, MIX_GBETA = 4, MIX_GEN = 8, MIX_GUNIT = 16 };

// MIX_GEN (one-vector passes): a general single-qubit layer instead.  Every
// active tile bit l gets its own complex 2x2 matrix m, (u, v) <- (m00 u + m01 v,
// m10 u + m11 v), read from PassArgs::gmat + qidx * kGenBlock + 8 l as
// (m00 re, im, m01 re, im, m10 re, im, m11 re, im); u is the amplitude whose
// bit is 0.  MIX_GUNIT: every matrix of the op has m00 = m11 = 1 (the host's
// unit-diagonal form), so (u, v) <- (u + m01 v, m10 u + v) at half the
// arithmetic, and the pending scale is multiplied by Op::b; a pass holds
// either only such ops or none (PassArgs::gen_unit selects the kernel).
constexpr int kGenBlock = 16 * 8;

// POINT flags, executed in this order.
enum PointFlags : int32_t {
    PT_REDUCE = 1,     // slots slot, slot+1, slot+2 += |psi|^2, E|psi|^2, [E = Emin]|psi|^2
    PT_LAM_INIT = 2,   // lam = E psi
    PT_GGAMMA = 4,     // slot2 += E Im(conj(lam) psi)
    PT_PHASE_PSI = 8,  // psi *= exp(-i gamma E)
    PT_PHASE_LAM = 16,  // lam *= exp(-i gamma E); two-vector passes phase both or neither
    PT_SPINZ = 32,      // spin sums: per tile, sum |psi|^2 s_l for every tile bit l and sum |psi|^2
    PT_E2 = 64,         // slot3 += E^2 |psi|^2 (with PT_REDUCE: the spread of E in the state)
    PT_ZETA = 128,      // one-vector passes: psi <- psi (1 + i t E), t = Op::b (after the reductions)
    PT_EFORM = 256      // one-vector passes: slot2 += E |psi|^2
};

// Per-tile spin partials (PT_SPINZ): kTF doubles per tile, entry l < T =
// sum over the tile of |psi|^2 s_l, entry kTF - 1 = sum of |psi|^2.
struct SpinArgs {
    const double* part;     // [ntiles][kTF]
    uint64_t ntiles;
    int32_t c, lo, g, T, n;
    int32_t qubit[16];      // tile bit -> qubit (-1: phantom)
    double* out;            // [n]: <sigma^z_i>
};

struct Op {
    int32_t kind;
    int32_t flags;
    int32_t slot;   // MIX: grad-beta slot; POINT: first reduce slot
    int32_t slot2;  // POINT: grad-gamma slot
    int32_t qidx;   // POINT: index of the (layout, gamma) phase table
    int32_t slot3;  // POINT: PT_E2 slot
    double a;       // MIX: tan(beta')   POINT: gamma
    double b;       // MIX: +-cos(beta')   POINT: t of PT_ZETA
};

// One layout of one tile geometry (device resident, read with uniform loads;
// everything a kernel reads per layout is a dword or wider, so it comes
// through the scalar cache without dependent per-byte vector loads).
struct GeoLayout {
    uint32_t reg_u[64];     // tile-local index of register r (thread part zero)
    uint32_t reg_lds[64];   // LDS byte offset (swizzled element index x element size) of reg_u[r] without the pivot bit
    uint64_t reg_goff[64];  // global element offset of reg_u[r]
    uint32_t tmask;         // tile bits held by the thread index: thread-id bit j -> j-th set bit of tmask
    uint32_t rbpack;        // register slot k -> tile bit (rbpack >> 4k) & 15
    uint32_t thr_off;       // per-thread coupling table: offset in doubles from the GeoBuf start (0: none)
    int32_t act_fwd;        // register slots butterflied when entering forward
    int32_t act_bwd;        // ... when walking the layouts backwards
    int32_t dpp;            // lane positions (bits 0, 1, 3 of the lane id) butterflied across lanes here
    double Q[64];           // sum of couplings among register bits, per register r
};

// Tile geometry table.  Instance geometries append, per layout, a per-thread
// coupling table of (R + 1) rows of 2^(T-R) doubles (thread t = column t):
//   row 0      sum over couplings between two thread bits of J s_a s_b
//   row 1 + k  sum over couplings between register slot k's bit and a thread bit l of J s_l
struct GeoBuf {
    int32_t P[kMaxT];  // tile bit -> global bit, -1 = phantom
    GeoLayout L[kMaxLayouts];
};

// Per-tile field table of an instance and a tile geometry: kTF doubles per
// tile, entry l < T = g_l (field seen by tile bit l from h and the couplings
// to bits outside the tile), entry kTF - 1 = E_fixed (fields and couplings
// among the bits outside the tile).  Requires T < kTF.
constexpr int kTF = 16;

// Device copy of an Ising instance.
struct IsingDev {
    const double* h;        // [n]
    const int32_t* adj_ptr; // [n+1] CSR over both endpoints of every coupling
    const int32_t* adj_nbr; // [2m]
    const double* adj_J;    // [2m]
    const int32_t* ei;      // [m]
    const int32_t* ej;      // [m]
    const double* J;        // [m]
    int32_t n, m;
};

// Per-call phase tables, built once by k_tables before the passes:
//   qph: exp(-i gamma Q[r]) for the register-bit couplings of one layout
//   lut: exp(-i gamma m) for integer m in [-L, L] (integer-valued instances)
struct TableJob {
    double gamma;
    const double* Q;        // device: the layout's Q[64]
    int32_t nr;             // registers per thread (2^R)
    int32_t L;              // lut half width (-1: no lut); entry m holds exp(-i gamma (m - L) qinv)
    double qinv;            // 1/q: energies on the grid Z / q
    uint32_t qph_off;       // double2 offset of qph in the table buffer
    uint32_t lut_off;       // double2 offset of lut[0] (the entry for m = -L)
};

struct PassArgs {
    void* psi;
    void* lam;
    const void* src;        // psi is loaded from here when non-null (out-of-place first pass), else from psi
    double* partials;       // [ntiles][nslots]
    const double2* ptab;    // phase tables (k_tables output)
    const GeoBuf* geo;
    const double* tf;       // per-tile field table (passes that evaluate E)
    uint64_t ntiles;
    int32_t n, c, lo, g;    // tile geometry
    uint32_t phantom;       // tile-local phantom bits
    int32_t nlayouts;
    int32_t load;           // bit0 load psi, bit1 load lam, bit2 init psi = |+>
    int32_t store;          // bit0 store psi, bit1 store lam
    int32_t nslots;
    int32_t nops;           // informational; ops[i].kind == 0 marks an absent slot
    int32_t need_e;         // the POINT op evaluates E (tile fields needed)
    int32_t nt;             // 3: nontemporal loads and stores (long contiguous runs), 0: plain
    int32_t swz;            // LDS slot swizzle width (the geometry tables use the same)
    int32_t grid;           // workgroups launched (< ntiles: persistent grid-stride walk), 0: one per tile
    int32_t stagger;        // persistent grids: start delay of the second half, in units of s_sleep(127)
    int32_t xcd;            // x > 0: with K = 8 * 2^(x-1), workgroup b takes tile (b mod K) * (ntiles / K)
                            // + b / K, so that each of the 8 XCDs (which receive workgroups round-robin)
                            // walks K / 8 contiguous stretches of the tiles; 0: tile = b
    int32_t nphase;
    int32_t lut_half;       // L of the phase tables (in units of 1/q), -1 for other real-valued instances
    double lut_q;           // q: table index = q * energy
    double* spin_part;      // [ntiles][kTF] spin partials (passes with PT_SPINZ)
    const double* gmat;     // general single-qubit layers (passes whose MIX ops carry MIX_GEN), else null
    int32_t gen_real;       // every general layer of the pass is real
    int32_t gen_unit;       // every general layer of the pass is in the unit-diagonal form (MIX_GUNIT)
    int32_t kc34;           // two-vector passes with three or four layouts: straight-line kernels
    int32_t qf;             // one-vector pass of the adjoint sweeps: 1 quadratic forms, 2 also PT_ZETA / PT_EFORM,
                            // 3 also PT_REDUCE before PT_ZETA
    int32_t occ4;           // complex64 14-bit tiles planned without lane position 4: kernel with
                            // four waves per SIMD (two workgroups per CU)
    uint32_t qph_off[kMaxPhase];
    uint32_t lut_off[kMaxPhase];
    double emin, etol;      // ground-state test |E - emin| <= etol
    double amp0;            // 2^{-n/2}
    Op ops[kMaxOps];
};

struct GroundArgs {
    const GeoBuf* geo;
    const double* tf;       // per-tile field table of the geometry
    uint64_t ntiles;
    int32_t n, c, lo, g;
    uint32_t phantom;
    int32_t mode;           // 0: minimum energy; 1: count and first index at emin
    double emin, etol;
    double* part_e;         // [ntiles]    mode 0
    uint64_t* part_cnt;     // [ntiles]    mode 1
    uint64_t* part_arg;     // [ntiles]    mode 1
};

// Build job of a per-tile field table.
struct TfArgs {
    IsingDev is;
    const GeoBuf* geo;      // any table of the geometry (uses P only)
    double* tf;             // [ntiles][kTF]
    uint64_t ntiles;
    int32_t T, c, lo, g;
};

// Launchers (sv_kernels.hip).  Return hipError_t as int.
int launch_pass(int dtype, int nv, int T, const PassArgs& a, void* stream);
int launch_tile_fields(const TfArgs& a, void* stream);
int launch_tables(const TableJob* jobs, int njobs, double2* out, void* stream);
int launch_spin_reduce(const SpinArgs& a, void* stream);
// stage: kReduceBlocks * kMaxSlots doubles of scratch for the first stage.
constexpr int kReduceBlocks = 256;
int launch_reduce_slots(const double* partials, uint64_t nrows, int nslots, const int* dst,
                        int accumulate, double* out, double* stage, void* stream);
int launch_ground(int dtype, const GroundArgs& a, void* stream);
// Streaming ceiling: in-place load/store of every tile of a geometry (T = 13
// for complex128, 14 for complex64), no arithmetic.
struct StreamArgs {
    uint64_t ntiles;
    int32_t c, lo, g;
    int32_t xcd;            // tile order as PassArgs::xcd
    uint64_t mask;          // 0: every amplitude is stored back unchanged (XOR with this mask)
};
int launch_stream(int dtype, void* p, const StreamArgs& a, void* stream);
int launch_ground_finish(const GroundArgs& a, double* out_e, uint64_t* out_cnt,
                         uint64_t* out_arg, void* stream);
// ---------------------------------------------------------------- batch scan
// One instance of the p = 1 landscape scan (device array of these).
struct BatchInst {
    int32_t n, m;
    int32_t hoff, coff;     // offsets into the packed fields / couplings
    uint64_t eoff;          // offset of this instance's energy table
    double emin, etol;      // ground-state test
    int32_t lut_lo, lut_n;  // integer energies lie in [lut_lo, lut_lo + lut_n); lut_n = 0: real
};

struct BatchArgs {
    const BatchInst* inst;
    int32_t ninst;
    const double* h;        // packed fields
    const int32_t* ei;      // packed couplings (instance-local spin indices)
    const int32_t* ej;
    const double* J;
    double* etab;           // energy tables, Sum 2^n_i entries
    uint16_t* eidx;         // integer-valued instances: E(z) - lut_lo per entry (same offsets)
    const int32_t* unit_inst;  // work unit -> instance (units sorted by n, largest first)
    const int32_t* unit_gam;   // work unit -> gamma index
    int32_t nunits;
    const double* gammas;
    int32_t ng;
    const double* betas;
    int32_t nb;
    double* out_e;          // [inst][gamma][beta]
    double* out_p;
    unsigned int* counter;  // work-queue head (zeroed before the launch)
    void* scratch;          // per-workgroup slices for states larger than LDS
    uint64_t scratch_elems; // elements per workgroup slot
    // sliced path (states with n > S, a launch at a time): state s of a launch is
    // the group state g = s_base + s, i.e. unit s_u0 + g / nb and beta index g % nb
    int32_t s_n;            // qubits of every state of the launch
    int32_t s_u0;           // first unit of the n-group
    int64_t s_base;         // first group state of the launch
    int32_t s_count;        // states in the launch
    void* slab;             // s_count x 2^s_n amplitudes
    double* part;           // s_count x 2^(s_n - S) x 2 partial sums
    // the previous launch, whose states the slice kernel of this one finishes
    // (f_count = 0: none)
    int32_t f_n, f_u0, f_count;
    int32_t f_nh;           // partial sums per state of the previous launch: 2^f_nh
    int64_t f_base;
    const double* f_part;
};

int launch_batch_energy(const BatchArgs& a, int max_n, void* stream);
int launch_batch_scan(int dtype, const BatchArgs& a, int grid, int wide, void* stream);
// Sliced path for states larger than the LDS tile: slices (which also finish
// the previous launch's states, a.f_*) and columns of one launch (a.s_*,
// a.slab, a.part); launch_batch_finish finishes the last launch's states.
int launch_batch_sliced(int dtype, const BatchArgs& a, int wide, void* stream);
int launch_batch_finish(const BatchArgs& a, void* stream);
int batch_lds_bits(int dtype, int wide);  // log2 of the LDS-resident state of a batch variant
int batch_lut_cap(int dtype, int wide);   // phase-table entries of a batch variant
int batch_slice_bits(int dtype, int n);   // log2 of the slice of an n-qubit state on the sliced path

// ---------------------------------------------------------------- fixed scratch
// Device region that a call which may not allocate uses instead of the state's
// work buffers: reduction partials, phase tables and the result array.
struct FixedScratch {
    double* part;           // reduction partials
    size_t part_doubles;
    double2* tab;           // phase tables
    size_t tab_entries;     // double2 entries
    double* out;            // results (device), each written by exactly one reduction
};


// Compile-time tile shapes per (dtype, vectors): T tile bits, R register bits.
struct Shape {
    int T, R;
};
Shape shape_for(int dtype, int nv, bool grad);

}  // namespace svk

// Host entry points shared between the C-ABI source files (sv_api.cpp).
// sv_qaoa_energy on a fixed scratch region: the same program and kernels,
// results (norm, energy, p_gs) written to fx.out on the state's stream, nothing
// allocated, no synchronisation.  device: the current HIP device, which must be
// the state's.
int sv_internal_qaoa_energy_fixed(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                                  int from_plus, int device, const svk::FixedScratch& fx);
// Set the thread-local message of sv_last_error; returns code.
int sv_internal_set_error(int code, const char* msg);
