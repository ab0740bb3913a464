// gfx950 kernels of libsv: tile passes over the state vector, ground-state
// enumeration and deterministic second-stage reductions.
//
// A tile pass streams 2^T amplitudes per workgroup from HBM into registers
// (2^R per thread), runs a short program of ops on them and streams them
// back.  MIX applies exp(-i beta sigma^x_q) to every active qubit q of the
// tile as a 2-component update on register-local pairs (Eq.
// twocomponentupdates); qubits that are thread bits in the current layout are
// made register-local by an LDS exchange into the next layout.  POINT works
// per amplitude with the Ising energy E(z) of Eq. HC, built from the bits of z
// as  E = E_fixed + sum_l g_l s_l + (couplings inside the tile)  where E_fixed
// and the fields g_l seen by the tile bits are computed once per workgroup.
#include <hip/hip_runtime.h>

#include "sv_internal.h"

namespace svk {

template <typename Real>
struct V2T;
template <>
struct V2T<double> {
    using type = double2;
};
template <>
struct V2T<float> {
    using type = float2;
};

// swizzle of a tile-local index into an LDS element index: bits >= G are folded
// into the low G bits so that 2^G consecutive lanes that differ in any G
// consecutive tile bits land in distinct 128-byte bank groups.
__device__ __forceinline__ uint32_t lds_swizzle(uint32_t u, int G) {
    uint32_t x = u >> G, f = 0;
#pragma unroll
    for (int i = 0; i < 6; i++) {
        f ^= x;
        x >>= G;
    }
    return u ^ (f & ((1u << G) - 1u));
}

// Streaming (nontemporal) accesses of one complex amplitude.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
    const nf2 v = __builtin_nontemporal_load(reinterpret_cast<const nf2*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2* p, double2 x) {
    nd2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, reinterpret_cast<nd2*>(p));
}
__device__ __forceinline__ void st_nt(float2* p, float2 x) {
    nf2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, reinterpret_cast<nf2*>(p));
}

// Tables that no kernel writes while it reads them (tile geometries, phase
// tables) are read through the constant address space: the compiler may then
// use scalar loads for their wave-uniform entries even after the kernel's own
// stores to the state, instead of one vector load per entry.
#define SV_CONST __attribute__((address_space(4)))
typedef const SV_CONST GeoBuf CGeoBuf;
typedef const SV_CONST GeoLayout CGeoLayout;
// entry i of a constant-space complex table (component loads: the vector type's
// operators take generic references)
__device__ __forceinline__ double2 ctab(const SV_CONST double* t, int i) {
    return make_double2(t[2 * i], t[2 * i + 1]);
}

__device__ __forceinline__ double spin_u(uint32_t u, int l) { return ((u >> l) & 1u) ? 1.0 : -1.0; }
__device__ __forceinline__ double spin_z(uint64_t z, int i) { return ((z >> i) & 1ull) ? 1.0 : -1.0; }

// Tile-local index of the thread part: thread-id bit j goes to the j-th set
// bit of the layout's (wave-uniform) thread mask.  No memory access.
template <int NTB>
__device__ __forceinline__ uint32_t thread_index_bits(uint32_t t, uint32_t tmask) {
    uint32_t u = 0, m = tmask;
#pragma unroll
    for (int j = 0; j < NTB; j++) {
        const uint32_t l = (uint32_t)__builtin_ctz(m);
        m &= m - 1u;
        u |= ((t >> j) & 1u) << l;
    }
    return u;
}

struct TileGeom {
    int c, lo, g;
    __device__ __forceinline__ bool in_tile(int i) const { return i < c || (i >= lo && i < lo + g); }
    __device__ __forceinline__ uint64_t gmap(uint32_t u) const {
        return (uint64_t)(u & ((1u << c) - 1u)) | ((uint64_t)(u >> c) << lo);
    }
    __device__ __forceinline__ uint64_t base(uint64_t w) const {
        const int nlow = lo - c;
        return ((w & ((1ull << nlow) - 1ull)) << c) | ((w >> nlow) << (lo + g));
    }
};

// Per-tile part of E(z) for one tile (one wave): E_fixed (fields and couplings
// among the bits outside the tile) and g_l = h_{P[l]} + sum of couplings from
// tile bit l to the fixed bits, written to the tile's row of the field table.
// Deterministic order.
__device__ void tile_fields_row(const IsingDev& is, const GeoBuf* geo, const TileGeom& tg, uint64_t base, int T,
                                double* __restrict__ row) {
    const int lane = threadIdx.x & 63;
    double part = 0.0;
    for (int i = lane; i < is.n; i += 64)
        if (!tg.in_tile(i)) part += is.h[i] * spin_z(base, i);
    for (int k = lane; k < is.m; k += 64) {
        const int i = is.ei[k], j = is.ej[k];
        if (!tg.in_tile(i) && !tg.in_tile(j)) part += is.J[k] * spin_z(base, i) * spin_z(base, j);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off);
    if (lane == kTF - 1) row[lane] = part;
    if (lane < kTF - 1) {
        const int P = lane < T ? geo->P[lane] : -1;
        double gv = 0.0;
        if (P >= 0) {
            gv = is.h[P];
            for (int q = is.adj_ptr[P]; q < is.adj_ptr[P + 1]; q++) {
                const int j = is.adj_nbr[q];
                if (!tg.in_tile(j)) gv += is.adj_J[q] * spin_z(base, j);
            }
        }
        row[lane] = gv;
    }
}

// Field table of an instance for one tile geometry, one wave per tile.
__global__ void __launch_bounds__(256) k_tile_fields(const TfArgs a) {
    const TileGeom tg{a.c, a.lo, a.g};
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    for (uint64_t w = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < a.ntiles; w += stride)
        tile_fields_row(a.is, a.geo, tg, tg.base(w), a.T, a.tf + w * kTF);
}

// Thread part of E for layout L: returns e0 = E at register index 0 and the
// register-bit fields f[k], so that E(r) = e0 + sum_{k: r_k = 1} 2 f[k] + Q[r].
// s_g holds the tile's g_l (l < T) and E_fixed (entry kTF - 1).  The couplings
// inside the tile that involve thread bits come from the layout's per-thread
// table (one coalesced load per row).
template <int R, int NTB>
__device__ __forceinline__ double thread_energy(CGeoLayout* L, CGeoBuf* geo, uint32_t t,
                                                const double* s_g, double (&f)[R]) {
    constexpr int NT = 1 << NTB;
    const uint32_t off = L->thr_off;
    const SV_CONST double* __restrict__ tab = reinterpret_cast<const SV_CONST double*>(geo) + off + t;
    double eth = s_g[kTF - 1];
    uint32_t m = L->tmask;
#pragma unroll
    for (int j = 0; j < NTB; j++) {
        const int l = __builtin_ctz(m);
        m &= m - 1u;
        const double gl = s_g[l];
        eth += ((t >> j) & 1u) ? gl : -gl;
    }
    if (off != 0) eth += tab[0];
    const uint32_t rbp = L->rbpack;
#pragma unroll
    for (int k = 0; k < R; k++) {
        double fv = s_g[(rbp >> (4 * k)) & 15u];
        if (off != 0) fv += tab[(1 + k) * NT];
        f[k] = fv;
        eth -= fv;
    }
    return eth;
}

// Wave-level sum of a per-lane value (fixed butterfly order), added by lane 0
// to this wave's row of the per-workgroup reduction array.
template <int NS>
__device__ __forceinline__ void wave_add(double (*s_red)[NS], int slot, double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6][slot] += v;
}

__device__ __forceinline__ double2 cmul(double2 x, double2 y) {
    return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

// One pair butterfly of exp(-i beta sigma^x) without its cos(beta) factor:
// (u, v) <- (u - i t v, v - i t u), t = tan(beta).
template <typename Real>
__device__ __forceinline__ void butterfly(Real& ar, Real& ai, Real& br, Real& bi, Real t) {
    const Real nar = fma(t, bi, ar), nai = fma(-t, br, ai);
    const Real nbr = fma(t, ai, br), nbi = fma(-t, ar, bi);
    ar = nar;
    ai = nai;
    br = nbr;
    bi = nbi;
}

// Value of the lane whose id differs in one bit, per 32-bit word: lane bit 3
// by a DPP row_ror:8 move (within a 16-lane row), lane bit 4 by a ds_swizzle
// in bit mode (and 0x1f, xor 0x10 within 32 lanes; no LDS storage).
constexpr int kLaneX8 = 0x128;
constexpr int kLaneX16 = 0x10000 | (0x10 << 10) | 0x1f;
template <int CTRL>
__device__ __forceinline__ int lane_xor_word(int w) {
    if constexpr (CTRL & 0x10000)
        return __builtin_amdgcn_ds_swizzle(w, CTRL & 0xffff);
    else
        return __builtin_amdgcn_update_dpp(0, w, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float lane_xor(float x) {
    return __int_as_float(lane_xor_word<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ __forceinline__ double lane_xor(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = lane_xor_word<CTRL>((int)(b & 0xffffffffll));
    const int hi = lane_xor_word<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Butterfly of one qubit held by a lane bit: both lanes of a pair apply
// x <- x - i t x_partner (the same form for the upper and the lower member).
// With gradient accumulation each lane adds Im(conj(lam_self) psi_partner), so
// that the pair sum of the register form is split over the two lanes.
template <int CTRL, typename Real, int R, int NV, bool QF = false>
__device__ __forceinline__ void lane_round(Real (&vr)[NV][1 << R], Real (&vi)[NV][1 << R], int flags, Real t,
                                           double cosb, double (&pend)[NV], double& gsum) {
    constexpr int NR = 1 << R;
    if constexpr (NV == 2) {
        if (flags & MIX_GBETA) {
            double gb = 0.0;
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const Real pr = lane_xor<CTRL>(vr[0][r]), pi = lane_xor<CTRL>(vi[0][r]);
                gb += (double)(vr[1][r] * pi - vi[1][r] * pr);
            }
            gsum += gb * pend[0] * pend[1];
        }
    }
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const bool mine = NV == 1 || (flags & (1 << v)) != 0;
        const Real tv = mine ? t : (Real)0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const Real pr = lane_xor<CTRL>(vr[v][r]), pi = lane_xor<CTRL>(vi[v][r]);
            vr[v][r] = fma(tv, pi, vr[v][r]);
            vi[v][r] = fma(-tv, pr, vi[v][r]);
        }
        pend[v] *= mine ? cosb : 1.0;
    }
    if constexpr (NV == 1 && QF) {
        if (flags & MIX_GBETA) {
            // one-vector quadratic form, taken after the butterfly (which leaves it unchanged)
            // in a loop of its own: each lane adds Re(conj(self) partner), so the two lanes
            // of a pair give 2 Re(conj(a) b)
            double gq[2] = {0.0, 0.0};
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const Real pr = lane_xor<CTRL>(vr[0][r]), pi = lane_xor<CTRL>(vi[0][r]);
                gq[r & 1] = fma((double)vr[0][r], (double)pr, gq[r & 1]);
                gq[r & 1] = fma((double)vi[0][r], (double)pi, gq[r & 1]);
                // keep the scheduler from hoisting every cross-lane move ahead of the sums
                // (their results would all be live at once)
                if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
            gsum += (gq[0] + gq[1]) * pend[0] * pend[0];
        }
    }
}

// Butterflies of every active register slot of the current layout; each slot
// multiplies the pending scale of the touched vectors by cos(beta).  With
// gradient accumulation the pair terms Im(conj(lam_a) psi_b) + Im(conj(lam_b) psi_a)
// are taken before each slot's butterfly, weighted by both pending scales.
template <typename Real, int R, int NV, bool QF = false>
__device__ __forceinline__ void mix_round(Real (&vr)[NV][1 << R], Real (&vi)[NV][1 << R], int act, int flags,
                                          Real t, double cosb, double (&pend)[NV], double& gsum) {
    constexpr int NR = 1 << R;
#pragma unroll
    for (int k = 0; k < R; k++) {
        // inactive slots run as identity butterflies (t = 0, no scale): branch-free
        // code keeps the amplitude registers in place
        const bool on = (act >> k) & 1;
        const Real tk = on ? t : (Real)0;
        if constexpr (NV == 2) {
            if ((flags & MIX_GBETA) && on) {
                double gb = 0.0;
                if constexpr (sizeof(Real) == 8) {
                    // complex128: the four products of each pair fused into two
                    // alternating FP64 accumulators
                    double g2 = 0.0;
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        if (r & (1 << k)) continue;
                        const int r2 = r | (1 << k);
                        double& acc = ((r >> (k == 0 ? 1 : 0)) & 1) ? g2 : gb;
                        acc = fma(vr[1][r], vi[0][r2], acc);
                        acc = fma(-vi[1][r], vr[0][r2], acc);
                        acc = fma(vr[1][r2], vi[0][r], acc);
                        acc = fma(-vi[1][r2], vr[0][r], acc);
                    }
                    gb += g2;
                } else {
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        if (r & (1 << k)) continue;
                        const int r2 = r | (1 << k);
                        // pair term in the storage precision, summed in FP64 (FP64 products
                        // change the complex64 gradient by ~1e-10 of the coefficient scale, far
                        // below the f32 rounding of the stored vectors, and spill the
                        // four-waves-per-SIMD kernels)
                        const Real q = vr[1][r] * vi[0][r2] - vi[1][r] * vr[0][r2] + vr[1][r2] * vi[0][r] -
                                       vi[1][r2] * vr[0][r];
                        gb += (double)q;
                    }
                }
                gsum += gb * pend[0] * pend[1];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
            // A vector the op does not touch runs identity butterflies (t = 0)
            // instead of a branch, which would force register copies at the
            // join.  One-vector passes always mix psi.
            const bool mine = NV == 1 || (flags & (1 << v)) != 0;
            const Real tv = mine ? tk : (Real)0;
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r & (1 << k)) continue;
                const int r2 = r | (1 << k);
                butterfly<Real>(vr[v][r], vi[v][r], vr[v][r2], vi[v][r2], tv);
            }
            pend[v] *= (on && mine) ? cosb : 1.0;
        }
    }
    if constexpr (NV == 1 && QF) {
        if (flags & MIX_GBETA) {
            // quadratic forms 2 Re(conj(a) b) of the pairs of every active slot.  A butterfly
            // on any qubit leaves the form of every other qubit unchanged, so all of them are
            // taken once, after the round, from the final values and pending scale.
            double g4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < R; k++) {
                if (!((act >> k) & 1)) continue;
                int j = 0;
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (r & (1 << k)) continue;
                    const int r2 = r | (1 << k);
                    double& acc = g4[j++ & 3];
                    acc = fma((double)vr[0][r], (double)vr[0][r2], acc);
                    acc = fma((double)vi[0][r], (double)vi[0][r2], acc);
                }
            }
            gsum += 2.0 * ((g4[0] + g4[1]) + (g4[2] + g4[3])) * pend[0] * pend[0];
        }
    }
}

// General single-qubit layer, register slots: slot k holds tile bit
// (rbpack >> 4k) & 15 and applies that bit's matrix M[l] to every register
// pair (bit k = 0, bit k = 1).  Inactive slots read the identity entry of tile
// bit 15 (never a qubit of a 13- or 14-bit tile), which keeps the code
// branch-free.  REALM: every matrix is real (two FMAs per amplitude instead
// of eight).  unit: every matrix has a unit diagonal (one FMA per amplitude
// for real matrices, four for complex ones).  The matrices are read through
// the constant address space (the host writes them before the launch): scalar
// loads of every slot's entries, issued together ahead of the butterflies.
template <typename Real, int R, bool REALM, bool UNIT>
__device__ __forceinline__ void gen_round(Real (&vr)[1][1 << R], Real (&vi)[1][1 << R], int act, uint32_t rbpack,
                                          const SV_CONST double* __restrict__ M) {
    constexpr int NR = 1 << R;
    if constexpr (UNIT) {
        // off-diagonal entries only: (u, v) <- (u + m01 v, m10 u + v)
        Real mo[R][4];  // slot k: m01 re, m10 re, m01 im, m10 im
#pragma unroll
        for (int k = 0; k < R; k++) {
            const bool on = (act >> k) & 1;
            const SV_CONST double* m = M + 8 * (on ? ((rbpack >> (4 * k)) & 15u) : 15u);
            mo[k][0] = (Real)m[2];
            mo[k][1] = (Real)m[4];
            if constexpr (!REALM) {
                mo[k][2] = (Real)m[3];
                mo[k][3] = (Real)m[5];
            }
        }
#pragma unroll
        for (int k = 0; k < R; k++) {
            const Real b0 = mo[k][0], c0 = mo[k][1];
            Real b1 = 0, c1 = 0;
            if constexpr (!REALM) {
                b1 = mo[k][2];
                c1 = mo[k][3];
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r & (1 << k)) continue;
                const int r2 = r | (1 << k);
                const Real ur = vr[0][r], ui = vi[0][r], wr = vr[0][r2], wi = vi[0][r2];
                if constexpr (REALM) {
                    vr[0][r] = fma(b0, wr, ur);
                    vi[0][r] = fma(b0, wi, ui);
                    vr[0][r2] = fma(c0, ur, wr);
                    vi[0][r2] = fma(c0, ui, wi);
                } else {
                    vr[0][r] = fma(b0, wr, fma(-b1, wi, ur));
                    vi[0][r] = fma(b0, wi, fma(b1, wr, ui));
                    vr[0][r2] = fma(c0, ur, fma(-c1, ui, wr));
                    vi[0][r2] = fma(c0, ui, fma(c1, ur, wi));
                }
            }
        }
    } else {
    Real me[R][8];  // slot k: a0 b0 c0 d0 (real parts), then a1 b1 c1 d1 (imaginary parts)
#pragma unroll
    for (int k = 0; k < R; k++) {
        const bool on = (act >> k) & 1;
        const SV_CONST double* m = M + 8 * (on ? ((rbpack >> (4 * k)) & 15u) : 15u);
#pragma unroll
        for (int j = 0; j < 4; j++) me[k][j] = (Real)m[2 * j];
        if constexpr (!REALM) {
#pragma unroll
            for (int j = 0; j < 4; j++) me[k][4 + j] = (Real)m[2 * j + 1];
        }
    }
#pragma unroll
    for (int k = 0; k < R; k++) {
        const Real a0 = me[k][0], b0 = me[k][1], c0 = me[k][2], d0 = me[k][3];
        Real a1 = 0, b1 = 0, c1 = 0, d1 = 0;
        if constexpr (!REALM) {
            a1 = me[k][4];
            b1 = me[k][5];
            c1 = me[k][6];
            d1 = me[k][7];
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r & (1 << k)) continue;
            const int r2 = r | (1 << k);
            const Real ur = vr[0][r], ui = vi[0][r], wr = vr[0][r2], wi = vi[0][r2];
            if constexpr (REALM) {
                vr[0][r] = fma(a0, ur, b0 * wr);
                vi[0][r] = fma(a0, ui, b0 * wi);
                vr[0][r2] = fma(c0, ur, d0 * wr);
                vi[0][r2] = fma(c0, ui, d0 * wi);
            } else {
                vr[0][r] = fma(a0, ur, fma(-a1, ui, fma(b0, wr, -b1 * wi)));
                vi[0][r] = fma(a0, ui, fma(a1, ur, fma(b0, wi, b1 * wr)));
                vr[0][r2] = fma(c0, ur, fma(-c1, ui, fma(d0, wr, -d1 * wi)));
                vi[0][r2] = fma(c0, ui, fma(c1, ur, fma(d0, wi, d1 * wr)));
            }
        }
    }
    }
}

// General single-qubit layer, lane bit POS (the partner lane is lane ^ 2^POS):
// the lane whose bit is 0 holds u and forms m00 u + m01 v, its partner forms
// m10 u + m11 v.  l is the tile bit of that lane position.  Both rows are read
// as scalars; each lane selects its own.  unit: unit diagonal, each lane adds
// its off-diagonal entry times the partner's value to its own.
template <int CTRL, int POS, typename Real, int R, bool REALM, bool UNIT>
__device__ __forceinline__ void gen_lane(Real (&vr)[1][1 << R], Real (&vi)[1][1 << R], int l,
                                         const SV_CONST double* __restrict__ M) {
    constexpr int NR = 1 << R;
    const SV_CONST double* m = M + 8 * l;
    const bool hi = ((threadIdx.x >> POS) & 1u) != 0;
    if constexpr (UNIT) {
        const double m2 = m[2], m4 = m[4];
        const Real orr = (Real)(hi ? m4 : m2);
        Real oi = (Real)0;
        if constexpr (!REALM) {
            const double m3 = m[3], m5 = m[5];
            oi = (Real)(hi ? m5 : m3);
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const Real pr = lane_xor<CTRL>(vr[0][r]), pi = lane_xor<CTRL>(vi[0][r]);
            const Real xr = vr[0][r], xi = vi[0][r];
            if constexpr (REALM) {
                vr[0][r] = fma(orr, pr, xr);
                vi[0][r] = fma(orr, pi, xi);
            } else {
                vr[0][r] = fma(orr, pr, fma(-oi, pi, xr));
                vi[0][r] = fma(orr, pi, fma(oi, pr, xi));
            }
        }
        return;
    }
    const double m0 = m[0], m2 = m[2], m4 = m[4], m6 = m[6];
    const Real sr = (Real)(hi ? m6 : m0), orr = (Real)(hi ? m4 : m2);
    Real si = (Real)0, oi = (Real)0;
    if constexpr (!REALM) {
        const double m1 = m[1], m3 = m[3], m5 = m[5], m7 = m[7];
        si = (Real)(hi ? m7 : m1);
        oi = (Real)(hi ? m5 : m3);
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const Real pr = lane_xor<CTRL>(vr[0][r]), pi = lane_xor<CTRL>(vi[0][r]);
        const Real xr = vr[0][r], xi = vi[0][r];
        if constexpr (REALM) {
            vr[0][r] = fma(sr, xr, orr * pr);
            vi[0][r] = fma(sr, xi, orr * pi);
        } else {
            vr[0][r] = fma(sr, xr, fma(-si, xi, fma(orr, pr, -oi * pi)));
            vi[0][r] = fma(sr, xi, fma(si, xr, fma(orr, pi, oi * pr)));
        }
    }
}

// Tile bit held by thread-index bit j of a layout (the j-th set bit of tmask).
__device__ __forceinline__ int tmask_bit(uint32_t tmask, int j) {
    for (int i = 0; i < j; i++) tmask &= tmask - 1u;
    return __builtin_ctz(tmask);
}

// Phase tables of one call: qph[r] = exp(-i gamma Q[r]) and, for instances whose
// energies lie on the grid Z / q (integer or half-integer coefficients),
// lut[m + L] = exp(-i gamma m / q), m = -L..L.  One workgroup per job.
struct TableJobs {
    TableJob j[64];
};

__global__ void __launch_bounds__(256) k_tables(const TableJobs jobs, double2* __restrict__ out) {
    const TableJob jb = jobs.j[blockIdx.x];
    for (int r = threadIdx.x; r < jb.nr; r += 256) {
        double sn, cs;
        sincos(jb.gamma * jb.Q[r], &sn, &cs);
        out[jb.qph_off + r] = make_double2(cs, -sn);
    }
    if (jb.L >= 0) {
        for (int m = threadIdx.x; m <= 2 * jb.L; m += 256) {
            double sn, cs;
            sincos(jb.gamma * ((double)(m - jb.L) * jb.qinv), &sn, &cs);
            out[jb.lut_off + m] = make_double2(cs, -sn);
        }
    }
}

// KC > 0: the pass geometry has exactly KC layouts (compile time, straight-line
// layout walks); KC == 0: generic kernel with a runtime layout count (used for
// states smaller than one tile and for real-valued instances).
template <typename Real, int T, int R, int NV, int NS, int MINB, bool PH, bool INTE, int KC, int NTM = 0,
          bool PERSIST = false, bool SPZ = PH, int GEN = 0, int QFM = 0>
__global__ void __launch_bounds__(1 << (T - R), MINB) k_pass(const PassArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int NT = 1 << (T - R);
    constexpr int NR = 1 << R;
    constexpr int NH = NR / 2;  // registers per pivot half
    constexpr int NW = NT / 64;

    // one-vector kernels exchange half a tile at a time (pivot layouts, two
    // workgroups per CU); two-vector kernels run one workgroup per CU (register
    // bound) and exchange whole tiles.
    constexpr bool FULLX = NV == 2;
    __shared__ V2 xbuf[FULLX ? (1 << T) : (1 << (T - 1))];
    __shared__ double s_g[kTF];  // tile fields g_l and E_fixed (entry kTF - 1)
    __shared__ double s_red[NW][NS];
    __shared__ double s_spin[NW][kTF];  // per-wave spin sums (PT_SPINZ)

    const uint32_t t = threadIdx.x;
    CGeoBuf* __restrict__ geo = (CGeoBuf*)a.geo;
    const TileGeom tg{a.c, a.lo, a.g};
    V2* __restrict__ psi = reinterpret_cast<V2*>(a.psi);
    V2* __restrict__ lam = reinterpret_cast<V2*>(a.lam);

    // Persistent launches (fewer workgroups than tiles) walk the tiles with a
    // grid stride; the second half of such a grid may start late, so that the
    // workgroups sharing a CU alternate between streaming and arithmetic
    // instead of loading and computing in lockstep.
    if (PERSIST && a.stagger > 0 && blockIdx.x >= gridDim.x / 2) {
        for (int i = 0; i < a.stagger; i++) __builtin_amdgcn_s_sleep(127);
    }
    uint64_t tile = blockIdx.x;
    if (!PERSIST && a.xcd > 0) {
        // K = 8 * 2^(xcd - 1) interleaved streams: workgroup b walks stream b mod K
        const int kb = 2 + a.xcd;
        if ((a.ntiles & ((1ull << kb) - 1ull)) == 0 && gridDim.x == a.ntiles)
            tile = (uint64_t)(blockIdx.x & ((1u << kb) - 1u)) * (a.ntiles >> kb) + (blockIdx.x >> kb);
    }
    do {
        const uint64_t base = tg.base(tile);

        // ---- load in layout 0 (issued before the per-tile field computation so
        // that the field loop overlaps the memory latency)
        int cur = 0;
        CGeoLayout* L = &geo->L[0];
        uint32_t thr_u = thread_index_bits<T - R>(t, L->tmask);
        uint64_t thr_goff = tg.gmap(thr_u);

        Real vr[NV][NR], vi[NV][NR];
        // Phantom bits exist only for states smaller than one tile (PH); full tiles
        // load without per-register tests.
        if (a.load & 4) {
#pragma unroll
            for (int r = 0; r < NR; r++) {
                bool valid = true;
                if constexpr (PH) valid = ((thr_u | L->reg_u[r]) & a.phantom) == 0u;
                vr[0][r] = valid ? (Real)a.amp0 : (Real)0;
                vi[0][r] = 0;
            }
        } else if (a.load & 1) {
            const V2* __restrict__ src = (a.src ? reinterpret_cast<const V2*>(a.src) : psi) + (base | thr_goff);
            if (NTM & 1) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    const V2 v = ld_nt(src + L->reg_goff[r]);
                    vr[0][r] = v.x;
                    vi[0][r] = v.y;
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    V2 v;
                    if constexpr (PH) {
                        v.x = 0;
                        v.y = 0;
                        if (((thr_u | L->reg_u[r]) & a.phantom) == 0u) v = src[L->reg_goff[r]];
                    } else {
                        v = src[L->reg_goff[r]];
                    }
                    vr[0][r] = v.x;
                    vi[0][r] = v.y;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; r++) {
                vr[0][r] = 0;
                vi[0][r] = 0;
            }
        }
        if constexpr (NV == 2) {
            const V2* __restrict__ src = lam + (base | thr_goff);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                V2 v;
                v.x = 0;
                v.y = 0;
                bool ok = (a.load & 2) != 0;
                if constexpr (PH) ok = ok && ((thr_u | L->reg_u[r]) & a.phantom) == 0u;
                if (ok) v = src[L->reg_goff[r]];
                vr[1][r] = v.x;
                vi[1][r] = v.y;
            }
        }

        if ((t & 63) == 0) {
#pragma unroll
            for (int q = 0; q < NS; q++) s_red[t >> 6][q] = 0.0;
#pragma unroll
            for (int q = 0; q < kTF; q++) s_spin[t >> 6][q] = 0.0;
        }
        double pend[NV];  // uniform scale every register of vector v still has to be multiplied by
#pragma unroll
        for (int v = 0; v < NV; v++) pend[v] = 1.0;

        // ---- fields seen by the tile bits (only passes that evaluate E need them)
        if (a.need_e && t < kTF) s_g[t] = a.tf[tile * kTF + t];
        __syncthreads();  // s_g ready

        // The pass program has a fixed shape: two mixer slots, one point slot, two
        // mixer slots (absent slots have kind 0).  A compile-time shape keeps the
        // amplitude registers in place across ops.
        constexpr int SLOT_KIND[kMaxOps] = {OP_MIX, OP_MIX, OP_POINT, OP_MIX, OP_MIX};
#pragma unroll
        for (int oi = 0; oi < kMaxOps; oi++) {
            const Op op = a.ops[oi];
            if (op.kind == 0) continue;
            if (SLOT_KIND[oi] == OP_MIX) {
                const int K = KC > 0 ? KC : a.nlayouts;
                const bool fwd = (cur == 0);
                double gsum = 0.0;
                auto round = [&](int step) {
                    const int j = fwd ? step : (K - 1 - step);
                    if (step > 0) {
                        // LDS exchange cur -> j: in two halves split by the pivot (register
                        // slot R-1) for one vector, as whole tiles for two vectors
                        CGeoLayout* Lt = &geo->L[j];
                        const uint32_t new_u = thread_index_bits<T - R>(t, Lt->tmask);
                        // byte offsets: one XOR with the table entry per access
                        const uint32_t src = lds_swizzle(thr_u, a.swz) * (uint32_t)sizeof(V2);
                        const uint32_t dst = lds_swizzle(new_u, a.swz) * (uint32_t)sizeof(V2);
                        char* xb = reinterpret_cast<char*>(xbuf);
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            constexpr int NHALF = FULLX ? 1 : 2;
                            constexpr int NQ = FULLX ? NR : NH;
#pragma unroll
                            for (int h = 0; h < NHALF; h++) {
                                __syncthreads();
#pragma unroll
                                for (int q = 0; q < NQ; q++) {
                                    const int r = h * NQ + q;
                                    V2 x;
                                    x.x = vr[v][r];
                                    x.y = vi[v][r];
                                    *reinterpret_cast<V2*>(xb + (src ^ L->reg_lds[r])) = x;
                                }
                                __syncthreads();
#pragma unroll
                                for (int q = 0; q < NQ; q++) {
                                    const int r = h * NQ + q;
                                    const V2 x = *reinterpret_cast<const V2*>(xb + (dst ^ Lt->reg_lds[r]));
                                    vr[v][r] = x.x;
                                    vi[v][r] = x.y;
                                }
                            }
                        }
                        cur = j;
                        L = Lt;
                        thr_u = new_u;
                        thr_goff = tg.gmap(thr_u);
                    }
                    const int act = fwd ? L->act_fwd : L->act_bwd;
                    if constexpr (GEN != 0) {
                        // general single-qubit layers (one vector, no pending scale)
                        static_assert(NV == 1, "general layers are one-vector passes");
                        const SV_CONST double* __restrict__ M =
                            (const SV_CONST double*)(a.gmat + op.qidx * kGenBlock);
                        // GEN: 1 complex, 2 real, 3 complex unit-diagonal, 4 real unit-diagonal
                        constexpr bool RM = GEN == 2 || GEN == 4;
                        constexpr bool UN = GEN >= 3;
                        gen_round<Real, R, RM, UN>(vr, vi, act, L->rbpack, M);
                        const int dl = L->dpp;
                        if (dl & 8) gen_lane<kLaneX8, 3, Real, R, RM, UN>(vr, vi, tmask_bit(L->tmask, 3), M);
                        if constexpr (sizeof(Real) == 4 && T == 14) {
                            if (dl & 16) gen_lane<kLaneX16, 4, Real, R, RM, UN>(vr, vi, tmask_bit(L->tmask, 4), M);
                        }
                        return;
                    }
                    mix_round<Real, R, NV, (QFM > 0)>(vr, vi, act, op.flags, (Real)op.a, op.b, pend, gsum);
                    // lane-bit butterflies (one-vector kernels): position 3 (DPP);
                    // position 4 (swizzle) for 14-bit complex64 tiles (a second branch
                    // in the complex128 kernel would exhaust its registers)
                    const int dl = L->dpp;
                    if constexpr (NV == 2) {
                        (void)dl;  // two-vector plans butterfly every qubit in registers
                    } else if constexpr (sizeof(Real) == 8) {
                        if (dl != 0)
                            lane_round<kLaneX8, Real, R, NV, (QFM > 0)>(vr, vi, op.flags, (Real)op.a, op.b, pend, gsum);
                    } else if constexpr (T == 14 && MINB <= 2) {
                        if (dl & 8)
                            lane_round<kLaneX8, Real, R, NV, (QFM > 0)>(vr, vi, op.flags, (Real)op.a, op.b, pend, gsum);
                        else if (dl & 16)
                            lane_round<kLaneX16, Real, R, NV, (QFM > 0)>(vr, vi, op.flags, (Real)op.a, op.b, pend, gsum);
                    } else {
                        // 13-bit complex64 tiles, and 14-bit tiles in the four-waves-per-SIMD
                        // kernel (the second branch would not fit its 128 registers), plan lane
                        // position 3 only
                        if (dl != 0)
                            lane_round<kLaneX8, Real, R, NV, (QFM > 0)>(vr, vi, op.flags, (Real)op.a, op.b, pend, gsum);
                    }
                };
                if constexpr (KC > 0) {
#pragma unroll
                    for (int step = 0; step < KC; step++) round(step);
                } else {
                    for (int step = 0; step < K; step++) round(step);
                }
                if (op.flags & MIX_GBETA) wave_add<NS>(s_red, op.slot, gsum);
                if constexpr (GEN >= 3) pend[0] *= op.b;  // unit-diagonal layers: product of the diagonal moduli
            } else {  // OP_POINT
                // Walk the registers in Gray-code order: consecutive registers differ in
                // one bit k, so E changes by +-2 f[k] and the phase by exp(-+2i gamma f[k]).
                double f[R];
                const double e0 = thread_energy<R, T - R>(L, geo, t, s_g, f);
                const int fl = op.flags;
                // E of register r = e0 + (Gray-walk sum of +-2 f[k]) + Q[r]
                if constexpr (QFM >= 2) {
                    // passes of the adjoint sweeps: zeta = psi (1 + i t E) in the first pass, the
                    // form sum E |zeta|^2 at the phase of each layer (nothing else is reduced)
                    // one loop per flag, so that no per-register select keeps the old and the
                    // new amplitudes alive together.  PT_REDUCE (norm, <H_C>, P_gs of the state
                    // the sweep starts from) comes before zeta is formed.
                    if (QFM == 3 && (fl & PT_REDUCE)) {
                        double r_n = 0.0, r_e = 0.0, r_p = 0.0, e_run = e0;
#pragma unroll
                        for (int i = 0; i < NR; i++) {
                            const int r = i ^ (i >> 1);
                            if (i > 0) {
                                const int k = __builtin_ctz(i);
                                e_run += ((r >> k) & 1) ? 2.0 * f[k] : -2.0 * f[k];
                            }
                            const double e = e_run + L->Q[r];
                            const double pr = (double)vr[0][r], pi = (double)vi[0][r];
                            const double p2 = fma(pr, pr, pi * pi);
                            r_n += p2;
                            r_e = fma(e, p2, r_e);
                            if (fabs(e - a.emin) <= a.etol) r_p += p2;
                        }
                        const double s2 = pend[0] * pend[0];
                        wave_add<NS>(s_red, op.slot, r_n * s2);
                        wave_add<NS>(s_red, op.slot + 1, r_e * s2);
                        wave_add<NS>(s_red, op.slot + 2, r_p * s2);
                    }
                    if (fl & PT_ZETA) {
                        const double zt = op.b;
                        double e_run = e0;
#pragma unroll
                        for (int i = 0; i < NR; i++) {
                            const int r = i ^ (i >> 1);
                            if (i > 0) {
                                const int k = __builtin_ctz(i);
                                e_run += ((r >> k) & 1) ? 2.0 * f[k] : -2.0 * f[k];
                            }
                            const double te = zt * (e_run + L->Q[r]);
                            const double pr = (double)vr[0][r], pi = (double)vi[0][r];
                            vr[0][r] = (Real)fma(-te, pi, pr);
                            vi[0][r] = (Real)fma(te, pr, pi);
                        }
                    }
                    if (fl & PT_EFORM) {
                        double r_f = 0.0, e_run = e0;
#pragma unroll
                        for (int i = 0; i < NR; i++) {
                            const int r = i ^ (i >> 1);
                            if (i > 0) {
                                const int k = __builtin_ctz(i);
                                e_run += ((r >> k) & 1) ? 2.0 * f[k] : -2.0 * f[k];
                            }
                            const double pr = (double)vr[0][r], pi = (double)vi[0][r];
                            r_f = fma(e_run + L->Q[r], fma(pr, pr, pi * pi), r_f);
                        }
                        wave_add<NS>(s_red, op.slot2, r_f * pend[0] * pend[0]);
                    }
                }
                constexpr int kRedFlags = QFM > 0 ? 0 : (PT_REDUCE | PT_LAM_INIT | PT_GGAMMA | PT_SPINZ | PT_E2);
                if (fl & kRedFlags) {
                    // one sweep over the registers feeds every reduction of the op
                    // (|psi|^2 is formed once; the spin sums of one-vector passes
                    // take it for each register bit k: +-|psi|^2 by bit k of r)
                    double r_n = 0.0, r_e = 0.0, r_p = 0.0, r_g = 0.0, r_e2 = 0.0;
                    double Sk[R];
#pragma unroll
                    for (int k = 0; k < R; k++) Sk[k] = 0.0;
                    // spin sums exist in the generic kernels and in dedicated fast variants
                    const bool spins = SPZ && NV == 1 && (fl & PT_SPINZ) != 0;
                    double e_run = e0;
#pragma unroll
                    for (int i = 0; i < NR; i++) {
                        const int r = i ^ (i >> 1);
                        if (i > 0) {
                            const int k = __builtin_ctz(i);
                            e_run += ((r >> k) & 1) ? 2.0 * f[k] : -2.0 * f[k];
                        }
                        const double e = e_run + L->Q[r];
                        const double pr = (double)vr[0][r], pi = (double)vi[0][r];
                        if (fl & (PT_REDUCE | PT_SPINZ | PT_E2)) {
                            const double p2 = pr * pr + pi * pi;
                            r_n += p2;
                            r_e += e * p2;
                            if (fl & PT_E2) r_e2 += e * e * p2;
                            if (fabs(e - a.emin) <= a.etol) r_p += p2;
                            if (spins) {
#pragma unroll
                                for (int k = 0; k < R; k++) Sk[k] += ((r >> k) & 1) ? p2 : -p2;
                            }
                        }
                        if constexpr (NV == 2) {
                            if (fl & PT_LAM_INIT) {
                                vr[1][r] = (Real)(e * pr);
                                vi[1][r] = (Real)(e * pi);
                            }
                            if (fl & PT_GGAMMA) {
                                const Real q = vr[1][r] * vi[0][r] - vi[1][r] * vr[0][r];
                                r_g += e * (double)q;
                            }
                        }
                    }
                    const double s2 = pend[0] * pend[0];
                    if (fl & PT_REDUCE) {
                        wave_add<NS>(s_red, op.slot, r_n * s2);
                        wave_add<NS>(s_red, op.slot + 1, r_e * s2);
                        wave_add<NS>(s_red, op.slot + 2, r_p * s2);
                    }
                    if (fl & PT_E2) wave_add<NS>(s_red, op.slot3, r_e2 * s2);
                    if constexpr (NV == 1 && SPZ) {
                        if (spins) {
                            // tile bit l: register bit k -> Sk[k]; thread bit j -> +-norm
                            const uint32_t rbp = L->rbpack;
#pragma unroll
                            for (int k = 0; k < R; k++) wave_add<kTF>(s_spin, (rbp >> (4 * k)) & 15u, Sk[k] * s2);
                            uint32_t m = L->tmask;
#pragma unroll
                            for (int j = 0; j < T - R; j++) {
                                const int l = __builtin_ctz(m);
                                m &= m - 1u;
                                wave_add<kTF>(s_spin, l, ((t >> j) & 1u) ? r_n * s2 : -r_n * s2);
                            }
                            wave_add<kTF>(s_spin, kTF - 1, r_n * s2);
                        }
                    }
                    if constexpr (NV == 2) {
                        if (fl & PT_LAM_INIT) pend[1] = pend[0];
                        if (fl & PT_GGAMMA) wave_add<NS>(s_red, op.slot2, r_g * pend[0] * pend[1]);
                    }
                }
                if (fl & (PT_PHASE_PSI | PT_PHASE_LAM)) {
                    const double gam = op.a;
                    const SV_CONST double* __restrict__ qph = (const SV_CONST double*)(a.ptab + a.qph_off[op.qidx]);
                    double2 gk[R];
                    double2 run;
                    if constexpr (INTE) {
                        // energies on the grid Z / q: factors from the table exp(-i gamma m / q)
                        const SV_CONST double* __restrict__ lut =
                            (const SV_CONST double*)(a.ptab + a.lut_off[op.qidx] + a.lut_half);
                        const int Lh = a.lut_half;
#pragma unroll
                        for (int k = 0; k < R; k++) {
                            const int m = min(max((int)(2.0 * f[k] * a.lut_q), -Lh), Lh);
                            gk[k] = ctab(lut, m);
                        }
                        run = ctab(lut, min(max((int)(e0 * a.lut_q), -Lh), Lh));
                    } else {
                        // One sincos at a time: the fma(0, previous sine, x) link (exact
                        // for finite values) keeps the scheduler from interleaving the
                        // R + 1 evaluations, which would exhaust the register file.
                        double link = 0.0;
#pragma unroll
                        for (int k = 0; k < R; k++) {
                            double sn, cs;
                            sincos(fma(0.0, link, 2.0 * gam * f[k]), &sn, &cs);
                            gk[k] = make_double2(cs, -sn);
                            link = sn;
                        }
                        double sn, cs;
                        sincos(fma(0.0, link, gam * e0), &sn, &cs);
                        run = make_double2(cs, -sn);
                    }
                    // the phase has modulus one: the pending scales stay pending (they are
                    // applied at the store)
#pragma unroll
                    for (int i = 0; i < NR; i++) {
                        const int r = i ^ (i >> 1);
                        if (i > 0) {
                            const int k = __builtin_ctz(i);
                            const double2 g = ((r >> k) & 1) ? gk[k] : make_double2(gk[k].x, -gk[k].y);
                            run = cmul(run, g);
                        }
                        const double2 ph = cmul(run, ctab(qph, r));
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            if constexpr (sizeof(Real) == 8) {
                                const double xr = vr[v][r], xi = vi[v][r];
                                vr[v][r] = xr * ph.x - xi * ph.y;
                                vi[v][r] = xr * ph.y + xi * ph.x;
                            } else {
                                const float cr = (float)ph.x, ci = (float)ph.y;
                                const float xr = vr[v][r], xi = vi[v][r];
                                vr[v][r] = xr * cr - xi * ci;
                                vi[v][r] = xr * ci + xi * cr;
                            }
                        }
                    }
                }
            }
        }

        // ---- store in the current layout (applying what is left of the pending scales)
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (!(a.store & (1 << v))) continue;
            V2* __restrict__ dst = (v == 0 ? psi : lam) + (base | thr_goff);
            const Real sc = (Real)pend[v];
            const bool unit = pend[v] == 1.0;
            if (NTM & 2) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    V2 x;
                    x.x = unit ? vr[v][r] : vr[v][r] * sc;
                    x.y = unit ? vi[v][r] : vi[v][r] * sc;
                    st_nt(dst + L->reg_goff[r], x);
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if constexpr (PH) {
                        if (((thr_u | L->reg_u[r]) & a.phantom) != 0u) continue;
                    }
                    V2 x;
                    x.x = unit ? vr[v][r] : vr[v][r] * sc;
                    x.y = unit ? vi[v][r] : vi[v][r] * sc;
                    dst[L->reg_goff[r]] = x;
                }
            }
        }

        // ---- per-tile partial sums, fixed order
        if (a.nslots > 0 || (SPZ && a.spin_part)) {
            __syncthreads();
            if ((int)t < a.nslots) {
                double v = 0.0;
                for (int ww = 0; ww < NW; ww++) v += s_red[ww][t];
                a.partials[tile * (uint64_t)a.nslots + t] = v;
            }
            if (SPZ && a.spin_part && t < kTF) {
                double v = 0.0;
                for (int ww = 0; ww < NW; ww++) v += s_spin[ww][t];
                a.spin_part[tile * kTF + t] = v;
            }
        }
        if constexpr (!PERSIST) break;
        tile += gridDim.x;
        if (tile < a.ntiles) __syncthreads();  // LDS reuse by the next tile
    } while (tile < a.ntiles);
}

// Column sums of partials[nrows][nslots] in a fixed order: out[dst[s]] (+)= sum.
// Two launches: kReduceBlocks workgroups each sum a contiguous run of rows
// (strided per thread, then a tree) into stage[block][slot]; one workgroup then
// adds the blocks' sums in a tree.  The order depends only on nrows.
struct SlotDst {
    int d[kMaxSlots];
};

__global__ void __launch_bounds__(256) k_reduce_rows(const double* __restrict__ partials, uint64_t nrows, int nslots,
                                                     double* __restrict__ stage) {
    __shared__ double sh[kMaxSlots][256];
    const int t = threadIdx.x;
    const uint64_t per = (nrows + gridDim.x - 1) / gridDim.x;
    const uint64_t r0 = (uint64_t)blockIdx.x * per;
    const uint64_t r1 = r0 + per < nrows ? r0 + per : nrows;
    double v[kMaxSlots];
#pragma unroll
    for (int q = 0; q < kMaxSlots; q++) v[q] = 0.0;
    for (uint64_t i = r0 + t; i < r1; i += 256)
#pragma unroll
        for (int q = 0; q < kMaxSlots; q++)
            if (q < nslots) v[q] += partials[i * nslots + q];
#pragma unroll
    for (int q = 0; q < kMaxSlots; q++) sh[q][t] = v[q];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < kMaxSlots; q++) sh[q][t] += sh[q][t + w];
        __syncthreads();
    }
    if (t < nslots) stage[blockIdx.x * kMaxSlots + t] = sh[t][0];
}

__global__ void __launch_bounds__(256) k_reduce_slots(const double* __restrict__ stage, int nblocks, int nslots,
                                                      SlotDst dst, int accumulate, double* __restrict__ out) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    for (int q = 0; q < nslots; q++) {
        sh[t] = t < nblocks ? stage[t * kMaxSlots + q] : 0.0;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) {
            const int d = dst.d[q];
            out[d] = accumulate ? out[d] + sh[0] : sh[0];
        }
        __syncthreads();
    }
}

// <sigma^z_i> from the per-tile spin partials, one workgroup per qubit in a fixed
// order: a qubit held by tile bit l sums entry l over the tiles; any other qubit
// is fixed within a tile, so it sums s_i(tile) times the tile's norm entry.
__global__ void __launch_bounds__(256) k_spin_reduce(const SpinArgs a) {
    __shared__ double sh[256];
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    int l = -1;
    for (int q = 0; q < a.T; q++)
        if (a.qubit[q] == i) l = q;
    const TileGeom tg{a.c, a.lo, a.g};
    double v = 0.0;
    for (uint64_t w = t; w < a.ntiles; w += 256) {
        const double* row = a.part + w * kTF;
        v += l >= 0 ? row[l] : spin_z(tg.base(w), i) * row[kTF - 1];
    }
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    if (t == 0) a.out[i] = sh[0];
}

int launch_spin_reduce(const SpinArgs& a, void* stream) {
    hipLaunchKernelGGL(k_spin_reduce, dim3((unsigned)a.n), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// Brute-force enumeration of E(z) over all basis states, tile by tile in layout 0.
template <int T, int R>
__global__ void __launch_bounds__(1 << (T - R)) k_ground(const GroundArgs a) {
    constexpr int NT = 1 << (T - R);
    constexpr int NR = 1 << R;
    constexpr int NW = NT / 64;
    constexpr int RLO = (R + 1) / 2;
    constexpr int RHI = R - RLO;
    __shared__ double s_g[kTF];
    __shared__ double s_e[NW];
    __shared__ unsigned long long s_c[NW], s_a[NW];

    const uint32_t t = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    CGeoBuf* __restrict__ geo = (CGeoBuf*)a.geo;
    const TileGeom tg{a.c, a.lo, a.g};
    const uint64_t base = tg.base(tile);
    if (t < kTF) s_g[t] = a.tf[tile * kTF + t];
    __syncthreads();

    CGeoLayout* L = &geo->L[0];
    const uint32_t thr_u = thread_index_bits<T - R>(t, L->tmask);
    const uint64_t thr_goff = tg.gmap(thr_u);
    double f[R];
    const double e0 = thread_energy<R, T - R>(L, geo, t, s_g, f);
    double elo[1 << RLO], ehi[1 << RHI];
    elo[0] = e0;
#pragma unroll
    for (int k = 0; k < RLO; k++)
#pragma unroll
        for (int r = 0; r < (1 << k); r++) elo[r | (1 << k)] = elo[r] + 2.0 * f[k];
    ehi[0] = 0.0;
#pragma unroll
    for (int k = 0; k < RHI; k++)
#pragma unroll
        for (int r = 0; r < (1 << k); r++) ehi[r | (1 << k)] = ehi[r] + 2.0 * f[RLO + k];

    double emin = INFINITY;
    unsigned long long cnt = 0, first = ~0ull;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const uint32_t u = thr_u | L->reg_u[r];
        if ((u & a.phantom) != 0u) continue;
        const double e = elo[r & ((1 << RLO) - 1)] + ehi[r >> RLO] + L->Q[r];
        if (a.mode == 0) {
            emin = fmin(emin, e);
        } else if (fabs(e - a.emin) <= a.etol) {
            const unsigned long long z = base | thr_goff | L->reg_goff[r];
            cnt++;
            first = z < first ? z : first;
        }
    }
    const int lane = t & 63, w = t >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        emin = fmin(emin, __shfl_xor(emin, off));
        cnt += __shfl_xor(cnt, off);
        const unsigned long long o = __shfl_xor(first, off);
        first = o < first ? o : first;
    }
    if (lane == 0) {
        s_e[w] = emin;
        s_c[w] = cnt;
        s_a[w] = first;
    }
    __syncthreads();
    if (t == 0) {
        double e = s_e[0];
        unsigned long long c2 = s_c[0], f2 = s_a[0];
        for (int ww = 1; ww < NW; ww++) {
            e = fmin(e, s_e[ww]);
            c2 += s_c[ww];
            f2 = s_a[ww] < f2 ? s_a[ww] : f2;
        }
        if (a.mode == 0) {
            a.part_e[tile] = e;
        } else {
            a.part_cnt[tile] = c2;
            a.part_arg[tile] = f2;
        }
    }
}

__global__ void __launch_bounds__(256) k_ground_finish(const GroundArgs a, double* out_e,
                                                       unsigned long long* out_cnt,
                                                       unsigned long long* out_arg) {
    __shared__ double se[256];
    __shared__ unsigned long long sc[256], sa[256];
    const int t = threadIdx.x;
    double e = INFINITY;
    unsigned long long c = 0, f = ~0ull;
    for (uint64_t i = t; i < a.ntiles; i += 256) {
        if (a.mode == 0) {
            e = fmin(e, a.part_e[i]);
        } else {
            c += a.part_cnt[i];
            f = a.part_arg[i] < f ? a.part_arg[i] : f;
        }
    }
    se[t] = e;
    sc[t] = c;
    sa[t] = f;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
            se[t] = fmin(se[t], se[t + w]);
            sc[t] += sc[t + w];
            sa[t] = sa[t + w] < sa[t] ? sa[t + w] : sa[t];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (a.mode == 0) {
            *out_e = se[0];
        } else {
            *out_cnt = sc[0];
            *out_arg = sa[0];
        }
    }
}

// ----------------------------------------------------------------------------- dispatch
// Tile shapes.  complex128: T = 13 (128 KiB tiles).  complex64: T = 14 for
// one-vector programs; adjoint programs use T = 13 for both vectors, the
// largest two-vector tile whose kernel fits the register file.
Shape shape_for(int dtype, int nv, bool grad) {
    if (dtype == 2) return nv == 1 ? Shape{13, 5} : Shape{13, 4};
    if (!grad) return Shape{14, 5};
    return nv == 1 ? Shape{13, 5} : Shape{13, 4};
}

// Full-tile general-layer passes: layout count, real or complex matrices, nontemporal hints.
template <typename Real, int T, int R, int NS, int GMB, int NTM, int GC = 1, int GR = 2>
static void launch_gen_fast(const PassArgs& a, dim3 grid, dim3 block, hipStream_t st) {
    if constexpr (GC == 1) {
        if (a.gen_unit) {  // unit-diagonal layers: the GEN = 3 / 4 kernels
            launch_gen_fast<Real, T, R, NS, GMB, NTM, 3, 4>(a, grid, block, st);
            return;
        }
    }
    const bool rm = a.gen_real != 0;
    // three or more layouts with complex matrices on complex128 amplitudes need the whole
    // register file (one workgroup per CU)
    constexpr int MB = (sizeof(Real) == 8 && GC == 1) ? 1 : GMB;
    if (a.nlayouts == 1) {
        if (rm) hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 1, NTM, false, false, GR>), grid, block,
                                   0, st, a);
        else hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 1, NTM, false, false, GC>), grid, block, 0,
                                st, a);
    } else if (a.nlayouts == 2) {
        if (rm) hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 2, NTM, false, false, GR>), grid, block,
                                   0, st, a);
        else hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 2, NTM, false, false, GC>), grid, block, 0,
                                st, a);
    } else if (a.kc34 && a.nlayouts == 3) {  // straight-line walk
        if (rm) hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 3, NTM, false, false, GR>), grid, block,
                                   0, st, a);
        else hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MB, false, true, 3, NTM, false, false, GC>), grid, block, 0,
                                st, a);
    } else {
        if (rm) hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, GMB, false, true, 0, NTM, false, false, GR>), grid, block,
                                   0, st, a);
        else hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MB, false, true, 0, NTM, false, false, GC>), grid, block, 0,
                                st, a);
    }
}

// Passes of the two one-vector adjoint sweeps: QFM = 1 mixer-only passes (quadratic forms),
// QFM = 2 passes that also form zeta or the E form at their POINT, QFM = 3 the first pass of
// the zeta_+ sweep, which also reduces norm, <H_C> and P_gs (each part that is not needed
// is left out: kernels with all of them spill).
template <typename Real, int T, int R, int NS, int MINB, int QFM>
static int launch_qf(const PassArgs& a, bool fast, dim3 grid, dim3 block, hipStream_t st) {
    constexpr int PMB = MINB > 2 ? 2 : MINB;
    if (!fast && a.lut_half >= 0) {  // states smaller than one tile
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, PMB, true, true, 0, 0, false, false, 0, QFM>), grid, block, 0, st,
                           a);
    } else if (!fast) {  // real-valued instances: FP64 sincos
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, 1, true, false, 0, 0, false, false, 0, QFM>), grid, block, 0, st,
                           a);
    } else if (a.nlayouts == 1) {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 1, 0, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else if (a.nlayouts == 2 && a.nt == 3) {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 2, 3, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else if (a.nlayouts == 2) {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 2, 0, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else if (sizeof(Real) == 4 && a.nlayouts == 3 && a.nt == 3) {
        // complex64: straight-line walk (the layout loop spills more there)
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 3, 3, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else if (sizeof(Real) == 4 && a.nlayouts == 3) {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 3, 0, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else if (a.nt == 3) {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 0, 3, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    } else {
        hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, MINB, false, true, 0, 0, false, false, 0, QFM>), grid, block, 0,
                           st, a);
    }
    return (int)hipGetLastError();
}

// Slot counts: one-vector passes carry up to 8 reduction slots (fused AQA
// steps); two-vector passes need at most 4 (3 for the turnaround reductions
// + 1 gradient slot, or 3 gradient slots).
template <typename Real, int T, int R, int NV, int NS, int MINB>
static int run_pass(const PassArgs& a, void* stream) {
    // persistent grids exist for the one-vector fast paths with >= 2 layouts
    const bool pers = NV == 1 && a.grid > 0 && (uint64_t)a.grid < a.ntiles && a.nlayouts >= 2 && a.phantom == 0 &&
                      (a.lut_half >= 0 || a.nphase == 0);
    const unsigned nwg = pers ? (unsigned)a.grid : (unsigned)a.ntiles;
    const dim3 grid(nwg), block(1 << (T - R));
    hipStream_t st = (hipStream_t)stream;
    const bool fast = a.phantom == 0 && (a.lut_half >= 0 || a.nphase == 0);
    // general-layer kernels exist for 13-bit complex128 and 14-bit complex64 tiles
    if constexpr (NV == 1 && ((sizeof(Real) == 8 && T == 13) || (sizeof(Real) == 4 && T == 14))) {
        if (a.gmat) {  // general single-qubit layers (real matrices: half the arithmetic)
            // general kernels need more registers than the four-waves-per-SIMD budget
            constexpr int GMB = MINB > 2 ? 2 : MINB;
            if (fast && !a.spin_part) {
                if (a.nt == 3)
                    launch_gen_fast<Real, T, R, NS, GMB, 3>(a, grid, block, st);
                else
                    launch_gen_fast<Real, T, R, NS, GMB, 0>(a, grid, block, st);
            } else if (a.gen_unit) {
                hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, 1, true, false, 0, 0, false, true, 3>), grid, block,
                                   0, st, a);
            } else {
                hipLaunchKernelGGL((k_pass<Real, T, R, 1, NS, 1, true, false, 0, 0, false, true, 1>), grid, block,
                                   0, st, a);
            }
            return (int)hipGetLastError();
        }
    }
    if (a.gmat) return (int)hipErrorInvalidValue;
    // passes of the two one-vector adjoint sweeps (quadratic forms, zeta, E forms) exist for
    // the default one-vector tiles: 13-bit complex128 and 14-bit complex64 with four waves per SIMD
    constexpr bool kQF = NV == 1 && ((sizeof(Real) == 8 && T == 13) || (sizeof(Real) == 4 && T == 14 && MINB == 4));
    if (a.qf && !kQF) return (int)hipErrorInvalidValue;
    if constexpr (kQF) {
        if (a.qf == 1) return launch_qf<Real, T, R, NS, MINB, 1>(a, fast, grid, block, st);
        if (a.qf == 2) return launch_qf<Real, T, R, NS, MINB, 2>(a, fast, grid, block, st);
        if (a.qf == 3) return launch_qf<Real, T, R, NS, MINB, 3>(a, fast, grid, block, st);
    }
    if (fast) {
        // one or two layouts: straight-line walks; three or more: a loop keeps
        // the register pressure below the two-workgroups-per-CU limit
        // (nontemporal variants for passes over long contiguous runs)
        if constexpr (NV == 1) {
            if (a.spin_part) {  // passes that also sum the spin expectations (more registers)
                constexpr int SMB = MINB > 2 ? 2 : MINB;
                if (a.nlayouts == 1)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, SMB, false, true, 1, 0, false, true>), grid, block,
                                       0, st, a);
                else if (a.nlayouts == 2)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, SMB, false, true, 2, 0, false, true>), grid, block,
                                       0, st, a);
                else
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, SMB, false, true, 0, 0, false, true>), grid, block,
                                       0, st, a);
                return (int)hipGetLastError();
            }
            if (pers) {
                if (a.nlayouts == 2)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 2, 0, true>), grid, block, 0, st,
                                       a);
                else if (a.nt == 3)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 0, 3, true>), grid, block, 0, st,
                                       a);
                else
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 0, 0, true>), grid, block, 0, st,
                                       a);
                return (int)hipGetLastError();
            }
        }
        if constexpr (NV == 2) {
            // two-vector passes (one workgroup per CU, the whole register file): three and
            // four layouts as straight-line walks
            if (a.kc34 && a.nlayouts == 3) {
                if (a.nt == 3)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 3, 3>), grid, block, 0, st, a);
                else
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 3>), grid, block, 0, st, a);
                return (int)hipGetLastError();
            }
            if (a.kc34 && a.nlayouts == 4) {
                if (a.nt == 3)
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 4, 3>), grid, block, 0, st, a);
                else
                    hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 4>), grid, block, 0, st, a);
                return (int)hipGetLastError();
            }
        }
        if (a.nlayouts == 1)
            hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 1>), grid, block, 0, st, a);
        else if (a.nlayouts == 2 && a.nt == 3)
            hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 2, 3>), grid, block, 0, st, a);
        else if (a.nlayouts == 2)
            hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 2>), grid, block, 0, st, a);
        else if (a.nt == 3)
            hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 0, 3>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, MINB, false, true, 0>), grid, block, 0, st, a);
    } else if (a.lut_half >= 0) {
        // states smaller than one tile (phantom bits): correctness over occupancy
        constexpr int PMB = MINB > 2 ? 2 : MINB;
        hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, PMB, true, true, 0>), grid, block, 0, st, a);
    } else {
        // real-valued instances: FP64 sincos per thread needs more registers;
        // one workgroup per CU lets the compiler keep them in the AGPR half
        hipLaunchKernelGGL((k_pass<Real, T, R, NV, NS, 1, true, false, 0>), grid, block, 0, st, a);
    }
    return (int)hipGetLastError();
}

int launch_pass(int dtype, int nv, int T, const PassArgs& a, void* stream) {
    if (nv == 2 && a.nslots > 4) return (int)hipErrorInvalidValue;
    if (a.nlayouts < 1 || a.nlayouts > kMaxLayouts) return (int)hipErrorInvalidValue;
    if (dtype == 2) {
        // 14-bit complex128 tiles: 512 threads, one workgroup per CU (128 KiB half-tile exchanges)
        if (nv == 1 && T == 14) return run_pass<double, 14, 5, 1, 8, 2>(a, stream);
        if (nv == 1) return run_pass<double, 13, 5, 1, 8, 2>(a, stream);
        return run_pass<double, 13, 4, 2, 4, 1>(a, stream);
    }
    if (nv == 1) {
        if (T == 14) return a.occ4 ? run_pass<float, 14, 5, 1, 8, 4>(a, stream) : run_pass<float, 14, 5, 1, 8, 2>(a, stream);
        return run_pass<float, 13, 5, 1, 8, 4>(a, stream);
    }
    if (T == 14) return run_pass<float, 14, 4, 2, 4, 4>(a, stream);  // 1024 threads
    return a.occ4 ? run_pass<float, 13, 4, 2, 4, 4>(a, stream) : run_pass<float, 13, 4, 2, 4, 1>(a, stream);
}

// Streaming ceiling of a tile geometry: every workgroup loads its tile (2^T
// amplitudes, the pass's lane order: thread t holds tile-local indices
// t + r 2^(T-R)) with nontemporal loads and stores it back unchanged, in the
// passes' XCD-aware tile order.  No arithmetic.
template <typename V2, int T, int R, int MINB>
__global__ void __launch_bounds__(1 << (T - R), MINB) k_stream(V2* __restrict__ p, const StreamArgs a) {
    constexpr int NT = 1 << (T - R);
    constexpr int NR = 1 << R;
    uint64_t tile = blockIdx.x;
    if (a.xcd > 0) {
        const int kb = 2 + a.xcd;
        if ((a.ntiles & ((1ull << kb) - 1ull)) == 0 && gridDim.x == a.ntiles)
            tile = (uint64_t)(blockIdx.x & ((1u << kb) - 1u)) * (a.ntiles >> kb) + (blockIdx.x >> kb);
    }
    const TileGeom tg{a.c, a.lo, a.g};
    V2* __restrict__ q = p + tg.base(tile);
    V2 v[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = ld_nt(q + tg.gmap(threadIdx.x + (uint32_t)r * NT));
    // XOR with a mask that is zero at run time: the stores cannot be proven to
    // write back what was loaded, so the compiler keeps them
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if constexpr (sizeof(v[r].x) == 8) {
            v[r].x = __longlong_as_double(__double_as_longlong(v[r].x) ^ (long long)a.mask);
            v[r].y = __longlong_as_double(__double_as_longlong(v[r].y) ^ (long long)a.mask);
        } else {
            v[r].x = __int_as_float(__float_as_int(v[r].x) ^ (int)a.mask);
            v[r].y = __int_as_float(__float_as_int(v[r].y) ^ (int)a.mask);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) st_nt(q + tg.gmap(threadIdx.x + (uint32_t)r * NT), v[r]);
}

int launch_stream(int dtype, void* p, const StreamArgs& a, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (dtype == 2)
        hipLaunchKernelGGL((k_stream<double2, 13, 5, 2>), dim3((unsigned)a.ntiles), dim3(256), 0, st,
                           (double2*)p, a);
    else
        hipLaunchKernelGGL((k_stream<float2, 14, 5, 4>), dim3((unsigned)a.ntiles), dim3(512), 0, st,
                           (float2*)p, a);
    return (int)hipGetLastError();
}

int launch_tables(const TableJob* jobs, int njobs, double2* out, void* stream) {
    for (int s = 0; s < njobs; s += 64) {
        TableJobs tj;
        const int cnt = njobs - s < 64 ? njobs - s : 64;
        for (int i = 0; i < cnt; i++) tj.j[i] = jobs[s + i];
        hipLaunchKernelGGL(k_tables, dim3(cnt), dim3(256), 0, (hipStream_t)stream, tj, out);
        const int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

int launch_reduce_slots(const double* partials, uint64_t nrows, int nslots, const int* dst, int accumulate,
                        double* out, double* stage, void* stream) {
    SlotDst d;
    for (int s = 0; s < kMaxSlots; s++) d.d[s] = s < nslots ? dst[s] : 0;
    const uint64_t want = (nrows + 2047) / 2048;  // about 2048 rows per workgroup
    const int nb = (int)(want < (uint64_t)kReduceBlocks ? (want > 0 ? want : 1) : kReduceBlocks);
    hipLaunchKernelGGL(k_reduce_rows, dim3(nb), dim3(256), 0, (hipStream_t)stream, partials, nrows, nslots, stage);
    hipLaunchKernelGGL(k_reduce_slots, dim3(1), dim3(256), 0, (hipStream_t)stream, stage, nb, nslots, d, accumulate,
                       out);
    return (int)hipGetLastError();
}

int launch_tile_fields(const TfArgs& a, void* stream) {
    const uint64_t blocks = (a.ntiles + 3) / 4;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_tile_fields, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_ground(int dtype, const GroundArgs& a, void* stream) {
    if (dtype == 2)
        hipLaunchKernelGGL((k_ground<13, 5>), dim3((unsigned)a.ntiles), dim3(256), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((k_ground<14, 5>), dim3((unsigned)a.ntiles), dim3(512), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_ground_finish(const GroundArgs& a, double* out_e, uint64_t* out_cnt, uint64_t* out_arg,
                         void* stream) {
    hipLaunchKernelGGL(k_ground_finish, dim3(1), dim3(256), 0, (hipStream_t)stream, a, out_e,
                       (unsigned long long*)out_cnt, (unsigned long long*)out_arg);
    return (int)hipGetLastError();
}

}  // namespace svk

// ============================================================================ batch scan
// p = 1 landscape over many small instances (Sec. III.C.1, Fig. 5): for each
// instance i and grid point (gamma_a, beta_b), psi = exp(-i beta_b H_D)
// exp(-i gamma_a H_C) |+>, then <H_C> and the ground-state probability.
namespace svk {

// Energy tables E_i(z) for every instance (Eq. HC), one thread per basis state;
// integer-valued instances also get the 16-bit table index E(z) - lut_lo.
__global__ void __launch_bounds__(256) k_batch_energy(const BatchArgs a) {
    const int i = blockIdx.y;
    const BatchInst in = a.inst[i];
    const uint64_t N = 1ull << in.n;
    for (uint64_t z = (uint64_t)blockIdx.x * 256 + threadIdx.x; z < N; z += (uint64_t)gridDim.x * 256) {
        double e = 0.0;
        for (int q = 0; q < in.n; q++) e += a.h[in.hoff + q] * (((z >> q) & 1) ? 1.0 : -1.0);
        for (int k = 0; k < in.m; k++) {
            const int u = a.ei[in.coff + k], v = a.ej[in.coff + k];
            const double su = ((z >> u) & 1) ? 1.0 : -1.0, sv = ((z >> v) & 1) ? 1.0 : -1.0;
            e += a.J[in.coff + k] * su * sv;
        }
        a.etab[in.eoff + z] = e;
        if (in.lut_n > 0) a.eidx[in.eoff + z] = (uint16_t)((int)e - in.lut_lo);
    }
}

// Minimum of each energy table (one workgroup per instance).
__global__ void __launch_bounds__(256) k_batch_emin(const BatchArgs a, BatchInst* inst) {
    __shared__ double sh[256];
    const int i = blockIdx.x;
    const BatchInst in = a.inst[i];
    const uint64_t N = 1ull << in.n;
    double e = INFINITY;
    for (uint64_t z = threadIdx.x; z < N; z += 256) e = fmin(e, a.etab[in.eoff + z]);
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) inst[i].emin = sh[0];
}

constexpr int kBatchUnroll = 4;  // table entries in flight per thread

// One workgroup per CU holds the LDS state, with NTH threads (complex128: four
// waves, its register blocks need more than the 256 registers that two waves
// per SIMD leave; complex64: four or eight).
template <typename Real>
struct BatchCfg {
    static constexpr int G = sizeof(Real) == 4 ? 4 : 3;  // LDS swizzle width
};

__device__ __forceinline__ uint32_t bswz(uint32_t z, int G) { return lds_swizzle(z, G); }

// Hides a per-thread value from loop-invariant code motion: the block addresses
// derived from it are then formed next to their use instead of being hoisted out
// of the slice and beta loops and kept live (and spilled) across them.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// exp(-i beta sigma^x) / cos(beta) on the NB index bits of 2^NB register values,
// t = tan(beta): the pair (a, b) becomes (a - i t b, b - i t a).  The scan applies
// the factor cos(beta)^{2n} to the reduced sums instead of to every amplitude.
template <typename Real, int NB>
__device__ __forceinline__ void reg_mix(typename V2T<Real>::type (&v)[1 << NB], Real t) {
#pragma unroll
    for (int k = 0; k < NB; k++) {
#pragma unroll
        for (int r = 0; r < (1 << NB); r++) {
            if (r & (1 << k)) continue;
            const int r2 = r | (1 << k);
            const Real ar = v[r].x, ai = v[r].y, br = v[r2].x, bi = v[r2].y;
            v[r].x = ar + t * bi;
            v[r].y = ai - t * br;
            v[r2].x = br + t * ai;
            v[r2].y = bi - t * ar;
        }
    }
}

// exp(-i beta sigma^x) / cos(beta) on every qubit of an LDS-resident state of 2^nb
// elements (bits 0..nb-1), in register blocks of 5 bits; t = tan(beta).
template <typename Real, int NTH>
__device__ void lds_mixer(typename V2T<Real>::type* st, int nb, Real t) {
    using V2 = typename V2T<Real>::type;
    constexpr int G = BatchCfg<Real>::G;
    const int nblk = (nb + 4) / 5;
    uint32_t done = 0;
    for (int j = 0; j < nblk; j++) {
        const int a0 = min(5 * j, nb - 5);
        uint32_t act = 0;
        for (int k = 0; k < 5; k++)
            if (!((done >> (a0 + k)) & 1u)) act |= 1u << k;
        done |= 31u << a0;
        const uint32_t nq = 1u << (nb - 5);
        for (uint32_t q = threadIdx.x; q < nq; q += NTH) {
            const uint32_t zb = (q & ((1u << a0) - 1u)) | ((q >> a0) << (a0 + 5));
            const uint32_t bz = bswz(zb, G);
            V2 v[32];
#pragma unroll
            for (int r = 0; r < 32; r++) v[r] = st[bz ^ bswz((uint32_t)r << a0, G)];
#pragma unroll
            for (int k = 0; k < 5; k++) {
                if (!((act >> k) & 1u)) continue;
#pragma unroll
                for (int r = 0; r < 32; r++) {
                    if (r & (1 << k)) continue;
                    const int r2 = r | (1 << k);
                    const Real ar = v[r].x, ai = v[r].y, br = v[r2].x, bi = v[r2].y;
                    v[r].x = ar + t * bi;
                    v[r].y = ai - t * br;
                    v[r2].x = br + t * ai;
                    v[r2].y = bi - t * ar;
                }
            }
#pragma unroll
            for (int r = 0; r < 32; r++) st[bz ^ bswz((uint32_t)r << a0, G)] = v[r];
        }
        __syncthreads();
    }
}

// Persistent scan: workgroups take (instance, gamma) units from a queue, largest
// n first, and evaluate every beta of the grid for that unit.  Integer-valued
// instances read 16-bit table indices (E(z) - lut_lo) and take the phase
// 2^{-n/2} exp(-i gamma E) from an LDS table; the others read E(z) in FP64 and
// take sincos.  Table reads are issued kBatchUnroll at a time per thread.
// SLOTS = false drops the slot code (registers for the LDS-resident path only):
// the variant for queues that hold only units with n <= S.
template <typename Real, int NTH, int S, int LUTN, int MINW = 1, bool SLOTS = true>
__global__ void __launch_bounds__(NTH, MINW) k_batch_scan(const BatchArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int G = BatchCfg<Real>::G;
    constexpr int U = kBatchUnroll;
    static_assert(S >= 10 && S <= 15, "slice rounds assume 10 <= S <= 15");
    __shared__ V2 st[1 << S];
    __shared__ V2 lut[LUTN];  // 2^{-n/2} exp(-i gamma E), rounded once to the storage type
    __shared__ double red[NTH / 64][2];
    __shared__ int s_unit;
    const int t = threadIdx.x;
    V2* slot = reinterpret_cast<V2*>(a.scratch) + (uint64_t)blockIdx.x * a.scratch_elems;

    for (;;) {
        if (t == 0) s_unit = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int u = s_unit;
        __syncthreads();
        if (u >= a.nunits) break;  // every wave of the workgroup sees the same u
        const BatchInst in = a.inst[a.unit_inst[u]];
        const double gam = a.gammas[a.unit_gam[u]];
        const int n = in.n;
        const double amp0 = exp2(-0.5 * n);
        const double* E = a.etab + in.eoff;
        const uint16_t* X = a.eidx + in.eoff;
        const bool intE = in.lut_n > 0;
        const int xmin = intE ? (int)in.emin - in.lut_lo : 0;  // table index of the ground energy
        if (intE) {
            for (int m = t; m < in.lut_n; m += NTH) {
                double sn, cs;
                sincos(gam * (double)(in.lut_lo + m), &sn, &cs);
                lut[m].x = (Real)(amp0 * cs);
                lut[m].y = (Real)(-amp0 * sn);
            }
            __syncthreads();
        }
        // phase state 2^{-n/2} exp(-i gamma E(z)) for U consecutive-stride entries z0 + j NTH
        auto phi_block = [&](uint64_t base, uint32_t z0, uint32_t lim, V2 (&out)[U]) {
            if (intE) {
                uint16_t x[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const uint32_t z = z0 + j * NTH;
                    x[j] = z < lim ? X[base + z] : (uint16_t)0;
                }
#pragma unroll
                for (int j = 0; j < U; j++) out[j] = lut[x[j]];
            } else {
                double e[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const uint32_t z = z0 + j * NTH;
                    e[j] = z < lim ? E[base + z] : 0.0;
                }
                // one sincos at a time (each needs many temporaries)
#pragma unroll 1
                for (int j = 0; j < U; j++) {
                    double sn, cs;
                    sincos(gam * e[j], &sn, &cs);
                    out[j].x = (Real)(amp0 * cs);
                    out[j].y = (Real)(-amp0 * sn);
                }
            }
        };
        // <H_C> and P_gs terms of U entries
        // (amplitude j sits at index z0 + j NTH; its energy is that of index (z0 + j NTH) ^ fl)
        auto obs_block = [&](uint64_t base, uint32_t z0, uint32_t lim, uint32_t fl, const V2 (&v)[U], double& r_e,
                             double& r_p) {
            if (intE) {
                uint16_t x[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const uint32_t z = z0 + j * NTH;
                    x[j] = z < lim ? X[base + (z ^ fl)] : (uint16_t)0;
                }
#pragma unroll
                for (int j = 0; j < U; j++) {
                    if (z0 + j * NTH >= lim) continue;
                    const double p2 = (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
                    r_e += (double)(in.lut_lo + (int)x[j]) * p2;
                    if ((int)x[j] == xmin) r_p += p2;
                }
            } else {
                double e[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const uint32_t z = z0 + j * NTH;
                    e[j] = z < lim ? E[base + (z ^ fl)] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < U; j++) {
                    if (z0 + j * NTH >= lim) continue;
                    const double p2 = (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
                    r_e += e[j] * p2;
                    if (fabs(e[j] - in.emin) <= in.etol) r_p += p2;
                }
            }
        };
        for (int b = 0; b < a.nb; b++) {
            // beta -> beta + pi multiplies the state by (-1)^n, and beta -> beta + pi/2
            // applies -i sigma^x to every qubit, which moves the amplitude of z to the
            // complement of z.  So beta is reduced to |beta| <= pi/4, the mixers run in
            // the tangent form (|tan| <= 1), the tables are read at z ^ fl, and the sums
            // take the factor cos(beta)^{2n} at the end.
            double bb = remainder(a.betas[b], M_PI);
            uint32_t fl = 0u;
            if (fabs(bb) > 0.25 * M_PI) {
                bb -= copysign(0.5 * M_PI, bb);
                fl = (uint32_t)((1ull << n) - 1ull);
            }
            const Real tq = (Real)tan(bb);
            double r_e = 0.0, r_p = 0.0;
            if (n <= S) {
                const uint32_t N = 1u << n;
                for (uint32_t z0 = t; z0 < N; z0 += NTH * U) {
                    V2 v[U];
                    phi_block(0, z0, N, v);
#pragma unroll
                    for (int j = 0; j < U; j++)
                        if (z0 + j * NTH < N) st[bswz(z0 + j * NTH, G)] = v[j];
                }
                __syncthreads();
                if (n >= 5) {
                    lds_mixer<Real, NTH>(st, n, tq);
                } else {
                    if (t == 0) {  // tiny states: plain pair loops
                        for (int q = 0; q < n; q++)
                            for (uint32_t z = 0; z < N; z++) {
                                if ((z >> q) & 1u) continue;
                                V2& x = st[bswz(z, G)];
                                V2& y = st[bswz(z | (1u << q), G)];
                                const Real ar = x.x, ai = x.y, br = y.x, bi = y.y;
                                x.x = ar + tq * bi;
                                x.y = ai - tq * br;
                                y.x = br + tq * ai;
                                y.y = bi - tq * ar;
                            }
                    }
                    __syncthreads();
                }
                for (uint32_t z0 = t; z0 < N; z0 += NTH * U) {
                    V2 v[U];
#pragma unroll
                    for (int j = 0; j < U; j++) {
                        const uint32_t z = z0 + j * NTH;
                        if (z < N) v[j] = st[bswz(z, G)];
                        else v[j].x = v[j].y = (Real)0;
                    }
                    obs_block(0, z0, N, fl, v, r_e, r_p);
                }
            } else if constexpr (SLOTS) {
                // low S bits slice by slice, written to this workgroup's slot: bits
                // S-5..S-1 in registers as the phases are formed, bits 0..4 in LDS,
                // bits 5..S-6 on the way from LDS to the slot
                const int nh = n - S;
                constexpr int LB = S - 5;
                constexpr int MB = S - 10;
                for (uint32_t sl = 0; sl < (1u << nh); sl++) {
                    const uint64_t off = (uint64_t)sl << S;
                    if (!intE) {
                        for (uint32_t z0 = t; z0 < (1u << S); z0 += NTH * U) {
                            V2 v[U];
                            phi_block(off, z0, 1u << S, v);
#pragma unroll
                            for (int j = 0; j < U; j++) st[bswz(z0 + j * NTH, G)] = v[j];
                        }
                        __syncthreads();
                    }
                    const uint16_t* Xs = X + off;  // uniform bases, 32-bit lane offsets
                    V2* Ss = slot + off;
                    for (uint32_t l = t; l < (1u << LB); l += NTH) {
                        const uint32_t bl = opaque(bswz(l, G));
                        V2 v[32];
                        if (intE) {
                            uint16_t x[32];
#pragma unroll
                            for (int r = 0; r < 32; r++) x[r] = Xs[l | ((uint32_t)r << LB)];
#pragma unroll
                            for (int r = 0; r < 32; r++) v[r] = lut[x[r]];
                        } else {
#pragma unroll
                            for (int r = 0; r < 32; r++) v[r] = st[bl ^ bswz((uint32_t)r << LB, G)];
                        }
                        reg_mix<Real, 5>(v, tq);
#pragma unroll
                        for (int r = 0; r < 32; r++) st[bl ^ bswz((uint32_t)r << LB, G)] = v[r];
                    }
                    __syncthreads();
                    for (uint32_t q = t; q < (1u << LB); q += NTH) {
                        const uint32_t bq = opaque(bswz(q << 5, G));
                        V2 v[32];
#pragma unroll
                        for (int r = 0; r < 32; r++) v[r] = st[bq ^ bswz((uint32_t)r, G)];
                        reg_mix<Real, 5>(v, tq);
#pragma unroll
                        for (int r = 0; r < 32; r++) st[bq ^ bswz((uint32_t)r, G)] = v[r];
                    }
                    __syncthreads();
                    for (uint32_t g = t; g < (1u << (S - MB)); g += NTH) {
                        const uint32_t zb = (g & 31u) | ((g >> 5) << (5 + MB));
                        const uint32_t bz = opaque(bswz(zb, G));
                        V2 v[1 << MB];
#pragma unroll
                        for (int r = 0; r < (1 << MB); r++) v[r] = st[bz ^ bswz((uint32_t)r << 5, G)];
                        reg_mix<Real, MB>(v, tq);
#pragma unroll
                        for (int r = 0; r < (1 << MB); r++) Ss[zb | ((uint32_t)r << 5)] = v[r];
                    }
                    __syncthreads();
                }
                // high bits: each thread holds the 2^nh amplitudes of one low index
                for (uint32_t l0 = t; l0 < (1u << S); l0 += NTH) {
                    const uint32_t l = opaque(l0);
                    V2 v[32];
#pragma unroll
                    for (int r = 0; r < 32; r++)
                        if (r < (1 << nh)) v[r] = slot[((uint32_t)r << S) | l];
#pragma unroll
                    for (int k = 0; k < 5; k++) {
                        if (k >= nh) continue;
#pragma unroll
                        for (int r = 0; r < 32; r++) {
                            if ((r & (1 << k)) || r >= (1 << nh)) continue;
                            const int r2 = r | (1 << k);
                            const Real ar = v[r].x, ai = v[r].y, br = v[r2].x, bi = v[r2].y;
                            v[r].x = ar + tq * bi;
                            v[r].y = ai - tq * br;
                            v[r2].x = br + tq * ai;
                            v[r2].y = bi - tq * ar;
                        }
                    }
                    if (intE) {
#pragma unroll
                        for (int r0 = 0; r0 < 32; r0 += U) {
                            uint16_t x[U];
#pragma unroll
                            for (int j = 0; j < U; j++)
                                x[j] = r0 + j < (1 << nh) ? X[(((uint32_t)(r0 + j) << S) | l) ^ fl] : (uint16_t)0;
#pragma unroll
                            for (int j = 0; j < U; j++) {
                                const int r = r0 + j;
                                if (r >= (1 << nh)) continue;
                                const double p2 = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
                                r_e += (double)(in.lut_lo + (int)x[j]) * p2;
                                if ((int)x[j] == xmin) r_p += p2;
                            }
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < 32; r++) {
                            if (r >= (1 << nh)) continue;
                            const double p2 = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
                            const double e = E[(((uint32_t)r << S) | l) ^ fl];
                            r_e += e * p2;
                            if (fabs(e - in.emin) <= in.etol) r_p += p2;
                        }
                    }
                }
                __syncthreads();  // slot reads done before the next beta overwrites it
            }
            // fixed-order workgroup sum
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                r_e += __shfl_xor(r_e, off);
                r_p += __shfl_xor(r_p, off);
            }
            if ((t & 63) == 0) {
                red[t >> 6][0] = r_e;
                red[t >> 6][1] = r_p;
            }
            __syncthreads();
            if (t == 0) {
                double se = 0.0, sp = 0.0;
                for (int w = 0; w < NTH / 64; w++) {
                    se += red[w][0];
                    sp += red[w][1];
                }
                const double cb = cos(bb), sc = pow(cb * cb, (double)n);  // the deferred cos(beta)^{2n}
                const uint64_t o = ((uint64_t)a.unit_inst[u] * a.ng + a.unit_gam[u]) * a.nb + b;
                a.out_e[o] = se * sc;
                a.out_p[o] = sp * sc;
            }
            __syncthreads();
        }
    }
}

int launch_batch_energy(const BatchArgs& a, int max_n, void* stream) {
    const unsigned gx = (unsigned)std::max(1, std::min(1024, (1 << max_n) / 256));
    hipLaunchKernelGGL(k_batch_energy, dim3(gx, a.ninst), dim3(256), 0, (hipStream_t)stream, a);
    int e = (int)hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_batch_emin, dim3(a.ninst), dim3(256), 0, (hipStream_t)stream, a,
                       const_cast<BatchInst*>(a.inst));
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------- sliced states
// States larger than the LDS tile (n > S) go through a slab of a few hundred MB
// that stays in the last-level cache between two kernels, instead of a
// per-workgroup slot of 2^n amplitudes that streams through HBM:
//   k_batch_slices  one workgroup per (state, slice of 2^S amplitudes): phase
//                   state of the slice, mixer on the low S bits, slice -> slab;
//   k_batch_columns one workgroup per (state, block of 2^S amplitudes taken as
//                   2^(S - nh) columns of the 2^nh high-bit values): mixer on
//                   the high bits, <H_C> and P_gs partial sums;
//   k_batch_finish  one thread per state: its partials in a fixed order, times
//                   the deferred cos(beta)^{2n}.
// Mixer in the tangent form on |beta| <= pi/4 as in k_batch_scan; fl flips the
// table index where beta was moved by pi/2.
__device__ __forceinline__ double batch_reduce_beta(double beta, int n, uint32_t& fl) {
    double bb = remainder(beta, M_PI);
    fl = 0u;
    if (fabs(bb) > 0.25 * M_PI) {
        bb -= copysign(0.5 * M_PI, bb);
        fl = (uint32_t)((1ull << n) - 1ull);
    }
    return bb;
}

// <H_C> and P_gs of state s of a launch (qubits n, first unit u0, first group
// state base): its 2^nh partial sums in a fixed order, times cos(beta)^{2n}.
__device__ void batch_finish_state(const BatchArgs& a, int nh, int n, int u0, int64_t base, const double* part,
                                   int s) {
    const int64_t g = base + s;
    const int u = u0 + (int)(g / a.nb);
    const int b = (int)(g % a.nb);
    uint32_t fl;
    const double bb = batch_reduce_beta(a.betas[b], n, fl);
    double se = 0.0, sp = 0.0;
    const double* P = part + ((uint64_t)s << nh) * 2;
    for (int k = 0; k < (1 << nh); k++) {
        se += P[2 * k];
        sp += P[2 * k + 1];
    }
    const double cb = cos(bb), sc = pow(cb * cb, (double)n);  // the deferred cos(beta)^{2n}
    const uint64_t o = ((uint64_t)a.unit_inst[u] * a.ng + a.unit_gam[u]) * a.nb + b;
    a.out_e[o] = se * sc;
    a.out_p[o] = sp * sc;
}

// B: bits of a register block (5: 2^13 slices in rounds of 5, 5 and 3 bits; 4: 2^12
// slices in three rounds of 4 bits)
template <typename Real, int NTH, int S, int LUTN, int MINW, int B = 5>
__global__ void __launch_bounds__(NTH, MINW) k_batch_slices(const BatchArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int G = BatchCfg<Real>::G;
    constexpr int U = kBatchUnroll;
    constexpr int NB = 1 << B;
    constexpr int LB = S - B;
    constexpr int MB = S - 2 * B;
    static_assert(MB >= 1 && MB <= B, "slice rounds assume B < S - B <= 2 B");
    static_assert((1 << S) % (NTH * kBatchUnroll) == 0, "phase loop assumes whole blocks");
    __shared__ V2 st[1 << S];
    __shared__ V2 lut[LUTN];  // 2^{-n/2} exp(-i gamma E), rounded once to the storage type
    const int t = threadIdx.x;
    const int n = a.s_n;
    const int nh = n - S;
    const uint32_t nsl = (uint32_t)a.s_count << nh;
    if (blockIdx.x >= nsl) {  // trailing workgroups: the previous launch's states
        const int fs = (int)(blockIdx.x - nsl) * NTH + t;
        if (fs < a.f_count) batch_finish_state(a, a.f_nh, a.f_n, a.f_u0, a.f_base, a.f_part, fs);
        return;
    }
    const uint32_t s = blockIdx.x >> nh;
    const uint32_t sl = blockIdx.x & ((1u << nh) - 1u);
    const int64_t g = a.s_base + s;
    const int u = a.s_u0 + (int)(g / a.nb);
    const int b = (int)(g % a.nb);
    const BatchInst in = a.inst[a.unit_inst[u]];
    const double gam = a.gammas[a.unit_gam[u]];
    const double amp0 = exp2(-0.5 * n);
    const bool intE = in.lut_n > 0;
    uint32_t fl;
    const Real tq = (Real)tan(batch_reduce_beta(a.betas[b], n, fl));
    const uint64_t off = in.eoff + ((uint64_t)sl << S);
    V2* __restrict__ Ss = reinterpret_cast<V2*>(a.slab) + ((uint64_t)s << n) + ((uint64_t)sl << S);
    if (intE) {
        for (int m = t; m < in.lut_n; m += NTH) {
            double sn, cs;
            sincos(gam * (double)(in.lut_lo + m), &sn, &cs);
            lut[m].x = (Real)(amp0 * cs);
            lut[m].y = (Real)(-amp0 * sn);
        }
    } else {
        const double* E = a.etab + off;
        for (uint32_t z0 = t; z0 < (1u << S); z0 += NTH * U) {
            double e[U];
#pragma unroll
            for (int j = 0; j < U; j++) e[j] = E[z0 + j * NTH];
#pragma unroll 1
            for (int j = 0; j < U; j++) {
                double sn, cs;
                sincos(gam * e[j], &sn, &cs);
                V2 v;
                v.x = (Real)(amp0 * cs);
                v.y = (Real)(-amp0 * sn);
                st[bswz(z0 + j * NTH, G)] = v;
            }
        }
    }
    __syncthreads();
    // bits S-B..S-1 in registers as the phases are formed
    const uint16_t* Xs = a.eidx + off;
    for (uint32_t l = t; l < (1u << LB); l += NTH) {
        const uint32_t bl = opaque(bswz(l, G));
        V2 v[NB];
        if (intE) {
            uint16_t x[NB];
#pragma unroll
            for (int r = 0; r < NB; r++) x[r] = Xs[l | ((uint32_t)r << LB)];
#pragma unroll
            for (int r = 0; r < NB; r++) v[r] = lut[x[r]];
        } else {
#pragma unroll
            for (int r = 0; r < NB; r++) v[r] = st[bl ^ bswz((uint32_t)r << LB, G)];
        }
        reg_mix<Real, B>(v, tq);
#pragma unroll
        for (int r = 0; r < NB; r++) st[bl ^ bswz((uint32_t)r << LB, G)] = v[r];
    }
    __syncthreads();
    // bits 0..B-1
    for (uint32_t q = t; q < (1u << LB); q += NTH) {
        const uint32_t bq = opaque(bswz(q << B, G));
        V2 v[NB];
#pragma unroll
        for (int r = 0; r < NB; r++) v[r] = st[bq ^ bswz((uint32_t)r, G)];
        reg_mix<Real, B>(v, tq);
#pragma unroll
        for (int r = 0; r < NB; r++) st[bq ^ bswz((uint32_t)r, G)] = v[r];
    }
    __syncthreads();
    // bits B..S-B-1 on the way from LDS to the slab
    for (uint32_t gq = t; gq < (1u << (S - MB)); gq += NTH) {
        const uint32_t zb = (gq & (NB - 1u)) | ((gq >> B) << (B + MB));
        const uint32_t bz = opaque(bswz(zb, G));
        V2 v[1 << MB];
#pragma unroll
        for (int r = 0; r < (1 << MB); r++) v[r] = st[bz ^ bswz((uint32_t)r << B, G)];
        reg_mix<Real, MB>(v, tq);
#pragma unroll
        for (int r = 0; r < (1 << MB); r++) Ss[zb | ((uint32_t)r << B)] = v[r];
    }
}

template <typename Real, int NTH, int S, int NH>
__global__ void __launch_bounds__(NTH) k_batch_columns(const BatchArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int U = kBatchUnroll;
    constexpr int NV = 1 << NH;  // high-bit values of one column
    __shared__ double red[NTH / 64][2];
    const int t = threadIdx.x;
    const int n = S + NH;
    const uint32_t s = blockIdx.x >> NH;
    const uint32_t cb = blockIdx.x & (NV - 1u);
    const int64_t g = a.s_base + s;
    const int u = a.s_u0 + (int)(g / a.nb);
    const int b = (int)(g % a.nb);
    const BatchInst in = a.inst[a.unit_inst[u]];
    const bool intE = in.lut_n > 0;
    const int xmin = intE ? (int)in.emin - in.lut_lo : 0;  // table index of the ground energy
    uint32_t fl;
    const Real tq = (Real)tan(batch_reduce_beta(a.betas[b], n, fl));
    const V2* __restrict__ Sv = reinterpret_cast<const V2*>(a.slab) + ((uint64_t)s << n);
    const uint16_t* X = a.eidx + in.eoff;
    const double* E = a.etab + in.eoff;
    constexpr uint32_t ncol = 1u << (S - NH);  // columns of this workgroup
    const uint32_t c0 = cb << (S - NH);
    double r_e = 0.0, r_p = 0.0;
    for (uint32_t lc = t; lc < ncol; lc += NTH) {
        const uint32_t l = opaque(c0 + lc);
        V2 v[NV];
#pragma unroll
        for (int r = 0; r < NV; r++) v[r] = Sv[((uint32_t)r << S) | l];
        reg_mix<Real, NH>(v, tq);
        if (intE) {
#pragma unroll
            for (int r0 = 0; r0 < NV; r0 += U) {
                constexpr int W = NV < U ? NV : U;
                uint16_t x[W];
#pragma unroll
                for (int j = 0; j < W; j++) x[j] = X[(((uint32_t)(r0 + j) << S) | l) ^ fl];
#pragma unroll
                for (int j = 0; j < W; j++) {
                    const int r = r0 + j;
                    const double p2 = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
                    r_e += (double)(in.lut_lo + (int)x[j]) * p2;
                    if ((int)x[j] == xmin) r_p += p2;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < NV; r++) {
                const double p2 = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
                const double e = E[(((uint32_t)r << S) | l) ^ fl];
                r_e += e * p2;
                if (fabs(e - in.emin) <= in.etol) r_p += p2;
            }
        }
    }
    // fixed-order workgroup sum
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r_e += __shfl_xor(r_e, o);
        r_p += __shfl_xor(r_p, o);
    }
    if ((t & 63) == 0) {
        red[t >> 6][0] = r_e;
        red[t >> 6][1] = r_p;
    }
    __syncthreads();
    if (t == 0) {
        double se = 0.0, sp = 0.0;
        for (int w = 0; w < NTH / 64; w++) {
            se += red[w][0];
            sp += red[w][1];
        }
        a.part[2 * (uint64_t)blockIdx.x] = se;
        a.part[2 * (uint64_t)blockIdx.x + 1] = sp;
    }
}

// Six high bits (64 values per column): each column is held by a lane pair, 32
// values per lane; row bits 0-4 in registers, row bit 5 across the pair (both
// members take x <- x - i t x_partner).
template <typename Real, int S>
__global__ void __launch_bounds__(128) k_batch_columns_pair(const BatchArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int U = kBatchUnroll;
    constexpr int NH = 6;
    constexpr int NTH = 128;
    static_assert(S - NH == 6, "a block of 64 columns per 128 threads");
    __shared__ double red[NTH / 64][2];
    const int t = threadIdx.x;
    const int n = S + NH;
    const uint32_t s = blockIdx.x >> NH;
    const uint32_t cb = blockIdx.x & ((1u << NH) - 1u);
    const int64_t g = a.s_base + s;
    const int u = a.s_u0 + (int)(g / a.nb);
    const int b = (int)(g % a.nb);
    const BatchInst in = a.inst[a.unit_inst[u]];
    const bool intE = in.lut_n > 0;
    const int xmin = intE ? (int)in.emin - in.lut_lo : 0;  // table index of the ground energy
    uint32_t fl;
    const Real tq = (Real)tan(batch_reduce_beta(a.betas[b], n, fl));
    const V2* __restrict__ Sv = reinterpret_cast<const V2*>(a.slab) + ((uint64_t)s << n);
    const uint16_t* X = a.eidx + in.eoff;
    const double* E = a.etab + in.eoff;
    const uint32_t h = (uint32_t)t & 1u;  // upper or lower 32 rows
    const uint32_t l = opaque((cb << (S - NH)) + ((uint32_t)t >> 1));
    const uint32_t r0 = h << 5;
    V2 v[32];
#pragma unroll
    for (int j = 0; j < 32; j++) v[j] = Sv[((r0 + (uint32_t)j) << S) | l];
    reg_mix<Real, 5>(v, tq);
#pragma unroll
    for (int j = 0; j < 32; j++) {
        const Real pr = __shfl_xor(v[j].x, 1), pi = __shfl_xor(v[j].y, 1);
        v[j].x = fma(tq, pi, v[j].x);
        v[j].y = fma(-tq, pr, v[j].y);
    }
    double r_e = 0.0, r_p = 0.0;
    if (intE) {
#pragma unroll
        for (int j0 = 0; j0 < 32; j0 += U) {
            uint16_t x[U];
#pragma unroll
            for (int j = 0; j < U; j++) x[j] = X[(((r0 + (uint32_t)(j0 + j)) << S) | l) ^ fl];
#pragma unroll
            for (int j = 0; j < U; j++) {
                const V2 w = v[j0 + j];
                const double p2 = (double)w.x * w.x + (double)w.y * w.y;
                r_e += (double)(in.lut_lo + (int)x[j]) * p2;
                if ((int)x[j] == xmin) r_p += p2;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 32; j++) {
            const double p2 = (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
            const double e = E[(((r0 + (uint32_t)j) << S) | l) ^ fl];
            r_e += e * p2;
            if (fabs(e - in.emin) <= in.etol) r_p += p2;
        }
    }
    // fixed-order workgroup sum
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r_e += __shfl_xor(r_e, o);
        r_p += __shfl_xor(r_p, o);
    }
    if ((t & 63) == 0) {
        red[t >> 6][0] = r_e;
        red[t >> 6][1] = r_p;
    }
    __syncthreads();
    if (t == 0) {
        a.part[2 * (uint64_t)blockIdx.x] = red[0][0] + red[1][0];
        a.part[2 * (uint64_t)blockIdx.x + 1] = red[0][1] + red[1][1];
    }
}

template <typename Real, int S>
static int launch_batch_columns(const BatchArgs& a, unsigned grid, hipStream_t st) {
    switch (a.s_n - S) {
        case 1: hipLaunchKernelGGL((k_batch_columns<Real, 256, S, 1>), dim3(grid), dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_batch_columns<Real, 256, S, 2>), dim3(grid), dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_batch_columns<Real, 256, S, 3>), dim3(grid), dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_batch_columns<Real, 256, S, 4>), dim3(grid), dim3(256), 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_batch_columns<Real, 256, S, 5>), dim3(grid), dim3(256), 0, st, a); break;
        case 6:
            if constexpr (S == 12) {
                hipLaunchKernelGGL((k_batch_columns_pair<Real, S>), dim3(grid), dim3(128), 0, st, a);
                break;
            }
            return (int)hipErrorInvalidValue;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

__global__ void __launch_bounds__(256) k_batch_finish(const BatchArgs a) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < a.f_count) batch_finish_state(a, a.f_nh, a.f_n, a.f_u0, a.f_base, a.f_part, s);
}

// Slice bits of the sliced path: complex128 states in 2^12-amplitude slices (72 KiB of
// LDS, two workgroups per CU; the column kernels then hold 2 to 6 high bits), complex64
// ones in 2^13 slices.
int batch_slice_bits(int dtype, int) { return dtype == 2 ? 12 : 13; }

int launch_batch_sliced(int dtype, const BatchArgs& a, int wide, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int S = batch_slice_bits(dtype, a.s_n);
    if (batch_lds_bits(dtype, wide) != 13 || a.s_n <= 13 || a.s_n > S + (S == 12 ? 6 : 5) || a.s_count < 1)
        return (int)hipErrorInvalidValue;
    const unsigned grid = (unsigned)a.s_count << (a.s_n - S);
    const unsigned fin = a.f_count > 0 ? (unsigned)((a.f_count + 255) / 256) : 0u;  // 256-thread workgroups
    if (dtype == 2)
        hipLaunchKernelGGL((k_batch_slices<double, 256, 12, 512, 2, 4>), dim3(grid + fin), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_batch_slices<float, 256, 13, 1024, 2>), dim3(grid + fin), dim3(256), 0, st, a);
    int e = (int)hipGetLastError();
    if (e) return e;
    return dtype == 2 ? launch_batch_columns<double, 12>(a, grid, st) : launch_batch_columns<float, 13>(a, grid, st);
}

int launch_batch_finish(const BatchArgs& a, void* stream) {
    if (a.f_count < 1) return 0;
    hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)((a.f_count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       a);
    return (int)hipGetLastError();
}

// Variants: complex128 2^13-amplitude LDS states, four waves (wide = 0) or eight (wide = 1);
// complex64 2^14 states with eight
// waves (wide = 1) or four (wide = 0), one workgroup per CU; complex64 2^13 states with four
// waves (wide = 2), two workgroups per CU.  Phase tables hold 1024 entries.
int batch_lds_bits(int dtype, int wide) { return dtype == 2 ? 13 : (wide == 2 ? 13 : 14); }
int batch_lut_cap(int dtype, int) { return dtype == 2 ? 512 : 1024; }  // complex128: the 2^12-slice kernel's table

int launch_batch_scan(int dtype, const BatchArgs& a, int grid, int wide, void* stream) {
    if (a.scratch_elems == 0 && ((dtype == 2 && wide == 1) || (dtype != 2 && wide == 2))) {  // LDS-resident units only
        if (dtype == 2)
            hipLaunchKernelGGL((k_batch_scan<double, 512, 13, 1024, 1, false>), dim3(grid), dim3(512), 0,
                               (hipStream_t)stream, a);
        else
            hipLaunchKernelGGL((k_batch_scan<float, 256, 13, 1024, 2, false>), dim3(grid), dim3(256), 0,
                               (hipStream_t)stream, a);
        return (int)hipGetLastError();
    }
    if (dtype == 2 && wide == 1)
        hipLaunchKernelGGL((k_batch_scan<double, 512, 13, 1024>), dim3(grid), dim3(512), 0, (hipStream_t)stream, a);
    else if (dtype == 2)
        hipLaunchKernelGGL((k_batch_scan<double, 256, 13, 1024>), dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    else if (wide == 1)
        hipLaunchKernelGGL((k_batch_scan<float, 512, 14, 1024>), dim3(grid), dim3(512), 0, (hipStream_t)stream, a);
    else if (wide == 2)
        hipLaunchKernelGGL((k_batch_scan<float, 256, 13, 1024, 2>), dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((k_batch_scan<float, 256, 14, 1024>), dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

}  // namespace svk
