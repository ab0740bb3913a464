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

__device__ __forceinline__ double spin_u(uint32_t u, int l) { return ((u >> l) & 1u) ? 1.0 : -1.0; }
__device__ __forceinline__ double spin_z(uint64_t z, int i) { return ((z >> i) & 1ull) ? 1.0 : -1.0; }

__device__ __forceinline__ uint32_t thread_index_bits(uint32_t t, const GeoLayout* L) {
    uint32_t u = 0;
    const int nt = L->ntb;
    for (int j = 0; j < nt; j++) u |= ((t >> j) & 1u) << L->tb[j];
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

// Per-workgroup part of E(z): E_fixed (fields and couplings among bits outside
// the tile) and g_l = h_{P[l]} + sum of couplings from tile bit l to fixed bits.
// Wave 0 only; deterministic order.
__device__ void tile_fields(const IsingDev& is, const GeoBuf* geo, const TileGeom& tg, uint64_t base,
                            int T, double* s_g, double* s_ew) {
    const int lane = threadIdx.x;
    if (is.h == nullptr) {  // mixer-only passes carry no instance
        if (lane == 0) *s_ew = 0.0;
        if (lane < T) s_g[lane] = 0.0;
        return;
    }
    double part = 0.0;
    for (int i = lane; i < is.n; i += 64)
        if (!tg.in_tile(i)) part += is.h[i] * spin_z(base, i);
    for (int k = lane; k < is.m; k += 64) {
        const int i = is.ei[k], j = is.ej[k];
        if (!tg.in_tile(i) && !tg.in_tile(j)) part += is.J[k] * spin_z(base, i) * spin_z(base, j);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) *s_ew = part;
    if (lane < T) {
        const int P = geo->P[lane];
        double gv = 0.0;
        if (P >= 0) {
            gv = is.h[P];
            for (int q = is.adj_ptr[P]; q < is.adj_ptr[P + 1]; q++) {
                const int j = is.adj_nbr[q];
                if (!tg.in_tile(j)) gv += is.adj_J[q] * spin_z(base, j);
            }
        }
        s_g[lane] = gv;
    }
}

// Thread part of E for layout L: returns e0 = E at register index 0 and the
// register-bit fields f[k], so that E(r) = e0 + sum_{k: r_k = 1} 2 f[k] + Q[r].
template <int R>
__device__ __forceinline__ double thread_energy(const GeoLayout* L, uint32_t thr_u, const double* s_g,
                                                double ew, double (&f)[R]) {
    double eth = ew;
    const int nt = L->ntb;
    for (int j = 0; j < nt; j++) {
        const int l = L->tb[j];
        eth += s_g[l] * spin_u(thr_u, l);
    }
    const int ntt = L->n_tt;
    for (int q = 0; q < ntt; q++) eth += L->tt_J[q] * spin_u(thr_u, L->tt_a[q]) * spin_u(thr_u, L->tt_b[q]);
#pragma unroll
    for (int k = 0; k < R; k++) {
        double fv = s_g[L->rb[k]];
        const int ntr = L->n_tr[k];
        for (int q = 0; q < ntr; q++) fv += L->tr_J[k][q] * spin_u(thr_u, L->tr_l[k][q]);
        f[k] = fv;
        eth -= fv;
    }
    return eth;
}

__device__ __forceinline__ void slot_add(double* acc, int slot, double v) {
#pragma unroll
    for (int s = 0; s < kMaxSlots; s++)
        if (s == slot) acc[s] += v;
}

__device__ __forceinline__ double2 cmul(double2 x, double2 y) {
    return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

template <typename Real, int T, int R, int NV>
__global__ void __launch_bounds__(1 << (T - R)) k_pass(const PassArgs a) {
    using V2 = typename V2T<Real>::type;
    constexpr int NT = 1 << (T - R);
    constexpr int NR = 1 << R;
    constexpr int NW = NT / 64;
    constexpr int G = (sizeof(Real) == 8) ? 3 : 4;
    constexpr int RLO = (R + 1) / 2;
    constexpr int RHI = R - RLO;

    __shared__ V2 xbuf[1 << T];
    __shared__ double s_g[kMaxT];
    __shared__ double s_ew;
    __shared__ double2 s_qph[kMaxPhase][NR];
    __shared__ double s_red[NW][kMaxSlots];

    const uint32_t t = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    const GeoBuf* __restrict__ geo = a.geo;
    const TileGeom tg{a.c, a.lo, a.g};
    const uint64_t base = tg.base(tile);
    V2* __restrict__ psi = reinterpret_cast<V2*>(a.psi);
    V2* __restrict__ lam = reinterpret_cast<V2*>(a.lam);

    // ---- prologue: tile fields and phase tables of the couplings among register bits
    if (t < 64) tile_fields(a.is, geo, tg, base, T, s_g, &s_ew);
    for (int idx = t; idx < a.nphase * NR; idx += NT) {
        const int q = idx / NR, r = idx % NR;
        const double th = a.phase_gamma[q] * geo->L[a.phase_layout[q]].Q[r];
        double sn, cs;
        sincos(th, &sn, &cs);
        s_qph[q][r] = make_double2(cs, -sn);
    }

    // ---- load in layout 0
    int cur = 0;
    const GeoLayout* L = &geo->L[0];
    uint32_t thr_u = thread_index_bits(t, L);
    uint64_t thr_goff = tg.gmap(thr_u);

    Real vr[NV][NR], vi[NV][NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const uint32_t u = thr_u | L->reg_u[r];
        const bool valid = (u & a.phantom) == 0u;
        const uint64_t z = base | thr_goff | L->reg_goff[r];
        Real xr = 0, xi = 0;
        if (valid) {
            if (a.load & 4) {
                xr = (Real)a.amp0;
            } else if (a.load & 1) {
                const V2 v = psi[z];
                xr = v.x;
                xi = v.y;
            }
        }
        vr[0][r] = xr;
        vi[0][r] = xi;
        if constexpr (NV == 2) {
            Real yr = 0, yi = 0;
            if (valid && (a.load & 2)) {
                const V2 v = lam[z];
                yr = v.x;
                yi = v.y;
            }
            vr[1][r] = yr;
            vi[1][r] = yi;
        }
    }

    double acc[kMaxSlots];
#pragma unroll
    for (int s = 0; s < kMaxSlots; s++) acc[s] = 0.0;

    __syncthreads();  // s_g, s_ew, s_qph ready

    for (int oi = 0; oi < a.nops; oi++) {
        const Op op = a.ops[oi];
        if (op.kind == OP_MIX) {
            const int K = a.nlayouts;
            const bool fwd = (cur == 0);
            const Real c = (Real)op.a, s = (Real)op.b;
            for (int step = 0; step < K; step++) {
                const int j = fwd ? step : (K - 1 - step);
                if (j != cur) {
                    // LDS exchange cur -> j, one vector at a time
                    const GeoLayout* Lt = &geo->L[j];
                    const uint32_t new_u = thread_index_bits(t, Lt);
                    const uint32_t src = lds_swizzle(thr_u, G);
                    const uint32_t dst = lds_swizzle(new_u, G);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        __syncthreads();
#pragma unroll
                        for (int r = 0; r < NR; r++) {
                            V2 x;
                            x.x = vr[v][r];
                            x.y = vi[v][r];
                            xbuf[src ^ L->reg_lds[r]] = x;
                        }
                        __syncthreads();
#pragma unroll
                        for (int r = 0; r < NR; r++) {
                            const V2 x = xbuf[dst ^ Lt->reg_lds[r]];
                            vr[v][r] = x.x;
                            vi[v][r] = x.y;
                        }
                    }
                    cur = j;
                    L = Lt;
                    thr_u = new_u;
                    thr_goff = tg.gmap(thr_u);
                }
                const int act = fwd ? L->act_fwd : L->act_bwd;
                double gb = 0.0;
#pragma unroll
                for (int k = 0; k < R; k++) {
                    if (!(act & (1 << k))) continue;
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        if (r & (1 << k)) continue;
                        const int r2 = r | (1 << k);
                        if constexpr (NV == 2) {
                            if (op.flags & MIX_GBETA) {
                                // Im(conj(lam_a) psi_b) + Im(conj(lam_b) psi_a)
                                gb += (double)vr[1][r] * (double)vi[0][r2] - (double)vi[1][r] * (double)vr[0][r2] +
                                      (double)vr[1][r2] * (double)vi[0][r] - (double)vi[1][r2] * (double)vr[0][r];
                            }
                        }
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            if (!(op.flags & (1 << v))) continue;
                            const Real ar = vr[v][r], ai = vi[v][r];
                            const Real br = vr[v][r2], bi = vi[v][r2];
                            vr[v][r] = c * ar + s * bi;
                            vi[v][r] = c * ai - s * br;
                            vr[v][r2] = c * br + s * ai;
                            vi[v][r2] = c * bi - s * ar;
                        }
                    }
                }
                if constexpr (NV == 2) {
                    if (op.flags & MIX_GBETA) slot_add(acc, op.slot, gb);
                }
            }
        } else {  // OP_POINT
            double f[R];
            const double e0 = thread_energy<R>(L, thr_u, s_g, s_ew, f);
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

            const int fl = op.flags;
            if (fl & (PT_REDUCE | PT_LAM_INIT | PT_GGAMMA)) {
                double r_n = 0.0, r_e = 0.0, r_p = 0.0, r_g = 0.0;
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    const double e = elo[r & ((1 << RLO) - 1)] + ehi[r >> RLO] + L->Q[r];
                    const double pr = (double)vr[0][r], pi = (double)vi[0][r];
                    if (fl & PT_REDUCE) {
                        const double p2 = pr * pr + pi * pi;
                        r_n += p2;
                        r_e += e * p2;
                        if (fabs(e - a.emin) <= a.etol) r_p += p2;
                    }
                    if constexpr (NV == 2) {
                        if (fl & PT_LAM_INIT) {
                            vr[1][r] = (Real)(e * pr);
                            vi[1][r] = (Real)(e * pi);
                        }
                        if (fl & PT_GGAMMA) r_g += e * ((double)vr[1][r] * pi - (double)vi[1][r] * pr);
                    }
                }
                if (fl & PT_REDUCE) {
                    slot_add(acc, op.slot, r_n);
                    slot_add(acc, op.slot + 1, r_e);
                    slot_add(acc, op.slot + 2, r_p);
                }
                if (fl & PT_GGAMMA) slot_add(acc, op.slot2, r_g);
            }
            if (fl & (PT_PHASE_PSI | PT_PHASE_LAM)) {
                const double gam = op.a;
                double2 plo[1 << RLO], phi[1 << RHI];
                {
                    double sn, cs;
                    sincos(gam * e0, &sn, &cs);
                    plo[0] = make_double2(cs, -sn);
                }
#pragma unroll
                for (int k = 0; k < RLO; k++) {
                    double sn, cs;
                    sincos(2.0 * gam * f[k], &sn, &cs);
                    const double2 gk = make_double2(cs, -sn);
#pragma unroll
                    for (int r = 0; r < (1 << k); r++) plo[r | (1 << k)] = cmul(plo[r], gk);
                }
                phi[0] = make_double2(1.0, 0.0);
#pragma unroll
                for (int k = 0; k < RHI; k++) {
                    double sn, cs;
                    sincos(2.0 * gam * f[RLO + k], &sn, &cs);
                    const double2 gk = make_double2(cs, -sn);
#pragma unroll
                    for (int r = 0; r < (1 << k); r++) phi[r | (1 << k)] = cmul(phi[r], gk);
                }
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    const double2 ph = cmul(cmul(plo[r & ((1 << RLO) - 1)], phi[r >> RLO]), s_qph[op.qidx][r]);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        if (!(fl & (v == 0 ? PT_PHASE_PSI : PT_PHASE_LAM))) continue;
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

    // ---- store in the current layout
    if (a.store) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const uint32_t u = thr_u | L->reg_u[r];
            if ((u & a.phantom) != 0u) continue;
            const uint64_t z = base | thr_goff | L->reg_goff[r];
            if (a.store & 1) {
                V2 x;
                x.x = vr[0][r];
                x.y = vi[0][r];
                psi[z] = x;
            }
            if constexpr (NV == 2) {
                if (a.store & 2) {
                    V2 x;
                    x.x = vr[1][r];
                    x.y = vi[1][r];
                    lam[z] = x;
                }
            }
        }
    }

    // ---- per-tile partial sums, fixed order
    if (a.nslots > 0) {
        const int lane = t & 63, w = t >> 6;
#pragma unroll
        for (int s = 0; s < kMaxSlots; s++) {
            double v = acc[s];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) s_red[w][s] = v;
        }
        __syncthreads();
        if ((int)t < a.nslots) {
            double v = 0.0;
            for (int ww = 0; ww < NW; ww++) v += s_red[ww][t];
            a.partials[tile * (uint64_t)a.nslots + t] = v;
        }
    }
}

// Column sums of partials[nrows][nslots] in a fixed order: out[dst[s]] (+)= sum.
struct SlotDst {
    int d[kMaxSlots];
};

__global__ void __launch_bounds__(256) k_reduce_slots(const double* __restrict__ partials, uint64_t nrows,
                                                      int nslots, SlotDst dst, int accumulate,
                                                      double* __restrict__ out) {
    __shared__ double sh[256];
    const int s = blockIdx.x;
    const int t = threadIdx.x;
    double v = 0.0;
    for (uint64_t i = t; i < nrows; i += 256) v += partials[i * nslots + s];
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) {
        const int d = dst.d[s];
        out[d] = accumulate ? out[d] + sh[0] : sh[0];
    }
}

// Brute-force enumeration of E(z) over all basis states, tile by tile in layout 0.
template <int T, int R>
__global__ void __launch_bounds__(1 << (T - R)) k_ground(const GroundArgs a) {
    constexpr int NT = 1 << (T - R);
    constexpr int NR = 1 << R;
    constexpr int NW = NT / 64;
    constexpr int RLO = (R + 1) / 2;
    constexpr int RHI = R - RLO;
    __shared__ double s_g[kMaxT];
    __shared__ double s_ew;
    __shared__ double s_e[NW];
    __shared__ unsigned long long s_c[NW], s_a[NW];

    const uint32_t t = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    const GeoBuf* __restrict__ geo = a.geo;
    const TileGeom tg{a.c, a.lo, a.g};
    const uint64_t base = tg.base(tile);
    if (t < 64) tile_fields(a.is, geo, tg, base, T, s_g, &s_ew);
    __syncthreads();

    const GeoLayout* L = &geo->L[0];
    const uint32_t thr_u = thread_index_bits(t, L);
    const uint64_t thr_goff = tg.gmap(thr_u);
    double f[R];
    const double e0 = thread_energy<R>(L, thr_u, s_g, s_ew, f);
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
Shape shape_for(int dtype, int nv) {
    if (dtype == 2) return nv == 1 ? Shape{13, 5} : Shape{13, 4};
    return Shape{14, 5};
}

template <typename Real, int T, int R, int NV>
static int run_pass(const PassArgs& a, void* stream) {
    hipLaunchKernelGGL((k_pass<Real, T, R, NV>), dim3((unsigned)a.ntiles), dim3(1 << (T - R)), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_pass(int dtype, int nv, const PassArgs& a, void* stream) {
    if (dtype == 2) {
        if (nv == 1) return run_pass<double, 13, 5, 1>(a, stream);
        return run_pass<double, 13, 4, 2>(a, stream);
    }
    if (nv == 1) return run_pass<float, 14, 5, 1>(a, stream);
    return run_pass<float, 14, 5, 2>(a, stream);
}

int launch_reduce_slots(const double* partials, uint64_t nrows, int nslots, const int* dst, int accumulate,
                        double* out, void* stream) {
    SlotDst d;
    for (int s = 0; s < kMaxSlots; s++) d.d[s] = s < nslots ? dst[s] : 0;
    hipLaunchKernelGGL(k_reduce_slots, dim3(nslots), dim3(256), 0, (hipStream_t)stream, partials, nrows, nslots,
                       d, accumulate, out);
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
