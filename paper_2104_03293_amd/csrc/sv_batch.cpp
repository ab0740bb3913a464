// libsv host: the batched p = 1 landscape scan (sv_batch_p1_scan).
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
            part_doubles = std::max(part_doubles, (size_t)states_per_launch(n) * 2 << (n - batch_slice_bits((int)dtype, n)));
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
                bs.f_nh = prev.s_count > 0 ? prev.s_n - batch_slice_bits((int)dtype, prev.s_n) : 0;
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

