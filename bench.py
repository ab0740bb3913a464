"""Benchmark: QAOA layers on one MI355X through the C ABI.

Workload (the one the headline metric is quoted on): p = 4 QAOA layers at
n = 32 qubits, complex128 amplitudes (64 GiB state), on a random Ising instance
G(32, 64) with integer J in [-2, 2] and h in {-1, 0, 1} (seeded), followed by
<H_C> and the ground-state probability.  One step = one energy evaluation of
the QAOA objective, sv_qaoa_energy(p = 4): the forward circuit with the
observables fused into its last pass (the final state is stored).
value = amplitude updates per second = p * 2^n * (n + 1) / t_step
(n butterflies and one phase per amplitude per layer).

Also reported (outside the timed steps): roofline of the dominant kernel
(tile pass) from per-launch HIP events on the launch stream, the complex64
rate, the adjoint gradient time against (2p + 1) forward evaluations, and the
FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--dtype", default="c128")
    ap.add_argument("--no-extras", action="store_true", help="skip gradient / c64 / CPU-baseline legs")
    ap.add_argument("--extras", default="all",
                    help="comma list of extra legs: grad,grad_p8,c64,exact_cover,hadamard,qsds,batch_scan,optimizer,full,cpu "
                         "(default all)")
    ap.add_argument("--cpu-sample-n", type=int, default=28)
    ap.add_argument("--cpu-sample-p", type=int, default=4)
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="set a plan knob of the library before the run (repeatable)")
    ap.add_argument("--tune-cache", default="",
                    help="autotuner cache to load (default: paper_2104_03293_amd/tune_cache.txt if present; "
                         "'none' for the built-in defaults)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (counter reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2104_03293_amd import inputs as I
    from paper_2104_03293_amd import sv

    torch.cuda.set_device(0)
    # the autotuner's choices (committed cache of tune.py), unless another is named
    cache = Path(args.tune_cache) if args.tune_cache else ROOT / "paper_2104_03293_amd" / "tune_cache.txt"
    if args.tune_cache != "none" and cache.exists():
        sv.tune_load(str(cache))
        log(f"[bench] tuned knobs from {cache.name}")
    for kv in args.knob:
        name, val = kv.split("=")
        sv.tune_set(name, int(val))
        log(f"[bench] knob {name}={int(val)}")
    if args.copy_ref_mib > 0:
        nel = args.copy_ref_mib << 18  # float32 elements
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] reference copy of {args.copy_ref_mib} MiB done")
        del src, dst
    n, p = args.n, args.p
    inst = I.full_size_instance(n) if n >= 33 else I.degree4_int2(n, 4 + n)
    H = sv.Ising.from_instance(inst)
    gam, bet = I.linear_ramp_params(p)
    log(f"[bench] n={n} p={p} dtype={args.dtype} ground...")
    emin, deg, _ = sv.ground(H)
    log(f"[bench] ground E_min={emin} degeneracy={deg}")
    s = sv.State(n, args.dtype)
    stream = torch.cuda.current_stream()

    def step():
        return sv.qaoa_energy(s, H, gam, bet)

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    sv.profile_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sv.profile_report()
    sv.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    updates = p * (1 << n) * (n + 1)
    value = updates / (ms * 1e-3)
    log(f"[bench] {ms:.3f} ms/step  {value:.4e} amp-updates/s  <H>={out[0]:.6f} P_gs={out[1]:.3e} norm={out[2]:.12f}")

    # roofline of the tile-pass kernel (the only kernel with non-trivial time)
    kind = f"pass_{args.dtype}_nv1"
    k = prof.get(kind, {"launches": 0, "ms": 0.0, "bytes": 0.0})
    avg_ms = k["ms"] / max(1, k["launches"])
    avg_bytes = k["bytes"] / max(1, k["launches"])
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = committed_traffic(args.dtype, n, p)
    # measured ceilings: the library's streaming kernel (in-place nontemporal read + write of the
    # state, no arithmetic) with the tile shape and tile order of each pass geometry of the plan
    ceil = stream_ceilings(sv, s, n, args.dtype)
    copy_gbs = ceil[f"c{ceil['T']}"]
    roof = {"bound": "hbm", "kernel": f"k_pass<{args.dtype}>", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "launches_per_step": k["launches"] / args.steps, "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": avg_bytes, "copy_ceiling": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4)}
    # fusion accounting: passes over the state per layer, the one-pass floor (read + write of
    # the state once per layer at peak) against the measured layer time, and the sweeps per layer
    # of a gate-by-gate scheme (n R_x + n R_z + m coupling gates)
    state_bytes = (1 << n) * (16 if args.dtype == "c128" else 8)
    t_layer = ms / p * 1e-3
    roof["passes_per_layer"] = round(k["launches"] / args.steps / p, 3)
    roof["one_pass_floor_frac"] = round(2 * state_bytes / (HBM_PEAK_GBS * 1e9) / t_layer, 4)
    roof["gate_sweeps_per_layer"] = 2 * n + len(inst["J"])
    # per tile geometry: T tile bits, c carrier bits (runs of 2^c amplitudes), L layouts, w write-only
    by_geo = {}
    for key, rec in sorted(prof.items()):
        if not key.startswith(kind + "/"):
            continue
        g_ms = rec["ms"] / max(1, rec["launches"])
        by_geo[key.split("/", 1)[1]] = {"launches_per_step": rec["launches"] / args.steps, "avg_ms": round(g_ms, 4),
                                        "GBps": round(rec["bytes"] / (rec["ms"] * 1e-3) / 1e9, 1)}
        log(f"[bench]   {key}: {by_geo[key.split('/', 1)[1]]}")
    roof["by_geometry"] = by_geo
    # streaming-ceiling time of the same passes (each pass's bytes at its geometry's ceiling)
    t_ceil = 0.0
    for gk, rec in by_geo.items():
        c_key = gk[gk.index("c"):gk.index("L")]
        rate = ceil.get(c_key)
        if rate:
            t_ceil += rec["GBps"] * rec["avg_ms"] * rec["launches_per_step"] / rate
    roof["stream_ceilings"] = {k: v for k, v in ceil.items() if k != "T"}
    pass_ms = sum(r["avg_ms"] * r["launches_per_step"] for r in by_geo.values())
    roof["frac_of_ceiling"] = round(t_ceil / pass_ms, 4) if pass_ms > 0 else None
    log(f"[bench] k_pass {achieved:.0f} GB/s; streaming ceilings {roof['stream_ceilings']}")

    extras = {}
    legs = set() if args.no_extras else (
        {"grad", "grad_p8", "c64", "exact_cover", "hadamard", "qsds", "batch_scan", "optimizer", "full", "cpu"}
        if args.extras == "all"
        else set(args.extras.split(",")))
    if "grad" in legs:
        # adjoint gradient vs finite differences (2p + 1 forward evaluations)
        lam = sv.State(n, args.dtype)
        sv.grad(s, lam, H, gam, bet)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            e, dg, db = sv.grad(s, lam, H, gam, bet)
        torch.cuda.synchronize()
        t_grad = (time.perf_counter() - t0) / reps * 1e3
        t_fd = (2 * p + 1) * ms
        extras["grad"] = {"ms": round(t_grad, 3), "forward_ms": round(ms, 3), "fd_forward_diff_ms": round(t_fd, 3),
                          "speedup_vs_fd": round(t_fd / t_grad, 3), "target": round((2 * p + 1) / 3, 3),
                          "max_abs_grad": float(max(np.max(np.abs(dg)), np.max(np.abs(db))))}
        log(f"[bench] grad {t_grad:.2f} ms vs FD {t_fd:.2f} ms")
        del lam
    if "grad_p8" in legs:
        # depth p = 8 (16 parameters) at n = 30 in complex64: forward <H_C> and the adjoint
        # gradient against 2p + 1 = 17 forward evaluations; the complex64 gradient's error
        # against the complex128 adjoint of the same instance, relative to max|g|
        n8, p8 = 30, 8
        H8 = sv.Ising.from_instance(I.degree4_int2(n8, 4 + n8))
        sv.ground(H8)
        g8, b8 = I.uniform_params(p8, 9, -0.9, 0.9)
        s8 = sv.State(n8, "c64")
        l8 = sv.State(n8, "c64")

        def med(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return sorted(ts)[reps // 2]

        t_f8 = med(lambda: sv.qaoa_energy(s8, H8, g8, b8))
        t_g8 = med(lambda: sv.grad(s8, l8, H8, g8, b8))
        _, dg8, db8 = sv.grad(s8, l8, H8, g8, b8)
        s8.close()
        l8.close()
        torch.cuda.empty_cache()
        r8, q8 = sv.State(n8, "c128"), sv.State(n8, "c128")
        _, rg8, rb8 = sv.grad(r8, q8, H8, g8, b8)
        r8.close()
        q8.close()
        ref8 = np.concatenate([rg8, rb8])
        err8 = float(np.max(np.abs(np.concatenate([dg8, db8]) - ref8)) / np.max(np.abs(ref8)))
        extras["grad_p8"] = {"workload": "QAOA p=8 (16 parameters), n=30 complex64, degree-4 Ising J in [-2,2]",
                             "forward_ms": round(t_f8, 3), "grad_ms": round(t_g8, 3),
                             "fd_forward_diff_ms": round((2 * p8 + 1) * t_f8, 3),
                             "speedup_vs_fd": round((2 * p8 + 1) * t_f8 / t_g8, 3),
                             "target": round((2 * p8 + 1) / 3, 3), "c64_grad_err_vs_c128_rel_max": err8}
        log(f"[bench] p=8 n=30 c64: forward {t_f8:.2f} ms, grad {t_g8:.2f} ms "
            f"({(2 * p8 + 1) * t_f8 / t_g8:.2f}x vs 17 forwards), c64 error {err8:.2e} of max|g|")
        del H8
        torch.cuda.empty_cache()
    if "c64" in legs:
        # complex64 storage, same instance
        s64 = sv.State(n, "c64")
        sv.qaoa_energy(s64, H, gam, bet)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o64 = sv.qaoa_energy(s64, H, gam, bet)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / args.steps
        extras["c64"] = {"ms_per_step": round(ms64, 3), "amp_updates_per_s": updates / (ms64 * 1e-3),
                         "energy_diff_vs_c128": abs(o64[0] - out[0])}
        log(f"[bench] c64 {ms64:.3f} ms/step")
        del s64
    if "exact_cover" in legs:
        # dense exact-cover-structured instance (F = 472 columns, half-integer
        # couplings between every pair of overlapping rows), rescaled angles
        a = I.exact_cover_matrix(n, 472, 4 + n)
        Hx, Cx = sv.Ising.exact_cover(a)
        rx = sv.rescale_factor(Hx)
        sv.ground(Hx)
        sv.qaoa_energy(s, Hx, gam / rx, bet)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ox = sv.qaoa_energy(s, Hx, gam / rx, bet)
        torch.cuda.synchronize()
        msx = (time.perf_counter() - t0) * 1e3 / args.steps
        extras["exact_cover"] = {"ms_per_step": round(msx, 3), "amp_updates_per_s": updates / (msx * 1e-3),
                                 "couplings": int(np.count_nonzero(np.triu(a.astype(np.int64) @ a.T.astype(np.int64), 1))),
                                 "rescale_r": rx, "energy_plus_C": ox[0] * 1.0 + Cx, "p_gs": ox[1]}
        log(f"[bench] exact cover {msx:.3f} ms/step")
        del Hx
    if "hadamard" in legs:
        # Hadamard benchmark circuit (H^{xN})^{11} (general single-qubit layers)
        had = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
        U = np.ascontiguousarray(np.broadcast_to(had, (11, n, 2, 2)))
        sv.init_plus(s)
        sv.profile_enable(True)
        sv.profile_report()
        sv.gate_layers(s, U)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            sv.gate_layers(s, U)
        torch.cuda.synchronize()
        msh = (time.perf_counter() - t0) * 1e3 / reps
        ph = sv.profile_report().get(f"pass_{args.dtype}_nv1", {"launches": 0, "ms": 0.0, "bytes": 0.0})
        sv.profile_enable(False)
        extras["hadamard"] = {"ms_per_circuit": round(msh, 3), "gates": 11 * n,
                              "gates_per_s": 11 * n / (msh * 1e-3),
                              "passes": ph["launches"] / (reps + 1),
                              "pass_GBps": ph["bytes"] / (ph["ms"] * 1e-3) / 1e9 if ph["ms"] > 0 else None}
        log(f"[bench] hadamard circuit {msh:.3f} ms")
    if "qsds" in legs:
        # Eq. AQA4 time stepping, 10 steps of the annealing Hamiltonian, no per-step observables
        reps = 3
        st = 10
        sg = np.arange(st) / st
        sv.qsds_run(s, H, 0.5, 1.0 - sg, sg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sv.qsds_run(s, H, 0.5, 1.0 - sg, sg)
        torch.cuda.synchronize()
        msq = (time.perf_counter() - t0) * 1e3 / reps
        extras["qsds"] = {"steps": st, "ms_per_run": round(msq, 3), "ms_per_step": round(msq / st, 3)}
        log(f"[bench] qsds {msq:.3f} ms for {st} steps")
    if "batch_scan" in legs:
        # batched p = 1 landscape: 2048 instances, n ~ U{10..18}, 3-regular +-1 couplings, 32 x 32 grid
        insts = I.batch_instances(2048)
        Hb = [sv.Ising.from_instance(x) for x in insts]
        gb, bb = I.batch_grid()
        for dt in ("c64", "c128"):
            sv.batch_p1_scan(Hb, gb, bb, dtype=dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sv.batch_p1_scan(Hb, gb, bb, dtype=dt)
            torch.cuda.synchronize()
            msb = (time.perf_counter() - t0) * 1e3
            ns = np.array([x["n"] for x in insts], dtype=np.float64)
            items = len(insts) * len(gb) * len(bb)
            upd = float(np.sum(2.0 ** ns * (ns + 1))) * len(gb) * len(bb)
            # floating-point work the kernel executes per amplitude: two FMAs per qubit in the
            # tangent-form mixer (4 flops) and |psi|^2, E |psi|^2 for the sums (6 flops)
            flops = float(np.sum(2.0 ** ns * (4 * ns + 6))) * len(gb) * len(bb)
            peak = 157.3e12 if dt == "c64" else 78.6e12
            # data movement of the scan per grid point: states above the 2^13-amplitude LDS slice
            # write and read their slab once (2 x amplitude bytes; the 256 MiB slab of a launch
            # stays in the last-level cache, so this is cache traffic, not HBM traffic) and read
            # the 16-bit energy index twice (phase, sums); LDS-resident states read the index twice
            es = 8 if dt == "c64" else 16
            big = ns > 13
            mem = float(np.sum(2.0 ** ns[big]) * (2 * es + 4) + np.sum(2.0 ** ns[~big]) * 4) * len(gb) * len(bb)
            extras[f"batch_scan_{dt}"] = {"ms": round(msb, 3), "items": items, "items_per_s": items / (msb * 1e-3),
                                          "amp_updates_per_s": upd / (msb * 1e-3),
                                          "valu_frac": flops / (msb * 1e-3) / peak,
                                          "slab_and_index_GBps": round(mem / (msb * 1e-3) / 1e9, 1),
                                          "batchslab_MiB": sv.tune_get("batchslab")}
            log(f"[bench] batch scan {dt}: {msb:.1f} ms for {items} items")
        del Hb
    if "optimizer" in legs:
        # optimisation loop of the paper (SLSQP, 200-call cap) at n = 26, p = 4:
        # adjoint gradients against scipy's finite differences of energy calls
        from paper_2104_03293_amd import optimize as O
        Ho = sv.Ising.from_instance(I.aqa_degree4_instance(26))
        dev = O.DeviceQAOA(Ho, args.dtype)
        g0, b0 = O.second_order_init(p, 0.5)
        opt, runs = {}, {}
        # the finite-difference run gets ten times the call budget so that it can reach the
        # energy the adjoint run ends at; the two are compared at equal energy
        for label, ug, cap in (("adjoint", True, 200), ("finite_diff", False, 2000)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = O.optimize_qaoa(dev, g0, b0, method="SLSQP", max_calls=cap, use_grad=ug)
            torch.cuda.synchronize()
            runs[label] = r
            opt[label] = {"seconds": round(time.perf_counter() - t0, 3), "max_calls": cap, "calls": r.calls,
                          "grad_calls": r.grad_calls, "energy": r.energy, "p_gs": r.p_gs,
                          "converged": r.converged, "fd_equivalent_calls": r.fd_equivalent_calls}
        # time to equal energy: the higher of the two final energies, which both runs reached
        target = max(runs["adjoint"].energy, runs["finite_diff"].energy) + 1e-9 * abs(runs["adjoint"].energy)
        tte = {k: O.time_to_energy(v, target) for k, v in runs.items()}
        e_init, _ = dev.energy(g0, b0)
        extras["optimizer"] = {"instance": "G(26,52), J in [-2,2], h in {-1,0,1}, seed 1", "p": p, "method": "SLSQP",
                               "initial_energy": e_init, **opt,
                               "equal_energy": {"target": target, **{k: v for k, v in tte.items()},
                                                "speedup": (tte["finite_diff"]["seconds"] / tte["adjoint"]["seconds"]
                                                            if tte["adjoint"] and tte["finite_diff"] else None)}}
        log(f"[bench] optimizer adjoint {opt['adjoint']['seconds']} s, FD {opt['finite_diff']['seconds']} s; "
            f"to E <= {target:.6f}: {tte}")
        dev.close()
        del Ho

    if "full" in legs:
        # the largest single-GPU states (one GPU's share of a run over several GPUs): n = 33
        # complex128 and n = 34 complex64, 128 GiB each (256 GiB with the adjoint's second vector)
        del s
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        extras["full_size"] = {}
        for nf, dtf in ((33, "c128"), (34, "c64")):
            extras["full_size"][f"n{nf}_{dtf}"] = full_size_leg(sv, I, nf, dtf, p)

    cpu = None
    if "cpu" in legs:
        cpu = cpu_baseline(args.cpu_sample_n, args.cpu_sample_p)

    res = {
        "metric": "amplitude-updates/s per QAOA layer at n=32 (HBM roofline of the layer kernel; grad vs FD)",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"QAOA p={p} energy evaluation (forward + fused <H_C>/P_gs), n={n} {args.dtype}, random Ising G(n,2n) "
                               f"J in [-2,2], h in {{-1,0,1}}", "n": n, "p": p, "amp_dtype": args.dtype},
        "roofline": roof,
        "tuned": tuned_knobs(sv, args.dtype, n),
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(res), flush=True)


def full_size_leg(sv, I, n: int, dtype: str, p: int) -> dict:
    """QAOA p-layer energy evaluation, AQA 10 steps and the p-layer adjoint
    gradient on a 128 GiB state: per-layer time, tile-pass GB/s against the
    HBM peak and the streaming ceilings of the plan."""
    import numpy as np
    import torch

    inst = I.full_size_instance(n)
    H = sv.Ising.from_instance(inst)
    sv.ground(H)
    s = sv.State(n, dtype)
    gam, bet = I.linear_ramp_params(p)
    sv.qaoa_energy(s, H, gam, bet)
    torch.cuda.synchronize()
    reps = 3
    sv.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        out = sv.qaoa_energy(s, H, gam, bet)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    prof = sv.profile_report()
    sv.profile_enable(False)
    k = prof.get(f"pass_{dtype}_nv1", {"launches": 0, "ms": 0.0, "bytes": 0.0})
    gbs = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
    by_geo = {key.split("/", 1)[1]: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
              for key, v in prof.items() if key.startswith(f"pass_{dtype}_nv1/")}
    ceil = stream_ceilings(sv, s, n, dtype)
    g_aqa, b_aqa = sv.schedule_linear(10, 0.5, paper_sign=True)
    sv.aqa_run(s, H, g_aqa, b_aqa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        sv.aqa_run(s, H, g_aqa, b_aqa)
    torch.cuda.synchronize()
    ms_aqa = (time.perf_counter() - t0) * 1e3 / 2
    res = {"ms_per_evaluation": round(ms, 3), "ms_per_layer": round(ms / p, 3),
           "amp_updates_per_s": p * (1 << n) * (n + 1) / (ms * 1e-3), "k_pass_GBps": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4), "by_geometry_GBps": by_geo,
           "stream_ceilings": {kk: v for kk, v in ceil.items() if kk != "T"},
           "passes_per_layer": k["launches"] / reps / p, "energy": out[0], "p_gs": out[1],
           "aqa10_ms": round(ms_aqa, 3), "aqa10_ms_per_step": round(ms_aqa / 10, 3)}
    free = torch.cuda.mem_get_info()[0]
    if free >= s.nbytes + (2 << 30):
        lam = sv.State(n, dtype)
        sv.grad(s, lam, H, gam, bet)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            sv.grad(s, lam, H, gam, bet)
        torch.cuda.synchronize()
        t_grad = (time.perf_counter() - t0) * 1e3 / 2
        res.update({"grad_ms": round(t_grad, 3), "grad_speedup_vs_fd": round((2 * p + 1) * ms / t_grad, 3)})
        del lam
    log(f"[bench] full size n={n} {dtype}: {ms:.1f} ms per p={p} evaluation, {gbs:.0f} GB/s, "
        f"AQA 10 steps {ms_aqa:.1f} ms, grad {res.get('grad_ms')} ms")
    del s, H
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def tuned_knobs(sv, dtype: str, n: int) -> dict:
    """Plan knobs in effect for (dtype, n): the tuned overrides where the cache has them."""
    d = sv.describe(n, dtype)
    return d.get("knobs_for_size", {})


def stream_ceilings(sv, s, n: int, dtype: str) -> dict:
    """GB/s of the library's streaming kernel (sv_stream_ceiling) for every tile
    geometry of the one-vector plan, keyed 'c<carrier bits>o<group start>'
    (and 'c<T>' for the contiguous tile)."""
    plan = sv.describe(n, dtype)["plans"]["nv1"]
    nbytes = 2 * (1 << n) * (16 if dtype == "c128" else 8)
    out = {"T": plan[0]["T"]}
    for g in plan:
        key = f"c{g['c']}" if g["g"] == 0 else f"c{g['c']}o{g['lo']}"
        sv.stream_ceiling(s, g["c"], g["lo"])
        ms = min(sv.stream_ceiling(s, g["c"], g["lo"]) for _ in range(3))
        out[key] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    return out


def committed_traffic(dtype: str, n: int, p: int):
    """HBM bytes per tile-pass launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload, or None when there is none or the
    kernel source changed since the counters were taken."""
    import hashlib
    import re

    f = ROOT / "profiles" / f"k_pass_{dtype}_traffic_n{n}_p{p}.md"
    if not f.exists():
        return None
    text = f.read_text()
    src = ROOT / "paper_2104_03293_amd" / "csrc" / "sv_kernels.hip"
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    m = re.search(r"kernel source sha256: ([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != sha:
        return None
    return float(t.group(1))


def cpu_baseline(n: int, p: int):
    """FP64 oracle on the host cores (a bounded sample of the same workload):
    oracle.c compiled here with -O3 -march=native (no fast-math) into a
    temporary directory; energy table + QAOA p-layer forward + observables,
    median of 3, on all cores at n and on one thread at n - 4."""
    import os
    import tempfile

    import numpy as np

    from oracle import build as obuild
    from oracle import oracle as orc
    from paper_2104_03293_amd import inputs as I

    tmp = Path(tempfile.mkdtemp(prefix="oracle_native_"))
    orc.use_library(obuild.build(out=tmp / "liboracle_native.so", native=True))
    g, b = I.linear_ramp_params(p)

    def rate(nn: int) -> tuple:
        inst = I.degree4_int2(nn, 4 + nn)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            E = orc.energies(inst)
            psi = orc.qaoa_state(inst, g, b, E=E)
            orc.observables(inst, psi, E=E, gs=(float(E.min()), 1, 0))
            ts.append(time.perf_counter() - t0)
            del psi, E
        dt = float(np.median(ts))
        return p * (1 << nn) * (nn + 1) / dt, dt

    threads = orc.num_threads()
    v_all, t_all = rate(n)
    orc.set_num_threads(1)
    v_one, t_one = rate(n - 4)
    orc.set_num_threads(threads)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0))
    log(f"[bench] cpu oracle (-O3 -march=native) n={n} p={p}: {t_all:.2f} s on {threads} threads; "
        f"n={n - 4}: {t_one:.2f} s on 1 thread ({model}, nproc {nproc})")
    return {"value": v_all, "unit": "amplitude-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"energy table + QAOA p={p} forward + observables at n={n} (FP64 C/OpenMP oracle, "
                      f"-O3 -march=native), median of 3 = {t_all:.2f} s",
            "one_thread": {"value": v_one, "n": n - 4, "seconds": round(t_one, 3)},
            "nproc": nproc, "cpu_model": model}


if __name__ == "__main__":
    main()
