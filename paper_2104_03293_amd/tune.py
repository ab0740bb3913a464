"""Autotuner for the plan knobs of libsv.

For each amplitude type and size it times the library's own workloads under
candidate knob values and writes the fastest choices to a cache file that libsv
reads from $SV_TUNE_CACHE (or via sv.tune_load), lines "<c64|c128> <n> <knob> <value>":

    python -m paper_2104_03293_amd.tune --n 26 30 32 --dtype c128 c64 --out tune_cache.txt

Targets (--targets, comma list):
  forward : one p-layer energy evaluation (sv_qaoa_energy: forward circuit with
            the fused observables).  Knobs: xcd (tile order), snake (group
            order), cmin128 / cmin64 (minimum carrier bits of the strided
            groups), ntmin (nontemporal threshold), ldsswz (LDS swizzle width),
            fuse, and c64occ / c64t13 (complex64 tile variants) or c128t14.
  grad    : one p-layer adjoint gradient (sv_grad).  Knobs: adjzeta (two
            one-vector sweeps or one two-vector sweep), kc34, and c64g4 /
            c64g14 (complex64 two-vector kernels).  The forward choices are
            kept while these are tuned.
  batch   : the p = 1 landscape scan over 2048 instances of n in 10..18 on a
            32 x 32 grid (size key 0).  Knobs: batchslab (MiB of the slab of
            one sliced launch, 0 = per-workgroup slots) and batchwide
            (complex64) or batch128 (complex128).
Search: coordinate descent from the built-in defaults (each knob in turn, the
others at their current best), two rounds, every candidate timed on the same
allocation as the median of --reps runs after one untimed run.  Knob values
that the library rejects for a size (an error) are skipped.  A JSON report of
every timing goes next to the cache (<out>.json).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from pathlib import Path

FORWARD = {
    "xcd": [-1, -2, 0, 1, 2, 3, 4],
    "snake": [1, 0, 2],
    "ntmin": [4, 3, 5, 6],
    "ldsswz": [4, 3, 5],
    "fuse": [1, 0],
}
FORWARD_C128 = {"cmin128": [3, 4, 5], "c128t14": [0, 1]}
FORWARD_C64 = {"cmin64": [4, 5, 6], "c64occ": [1, 0], "c64t13": [0, 1]}
GRAD = {"adjzeta": [-1, 0, 1], "kc34": [1, 0]}
GRAD_C64 = {"c64g4": [1, 0], "c64g14": [2, 0, 1]}
BATCH = {"c64": {"batchslab": [256, 128, 192, 384, 0], "batchwide": [2, 1, 0]},
         "c128": {"batchslab": [256, 128, 192, 384, 0], "batch128": [1, 0]}}


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _timer(fn, reps):
    import torch

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return _median(ts)


def coordinate_descent(sv, space: dict, measure, log, label: str, rounds: int = 2):
    """Tune the knobs of `space` one at a time; returns (best values, best time, trace)."""
    best = {k: sv.tune_get(k) for k in space}
    for k, v in best.items():
        sv.tune_set(k, v)
    t_best = measure()
    trace = [{"knobs": dict(best), "ms": t_best * 1e3}]
    log(f"[tune] {label} start {best}: {t_best * 1e3:.3f} ms")
    for _ in range(rounds):
        changed = False
        for k, values in space.items():
            for v in values:
                if v == best[k]:
                    continue
                try:
                    sv.tune_set(k, v)
                    t = measure()
                except Exception as e:  # a value the library rejects for this size
                    log(f"[tune] {label} {k}={v}: skipped ({e})")
                    sv.tune_set(k, best[k])
                    continue
                trace.append({"knobs": {**best, k: v}, "ms": t * 1e3})
                log(f"[tune] {label} {k}={v}: {t * 1e3:.3f} ms")
                if t < t_best * 0.995:  # keep a change only for a clear gain
                    t_best, best[k], changed = t, v, True
                sv.tune_set(k, best[k])
        if not changed:
            break
    log(f"[tune] {label} best {best}: {t_best * 1e3:.3f} ms")
    return best, t_best, trace


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[26, 30, 32])
    ap.add_argument("--dtype", nargs="+", default=["c128", "c64"])
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--targets", default="forward,grad,batch")
    ap.add_argument("--out", default="tune_cache.txt")
    args = ap.parse_args(argv)
    targets = set(args.targets.split(","))

    root = Path(__file__).resolve().parents[1]
    if str(root) not in sys.path:
        sys.path.insert(0, str(root))
    import torch

    from paper_2104_03293_amd import inputs as I
    from paper_2104_03293_amd import sv

    def log(msg):
        print(msg, flush=True)

    torch.cuda.set_device(0)
    sv.tune_load(None)  # tune against the built-in defaults
    every = {**FORWARD, **FORWARD_C128, **FORWARD_C64, **GRAD, **GRAD_C64, "batchwide": [], "batch128": [],
             "batchslab": []}
    defaults = {k: sv.tune_get(k) for k in every}
    lines, report = [], {}
    for dtype in args.dtype:
        for n in args.n:
            if dtype == "c128" and n > 33:
                continue
            inst = I.degree4_int2(n, 4 + n)
            H = sv.Ising.from_instance(inst)
            sv.ground(H)
            gam, bet = I.linear_ramp_params(args.p)
            s = sv.State(n, dtype)
            chosen = {}
            if "forward" in targets:
                space = {**FORWARD, **(FORWARD_C128 if dtype == "c128" else FORWARD_C64)}
                best, t, trace = coordinate_descent(
                    sv, space, lambda: _timer(lambda: sv.qaoa_energy(s, H, gam, bet), args.reps), log,
                    f"{dtype} n={n} forward")
                chosen.update(best)
                report[f"{dtype} {n} forward"] = {"best": best, "ms": t * 1e3, "trace": trace}
            if "grad" in targets:
                free = torch.cuda.mem_get_info()[0]
                if free >= s.nbytes + (2 << 30):
                    lam = sv.State(n, dtype)
                    space = {**GRAD, **(GRAD_C64 if dtype == "c64" else {})}
                    best, t, trace = coordinate_descent(
                        sv, space, lambda: _timer(lambda: sv.grad(s, lam, H, gam, bet), args.reps), log,
                        f"{dtype} n={n} grad")
                    chosen.update(best)
                    report[f"{dtype} {n} grad"] = {"best": best, "ms": t * 1e3, "trace": trace}
                    lam.close()
            for k, v in chosen.items():
                lines.append(f"{dtype} {n} {k} {v}")
            for k, v in defaults.items():
                sv.tune_set(k, v)
            s.close()
            H.close()
            torch.cuda.empty_cache()
    if "batch" in targets:
        insts = I.batch_instances(2048)
        Hb = [sv.Ising.from_instance(x) for x in insts]
        gb, bb = I.batch_grid()
        for dtype in args.dtype:
            best, t, trace = coordinate_descent(
                sv, BATCH[dtype], lambda: _timer(lambda: sv.batch_p1_scan(Hb, gb, bb, dtype=dtype), args.reps), log,
                f"{dtype} batch scan", rounds=1)
            for k, v in best.items():
                lines.append(f"{dtype} 0 {k} {v}")
            report[f"{dtype} batch"] = {"best": best, "ms": t * 1e3, "trace": trace}
            for k, v in defaults.items():
                sv.tune_set(k, v)
    Path(args.out).write_text("\n".join(lines) + "\n")
    Path(str(args.out) + ".json").write_text(json.dumps(report, indent=1))
    log(f"[tune] wrote {args.out}")


if __name__ == "__main__":
    main()
