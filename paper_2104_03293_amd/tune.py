"""Autotuner for the tile-pass plans.

For each (amplitude type, n) it times a p-layer QAOA forward pass plus the
expectation under every candidate plan knob setting and writes the fastest to
a cache file that libsv reads from $SV_TUNE_CACHE (or via sv.tune_load):

    python -m paper_2104_03293_amd.tune --n 26 30 32 --dtype c128 c64 --out tune_cache.txt

Knobs swept:
  cmin128 / cmin64 : minimum carrier bits of the high tile groups (contiguous
                     runs of 2^c amplitudes; larger runs stream better but give
                     smaller groups, i.e. possibly more passes per layer)
  fuse             : snake-fused passes (1) or one mixer per pass (0)
  snake            : the contiguous group in the middle of each layer's order (1) or first (0)
  c64occ / c64t13  : complex64 only: 14-bit tiles without lane position 4 (two
                     workgroups per CU) or with it; 13-bit tiles (four groups)
Timing uses the library's per-launch HIP events (sv.profile_*) plus wall time.
"""
from __future__ import annotations

import argparse
import itertools
import sys
import time
from pathlib import Path


def candidates(dtype: str):
    key = "cmin128" if dtype == "c128" else "cmin64"
    base = 3 if dtype == "c128" else 4
    for c, f, sn in itertools.product([base, base + 1, base + 2], [1, 0], [1, 0]):
        if dtype == "c128":
            yield {key: c, "fuse": f, "snake": sn}
        else:
            for occ, t13 in ((1, 0), (0, 0), (1, 1)):
                yield {key: c, "fuse": f, "snake": sn, "c64occ": occ, "c64t13": t13}


def time_plan(sv, H, n, dtype, gam, bet, reps):
    import torch

    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, gam, bet)
    sv.expect(s, H)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sv.qaoa_forward(s, H, gam, bet)
        sv.expect(s, H)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    s.close()
    return dt


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[26, 30, 32])
    ap.add_argument("--dtype", nargs="+", default=["c128", "c64"])
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default="tune_cache.txt")
    args = ap.parse_args(argv)

    root = Path(__file__).resolve().parents[1]
    if str(root) not in sys.path:
        sys.path.insert(0, str(root))
    import torch

    from paper_2104_03293_amd import inputs as I
    from paper_2104_03293_amd import sv

    torch.cuda.set_device(0)
    sv.tune_load(None)  # tune against the built-in defaults
    defaults = {k: sv.tune_get(k) for k in ("fuse", "cmin128", "cmin64", "snake", "c64occ", "c64t13")}
    lines = []
    for dtype in args.dtype:
        for n in args.n:
            if dtype == "c128" and n > 33:
                continue
            inst = I.degree4_int2(n, 4 + n)
            H = sv.Ising.from_instance(inst)
            gam, bet = I.linear_ramp_params(args.p)
            best = None
            for cand in candidates(dtype):
                for k, v in cand.items():
                    sv.tune_set(k, v)
                dt = time_plan(sv, H, n, dtype, gam, bet, args.reps)
                print(f"[tune] {dtype} n={n} {cand}: {dt * 1e3:.3f} ms", flush=True)
                if best is None or dt < best[0]:
                    best = (dt, dict(cand))
                for k, v in defaults.items():
                    sv.tune_set(k, v)
            print(f"[tune] {dtype} n={n} best {best[1]} {best[0] * 1e3:.3f} ms", flush=True)
            for k, v in best[1].items():
                lines.append(f"{dtype} {n} {k} {v}")
    Path(args.out).write_text("\n".join(lines) + "\n")
    print(f"[tune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
