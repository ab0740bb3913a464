"""The autotuner on the GPU: a short coordinate-descent run over the forward and
gradient knobs writes a cache; loaded, the tuned plans give results that match
the FP64 oracle (state, <H_C>, P_gs and the adjoint gradient)."""
import sys

import numpy as np
import pytest

from paper_2104_03293_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2104_03293_amd import sv as m

    return m


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_tuned_cache_matches_oracle(sv, orc, tmp_path, record_error):
    from paper_2104_03293_amd import tune

    n, p = 18, 4
    out = tmp_path / "cache.txt"
    tune.main(["--n", str(n), "--dtype", "c128", "c64", "--reps", "1", "--targets", "forward,grad",
               "--out", str(out)])
    lines = [l.split() for l in out.read_text().splitlines() if l.strip()]
    assert lines and all(len(l) == 4 and l[0] in ("c128", "c64") and l[1] == str(n) for l in lines)
    inst = I.degree4_int2(n, 4 + n)  # the tuner's instance
    g, b = I.linear_ramp_params(p)
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, g, b, E=E)
    _, ren, rpg = orc.observables(inst, ref, E=E)
    _, rg, rb = orc.grad_tangent(inst, g, b, E=E)
    scale = max(float(np.max(np.abs(np.concatenate([rg, rb])))), orc.coeff_scale(inst))
    sv.tune_load(str(out))
    try:
        H = sv.Ising.from_instance(inst)
        for dtype, amp_tol, gtol in (("c128", 1e-11, 1e-6), ("c64", 2e-5, 5e-6)):
            s = sv.State(n, dtype)
            e, pg, nrm = sv.qaoa_energy(s, H, g, b)
            err = float(np.max(np.abs(s.to_numpy() - ref)))
            record_error(f"amp max-abs {dtype}", err)
            assert err <= amp_tol
            assert abs(e - ren) <= 1e-6 * max(abs(ren), orc.coeff_scale(inst))
            lam = sv.State(n, dtype)
            ge, dg, db = sv.grad(s, lam, H, g, b)
            gerr = max(np.max(np.abs(dg - rg)), np.max(np.abs(db - rb))) / scale
            record_error(f"grad / scale {dtype}", gerr)
            assert gerr <= gtol
    finally:
        sv.tune_load(None)
