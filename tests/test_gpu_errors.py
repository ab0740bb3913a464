"""Error paths of the C ABI on the GPU: allocation beyond the free device memory
and the failed state a launch error leaves behind.

The launch failure is forced from the host (knob fail_next_launch: the next
tile-pass launch reports hipErrorLaunchFailure and nothing is launched), so no
kernel ever faults.
"""
import sys

import numpy as np
import pytest

from paper_2104_03293_amd import inputs as I

pytestmark = pytest.mark.gpu
GIB = 1 << 30


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


def test_alloc_beyond_free_memory_is_oom_and_allocates_nothing(sv):
    """sv_alloc checks hipMemGetInfo first: 128 GiB states (complex64, n = 34) are
    taken until the next one does not fit; that request fails with SV_ERR_OOM and
    leaves the free memory unchanged; afterwards small states work."""
    import torch

    big = (1 << 34) * 8
    held = []
    try:
        while torch.cuda.mem_get_info()[0] >= big and len(held) < 4:
            held.append(sv.State(34, "c64", owner="lib"))
        free0 = torch.cuda.mem_get_info()[0]
        assert free0 < big, free0
        with pytest.raises(sv.SVError) as e:
            sv.State(34, "c64", owner="lib")
        assert e.value.code == 2, e.value
        assert "free" in str(e.value)
        assert abs(torch.cuda.mem_get_info()[0] - free0) <= 64 * (1 << 20)
    finally:
        for h in held:
            h.close()
    s = sv.State(12, "c128", owner="lib")
    sv.init_plus(s)
    assert np.max(np.abs(s.to_numpy() - 2.0 ** -6)) == 0.0
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_launch_failure_leaves_state_failed(sv, dtype):
    """A launch error marks the state failed: every later call on it returns
    SV_ERR_HIP without running, other states and instances keep working, and
    the handle can still be freed."""
    n = 16
    inst = I.degree4_int2(n, 3)
    H = sv.Ising.from_instance(inst)
    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, [0.3], [0.2])
    sv.tune_set("fail_next_launch", 1)
    with pytest.raises(sv.SVError) as e:
        sv.qaoa_forward(s, H, [0.3, 0.1], [0.2, -0.4])
    assert e.value.code == 3 and "launch" in str(e.value)
    assert sv.tune_get("fail_next_launch") == 0  # consumed by that launch
    calls = [lambda: sv.qaoa_forward(s, H, [0.1], [0.2]), lambda: sv.expect(s, H), lambda: sv.mixer(s, 0.3),
             lambda: sv.cost_phase(s, H, 0.2), lambda: s.to_numpy(), lambda: sv.qaoa_energy(s, H, [0.1], [0.1]),
             lambda: sv.init_plus(s), lambda: sv.spin_z(s)]
    for call in calls:
        with pytest.raises(sv.SVError) as e:
            call()
        assert e.value.code == 3, e.value
    # the adjoint refuses a failed state as either vector
    ok = sv.State(n, dtype)
    with pytest.raises(sv.SVError) as e:
        sv.grad(s, ok, H, [0.1], [0.2])
    assert e.value.code == 3
    with pytest.raises(sv.SVError) as e:
        sv.grad(ok, s, H, [0.1], [0.2])
    assert e.value.code == 3
    # other objects are unaffected
    e1, pg, nrm = sv.qaoa_energy(ok, H, [0.3], [0.2])
    assert abs(nrm - 1.0) <= 1e-5
    s.close()
    ok.close()
