"""ai_integrate_static_async, the entry point that allocates nothing (its
schedule workspace and queue counter live in a static device array of the
library): through the C ABI, each call's results equal ai_integrate_async's on
the same inputs, bitwise (the same kernels run), on two calls in a row whose
second is smaller, for the scheduled plain kernel, the scheduled persistent
kernel and the unscheduled persistent kernel; sizes beyond the scheduled
maximum are refused before any work is enqueued."""
import ctypes

import numpy as np
import pytest

from paper_2509_12381_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    return _torch


@pytest.fixture(scope="module")
def ai(torch):
    from paper_2509_12381_amd import binding
    binding.load()
    return binding


def _outputs(torch, n):
    fin = torch.full((12, n), -7.0, dtype=torch.float64, device="cuda")
    obs = torch.full((13, n), -7.0, dtype=torch.float64, device="cuda")
    return fin, obs


def _pair(ai, torch, wl, y0, kernel, schedule, refill_min=0):
    """(static results, allocating results) of one ensemble."""
    n = y0.shape[1]
    out = []
    for call in (ai.ai_integrate_static_async, ai.ai_integrate_async):
        fin, obs = _outputs(torch, n)
        torch.cuda.synchronize()
        rc = call(wl.system, y0, wl.t0, wl.tmax, wl.rtol, wl.atol, fin, obs, kernel=kernel,
                  schedule=schedule, refill_min=refill_min)
        torch.cuda.synchronize()
        assert rc == 0
        out.append((fin.cpu().numpy(), obs.cpu().numpy()))
    return out


@pytest.mark.parametrize("kernel,schedule,sizes", [
    ("plain", "longest-first", (100_000, 3_001)),
    ("persistent", "longest-first", (40_000, 777)),
    ("persistent", None, (30_000, 65)),
])
def test_static_calls_equal_allocating_calls(ai, torch, kernel, schedule, sizes):
    wl = W.thermal_workload(max(sizes))
    pool = torch.from_numpy(wl.initial_states()).cuda()
    for n in sizes:
        print(f"[no-alloc] {kernel} schedule={schedule} n={n}", flush=True)
        y0 = pool[:, :n].contiguous()
        (sf, so), (af, ao) = _pair(ai, torch, wl, y0, kernel, schedule, refill_min=16)
        assert np.array_equal(sf, af) and np.array_equal(so, ao), (kernel, schedule, n)
        assert np.all(so[W.OBS["status"]] > 0)


def test_static_call_refuses_sizes_beyond_its_scratch(ai, torch):
    wl = W.thermal_workload(1024)
    n = (1 << 20) + 1
    y0 = torch.zeros((12, n), dtype=torch.float64, device="cuda")
    fin, obs = _outputs(torch, n)
    torch.cuda.synchronize()
    with pytest.raises(ai.AiError) as err:
        ai.ai_integrate_static_async(wl.system, y0, wl.t0, wl.tmax, wl.rtol, wl.atol, fin, obs,
                                     kernel="plain", schedule="longest-first")
    assert err.value.rc == -1 and "at most" in str(err.value)
    torch.cuda.synchronize()
    assert float(obs.min()) == -7.0 == float(obs.max())  # nothing was launched
    with pytest.raises(ai.AiError):
        ai.ai_integrate_static_async(wl.system, y0, wl.t0, wl.tmax, wl.rtol, wl.atol, fin, obs,
                                     kernel=ai.kernel_code("plain") | ai.TIME_KERNEL)
    # the largest scheduled size is accepted (its workspace fits the scratch)
    m = 1 << 20
    rc = ai.ai_integrate_static_async(wl.system, y0[:, :m].contiguous(), wl.t0, wl.t0 + 1e6,
                                      wl.rtol, wl.atol, fin[:, :m].contiguous(),
                                      obs[:, :m].contiguous(), kernel="plain",
                                      schedule="longest-first")
    torch.cuda.synchronize()
    assert rc in (0, 1)
