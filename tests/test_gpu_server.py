"""The serving entry points (ai_server_*): requests queued while the GPU is
busy share the next batched launch, and every request's results are bitwise
those of ai_integrate on that request alone ("alone = in-mix")."""
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


def _request(torch, wl, y0, t0=None, tmax=None, rtol=None, atol=None, ld=None):
    n = y0.shape[1]
    ld = n if ld is None else ld
    y0p = np.zeros((12, ld))
    y0p[:, :n] = y0
    d = torch.from_numpy(y0p).cuda()
    fin = torch.full((12, ld), -7.0, dtype=torch.float64, device="cuda")
    obs = torch.full((13, ld), -7.0, dtype=torch.float64, device="cuda")
    return dict(item=(wl.system, d, fin, obs, wl.t0 if t0 is None else t0,
                      wl.tmax if tmax is None else tmax, wl.rtol if rtol is None else rtol,
                      wl.atol if atol is None else atol, n),
                fin=fin, obs=obs, n=n)


def _alone(ai, torch, req, precision="fp64"):
    system, d, _, _, t0, tmax, rtol, atol, n = req["item"]
    fin = torch.full_like(req["fin"], -7.0)
    obs = torch.full_like(req["obs"], -7.0)
    ai.ai_integrate(system, d, t0, tmax, rtol, atol, fin, obs, "plain", n=n,
                    schedule="longest-first", precision=precision)
    torch.cuda.synchronize()
    return fin.cpu().numpy(), obs.cpu().numpy()


def _mix(torch):
    """A first request whose slow trajectories keep the GPU busy for several
    milliseconds, then requests of other systems, sizes, spans and tolerances
    (and an empty one) that queue behind it."""
    full = W.full_ensemble()
    grid = W.batch_grid(scale=1.0 / 64)
    reqs = [_request(torch, full, full.initial_states(4096))]
    for k in (0, 12, 21, 45, 63):
        wl = grid[k]
        reqs.append(_request(torch, wl, wl.initial_states(), ld=wl.n + 5))
    wl = grid[30]
    reqs.append(_request(torch, wl, wl.initial_states(), rtol=1e-10, atol=1e-12))
    reqs.append(_request(torch, wl, wl.initial_states(), t0=0.2 * wl.tmax, tmax=0.7 * wl.tmax))
    reqs.append(_request(torch, wl, wl.initial_states(1)[:, :0]))
    return reqs


def test_server_alone_equals_in_mix(ai, torch):
    reqs = _mix(torch)
    with ai.Server(schedule="longest-first") as srv:
        tickets = [srv.submit(r["item"]) for r in reqs]
        infos = [srv.wait(t) for t in tickets]
    assert all(i["rc"] == 0 and i["error"] == "" for i in infos), infos
    # the requests behind the first one were served together
    assert max(i["batch_size"] for i in infos) > 1, [i["batch_size"] for i in infos]
    assert infos[-1]["batch_id"] == -1                      # the empty request
    for i in infos:
        assert i["submit_s"] <= i["start_s"] <= i["end_s"]
    for r, i in zip(reqs, infos):
        fin, obs = _alone(ai, torch, r)
        np.testing.assert_array_equal(r["fin"].cpu().numpy(), fin)
        np.testing.assert_array_equal(r["obs"].cpu().numpy(), obs)
        assert np.all(r["obs"].cpu().numpy()[:, r["n"]:] == -7.0)


def test_server_requests_that_run_alone(ai, torch):
    """Single-precision stages and potentials with other exponents do not run
    in the batched kernel: such a request gets a launch of its own."""
    import dataclasses
    wl = W.small_ensemble()
    wl612 = dataclasses.replace(wl, system=dataclasses.replace(
        wl.system, n=6, m=12, Cn=8200.0 * 2.0, Cm=4.1e9))
    y = wl.initial_states()
    reqs = [_request(torch, wl, y[:, :300]), _request(torch, wl, y[:, 300:700]),
            _request(torch, wl, y[:, 700:900]), _request(torch, wl612, y[:, 900:])]
    precisions = ["fp64", "fp32-stages", "fp64", "fp64"]
    with ai.Server(workers=1) as srv:
        tickets = [srv.submit(r["item"], p) for r, p in zip(reqs, precisions)]
        infos = [srv.wait(t) for t in tickets]
    for k in (1, 3):
        assert infos[k]["batch_size"] == 1
        assert sum(i["batch_id"] == infos[k]["batch_id"] for i in infos) == 1
    for r, p in zip(reqs, precisions):
        fin, obs = _alone(ai, torch, r, p)
        np.testing.assert_array_equal(r["fin"].cpu().numpy(), fin)
        np.testing.assert_array_equal(r["obs"].cpu().numpy(), obs)


def test_server_launch_cap_and_close_finishes_queued_work(ai, torch):
    """max_batch caps a launch's trajectories (a larger request still runs,
    alone); closing the server serves what is queued before it returns."""
    wl = W.small_ensemble()
    y = wl.initial_states()
    reqs = [_request(torch, wl, y[:, i:i + 256]) for i in range(0, 1024, 256)]
    big = _request(torch, wl, y)
    srv = ai.Server(max_batch=512, workers=1)
    tickets = [srv.submit(r["item"]) for r in reqs + [big]]
    infos = [srv.wait(t) for t in tickets[:2]]
    srv.close()
    assert all(i["batch_trajectories"] <= 512 for i in infos)
    for r in reqs + [big]:
        fin, obs = _alone(ai, torch, r)
        np.testing.assert_array_equal(r["fin"].cpu().numpy(), fin)
        np.testing.assert_array_equal(r["obs"].cpu().numpy(), obs)


def test_server_errors_and_timeouts(ai, torch):
    wl = W.small_ensemble()
    good = _request(torch, wl, wl.initial_states())
    bad = _request(torch, wl, wl.initial_states(), rtol=-1.0)
    with ai.Server() as srv:
        with pytest.raises(ai.AiError) as e:
            srv.submit(bad["item"])
        assert e.value.rc == ai.EINVAL
        with pytest.raises(ai.AiError) as e:
            srv.wait(12345)
        assert e.value.rc == ai.EINVAL
        t = srv.submit(good["item"])
        first = srv.wait(t, timeout=0.0)                  # None while it runs
        info = first if first is not None else srv.wait(t)
        assert info["rc"] == 0
        with pytest.raises(ai.AiError):
            srv.wait(t)                                   # a ticket is waited for once
