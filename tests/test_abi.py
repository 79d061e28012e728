"""The C ABI library loads on a host without a GPU and exports every entry
point include/ai.h declares (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ai.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ai_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2509_12381_amd import binding, build
    if build.stale():
        build.build()
    return ctypes.CDLL(binding.LIB_PATH)


def test_header_declares_the_entry_points():
    names = declared_functions()
    assert names == sorted(["ai_integrate", "ai_integrate_async", "ai_integrate_static_async",
                            "ai_integrate_batch",
                            "ai_integrate_batch_async", "ai_batch_plan_create",
                            "ai_batch_plan_launch", "ai_batch_plan_destroy", "ai_tune",
                            "ai_tune_batch",
                            "ai_trace",
                            "ai_server_create",
                            "ai_server_submit",
                            "ai_server_wait", "ai_server_destroy", "ai_kernel_time",
                            "ai_get_kernel_info",
                            "ai_last_error", "ai_nobs", "ai_version"])


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2509_12381_amd import binding
    assert sorted(binding.SYMBOLS) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(binding, name))


def test_struct_layout_matches_header():
    from paper_2509_12381_amd import binding
    # ai_params: 2 doubles, 2 int32, 2 doubles, 2 x 3 doubles, 3 doubles, int64, double
    assert ctypes.sizeof(binding.AiParams) == 8 * 2 + 4 * 2 + 8 * 2 + 8 * 6 + 8 * 3 + 8 + 8
    assert binding.AiParams.max_steps.offset == 8 * 2 + 4 * 2 + 8 * 2 + 8 * 6 + 8 * 3
    assert ctypes.sizeof(binding.AiKernelInfo) == 6 * 4 + 8
    # ai_batch_item: ai_params, pointer, 2 int64, 4 doubles, 2 pointers
    assert ctypes.sizeof(binding.AiBatchItem) == ctypes.sizeof(binding.AiParams) + 8 * 9


def test_struct_layout_against_the_c_compiler(tmp_path):
    """sizeof and field offsets of every ABI struct as gcc lays them out from
    include/ai.h, against the binding's ctypes declarations."""
    from paper_2509_12381_amd import binding
    structs = {"ai_params": binding.AiParams, "ai_batch_item": binding.AiBatchItem,
               "ai_server_config": binding.AiServerConfig,
               "ai_request_info": binding.AiRequestInfo, "ai_kernel_info": binding.AiKernelInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ai.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, what, value = line.split()
        cls = structs[cname]
        got = ctypes.sizeof(cls) if what == "sizeof" else getattr(cls, what).offset
        assert got == int(value), (cname, what, got, value)


def test_trace_argument_errors_without_gpu(lib):
    """ai_trace refuses a NULL point count, a negative capacity, refine < 1 and
    missing point buffers before any device call."""
    from paper_2509_12381_amd import binding, workload as W
    L = binding.load()
    p = binding.params(W.small_ensemble().system)
    pts = ctypes.c_int64(7)
    assert L.ai_trace(ctypes.byref(p), None, 0.0, 1.0, 1e-8, 1e-10, 1, 0, None, None, None,
                      None, None) == binding.EINVAL
    assert L.ai_trace(ctypes.byref(p), None, 0.0, 1.0, 1e-8, 1e-10, 1, -1, None, None, None,
                      None, ctypes.byref(pts)) == binding.EINVAL
    assert pts.value == 0
    assert L.ai_trace(ctypes.byref(p), None, 0.0, 1.0, 1e-8, 1e-10, 0, 5, None, None, None,
                      None, ctypes.byref(pts)) == binding.EINVAL
    assert L.ai_trace(ctypes.byref(p), None, 0.0, 1.0, 1e-8, 1e-10, 1, 5, None, None, None,
                      None, ctypes.byref(pts)) == binding.EINVAL
    assert b"point buffer" in L.ai_last_error()


def test_kernel_time_without_a_timed_call(lib):
    """The timing record is per thread: a thread that made no call with
    AI_TIME_KERNEL gets AI_EINVAL (checked on a fresh thread, whatever other
    tests in this process have done)."""
    import threading
    from paper_2509_12381_amd import binding
    L = binding.load()
    out = {}

    def probe():
        ms = ctypes.c_float(1.0)
        out["null"] = L.ai_kernel_time(0, None)
        out["rc"] = L.ai_kernel_time(0, ctypes.byref(ms))
        out["ms"] = ms.value

    t = threading.Thread(target=probe)
    t.start()
    t.join()
    assert out["null"] == binding.EINVAL
    assert out["rc"] == binding.EINVAL and out["ms"] == 0.0


def test_server_argument_errors_without_gpu(lib):
    """Null handles and bad configurations are refused before any device call;
    creating a server on a host without a GPU reports the HIP error."""
    from paper_2509_12381_amd import binding
    L = binding.load()
    h = ctypes.c_void_p()
    assert L.ai_server_create(None, None) == binding.EINVAL
    bad = binding.AiServerConfig(-1, 0, 0)
    assert L.ai_server_create(ctypes.byref(bad), ctypes.byref(h)) == binding.EINVAL
    bad = binding.AiServerConfig(0, 1, 0)
    assert L.ai_server_create(ctypes.byref(bad), ctypes.byref(h)) == binding.EINVAL
    bad = binding.AiServerConfig(0, 0, 17)
    assert L.ai_server_create(ctypes.byref(bad), ctypes.byref(h)) == binding.EINVAL
    for field, value in (("mode", 2), ("ring", -1), ("ring", 65537), ("slab_bytes", -1),
                         ("idle_ms", -1.0), ("idle_ms", float("nan")), ("refill_min", 65),
                         ("reserved", 1)):
        bad = binding.AiServerConfig(0, 0, 0, 1)
        setattr(bad, field, value)
        assert L.ai_server_create(ctypes.byref(bad), ctypes.byref(h)) == binding.EINVAL, field
    assert h.value is None
    t = ctypes.c_uint64()
    info = binding.AiRequestInfo()
    assert L.ai_server_submit(None, None, 0, ctypes.byref(t)) == binding.EINVAL
    assert L.ai_server_wait(None, 1, 0.0, ctypes.byref(info)) == binding.EINVAL
    assert L.ai_server_destroy(None) == binding.EINVAL
    if not _gpu_visible():
        rc = L.ai_server_create(None, ctypes.byref(h))
        assert rc == binding.EHIP and h.value is None


def test_batch_plan_argument_errors_without_gpu(lib):
    """ai_batch_plan_*: a NULL out pointer, a negative count, a kernel other
    than the plain double one (timing included), an invalid item and NULL
    plans are refused before any device call; an empty plan without a GPU
    reports the HIP error."""
    from paper_2509_12381_amd import binding, workload as W
    L = binding.load()
    p = binding.params(W.liyb_system())
    h = ctypes.c_void_p()
    items = (binding.AiBatchItem * 2)()
    for it in items:
        it.params = p
        it.n, it.ld, it.t0, it.tmax, it.rtol, it.atol = 0, 0, 0.0, 1.0, 1e-8, 1e-10
    assert L.ai_batch_plan_create(items, 2, 0, None) == binding.EINVAL
    assert L.ai_batch_plan_create(None, -1, 0, ctypes.byref(h)) == binding.EINVAL
    assert L.ai_batch_plan_create(items, 2, binding.TIME_KERNEL,
                                  ctypes.byref(h)) == binding.EUNSUPPORTED
    assert L.ai_batch_plan_create(items, 2, 1, ctypes.byref(h)) == binding.EUNSUPPORTED
    items[1].tmax = -1.0
    assert L.ai_batch_plan_create(items, 2, 0, ctypes.byref(h)) == binding.EINVAL
    assert binding.ai_last_error().startswith("item 1:")
    assert h.value is None
    assert L.ai_batch_plan_launch(None, None) == binding.EINVAL
    assert L.ai_batch_plan_destroy(None) == binding.EINVAL
    if not _gpu_visible():
        items[1].tmax = 1.0
        assert L.ai_batch_plan_create(items, 2, 0, ctypes.byref(h)) == binding.EHIP
        assert h.value is None


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_constants_without_gpu(lib):
    lib.ai_nobs.restype = ctypes.c_int
    lib.ai_version.restype = ctypes.c_int
    assert lib.ai_nobs() == 13
    assert lib.ai_version() >= 1


def test_invalid_arguments_are_refused_before_any_device_call(lib):
    from paper_2509_12381_amd import binding
    from paper_2509_12381_amd import workload as W
    b = binding.load()
    p = binding.params(W.liyb_system())
    # tmax <= t0 is refused during validation, before any HIP call
    rc = b.ai_integrate(ctypes.byref(p), None, 0, 0, 1.0, 0.0, 1e-8, 1e-10, None, None, 0)
    assert rc == binding.EINVAL
    assert "t0 < tmax" in binding.ai_last_error()
    rc = b.ai_integrate(ctypes.byref(p), None, -1, 0, 0.0, 1.0, 1e-8, 1e-10, None, None, 0)
    assert rc == binding.EINVAL
    rc = b.ai_integrate(ctypes.byref(p), None, 0, 0, 0.0, 1.0, 1e-8, 1e-10, None, None, 7)
    assert rc == binding.EINVAL
    # batches: a negative count, a NULL item array, an unsupported kernel, and an
    # invalid item (named in the message) are refused before any device call
    assert b.ai_integrate_batch(None, -1, 0) == binding.EINVAL
    assert b.ai_integrate_batch(None, 2, 0) == binding.EINVAL
    items = (binding.AiBatchItem * 2)()
    assert b.ai_integrate_batch(items, 2, 1) == binding.EUNSUPPORTED
    for it in items:
        it.params = p
        it.n, it.ld, it.t0, it.tmax, it.rtol, it.atol = 0, 0, 0.0, 1.0, 1e-8, 1e-10
    items[1].tmax = -1.0
    assert b.ai_integrate_batch(items, 2, 0) == binding.EINVAL
    assert binding.ai_last_error().startswith("item 1:")
    assert b.ai_integrate_batch_async(items, 0, 0, None) == binding.OK  # nothing enqueued



def test_static_entry_point_argument_errors_without_gpu(lib):
    """ai_integrate_static_async refuses what ai_integrate refuses (NULL
    parameters, n < 0, ld < n) before any device call."""
    from paper_2509_12381_amd import binding, workload as W
    L = binding.load()
    p = binding.params(W.small_ensemble().system)
    f = L.ai_integrate_static_async
    assert f(None, None, 0, 0, 0.0, 1.0, 1e-8, 1e-10, None, None, 0, None) == binding.EINVAL
    assert f(ctypes.byref(p), None, -1, 0, 0.0, 1.0, 1e-8, 1e-10, None, None, 0,
             None) == binding.EINVAL
    assert f(ctypes.byref(p), None, 5, 4, 0.0, 1.0, 1e-8, 1e-10, None, None, 0,
             None) == binding.EINVAL
