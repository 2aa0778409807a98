"""GPU test of nsfrb_inject_boxcars_static, the injection entry point that
allocates nothing (its tables go to a static device array).

Called through the C ABI, it must give the same cubes as nsfrb_inject_boxcars,
bit for bit, on two calls in a row, the second with fewer cubes, fewer records
and fewer sub-bands than the first (the static array still holds the first
call's tables when the second starts). Sizes beyond the documented limit are
refused with INVALID_ARG before anything is copied or launched.
"""
import ctypes

import numpy as np
import pytest

from paper_2510_18136_amd import nsfrb
from tests._lib import ensure_built

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def _cubes(n_cubes, n_pix, n_sub, n_time, dtype, seed):
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    stream = torch.cuda.current_stream().cuda_stream
    a = []
    for k in range(n_cubes):
        x = torch.empty(n_time * n_sub * n_pix, dtype=tdt, device="cuda")
        nsfrb.generate_noise(x.data_ptr(), dtype, "tsp", n_pix, n_sub, n_time, seed=seed + k, stream=stream)
        a.append(x)
    torch.cuda.synchronize()
    return a, [x.clone() for x in a]


def _records(rng, n, n_cubes, n_pix, n_sub, n_time):
    keys = rng.choice(n_cubes * n_pix, size=n, replace=False)
    recs = [(int(k) // n_pix, int(k) % n_pix, int(rng.integers(-4, n_time + 4)), int(rng.integers(1, 20)),
             float(rng.normal(0, 3))) for k in keys]
    offsets = rng.integers(0, 12, size=(n, n_sub)).astype(np.int32)
    return recs, offsets


@pytest.mark.parametrize("calls", [
    # (n_cubes, n_pix, n_sub, n_time, dtype, n_records): the second call is smaller in every table
    [(3, 300, 16, 96, "f32", 200), (2, 40, 4, 33, "f16", 9)],
])
def test_static_injection_equals_allocating_injection(calls):
    rng = np.random.default_rng(11)
    stream = torch.cuda.current_stream().cuda_stream
    for i, (n_cubes, n_pix, n_sub, n_time, dtype, n) in enumerate(calls):
        print(f"[gpu] static injection call {i}: {n_cubes} cubes, {n} records, {n_sub} sub-bands, {dtype}",
              flush=True)
        got, ref = _cubes(n_cubes, n_pix, n_sub, n_time, dtype, seed=100 + 10 * i)
        recs, offsets = _records(rng, n, n_cubes, n_pix, n_sub, n_time)
        nsfrb.inject_boxcars([x.data_ptr() for x in got], dtype, "tsp", n_pix, n_sub, n_time, recs, offsets,
                             stream=stream, static=True)
        nsfrb.inject_boxcars([x.data_ptr() for x in ref], dtype, "tsp", n_pix, n_sub, n_time, recs, offsets,
                             stream=stream)
        torch.cuda.synchronize()
        changed = 0
        for g, r in zip(got, ref):
            gb, rb = g.view(torch.int16 if dtype != "f32" else torch.int32), r.view(
                torch.int16 if dtype != "f32" else torch.int32)
            assert torch.equal(gb, rb)
        # the injection did something (not two untouched cubes compared)
        fresh, _ = _cubes(n_cubes, n_pix, n_sub, n_time, dtype, seed=100 + 10 * i)
        for g, f in zip(got, fresh):
            changed += int((g.float() != f.float()).sum().item())
        assert changed > 0


def test_static_injection_refuses_sizes_beyond_the_limit():
    # the cube holds every shape named below, so even a launch would stay in bounds
    x = torch.zeros(4096 * 64, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    # more than 4096 records
    with pytest.raises(nsfrb.NsfrbError) as e:
        nsfrb.inject_boxcars([x.data_ptr()], "f32", "tsp", 4097, 8, 1,
                             [(0, p, 0, 1, 1.0) for p in range(4097)], np.zeros((4097, 8), np.int32),
                             stream=stream, static=True)
    assert e.value.status == nsfrb.INVALID_ARG and "4096" in str(e.value)
    # tables beyond 1 MiB: 4096 records x 64 sub-bands of offsets alone fill it
    with pytest.raises(nsfrb.NsfrbError) as e:
        nsfrb.inject_boxcars([x.data_ptr()], "f32", "tsp", 4096, 64, 1,
                             [(0, p, 0, 1, 1.0) for p in range(4096)], np.zeros((4096, 64), np.int32),
                             stream=stream, static=True)
    assert e.value.status == nsfrb.INVALID_ARG and "1 MiB" in str(e.value)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(x).item()) == 0


def test_static_injection_is_exported_through_the_c_abi():
    L = nsfrb.lib()
    fn = L.nsfrb_inject_boxcars_static
    assert fn.restype == ctypes.c_int and len(fn.argtypes) == 11
