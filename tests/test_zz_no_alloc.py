"""The allocation-free harmonics entry point, hb_ugks_harmonics_out_noalloc,
through the C ABI:

- two calls in a row, the second on a smaller case than the first (the
  static scratch then still holds the first call's values beyond the second's
  extent), each bit-identical to hb_ugks_harmonics_out on the same handle
  (same kernels, same data), with the device's free memory and the handle's
  footprint unchanged by either call;
- a case that needs more than the static scratch is refused with HB_ENOMEM.
No test here makes a kernel run outside its buffers: the refusal happens on
the host before any launch."""
import ctypes

import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu
_DP = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def gpu():
    import paper_2605_03479_amd as hb
    hb.load_library()
    return hb


def _free_bytes():
    """Free device memory from the HIP runtime the library runs on."""
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipDeviceSynchronize() == 0
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _call(L, fn, h, mask, n):
    re = np.zeros(n)
    im = np.zeros(n)
    rc = getattr(L, fn)(h, mask, re.ctypes.data_as(_DP), im.ctypes.data_as(_DP), n)
    return rc, re, im


def test_noalloc_matches_harmonics_out_on_two_calls(gpu):
    L = gpu.load_library()
    big = Case(12, 10, 16, 5.0, 0.5, 2.0, 3, hbcases.thermal_walls(0.3, 0, "sin"), name="big")
    small = Case(6, 5, 12, 4.0, 1.0, 1.0, 1, hbcases.lid_walls(0.02), name="small")
    runs = []
    for case, prec, mask in ((big, gpu.HB_MIXED, 0x7F), (small, gpu.HB_FP64, 0x5B)):
        s = gpu.Solver(case, precision=prec)
        s.step(25)
        n = bin(mask).count("1") * (case.NH + 1) * case.nc
        rc, re, im = _call(L, "hb_ugks_harmonics_out", s.h, mask, n)
        assert rc == gpu.HB_OK
        assert np.any(re != 0.0)
        runs.append((s, mask, n, re, im))
    print(f"  noalloc on {big.name} ({big.nc} cells, N_T {big.NT}) then {small.name} ({small.nc} cells, "
          f"N_T {small.NT})", flush=True)
    for s, mask, n, re, im in runs:
        before, fp = _free_bytes(), s.device_bytes()
        rc, re2, im2 = _call(L, "hb_ugks_harmonics_out_noalloc", s.h, mask, n)
        after = _free_bytes()
        assert rc == gpu.HB_OK
        assert np.array_equal(re2, re) and np.array_equal(im2, im)
        assert after == before and s.device_bytes() == fp
    for s, *_ in runs:
        s.close()


def test_noalloc_refuses_cases_beyond_its_scratch(gpu):
    L = gpu.load_library()
    # 200 x 200 cells at N_T = 11 need 161 * 40000 doubles, more than the 4 Mi of the scratch
    case = Case(200, 200, 4, 4.0, 1.0, 1.0, 5, hbcases.lid_walls(0.01), name="too_big")
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    n = 7 * (case.NH + 1) * case.nc
    rc, _, _ = _call(L, "hb_ugks_harmonics_out_noalloc", s.h, 0x7F, n)
    assert rc == gpu.HB_ENOMEM
    rc, _, _ = _call(L, "hb_ugks_harmonics_out", s.h, 0x7F, n)  # the handle's own scratch still serves it
    assert rc == gpu.HB_OK
    s.close()
