"""Error paths of the C ABI on the device (hb_ugks.h conventions):

- HB_EDIVERGED: a NaN loaded through state_in reaches the residual, which
  then reports divergence on the single handle and in a batch, and keeps
  reporting it; the state stays readable.
- HB_ENOMEM: a handle's hbm_budget_bytes below the case's footprint refuses
  set_case; at the footprint it is accepted (harmonics scratch included).
- HB_ECAPACITY: buffers shorter than the result for harmonics_out and
  state_out.
- HB_ESTATE: stepping, reading or copying before set_case.
- HB_EINVAL for a velocity grid whose v axis is odd, too short or too long,
  or whose update tables (16 N_T max(M, M_v) words) exceed the LDS.
No error here comes from a device fault: every kernel runs to its end (a NaN
is ordinary floating-point data to them)."""
import ctypes

import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import paper_2605_03479_amd as hb
    hb.load_library()
    return hb


def _small():
    return Case(6, 5, 8, 4.0, 1.0, 1.0, 1, hbcases.lid_walls(0.01), name="err6x5")


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_nan_state_reports_diverged(gpu, prec):
    case = _small()
    s = gpu.Solver(case, precision=prec)
    s.step(2)
    assert np.all(np.isfinite(s.residual()))
    W, h, b = s.state()
    h[7, 1, 5] = np.nan
    print(f"  NaN in h of cell 7, level 1, velocity 5 (prec {prec})", flush=True)
    s.set_state(W, h, b)
    s.step(1)
    with pytest.raises(gpu.HBError) as e:
        s.residual()
    assert e.value.code == gpu.HB_EDIVERGED
    s.step(1)  # further steps are accepted; divergence stays reported
    rc, r, k = gpu.hb_ugks_residual(s.h)
    assert rc == gpu.HB_EDIVERGED and k == 4
    W2 = s.macro()  # the state is kept for state_out
    assert np.isnan(W2).any()
    s.close()


def test_nan_in_batch_flags_only_that_case(gpu):
    B = gpu.Batch(max_cases=4)
    a = B.add(_small(), gpu.HB_FP64)
    c = B.add(_small().with_(nx=7, name="err7x5"), gpu.HB_FP64)
    B.step(1)
    W, h, b = a.state()
    W[3, 0, 0] = np.nan
    a.set_state(W, h, b)
    B.step(2)
    res = B.residuals()
    assert res[a.cid][2] is True and res[c.cid][2] is False
    assert np.all(np.isfinite(res[c.cid][0]))
    with pytest.raises(gpu.HBError) as e:
        a.residual()
    assert e.value.code == gpu.HB_EDIVERGED
    B.close()


def test_budget_refuses_then_accepts(gpu):
    case = hbcases.shear_small()
    probe = gpu.Solver(case)
    need = probe.device_bytes()
    probe.close()
    assert need > 0
    with pytest.raises(gpu.HBError) as e:
        gpu.Solver(case, hbm_budget_bytes=need - 1)
    assert e.value.code == gpu.HB_ENOMEM
    s = gpu.Solver(case, hbm_budget_bytes=need)
    s.step(3)
    re, im = s.harmonics()  # its scratch is part of the footprint: no allocation here
    assert np.all(np.isfinite(re)) and s.device_bytes() == need
    s.close()


def test_short_buffers(gpu):
    L = gpu.load_library()
    case = _small()
    s = gpu.Solver(case)
    s.step(1)
    nx, ny, nc, M, nv, NT = s.sizes
    per = (case.NH + 1) * nc
    re = np.zeros(2 * per)
    im = np.zeros(2 * per)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = L.hb_ugks_harmonics_out(s.h, 0x3, re.ctypes.data_as(dp), im.ctypes.data_as(dp), 2 * per - 1)
    assert rc == gpu.HB_ECAPACITY
    rc = L.hb_ugks_harmonics_out(s.h, 0x3, re.ctypes.data_as(dp), im.ctypes.data_as(dp), 2 * per)
    assert rc == gpu.HB_OK and np.any(re != 0.0)
    hh = np.zeros(nc * NT * nv)
    rc = L.hb_ugks_state_out(s.h, None, hh.ctypes.data_as(dp), None, hh.size - 1)
    assert rc == gpu.HB_ECAPACITY
    rc = L.hb_ugks_state_out(s.h, None, hh.ctypes.data_as(dp), None, hh.size)
    assert rc == gpu.HB_OK
    names = (ctypes.c_char_p * 2)()
    assert L.hb_ugks_kernel_times(s.h, names, None, None, 2) == gpu.HB_ECAPACITY
    s.close()


def test_calls_before_set_case(gpu):
    L = gpu.load_library()
    h = gpu.hb_ugks_create()
    out = np.zeros(4)
    dp = ctypes.POINTER(ctypes.c_double)
    assert L.hb_ugks_pseudo_step(h, 1) == gpu.HB_ESTATE
    assert L.hb_ugks_residual(h, out.ctypes.data_as(dp), None) == gpu.HB_ESTATE
    assert L.hb_ugks_harmonics_out(h, 1, out.ctypes.data_as(dp), out.ctypes.data_as(dp), 4) == gpu.HB_ESTATE
    assert L.hb_ugks_state_out(h, out.ctypes.data_as(dp), None, None, 0) == gpu.HB_ESTATE
    assert L.hb_ugks_pseudo_step(h, -1) == gpu.HB_ESTATE
    gpu.hb_ugks_destroy(h)


@pytest.mark.parametrize("grid,prec,ok", [
    (dict(Mv=7), 0, False),                 # odd node count along v
    (dict(Mv=-2), 0, False),
    (dict(Mv=2), 1, False),                 # fewer than 4 nodes
    (dict(Mv=130), 1, False),               # more than 128
    (dict(M=16, Mv=128, NH=5), 0, False),   # FP64 tables 16 x 11 x 128 x 8 B = 180 KB > 160 KB of LDS
    (dict(M=16, Mv=128, NH=5), 1, True),    # the same tables in FP32: 90 KB
], ids=["odd", "negative", "two", "130", "fp64-lds", "mixed-lds"])
def test_rectangular_grid_arguments(gpu, grid, prec, ok):
    """hb_vgrid's v axis is checked like the u axis, and the update tables'
    size bound takes the longer axis."""
    case = _small().with_(**grid)
    h = gpu.hb_ugks_create(precision=prec)
    try:
        if ok:
            gpu.hb_ugks_set_case(h, case)
            assert gpu.hb_ugks_sizes(h)[4] == case.M * case.Mv
        else:
            with pytest.raises(gpu.HBError) as e:
                gpu.hb_ugks_set_case(h, case)
            assert e.value.code == gpu.HB_EINVAL
    finally:
        gpu.hb_ugks_destroy(h)
