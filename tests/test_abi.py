"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host-side error paths behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2605_03479_amd as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hb_ugks.h")).read()
    return sorted(set(re.findall(r"\b(hb_(?:ugks|batch|serve|vgrid)_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_03479_amd import build as b
    if b.stale():
        b.build()
    return hb.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 27
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hb.EXPORTS)


def _header_structs():
    """{name: [field, ...]} of every typedef struct in the header."""
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "hb_ugks.h")).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", src, flags=re.S):
        fields = []
        for decl in filter(None, (d.strip() for d in body.split(";"))):
            decl = re.sub(r"\[[^\]]*\]", "", decl)
            m = re.match(r"((?:const\s+)?(?:unsigned\s+)?\w+(?:\s*\*)*)\s+(.*)", decl, flags=re.S)
            fields += [re.sub(r"[\s*]", "", x) for x in m.group(2).split(",")]
        out[name] = fields
    return out


def test_binding_structs_match_header(tmp_path):
    """The ctypes mirrors of the header's structs: same fields in the same
    order, and the same size and offsets as the C compiler lays them out."""
    structs = _header_structs()
    assert {"hb_vgrid", "hb_geometry", "hb_wall", "hb_numerics", "hb_request", "hb_result"} <= set(structs)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hb_ugks.h"', "int main(void) {"]
    for name, fields in structs.items():
        cls = getattr(hb, name)
        assert [f[0] for f in cls._fields_] == fields, name
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, fields in structs.items():
        cls = getattr(hb, name)
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in fields:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_strerror_and_defaults(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.hb_ugks_strerror(code)
    assert b"unknown" in lib.hb_ugks_strerror(-99)
    n = hb.default_numerics()
    assert n.cfl == 0.5 and n.face_dt == 0 and abs(n.Pr - 2 / 3) < 1e-15 and n.K_int == 1
    assert n.macro_flux_mode == 0 and n.level_mass == 1 and n.dt_mode == 0


def test_null_and_state_errors(lib):
    assert lib.hb_ugks_create(None, None) == hb.HB_EINVAL
    assert lib.hb_ugks_pseudo_step(None, 1) == hb.HB_EINVAL
    assert lib.hb_ugks_set_case(None, None, 1.0, 1.0, 1, None, None, None) == hb.HB_EINVAL
    out = (ctypes.c_double * 4)()
    assert lib.hb_ugks_residual(None, out, None) == hb.HB_EINVAL
    assert lib.hb_ugks_td_step(None, 1) == hb.HB_EINVAL
    assert lib.hb_ugks_td_period(None, 1, out) == hb.HB_EINVAL
    assert lib.hb_ugks_time(None, ctypes.byref(ctypes.c_double())) == hb.HB_EINVAL
    assert lib.hb_ugks_wall_harmonic(None, 2, 1, 1, out) == hb.HB_EINVAL
    lib.hb_ugks_destroy(None)  # no-op


def test_batch_null_and_argument_errors(lib):
    b = ctypes.c_void_p()
    assert lib.hb_batch_create(None, 0, 0, ctypes.byref(b)) == hb.HB_EINVAL
    assert lib.hb_batch_create(None, 0, 4, None) == hb.HB_EINVAL
    o = hb.hb_create_opts(4096, None, 0, 0)
    assert lib.hb_batch_create(ctypes.byref(o), 0, 4, ctypes.byref(b)) == hb.HB_EDEVICE
    assert lib.hb_batch_step(None, 1) == hb.HB_EINVAL
    assert lib.hb_batch_remove(None, 0) == hb.HB_EINVAL
    assert lib.hb_batch_set_active(None, 0, 1) == hb.HB_EINVAL
    assert lib.hb_batch_tune(None, 1) == hb.HB_EINVAL
    assert lib.hb_batch_residuals(None, None, None, None, None, 0) == hb.HB_EINVAL
    h = ctypes.c_void_p()
    assert lib.hb_batch_case(None, 0, ctypes.byref(h)) == hb.HB_EINVAL
    lib.hb_batch_destroy(None)  # no-op


def test_create_bad_precision_or_device(lib):
    o = hb.hb_create_opts(0, None, 7, 0)
    h = ctypes.c_void_p()
    assert lib.hb_ugks_create(ctypes.byref(o), ctypes.byref(h)) == hb.HB_EINVAL
    o = hb.hb_create_opts(4096, None, 0, 0)
    assert lib.hb_ugks_create(ctypes.byref(o), ctypes.byref(h)) == hb.HB_EDEVICE


def test_vgrid_nodes_host(lib, oracle_mod):
    """Velocity rules of the library (host only): the trapezoid nodes and
    weights equal the oracle's; the Gauss-Hermite rule is exact for
    exp(-u^2) u^(2j), j < m (closed form Gamma(j + 1/2)) and matches the
    oracle's independent rule; bad arguments are refused."""
    import mpmath as mp
    import numpy as np
    u, w = hb.hb_vgrid_nodes(16, 4.0, hb.HB_RULE_TRAPEZOID)
    uo, wo = oracle_mod.velocity_grid(16, 4.0)
    np.testing.assert_allclose(u, uo, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, wo, rtol=0, atol=1e-15)
    for m in (4, 28, 64, 128):
        u, w = hb.hb_vgrid_nodes(m, 0.0, hb.HB_RULE_GAUSS_HERMITE)
        assert np.all(np.diff(u) > 0) and np.all(w > 0)
        g = w * np.exp(-u * u)
        for j in range(min(m, 40)):
            ref = float(mp.gamma(j + 0.5))
            assert abs(np.sum(g * u ** (2 * j)) - ref) <= 1e-12 * ref * max(1.0, 2.0 ** j), (m, j)
        if m <= 64:
            uo, wo = oracle_mod.gauss_hermite(m)
            np.testing.assert_allclose(u, uo, rtol=0, atol=1e-13 * np.max(np.abs(uo)))
            np.testing.assert_allclose(w, wo, rtol=1e-11)
    for m, umax, rule in ((5, 4.0, 0), (2, 4.0, 1), (16, 0.0, 0), (16, 4.0, 7)):
        with pytest.raises(hb.HBError):
            hb.hb_vgrid_nodes(m, umax, rule)
