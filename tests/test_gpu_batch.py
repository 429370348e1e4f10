"""Batched form on the GPU.

A case keeps exactly its single-case decomposition inside a batch (same
per-cell bodies, same residual partial sums in the same order), so the
result of every case must be bit-identical alone and in a heterogeneous
batch, in both precisions, with or without the captured graph, after the
tuner has changed launch shapes, and while other cases join, leave or sleep.
"""
import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def hb():
    import paper_2605_03479_amd as m
    m.load_library()
    return m


CASES = [
    (Case(12, 10, 16, 4.0, 1.0, 1.0, 1, hbcases.lid_walls(0.01), Pr=1.0), 0),
    (Case(9, 11, 12, 5.0, 0.3, 2.0, 2, hbcases.thermal_walls(0.4, 0, "sin")), 1),
    (Case(16, 16, 20, 4.0, 0.05, 0.5, 3, hbcases.lid_walls(0.02)), 0),
    (Case(10, 8, 16, 4.0, 5.0, 8.0, 1, hbcases.lid_walls(0.01)), 1),
    (Case(7, 7, 24, 5.0, 1.0, 1.0, 4, hbcases.thermal_walls(0.2, 2, "cos")), 1),
    # Gauss-Hermite velocities on a wall-refined mesh
    (Case(10, 9, 14, 0.0, 0.1, 3.0, 1, hbcases.lid_walls(0.01), x_faces=hbcases.stretched_faces(10, 1.0, 0.02),
          y_faces=hbcases.stretched_faces(9, 1.0, 0.02), vrule=1), 0),
    # rectangular velocity grids: wider along v (mixed), wider along u (FP64)
    (Case(8, 10, 12, 4.0, 0.5, 2.0, 1, hbcases.lid_walls(0.01), Mv=20, vmax=5.0), 1),
    (Case(9, 8, 22, 5.0, 0.2, 1.0, 2, hbcases.thermal_walls(0.3, 0, "sin"), Mv=10, vmax=4.0), 0),
]


def _solo(hb, case, prec, steps):
    s = hb.Solver(case, precision=prec)
    s.step(steps)
    out = s.state(), s.residual()
    s.close()
    return out


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batch_matches_solo_bitwise(hb):
    steps = 7
    B = hb.Batch(max_cases=8, pool_bytes=1 << 30)
    bc = [B.add(c, p) for c, p in CASES]
    B.step(steps)
    res = B.residuals()
    for (case, prec), h in zip(CASES, bc):
        st, r = _solo(hb, case, prec, steps)
        assert _same(h.state(), st), (case, prec)
        assert np.array_equal(h.residual(), r)
        assert np.array_equal(res[h.cid][0], r) and res[h.cid][1] == steps
        _say(f"  case {h.cid} ({case.nx}x{case.ny}, M={case.M}, NH={case.NH}, prec={prec}): bit-identical")
    B.close()


def test_graph_replays_match_eager_every_step(hb):
    A = hb.Batch(max_cases=8, pool_bytes=1 << 30)
    E = hb.Batch(max_cases=8, pool_bytes=1 << 30)
    E.use_graph(False)
    ca = [A.add(c, p) for c, p in CASES[:3]]
    ce = [E.add(c, p) for c, p in CASES[:3]]
    for k in range(5):
        A.step(1)  # graph replay
        E.step(1)  # direct launches
        for x, y in zip(ca, ce):
            assert _same(x.state(), y.state()), k  # synchronises between replays
    A.close()
    E.close()


def test_membership_changes_keep_results(hb):
    B = hb.Batch(max_cases=8, pool_bytes=1 << 30)
    c0 = B.add(*CASES[0])
    c1 = B.add(*CASES[1])
    B.step(3)
    c2 = B.add(*CASES[2])  # joins late
    B.set_active(c1, False)  # sleeps for 2 steps
    B.step(2)
    B.set_active(c1, True)
    B.remove(c0)  # leaves
    B.step(2)
    assert _same(c1.state(), _solo(hb, *CASES[1], 5)[0])
    assert _same(c2.state(), _solo(hb, *CASES[2], 4)[0])
    assert c1.step_index() == 5 and c2.step_index() == 4
    B.close()


def test_pool_admission_by_footprint(hb):
    case, prec = CASES[2]
    B = hb.Batch(max_cases=8, pool_bytes=64 << 20)
    need = B.case_bytes(case, prec)
    cap, used, _ = B.pool_info()
    assert used == 0 and need > 0
    n = 0
    while True:
        try:
            B.add(case, prec)
        except hb.HBError as e:
            assert e.code == hb.HB_ENOMEM
            break
        n += 1
        assert B.pool_info()[1] == n * need
        assert n < 8
    assert n == cap // need
    B.close()


def test_tuned_shapes_keep_results(hb):
    B = hb.Batch(max_cases=8, pool_bytes=1 << 30)
    bc = [B.add(c, p) for c, p in CASES]
    B.tune(2)  # takes one batch step
    shapes = B.shapes()
    _say("  tuned update shapes:", shapes)
    assert {(s["precision"], s["NT"]) for s in shapes} == {(p, c.NT) for c, p in CASES}
    assert all(s["threads"] in (64, 128, 256) for s in shapes)
    B.step(4)
    for (case, prec), h in zip(CASES, bc):
        assert _same(h.state(), _solo(hb, case, prec, 5)[0])
    B.close()


def test_streaming_store_case_matches_solo(hb):
    """A mixed case whose state exceeds 128 MiB (48^2 cells x 48^2 velocities x
    9 levels: 382 MB of FP32 h and b) stores its update non-temporally, in the
    single-case kernels through buffer resources and in the batched ones
    through global stores; beside a small cached-store case in one batch it
    must still give the bits it gives alone."""
    big = Case(48, 48, 48, 5.0, 1.0, 1.0, 4, hbcases.thermal_walls(0.5, 0, "sin"))
    small = CASES[1]
    assert big.nc * big.NT * 4 * 576 * 2 * 4 > 128 << 20
    B = hb.Batch(max_cases=2, pool_bytes=2 << 30)
    hb_big = B.add(big, hb.HB_MIXED)
    hb_small = B.add(*small)
    B.step(4)
    assert _same(hb_big.state(), _solo(hb, big, hb.HB_MIXED, 4)[0])
    assert _same(hb_small.state(), _solo(hb, *small, 4)[0])
    B.close()
