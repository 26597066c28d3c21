"""Several trips in one persistent launch (teams, per-tile counters of
completed trips, looseness d_u) against the CPU oracle: bitwise FP64 for
every t, looseness and team count, with remainder trips, several k segments
and ragged tiles; graph replay; the bounded spin forced from the host."""

import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _run(box, n, **kw):
    from paper_1006_3148_amd import Jacobi
    j = Jacobi(box, **kw)
    j.sweep(n)
    out = j.box()
    j.close()
    return out


def _assert_same(got, want, what):
    if not np.array_equal(got.view(np.uint64), want.view(np.uint64)):
        diff = np.argwhere(got != want)
        raise AssertionError("%s: %d cells differ, first at (k,j,i)=%s" %
                             (what, len(diff), tuple(diff[0])))


@pytest.mark.parametrize("looseness", [-1, 0, 1, 3])
@pytest.mark.parametrize("t", [1, 3, 5, 8])
@pytest.mark.parametrize("dims", [(70, 45, 37), (130, 67, 21), (3, 2, 5)])
def test_teams_bitwise(dims, t, looseness):
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=400 + t)
    n = 5 * t + 2   # two launches of teams (3 + 2 trips) and a remainder trip
    print("case teams dims=%s t=%d d_u=%d n=%d" % (dims, t, looseness, n), flush=True)
    want = oracle.sweeps_f64(box, n)
    got = _run(box, n, t=t, teams=3, looseness=looseness)
    _assert_same(got, want, "teams dims=%s t=%d d_u=%d" % (dims, t, looseness))


def test_teams_many_segments_and_tile_shapes():
    box = synth.uniform_box(150, 97, 41, seed=410)
    for t, rows, rpw, seg in ((4, 36, 3, 9), (5, 32, 4, 11), (2, 64, 4, 5)):
        n = 6 * t + 1
        print("case teams 150x97x41 t=%d rows=%d seg=%d" % (t, rows, seg), flush=True)
        want = oracle.sweeps_f64(box, n)
        got = _run(box, n, t=t, tile_rows=rows, rows_per_wave=rpw, seg_len=seg,
                   teams=6, looseness=-1)
        _assert_same(got, want, "teams t=%d rows=%d" % (t, rows))


def test_teams_single_sweep_64cube_100_sweeps():
    """The 64^3 x 100 single-sweep configuration as 100 teams of t=1 in one
    launch."""
    box = synth.uniform_box(64, 64, 64, seed=1)
    print("case teams 64^3 x 100 t=1", flush=True)
    want = oracle.sweeps_f64(box, 100)
    got = _run(box, 100, t=1, teams=100, looseness=-1)
    _assert_same(got, want, "64^3 teams t=1")


def test_teams_graph_replay():
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(90, 61, 33, seed=31)
    print("case teams graph replay 90x61x33", flush=True)
    g = Jacobi(box, t=4, use_graph=True, teams=4, looseness=1)
    total = 0
    for n in (17, 17, 9, 17):
        g.sweep(n)
        total += n
        g.residual()
        _assert_same(g.box(), oracle.sweeps_f64(box, total), "teams graph %d" % total)
    g.close()


def test_teams_timeout_forced_from_host():
    """Spin bound 1: some wait gives up, the kernel exits normally and the
    handle reports JACOBI_ETIMEOUT; a fresh handle is bitwise again."""
    from paper_1006_3148_amd._lib import JacobiError
    box = synth.uniform_box(300, 200, 90, seed=22)
    print("case teams spin bound 1, 300x200x90", flush=True)
    from paper_1006_3148_amd import Jacobi
    timed_out = False
    os.environ["JACOBI_SPIN_LIMIT"] = "1"
    try:
        for _ in range(3):
            j = Jacobi(box, t=3, teams=4, looseness=0)
            try:
                j.sweep(12)
                j.sync()
            except JacobiError as e:
                assert e.code == -5, e
                timed_out = True
            j.close()
            if timed_out:
                break
    finally:
        del os.environ["JACOBI_SPIN_LIMIT"]
    assert timed_out
    want = oracle.sweeps_f64(box, 12)
    _assert_same(_run(box, 12, t=3, teams=4, looseness=0), want, "after timeout")
