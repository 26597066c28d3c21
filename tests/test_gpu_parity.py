"""GPU parity of the HIP trip kernels against the CPU oracle (bitwise FP64).

Sizes span several tiles in i and j, several k segments and ragged tails;
degenerate boxes (1-cell dims) and sweep counts that are not multiples of t
(remainder trips) are included.  Every case prints its name before running.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _bits(a):
    return a.view(np.uint64)


def _run(box, n, **kw):
    from paper_1006_3148_amd import Jacobi
    j = Jacobi(box, **kw)
    j.sweep(n)
    out = j.box()
    info = j.info()
    j.close()
    return out, info


def _assert_same(got, want, what):
    if not np.array_equal(_bits(got), _bits(want)):
        diff = np.argwhere(got != want)
        raise AssertionError("%s: %d cells differ, first at (k,j,i)=%s: got %r "
                             "want %r" % (what, len(diff), tuple(diff[0]),
                                          got[tuple(diff[0])], want[tuple(diff[0])]))


DIMS = [(70, 45, 37), (1, 1, 1), (3, 2, 5), (130, 67, 21), (64, 64, 64)]


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dims", DIMS)
def test_ab_trips_bitwise(t, dims):
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=100 + t)
    n = 2 * t + 1
    print("case ab t=%d dims=%s n=%d" % (t, dims, n), flush=True)
    want = oracle.sweeps_f64(box, n)
    got, _ = _run(box, n, t=t, layout="ab")
    _assert_same(got, want, "ab t=%d %s" % (t, dims))


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dims", [(70, 45, 37), (2, 3, 1), (130, 67, 40)])
def test_compressed_trips_bitwise(t, dims):
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=200 + t)
    # 3t+2 sweeps: forward and backward trips plus a short trip that brings the
    # shift offset back before a full backward trip.
    n = 3 * t + 2
    print("case compressed t=%d dims=%s n=%d" % (t, dims, n), flush=True)
    want = oracle.sweeps_f64(box, n)
    got, _ = _run(box, n, t=t, layout="compressed")
    _assert_same(got, want, "compressed t=%d %s" % (t, dims))


@pytest.mark.parametrize("layout", ["ab", "compressed"])
@pytest.mark.parametrize("t", [1, 3, 5, 8])
@pytest.mark.parametrize("dims", [(70, 45, 37), (2, 3, 1)])
def test_full_random_box_bitwise(layout, t, dims):
    """Every cell random: a nonzero starting interior, and edges and corners of
    the boundary layer that the 7-point update never reads but must pass
    through unchanged."""
    box = synth.full_random_box(*dims, seed=500 + t)
    n = 2 * t + 1
    print("case full random %s t=%d dims=%s n=%d" % (layout, t, dims, n), flush=True)
    got, _ = _run(box, n, t=t, layout=layout)
    _assert_same(got, oracle.sweeps_f64(box, n), "full random %s t=%d %s" % (layout, t, dims))


@pytest.mark.parametrize("t,dims,seg_len", [
    (5, (70, 45, 37), 0),       # E = 2t, one k segment
    (5, (130, 67, 90), 30),     # E = 2t, three segments of 30 planes
    (4, (70, 45, 60), 11),      # E capped at seg_len - 2t = 3
    (3, (41, 70, 52), 0),
    (6, (70, 45, 37), 0),       # t > 5: backward trips stream upwards, E = 0
])
def test_compressed_uneven_calls_bitwise(t, dims, seg_len):
    """Compressed trips over sweep counts that are not multiples of t, in
    uneven calls: remainder trips, trips the planner shortens to keep both
    shift offsets in range, backward trips in the k-mirrored view and the
    extra shift along k (planes of shift room per the layout)."""
    from paper_1006_3148_amd import Jacobi
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=400 + t)
    calls = [1, 7, 3, 2 * t, 5, 1, 4 * t + 3]
    print("case compressed uneven t=%d dims=%s seg_len=%d calls=%s"
          % (t, dims, seg_len, calls), flush=True)
    j = Jacobi(box, t=t, layout="compressed", seg_len=seg_len)
    done = 0
    for c in calls:
        j.sweep(c)
        done += c
        _assert_same(j.box(), oracle.sweeps_f64(box, done),
                     "compressed uneven t=%d %s after %d" % (t, dims, done))
    j.close()


@pytest.mark.parametrize("env", [{"JACOBI_KREV": "0"}, {"JACOBI_XCD_ORDER": "0"},
                                 {"JACOBI_ZEXTRA": "0"}])
def test_compressed_variants_same_bits(env, monkeypatch):
    """Backward trips streaming upwards (no extra k shift), one ticket counter
    instead of the per-XCD claim groups, and no extra k shift all give the
    default path's bits."""
    box = synth.uniform_box(130, 67, 60, seed=431)
    n = 23
    print("case compressed variant %s" % env, flush=True)
    want, _ = _run(box, n, t=5, layout="compressed")
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    got, _ = _run(box, n, t=5, layout="compressed")
    _assert_same(got, want, "compressed variant %s" % env)
    _assert_same(got, oracle.sweeps_f64(box, n), "compressed variant %s vs oracle" % env)


@pytest.mark.parametrize("t,dims,seg_len", [(5, (300, 250, 60), 8), (4, (200, 130, 90), 4)])
def test_ab_band_order_bitwise(t, dims, seg_len, monkeypatch):
    """A/B trips with several generations of workgroups (more tiles than CUs)
    take tiles in band order with a split tail: bitwise the oracle and the
    one-range-per-XCD order."""
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=500 + t)
    n = 2 * t + 3
    print("case ab band order t=%d dims=%s seg_len=%d" % (t, dims, seg_len), flush=True)
    got, info = _run(box, n, t=t, layout="ab", seg_len=seg_len)
    _assert_same(got, oracle.sweeps_f64(box, n), "ab band order t=%d %s" % (t, dims))
    monkeypatch.setenv("JACOBI_AB_BANDS", "0")
    ranges, _ = _run(box, n, t=t, layout="ab", seg_len=seg_len)
    _assert_same(got, ranges, "ab band order vs ranges t=%d %s" % (t, dims))


def _compiled_shapes():
    from paper_1006_3148_amd.solver import tile_supported
    out = []
    for t in range(1, 9):
        for rpw in (2, 3, 4):
            for waves in (8, 12, 16):
                if tile_supported(t, rpw * waves, rpw):
                    out.append((t, rpw * waves, rpw))
    return out


@pytest.mark.parametrize("layout", ["ab", "compressed"])
def test_every_compiled_tile_shape_bitwise(layout):
    """Each compiled (t, rows, rows per wave) kernel on a box of several tiles
    in i and j with ragged tails and several k segments."""
    box = synth.uniform_box(150, 97, 41, seed=300)
    shapes = _compiled_shapes()
    assert len(shapes) >= 20
    for t, rows, rpw in shapes:
        n = 3 * t + 2
        print("case %s t=%d rows=%d rpw=%d n=%d" % (layout, t, rows, rpw, n), flush=True)
        want = oracle.sweeps_f64(box, n)
        got, info = _run(box, n, t=t, layout=layout, tile_rows=rows,
                         rows_per_wave=rpw, seg_len=max(2 * t, 13))
        _assert_same(got, want, "%s t=%d rows=%d rpw=%d" % (layout, t, rows, rpw))


def test_single_sweep_config_64cube_100_sweeps():
    box = synth.uniform_box(64, 64, 64, seed=1)
    print("case 64^3 x 100, t=1", flush=True)
    want = oracle.sweeps_f64(box, 100)
    got, _ = _run(box, 100, t=1, layout="ab")
    _assert_same(got, want, "64^3 t=1")


def test_residual_matches_oracle_and_is_deterministic():
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(90, 70, 50, seed=7)
    print("case residual 90x70x50", flush=True)
    j = Jacobi(box, t=4)
    j.sweep(9)
    r1, m1 = j.residual()
    r2, m2 = j.residual()
    u = j.box()
    j.close()
    assert r1 == r2 and m1 == m2
    ro = oracle.residual_norm(u)
    assert abs(r1 - ro) <= 1e-12 * ro
    assert m1 == float(np.max(np.abs(oracle.residual_f64(u))))


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 1), (61, 16, 3), (62, 17, 4),
                                  (63, 15, 33), (125, 47, 20)])
def test_residual_block_edges_match_oracle(dims):
    """The residual's blocks are 62 i-columns (lanes 0 and 63 the halo) by 16
    j-rows (4 waves of 4) by a k segment: boxes one cell wide, widths around
    62 and heights around 16 exercise the clamped halo lanes and rows."""
    from paper_1006_3148_amd import Jacobi
    box = synth.full_random_box(*dims, seed=600 + sum(dims))
    print("case residual %s" % (dims,), flush=True)
    j = Jacobi(box, t=2)
    r1, m1 = j.residual()
    j.sweep(3)
    r2, m2 = j.residual()
    u = j.box()
    j.close()
    for r, m, field in ((r1, m1, box), (r2, m2, u)):
        ro = oracle.residual_norm(field)
        assert abs(r - ro) <= 1e-12 * ro, (dims, r, ro)
        assert m == float(np.max(np.abs(oracle.residual_f64(field)))), dims


@pytest.mark.parametrize("layout", ["ab", "compressed"])
def test_split_of_sweeps_does_not_change_bits(layout):
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(50, 41, 33, seed=9)
    print("case split", layout, flush=True)
    j = Jacobi(box, t=4, layout=layout)
    for n in (1, 5, 3, 4, 2):
        j.sweep(n)
    got = j.box()
    j.close()
    _assert_same(got, oracle.sweeps_f64(box, 15), "split " + layout)


@pytest.mark.parametrize("layout", ["ab", "compressed"])
def test_f32_refined_matches_oracle(layout):
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(40, 33, 29, seed=12)
    m_in, outer = 6, 3
    print("case f32 refined", layout, flush=True)
    want = oracle.refine_f32(box, m_in, outer)
    j = Jacobi(box, t=4, layout=layout, dtype="f32_refined", inner_sweeps=m_in)
    j.sweep(m_in * outer)
    got = j.box()
    j.close()
    _assert_same(got, want, "f32 refined " + layout)


@pytest.mark.parametrize("layout", ["ab", "compressed"])
def test_solve_to_tolerance_matches_oracle(layout):
    """Run to ||r|| <= 1e-8 ||r0|| checking every 64 sweeps: the same sweep
    count and the same field, bit for bit, as the oracle's driver."""
    from paper_1006_3148_amd import Jacobi
    box = synth.sine_face_box(30, 26, 22, seed=3)
    print("case solve %s 30x26x22" % layout, flush=True)
    want, wdone, wrn, r0 = oracle.solve_to_tol(box, 1e-8, check_every=64, max_sweeps=20000)
    j = Jacobi(box, t=4, layout=layout)
    done, fin = j.solve(1e-8, 20000, 64)
    got = j.box()
    j.close()
    assert done == wdone and 0 < done < 20000
    _assert_same(got, want, "solve %s" % layout)
    assert abs(fin - wrn) <= 1e-12 * wrn
    # an unreachable tolerance stops at max_sweeps (not a multiple of the check)
    want2, wdone2, _, _ = oracle.solve_to_tol(box, 1e-300, check_every=64, max_sweeps=150)
    j = Jacobi(box, t=4, layout=layout)
    done2, _ = j.solve(1e-300, 150, 64)
    got2 = j.box()
    j.close()
    assert done2 == wdone2 == 150
    _assert_same(got2, want2, "solve cap %s" % layout)


def test_compressed_spin_bound_reports_timeout_and_recovers():
    """With the progress-wait spin bound forced to 1 from the host, a waiting
    tile gives up, the kernel still exits normally and the call reports
    JACOBI_ETIMEOUT; a handle made afterwards with the normal bound is exact."""
    import os
    from paper_1006_3148_amd import Jacobi
    from paper_1006_3148_amd._lib import JacobiError
    box = synth.uniform_box(300, 200, 90, seed=21)
    print("case spin bound 1, compressed 300x200x90", flush=True)
    timed_out = False
    os.environ["JACOBI_SPIN_LIMIT"] = "1"
    try:
        for _ in range(3):
            j = Jacobi(box, t=4, layout="compressed", seg_len=8)
            try:
                j.sweep(8)
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
    want = oracle.sweeps_f64(box, 8)
    got, _ = _run(box, 8, t=4, layout="compressed", seg_len=8)
    _assert_same(got, want, "after timeout")


def test_graph_replay_matches_eager_every_call():
    """A/B FP64 sweeps replayed from captured graphs (two starting grids, two
    sweep counts) with eager work and synchronisation between the calls: each
    call is checked against an eager handle."""
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(90, 61, 33, seed=31)
    print("case graph replay 90x61x33", flush=True)
    g = Jacobi(box, t=4, use_graph=True)
    e = Jacobi(box, t=4)
    total = 0
    for n in (9, 9, 9, 5, 9, 5):
        g.sweep(n)
        e.sweep(n)
        total += n
        gl2, _ = g.residual()
        el2, _ = e.residual()
        g.sync()
        e.sync()
        _assert_same(g.box(), e.box(), "graph after %d sweeps" % total)
        assert gl2 == el2
        assert g.info()["sweeps"] == total
    _assert_same(g.box(), oracle.sweeps_f64(box, total), "graph vs oracle")
    g.close()
    e.close()


def test_solve_with_graph_replay_matches_eager():
    """Run-to-tolerance on a handle that replays captured graphs: the same
    sweep count and field as the eager handle and the oracle."""
    from paper_1006_3148_amd import Jacobi
    box = synth.sine_face_box(28, 21, 25, seed=8)
    print("case solve with graphs 28x21x25", flush=True)
    want, wdone, wrn, _ = oracle.solve_to_tol(box, 1e-8, check_every=48, max_sweeps=20000)
    g = Jacobi(box, t=5, use_graph=True)
    done, fin = g.solve(1e-8, 20000, 48)
    got = g.box()
    g.close()
    assert done == wdone
    _assert_same(got, want, "solve with graphs")
    assert abs(fin - wrn) <= 1e-12 * wrn


def test_autotune_t0_picks_fastest_and_stays_bitwise():
    """t=0 (A/B FP64): the first call of >= 96 sweeps times every candidate on
    real sweeps, keeps the fastest, and the result is bitwise the plain
    sweeps."""
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(150, 97, 41, seed=320)
    print("case autotune t=0 150x97x41", flush=True)
    j = Jacobi(box, t=0)
    j.sweep(10)                    # below the tuning threshold: default t
    assert j.tune_log()[0] == []
    j.sweep(200)
    log, ms = j.tune_log()
    info = j.info()
    got = j.box()
    j.close()
    assert len(log) == 6 and ms > 0
    best = max(log, key=lambda e: e["glups"])
    assert (info["t"], info["tile_rows"]) == (best["t"], best["tile_rows"])
    _assert_same(got, oracle.sweeps_f64(box, 210), "autotune t=0")
