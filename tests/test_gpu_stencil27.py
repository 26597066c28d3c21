"""GPU parity of the 27-point trip kernels against the CPU oracle (bitwise
FP64): several tiles in i and j, several k segments, ragged tails, 1-cell
boxes, remainder trips, every compiled tile shape, uneven calls, graph
replay, and the full 512^3 box.  Every case prints its name before running."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _assert_same(got, want, what):
    if not _same(got, want):
        diff = np.argwhere(got != want)
        raise AssertionError("%s: %d cells differ, first at (k,j,i)=%s: got %r want %r"
                             % (what, len(diff), tuple(diff[0]), got[tuple(diff[0])],
                                want[tuple(diff[0])]))


def _run(box, calls, **kw):
    from paper_1006_3148_amd import Jacobi
    j = Jacobi(box, layout="ab", stencil=27, **kw)
    for n in calls:
        j.sweep(n)
    out = j.box()
    info = j.info()
    j.close()
    return out, info


@pytest.mark.parametrize("t", [1, 2, 3, 4])
@pytest.mark.parametrize("dims", [(70, 45, 37), (1, 1, 1), (3, 2, 5), (130, 67, 21),
                                  (64, 64, 64)])
def test_s27_trips_bitwise(t, dims):
    box = synth.uniform_box(*dims, seed=300 + t)
    n = 2 * t + 1  # two full trips and a remainder trip
    print("case s27 t=%d dims=%s n=%d" % (t, dims, n), flush=True)
    got, info = _run(box, [n], t=t)
    assert info["t"] == t
    _assert_same(got, oracle.sweeps27_f64(box, n), "s27 t=%d %s" % (t, dims))


@pytest.mark.parametrize("t", [1, 2, 3, 4])
@pytest.mark.parametrize("dims", [(70, 45, 37), (1, 1, 1), (2, 3, 1), (130, 67, 21)])
def test_s27_full_random_box_bitwise(t, dims):
    """Every cell random, the edges and corners of the boundary layer and the
    interior included: the update reads the box's edges and corners, which
    the boundary-only boxes above hold at zero."""
    box = synth.full_random_box(*dims, seed=340 + t)
    n = 2 * t + 1
    print("case s27 full random t=%d dims=%s n=%d" % (t, dims, n), flush=True)
    got, _ = _run(box, [n], t=t)
    _assert_same(got, oracle.sweeps27_f64(box, n), "s27 full random t=%d %s" % (t, dims))


SHAPES = [(1, 32, 4), (2, 32, 4), (2, 36, 3), (2, 32, 2), (3, 24, 3), (3, 32, 4),
          (4, 24, 3)]


@pytest.mark.parametrize("t,rows,rpw", SHAPES)
def test_s27_every_compiled_shape_bitwise(t, rows, rpw):
    dims = (130, 75, 40)
    box = synth.uniform_box(*dims, seed=310 + t)
    n = t + 1
    print("case s27 shape t=%d rows=%d rpw=%d n=%d" % (t, rows, rpw, n), flush=True)
    got, info = _run(box, [n], t=t, tile_rows=rows, rows_per_wave=rpw)
    assert info["tile_rows"] == rows
    _assert_same(got, oracle.sweeps27_f64(box, n), "s27 shape %s" % ((t, rows, rpw),))


@pytest.mark.parametrize("t,seg_len", [(2, 7), (3, 5), (4, 0)])
def test_s27_segments_and_uneven_calls_bitwise(t, seg_len):
    """Short k segments (k ghost planes between segments) and sweep counts
    split over uneven calls."""
    dims = (90, 70, 33)
    box = synth.sine_face_box(*dims, seed=320 + t)
    calls = [3, 1, 2 * t + 1, 4]
    print("case s27 segments t=%d seg_len=%d calls=%s" % (t, seg_len, calls), flush=True)
    got, _ = _run(box, calls, t=t, seg_len=seg_len)
    _assert_same(got, oracle.sweeps27_f64(box, sum(calls)), "s27 segments t=%d" % t)


def test_s27_graph_replay_matches_oracle_every_call():
    from paper_1006_3148_amd import Jacobi
    dims = (100, 60, 30)
    box = synth.uniform_box(*dims, seed=330)
    print("case s27 graph replay", flush=True)
    j = Jacobi(box, t=2, layout="ab", stencil=27, use_graph=True)
    want = box
    for q in range(3):
        j.sweep(5)
        want = oracle.sweeps27_f64(want, 5)
        _assert_same(j.box(), want, "s27 replay %d" % q)
    j.close()


def test_s27_autotune_t0_stays_bitwise():
    """t = 0 times the 27-point candidates on the first call's real sweeps
    (every candidate gives the same bits) and keeps the fastest."""
    from paper_1006_3148_amd import Jacobi
    dims = (120, 90, 50)
    box = synth.uniform_box(*dims, seed=332)
    print("case s27 autotune", flush=True)
    j = Jacobi(box, t=0, layout="ab", stencil=27)
    j.sweep(100)
    j.sweep(7)
    log, _ = j.tune_log()
    info = j.info()
    got = j.box()
    j.close()
    assert len(log) == 4 and {e["t"] for e in log} == {2, 3, 4}
    assert info["t"] in (2, 3, 4)
    _assert_same(got, oracle.sweeps27_f64(box, 107), "s27 autotune")


def test_s27_residual_is_refused():
    from paper_1006_3148_amd import Jacobi
    from paper_1006_3148_amd._lib import JacobiError
    box = synth.uniform_box(20, 20, 20, seed=331)
    j = Jacobi(box, t=2, layout="ab", stencil=27)
    with pytest.raises(JacobiError) as e:
        j.residual()
    assert e.value.code == -2
    j.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("t", [2, 3])
def test_s27_512cube_bitwise(t):
    print("case s27 512^3 t=%d" % t, flush=True)
    box = synth.uniform_box(512, 512, 512, seed=2)
    n = 4 * t
    got, info = _run(box, [n], t=t)
    # t=3: 261 tile columns, planned as a split trip (256 whole columns of
    # 514 planes, then the 5 left); t=2: equal segments
    assert (info["seg_len"] == 514) == (t == 3), info
    want = oracle.sweeps27_f64(box, n)
    assert _same(got, want)


@pytest.mark.timeout(600)
def test_s27_1024cube_bitwise():
    """The 1024^3 configuration the bench extra times (t=3, 3 rows x 8 waves,
    sine-mode faces): the whole field after two trips."""
    print("case s27 1024^3 t=3 x 6", flush=True)
    box = synth.sine_face_box(1024, 1024, 1024, seed=3)
    got, info = _run(box, [6], t=3, tile_rows=24, rows_per_wave=3)
    assert info["tile_rows"] == 24
    want = oracle.sweeps27_f64(box, 6)
    del box
    assert _same(got, want)


@pytest.mark.parametrize("t,dims,split", [
    (3, (70, 45, 37), "4"), (4, (70, 45, 37), "4"), (2, (130, 67, 21), "4"),
    (2, (200, 150, 90), "8"), (3, (150, 40, 300), "4"), (4, (64, 64, 64), "4"),
    (3, (120, 90, 50), "4"), (3, (70, 45, 37), "0"), (3, (1, 1, 1), "4")])
def test_s27_split_trips_bitwise(t, dims, split, monkeypatch):
    """Split trips: the first multiple-of-n tile columns run whole in one
    launch, the columns left in a second launch, cut into segments of at
    least 2t planes (JACOBI_KSPLIT=n forces it with rounds of n columns; 0
    turns it off); remainder trips and uneven calls included."""
    monkeypatch.setenv("JACOBI_KSPLIT", split)
    box = synth.full_random_box(*dims, seed=360 + t)
    calls = [2 * t + 1, 3]
    print("case s27 split=%s t=%d dims=%s calls=%s" % (split, t, dims, calls), flush=True)
    got, _ = _run(box, calls, t=t)
    _assert_same(got, oracle.sweeps27_f64(box, sum(calls)),
                 "s27 split=%s t=%d %s" % (split, t, dims))


def test_s27_split_graph_and_autotune_bitwise(monkeypatch):
    monkeypatch.setenv("JACOBI_KSPLIT", "4")
    from paper_1006_3148_amd import Jacobi
    box = synth.uniform_box(120, 90, 50, seed=362)
    print("case s27 split graph replay + autotune", flush=True)
    j = Jacobi(box, t=3, layout="ab", stencil=27, use_graph=True)
    want = box
    for q in range(3):
        j.sweep(7)
        want = oracle.sweeps27_f64(want, 7)
        _assert_same(j.box(), want, "s27 split replay %d" % q)
    j.close()
    j = Jacobi(box, t=0, layout="ab", stencil=27)
    j.sweep(100)
    j.sweep(7)
    got = j.box()
    j.close()
    _assert_same(got, oracle.sweeps27_f64(box, 107), "s27 split autotune")
