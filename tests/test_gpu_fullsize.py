"""Full-size parity at the benchmarked configurations (bitwise FP64 against the
CPU oracle run with all host threads)."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


# ("ab", 5) is the headline bench configuration (4 x 8 tile, one 514-plane
# segment per tile column).
@pytest.mark.parametrize("layout,t", [("ab", 5), ("ab", 3), ("compressed", 5), ("ab", 0)])
def test_512cube_200_sweeps_bitwise(layout, t):
    from paper_1006_3148_amd import Jacobi
    print("case 512^3 x 200 %s t=%d" % (layout, t), flush=True)
    box = synth.uniform_box(512, 512, 512, seed=2)
    j = Jacobi(box, t=t, layout=layout)
    j.sweep(200)
    got = j.box()
    info = j.info()
    j.close()
    if layout == "ab" and t == 5:
        # the planner keeps the 4 x 8 tile here (one generation of 240 tiles)
        assert info["tile_rows"] == 32, info
    want = oracle.sweeps_f64(box, 200)
    assert _same(got, want)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("layout,t,sweeps", [("compressed", 4, 16), ("compressed", 5, 16),
                                             ("ab", 5, 15)])
def test_1024cube_bitwise(layout, t, sweeps):
    from paper_1006_3148_amd import Jacobi
    print("case 1024^3 %s t=%d x %d" % (layout, t, sweeps), flush=True)
    box = synth.sine_face_box(1024, 1024, 1024, seed=3)
    j = Jacobi(box, t=t, layout=layout)
    j.sweep(sweeps)
    got = j.box()
    info = j.info()
    j.close()
    if layout == "ab" and t == 5:
        # the planner picks the 3 x 12 tile here (3 rounds of one segment)
        assert info["tile_rows"] == 36, info
    want = oracle.sweeps_f64(box, sweeps)
    del box
    assert _same(got, want)


def test_batched_256_problems_500_sweeps_bitwise():
    from paper_1006_3148_amd import JacobiBatch
    print("case batched 256 x 500", flush=True)
    probs = list(synth.batch_problems(256, 4))
    boxes = [p[3] for p in probs]
    b = JacobiBatch(boxes, t=0)
    b.sweep(500)
    bad = []
    for q, box in enumerate(boxes):
        if not _same(b.box(q), oracle.sweeps_f64(box, 500)):
            bad.append((q, probs[q][:3]))
    b.close()
    assert not bad, bad[:5]
