"""GPU parity of the batched persistent launch (bitwise per problem against the
oracle run alone), autotuned and fixed configurations, graph and eager."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _problems(count, seed, lo=3, step=7, nsteps=10):
    return [(nx, ny, nz, box) for nx, ny, nz, box in
            synth.batch_problems(count, seed, lo=lo, step=step, nsteps=nsteps)]


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("t,use_graph", [(3, True), (5, False), (1, True), (0, True)])
def test_batch_f64_bitwise(t, use_graph):
    from paper_1006_3148_amd import JacobiBatch
    probs = _problems(11, seed=40 + t)
    boxes = [p[3] for p in probs]
    print("case batch f64 t=%d graph=%s dims=%s" % (t, use_graph,
                                                    [p[:3] for p in probs]), flush=True)
    b = JacobiBatch(boxes, t=t, use_graph=use_graph)
    # two calls with the same n (graph replay) and one with a different n
    plan = [40, 40, 7]
    for n in plan:
        b.sweep(n)
    total = sum(plan)
    l2, mx = b.residual()
    for q, box in enumerate(boxes):
        want = oracle.sweeps_f64(box, total)
        got = b.box(q)
        assert _same(got, want), "problem %d %s differs" % (q, probs[q][:3])
        ro = oracle.residual_norm(want)
        assert abs(l2[q] - ro) <= 1e-12 * max(ro, 1e-300)
    info = b.info()
    assert info["sweeps"] == total
    if t == 0:
        log = b.tune_log()
        assert len(log) >= 1 and all(e["glups"] > 0 for e in log)
    b.close()


def test_batch_f32_refined_bitwise():
    from paper_1006_3148_amd import JacobiBatch
    probs = _problems(7, seed=77)
    boxes = [p[3] for p in probs]
    m_in, outer = 5, 3
    print("case batch f32 refined", [p[:3] for p in probs], flush=True)
    b = JacobiBatch(boxes, t=0, dtype="f32_refined", inner_sweeps=m_in)
    b.sweep(m_in * outer)
    for q, box in enumerate(boxes):
        want = oracle.refine_f32(box, m_in, outer)
        assert _same(b.box(q), want), "problem %d differs" % q
    b.close()


def test_batch_equals_standalone_handles():
    from paper_1006_3148_amd import Jacobi, JacobiBatch
    probs = _problems(5, seed=5, lo=20, step=16, nsteps=4)
    boxes = [p[3] for p in probs]
    print("case batch vs standalone", [p[:3] for p in probs], flush=True)
    b = JacobiBatch(boxes, t=4)
    b.sweep(13)
    for q, box in enumerate(boxes):
        j = Jacobi(box, t=2)
        j.sweep(13)
        assert _same(b.box(q), j.box())
        j.close()
    b.close()


def test_batch_graph_replays_each_match_eager():
    """Several replays of one captured schedule, with eager work and
    synchronisation between them; every replay is checked against the same
    schedule run eagerly."""
    from paper_1006_3148_amd import JacobiBatch
    probs = _problems(6, seed=91)
    boxes = [p[3] for p in probs]
    print("case batch graph replays", [p[:3] for p in probs], flush=True)
    g = JacobiBatch(boxes, t=4, use_graph=True)
    e = JacobiBatch(boxes, t=4, use_graph=False)
    for rep in range(4):
        g.sweep(9)
        e.sweep(9)
        gl2, _ = g.residual()   # eager work between replays
        el2, _ = e.residual()
        g.sync()
        e.sync()
        for q in range(len(boxes)):
            assert _same(g.box(q), e.box(q)), "replay %d problem %d" % (rep, q)
        assert np.array_equal(np.asarray(gl2), np.asarray(el2))
    want = oracle.sweeps_f64(boxes[0], 36)
    assert _same(g.box(0), want)
    g.close()
    e.close()


def test_batch_solve_counts_match_oracle():
    from paper_1006_3148_amd import JacobiBatch
    boxes = [synth.sine_face_box(n1, n2, n3, seed=60 + q)
             for q, (n1, n2, n3) in enumerate([(20, 17, 23), (31, 12, 18), (9, 9, 9),
                                                (26, 30, 14)])]
    print("case batch solve", [b.shape for b in boxes], flush=True)
    b = JacobiBatch(boxes, t=3)
    done, fin = b.solve(1e-8, 20000, 32)
    b.close()
    for q, box in enumerate(boxes):
        _, wdone, wrn, _ = oracle.solve_to_tol(box, 1e-8, check_every=32, max_sweeps=20000)
        assert done[q] == wdone, (q, done[q], wdone)
        assert abs(fin[q] - wrn) <= 1e-12 * wrn
