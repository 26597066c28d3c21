"""The multigrid correction solve (weighted-Jacobi smoother in an FP32
V-cycle inside the FP64 defect correction) against the oracle: bitwise
after one and several outer steps, the same outer-step count to a 1e-10
relative residual, and the closed-form solution within the residual bound."""

import numpy as np
import pytest

import oracle
import synth
from oracle import multigrid as omg
from tests import closed_form as cf

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("n,steps", [(3, 2), (7, 1), (15, 2), (31, 3), (63, 2), (127, 1), (255, 2), (511, 1)])
def test_multigrid_steps_bitwise(n, steps):
    from paper_1006_3148_amd import Jacobi
    print("case multigrid n=%d steps=%d" % (n, steps), flush=True)
    box = synth.sine_face_box(n, n, n, seed=40 + n)
    j = Jacobi(box, dtype="f32_multigrid")
    j.sweep(steps)
    got = j.box()
    j.close()
    want = omg.mg_refine(box, steps)
    assert _same(got, want), np.max(np.abs(got - want))


def test_multigrid_solve_matches_oracle_and_closed_form():
    from paper_1006_3148_amd import Jacobi
    n = 31
    print("case multigrid solve n=31", flush=True)
    box = synth.sine_face_box(n, n, n, seed=7)
    j = Jacobi(box, dtype="f32_multigrid")
    r0, _ = j.residual()
    done, fin = j.solve(1e-10, 40, 1, r0)
    got = j.box()
    j.close()
    u, k = box, 0
    while oracle.residual_norm(u) > 1e-10 * r0 and k < 40:
        u, _s, _m = omg.mg_outer(u)
        k += 1
    assert done == k and _same(got, u)
    ustar = cf.harmonic_from_sine_faces(n, n, n, synth.sine_face_modes(7))
    err = np.linalg.norm((got - ustar)[1:-1, 1:-1, 1:-1])
    assert err <= cf.laplace_error_bound(n, n, n, fin) * 1.01 + 1e-12
