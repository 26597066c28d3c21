"""What the trained network's guess saves on held-out problems, against the
zero start and against the non-learned face blend that the network corrects
(small-scale version of the 128^3 experiment run by
``python -m paper_1006_3148_amd.learned``).

The gain over the zero start is significant.  Against the blend the network
is on par: at 128^3 (64 held-out problems) it saves 320 +/- 916 sweeps
(CI95), not a significant gain.  The test therefore asserts the gain over
the zero start and that the learned start is not significantly worse than
the blend, and prints the paired learned-vs-blend difference."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_learned_guess_saves_sweeps():
    from paper_1006_3148_amd import GuessNet, init_params, learned
    n, levels, pmax = 32, 3, 4
    print("case learned gain n=32", flush=True)
    U, basis = learned.solve_basis(n, pmax, check_every=128)
    assert basis["converged"]
    net = GuessNet(n, levels, init_params(levels, 2))
    tr = learned.train(net, U, n, pmax, list(range(1000, 1768)), epochs=5, lr=3e-3,
                       accum=2, val_seeds=list(range(5000, 5016)))
    print("train", tr["train_loss"], tr["val_rel_mse"], flush=True)
    assert tr["train_loss"][-1] < tr["train_loss"][0]
    assert tr["val_rel_mse"] < 0.2
    ev = learned.evaluate(net, n, list(range(900000, 900032)), check_every=32,
                          single=1)
    print({k: v for k, v in ev.items() if not isinstance(v, list)}, flush=True)
    assert ev["all_converged"]
    # fewer sweeps than the zero start, beyond the 95% interval of the mean
    assert ev["sweeps_saved_mean"] > ev["sweeps_saved_ci95"] > 0
    assert ev["sweeps_learned_mean"] < ev["sweeps_zero_mean"]
    # against the blend: report the paired difference; the learned start must
    # not be significantly worse (a significant gain is not claimed)
    vb, ci = ev["sweeps_saved_vs_blend_mean"], ev["sweeps_saved_vs_blend_ci95"]
    print("learned vs blend: %.1f +/- %.1f sweeps saved (CI95), %d/%d problems better"
          % (vb, ci, ev["problems_better_than_blend"], ev["problems"]), flush=True)
    assert vb > -ci, (vb, ci)
