"""What the learned warm start gains (marker: gpu).

Trains the warm-start network on the GPU (project kernels: forward,
backward, Adam) from 2048 cold solves of the n=32, l=4, dp=1, d=2 family
(labels: the iterate at relative gap 1e-1), then solves 128 held-out systems
warm and cold.  The warm runs must give every held-out system the cold
verdict (the library falls back to a cold solve when a warm run is not
certified) and must need fewer IPM iterations on average, fallbacks
included.
"""
import numpy as np
import pytest

from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_learned_warm_start_gain():
    from paper_1411_3769_amd import learned as Lm
    from paper_1411_3769_amd import polyaipm as P
    P.load()
    log = lambda m: print(m, flush=True)
    tr = [W.warm_system(s) for s in range(2048)]
    te = [W.warm_system(10**6 + s) for s in range(128)]
    dtr = Lm.solve_cold(tr, log=log)
    dte = Lm.solve_cold(te, log=log)
    assert dtr.reached.all()
    model = Lm.train(dtr, K=2112, epochs=100, log=log)
    assert model.history[-1] < 0.7 * model.history[0]
    ev = Lm.evaluate(model, te, dte, log=log)
    log(str(ev))
    assert ev["verdicts_agree"] == ev["systems"]
    assert ev["warm_iters_mean"] < ev["cold_iters_mean"] - 2.0
    model.net.close()
