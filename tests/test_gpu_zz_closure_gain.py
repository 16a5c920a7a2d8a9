"""What the trained closure gains over the plain k = 1 scheme (the full
experiment, about two minutes on one GPU).

Data: a k = 2 run on 128^3 cells (turbulence surrogate at Mach 0.3 with the
driving), 16 snapshots restricted to k = 1 on 64^3; targets
c = R_c(P y_f) - P R_f(y_f).  Training: 3000 Adam steps, batch 4096, input
noise 0.1, all on the GPU through the library's kernels.  The correction scale
is chosen on a validation window; the test window comes after it in time.

Pass bar on the test window:
* the corrected operator is closer to the restricted fine operator than the
  plain one, in every field (a-priori);
* over the horizon (0.1 time units), the evolution of the corrected coarse run
  is closer to the restricted fine evolution than the plain run's, on average
  over the five fields (a-posteriori), and no field's evolution error exceeds
  the plain run's by more than 2% (the training is stochastic; the density
  row, whose correction is the smallest, may gain nothing), with the total mass
  conserved;
* accuracy per DOF: a plain k = 1 run with 8x the cells (the fine mesh, from
  the fine state's degree-1 modes) sets the other end of a DOF ladder; the
  closure's effective DOF gain per field is read off between the two plain
  runs and reported.
The outcome is stochastic training in FP32: parity is not claimed, only the gain.
"""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.timeout(600)
def test_closure_gains_over_plain_scheme():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_09079_amd import closure, dg
    dg.lib()
    res = closure.run(closure.Config(), log=lambda *a: print(*a, flush=True))
    print(json.dumps(res))
    hist = res["loss_history"]
    assert hist[-1][1] < 0.7 * hist[0][1]
    test = res["test"]
    plain = test["plain"]
    cl = test[f"alpha={res['alpha']}"]
    assert np.all(np.array(cl["rhs_err"]) < np.array(plain["rhs_err"])), (cl["rhs_err"], plain["rhs_err"])
    assert np.mean(cl["err"]) < np.mean(plain["err"]), (cl["err"], plain["err"])
    assert np.all(np.array(cl["err"]) <= 1.02 * np.array(plain["err"])), (cl["err"], plain["err"])
    assert cl["fallback_rate"] < 0.05
    # the DOF ladder: plain k = 1 with 8x the cells is closer to the reference in every field, and the
    # closure's effective DOF gain is read off between the two plain runs (reported unclipped: below 1
    # where the closure loses); it gains on some field
    assert np.all(np.array(test["plain_8x_dof"]["err"]) < np.array(plain["err"]))
    g = np.array(res["effective_dof_gain"])
    assert np.all(np.isfinite(g)) and np.max(g) > 1.0, g
    assert cl["totals_drift"][0] < 1e-5  # mass: the driving adds momentum and energy, never mass
