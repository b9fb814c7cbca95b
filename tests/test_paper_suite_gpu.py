"""The paper's own workloads (section 3) on the GPU: every run equals the FP64
oracle, and shows what the paper says it shows (circle and sphere radii
follow Eq. exactradiusEQ; the star's tips move in and its gaps out until it
is round; the torus' hole closes first and the disc left follows the circle
law; the 2D dumbbell shrinks but keeps its lobes and bar; the 3D dumbbell's
handle pinches off before the end spheres vanish; random starts separate)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import diagnostics as D
from paper_2105_09671_amd import paper_suite as S

pytestmark = pytest.mark.gpu

THREADS = min(32, max(1, oracle.cpus_available()))


@pytest.mark.parametrize("name", list(S.CASES))
def test_paper_case(name):
    c = S.CASES[name]
    res = S.run(c, torch.float64)
    step = oracle.step2d if c.dim == 2 else oracle.step3d
    ref = step(np.ascontiguousarray(res["initial"], dtype=np.float64), c.h, c.dt, c.eps, c.steps, THREADS)
    err = D.rel_linf(res["final"].cpu().numpy(), ref)
    print(name, "rel Linf %.3g" % err, res["check"])
    assert err <= 1e-12
    assert res["check"]["ok"], res["check"]
