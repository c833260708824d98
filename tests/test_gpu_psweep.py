"""p-refinement on a fixed mesh through the GPU pipeline (Section 10, Table 4, eq 10.3):
for k = 0..6 the errors of eq 10.1 computed from the library's q, u and uhat (condensation,
boundary data, PCG to 1e-13, reconstruction) equal the oracle's errors on the same mesh, so
the library reproduces the oracle's p-convergence and its eq 10.3 ratios."""
import math

import numpy as np
import pytest

from hdg_inputs import manufactured_sin_xyz
from oracle import globalsys as OGS
from test_oracle_psweep import KS, psweep_mesh, ratios
from _gpu_helpers import gpu_system, oracle_expand

pytestmark = pytest.mark.gpu


def test_gpu_p_convergence_matches_oracle():
    m = psweep_mesh()
    ex = oracle_expand(m)
    pb = manufactured_sin_xyz("c1", "c1")
    gpu = {a: [] for a in ("e_q", "e_u", "e_uhat")}
    ora = {a: [] for a in gpu}
    for k in KS:
        print(f"p-sweep k={k}", flush=True)
        S = gpu_system(m, k, pb)
        r = S.run(rtol=1e-13)
        assert r["info"]["rel_residual"] <= 1e-13
        eg = OGS.errors(ex, pb, k, r["q"].cpu().numpy(), r["u"].cpu().numpy(), S.uhat.cpu().numpy())
        out = OGS.solve_problem(ex, pb, k, with_post=False)
        eo = OGS.errors(ex, pb, k, out["q"], out["u"], out["uhat"])
        for a in gpu:
            gpu[a].append(eg[a])
            ora[a].append(eo[a])
            assert abs(eg[a] - eo[a]) <= 1e-8 * eo[a], (k, a, eg[a], eo[a])
    for a in gpu:
        assert np.allclose(ratios(gpu[a]), ratios(ora[a]), rtol=1e-6, atol=0)
        assert all(gpu[a][i + 1] < 0.5 * gpu[a][i] for i in range(len(KS) - 1))
