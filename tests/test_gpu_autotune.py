"""GPU: the measured cost model (autotune.calibrate) is sane and the segment
counts it picks give solutions that match the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def test_measured_cost_model_and_its_choice(tmp_path, monkeypatch):
    from paper_2511_00946_amd import autotune, kkt
    monkeypatch.setenv("KKT_CACHE_DIR", str(tmp_path))
    print("gpu case: autotune calibration", file=sys.stderr, flush=True)
    m = autotune.cost_model(refresh=True, verbose=True)
    for k in ("t_first", "t_fill", "t_red", "workers", "workers_seg"):
        assert all(np.isfinite(v) and v > 0 for v in m[k]), (k, m[k])
    assert autotune.cost_model() == m                    # cached
    s = workloads.single("race")
    print("gpu case: race system N=%d b=%d ng=%d with measured model" % (s.N, s.b, s.ng), file=sys.stderr,
          flush=True)
    plan = kkt.Plan([(s.N, s.b, s.ng, 0)], nrhs=s.r.shape[1], cost_model=m)
    (p,) = plan.segments()
    assert p > 1
    d = kkt.pack_to_device(workloads.pack([s]))
    ws = plan.new_workspace()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = d["r"].clone()
    plan.factor_solve(d["D"], d["C"], d["B"], d["corner"], ws, x, info)
    torch.cuda.synchronize()
    assert plan.workspace_error(ws) == 0 and info.item() == 0
    xs = x.cpu().numpy().reshape(s.n, -1)
    xo = okkt.solve(s.D, s.C, s.B, s.corner, s.r, plan.segment_lengths(0))
    assert np.max(np.abs(xs - xo)) <= 1e-10 * np.max(np.abs(xo))
