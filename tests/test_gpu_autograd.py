"""GPU: the differentiable solve (torch.autograd.Function over kkt_factor_solve /
kkt_solve_adjoint) against the oracle's closed-form adjoint, torch's finite
differences on a tiny system, and a directional finite difference at the
differentiation workload's shape (N = 64, b = 24, ng = 4)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _uniform(seed, S, N, b, ng, nrhs):
    rng = np.random.default_rng(seed)
    sy = [workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.05, s_B=0.05, with_w=True)
          for _ in range(S)]
    st = lambda k: torch.from_numpy(np.stack([getattr(s, k) for s in sy])).cuda()
    return sy, st("D"), st("C"), st("B"), st("corner"), st("r"), st("w")


@pytest.mark.parametrize("segments", [1, 3])
def test_autograd_matches_oracle_adjoint(segments):
    from paper_2511_00946_amd.autograd import kkt_solve, plan_for
    _say("gpu case: autograd S=3 N=10 b=6 ng=3 nrhs=2 p=%d" % segments)
    sy, D, C, B, corner, r, w = _uniform(41, 3, 10, 6, 3, 2)
    leaves = [t.clone().requires_grad_(True) for t in (D, C, B, corner, r)]
    x, info = kkt_solve(*leaves, segments=segments)
    (x * w).sum().backward()
    torch.cuda.synchronize()
    assert (info.cpu() == 0).all()
    xh = x.detach().cpu().numpy()
    for s, sysm in enumerate(sy):
        seg = plan_for([(10, 6, 3, segments)] * 3, 2).segment_lengths(s)
        xo = okkt.solve(sysm.D, sysm.C, sysm.B, sysm.corner, sysm.r, seg)
        assert np.max(np.abs(xh[s] - xo)) <= 1e-10 * np.max(np.abs(xo))
        ref = okkt.adjoint(sysm.D, sysm.C, sysm.B, sysm.corner, xh[s], sysm.w, seg)
        lam, dD, dC, dB, dcorner = ref
        for name, leaf, want in zip(("dD", "dC", "dB", "dcorner", "dr"), leaves, (dD, dC, dB, dcorner, lam)):
            got = leaf.grad[s].cpu().numpy()
            err = float(np.max(np.abs(got - want)) / max(1e-300, np.max(np.abs(want))))
            assert err < 1e-9, (name, s, err)


def test_autograd_gradcheck_tiny():
    from paper_2511_00946_amd.autograd import kkt_solve
    _say("gpu case: gradcheck S=2 N=4 b=2 ng=1 nrhs=1 p=2")
    sy, D, C, B, corner, r, w = _uniform(42, 2, 4, 2, 1, 1)
    leaves = tuple(t.clone().requires_grad_(True) for t in (D, C, B, corner, r))

    def f(*a):
        return kkt_solve(*a, segments=2)[0]

    assert torch.autograd.gradcheck(f, leaves, eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_directional_derivative_full_shape():
    """<grad, delta> against a central difference of the loss along delta, for 8
    systems of the differentiation workload's shape."""
    from paper_2511_00946_amd.autograd import kkt_solve
    _say("gpu case: directional FD S=8 N=64 b=24 ng=4 nrhs=1 p=4")
    sy, D, C, B, corner, r, w = _uniform(43, 8, 64, 24, 4, 1)
    leaves = [t.clone().requires_grad_(True) for t in (D, C, B, corner, r)]
    x, info = kkt_solve(*leaves, segments=4)
    (x * w).sum().backward()
    g = torch.Generator(device="cpu").manual_seed(44)
    deltas = [torch.randn(t.shape, generator=g, dtype=torch.float64).cuda() for t in leaves]
    ana = sum(float((l.grad * d).sum()) for l, d in zip(leaves, deltas))
    h = 1e-5

    def loss(sign):
        with torch.no_grad():
            a = [t.detach() + sign * h * d for t, d in zip(leaves, deltas)]
            return float((kkt_solve(*a, segments=4)[0] * w).sum())

    fd = (loss(1.0) - loss(-1.0)) / (2 * h)
    torch.cuda.synchronize()
    assert abs(fd - ana) <= 1e-6 * max(1.0, abs(ana)), (fd, ana)
