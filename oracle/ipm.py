"""Oracle interior-point loop for a multistage QP -- test infrastructure only.

The paper runs its KKT solver inside PIQP, whose iteration it does not describe;
this oracle follows the reading used on the GPU: a primal-dual interior-point
method with Mehrotra's predictor-corrector on

    min 1/2 x^T P x + c^T x   s.t.   A x = beq,   G x + s = h,  s >= 0

(P, A, G from ``oracle.qp.dense_parts``; c, beq, h stacked stage by stage, g
last), whose Newton systems are the regularised ones of ``oracle.qp`` with the
proximal centres at the current iterate (the regularisation terms vanish in the
residuals, so the fixed point is the exact KKT point).  The regularisation falls
as the iterate converges, as proximal methods do: the start step uses rho_0 and
delta_0, iteration k uses rho_0 f, delta_0 f with f = max(1e-4, 10^-(k+1)) (a
fixed delta leaves an equality residual of about delta |dy| per step, which
contracts ever more slowly as the horizon grows).

  start: from x = 0, y = 0, s = z = 1 take the full predictor step (below) and
  move s and z into the interior by Mehrotra's heuristic (the starting point of
  primal-dual methods in Nocedal & Wright, Numerical Optimization, Sec. 14.2):
    s += max(-1.5 min s, 0), z += max(-1.5 min z, 0), then with t = s^T z
    s += t / (2 sum z), z += t / (2 sum s)   (both shifts from the same s, z);
  skipped without inequality rows.  Then per iteration
    r_d = P x + c + A^T y + G^T z,   r_p = A x - beq,   r_s = G x + s - h,
    mu = s^T z / m (m inequality rows; 0 without any);
    stop when max(|r_d|, |r_p|, |r_s|)_inf <= tol and mu <= tol;
    w = z / (s + delta z)                       (W^-1 = S Z^-1 + delta I)
    predictor: rx = -r_d, ry = -r_p, rz = -r_s + s; solve; ds = -r_s - rz - dz / w
    alpha_aff = the largest step in (0, 1] keeping s, z >= 0;
    mu_aff = (s + alpha_aff ds)^T (z + alpha_aff dz) / m, sigma = (mu_aff / mu)^3
    corrector: rz = -r_s - rc / z, rc = -s z + sigma mu - ds_aff dz_aff; solve; ds
    alpha = min(1, 0.99 * the largest step keeping s, z >= 0);
    x, y, z, s += alpha (dx, dy, dz, ds).
"""
import numpy as np

from . import qp as oqp


def _step_to_boundary(v, dv):
    """Largest a in (0, 1] with v + a dv >= 0 (v > 0)."""
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-v[neg] / dv[neg])))


def newton(qp, rho, delta, w, rx, ry, rz):
    """The regularised Newton step (dense, LAPACK): dx from Psi, then dy, dz."""
    _, _, _, _, Psi = oqp.assemble(dict(qp, w=w), rho, delta)
    r = oqp.reduce_rhs(dict(qp, w=w), delta, rx, ry, rz)
    dx = np.linalg.solve(Psi, r)
    dy, dz = oqp.recover(dict(qp, w=w), delta, dx, ry, rz)
    return dx, dy, dz


def solve(qp, c, beq, h, rho=1e-6, delta=1e-6, tol=1e-9, max_iter=60):
    """Run the loop above.  c: n vector (stages then g), beq: N pe, h: N me.
    Returns dict(x, y, z, s, iterations, converged, history of (res, mu))."""
    P, A, G = oqp.dense_parts(qp)
    n, ma, mg = P.shape[0], A.shape[0], G.shape[0]
    c, beq, h = (np.asarray(v, dtype=np.float64).reshape(-1) for v in (c, beq, h))
    x, y = np.zeros(n), np.zeros(ma)
    s, z = np.ones(mg), np.ones(mg)
    if mg:
        rd = P @ x + c + A.T @ y + G.T @ z
        rp = A @ x - beq
        rs = G @ x + s - h
        w = z / (s + delta * z)
        rz = -rs + s
        dx, dy, dz = newton(qp, rho, delta, w, -rd[:, None], -rp[:, None], rz[:, None])
        x, y = x + dx[:, 0], y + dy[:, 0]
        s = s + (-rs - rz - dz[:, 0] / w)
        z = z + dz[:, 0]
        s = s + max(-1.5 * float(np.min(s)), 0.0)
        z = z + max(-1.5 * float(np.min(z)), 0.0)
        t = float(s @ z)
        s, z = s + 0.5 * t / float(np.sum(z)), z + 0.5 * t / float(np.sum(s))
    hist = []
    converged = False
    it = 0
    for it in range(max_iter + 1):
        rd = P @ x + c + A.T @ y + G.T @ z
        rp = A @ x - beq
        rs = G @ x + s - h
        mu = float(s @ z / mg) if mg else 0.0
        res = max(np.max(np.abs(rd), initial=0.0), np.max(np.abs(rp), initial=0.0), np.max(np.abs(rs), initial=0.0))
        hist.append((res, mu))
        if res <= tol and mu <= tol:
            converged = True
            break
        if it == max_iter:
            break
        f = max(1e-4, 10.0 ** -(it + 1))
        rk, dk = rho * f, delta * f
        w = z / (s + dk * z)
        rx, ry = -rd, -rp
        rz = -rs + s
        dx, dy, dz = newton(qp, rk, dk, w, rx[:, None], ry[:, None], rz[:, None])
        dx, dy, dz = dx[:, 0], dy[:, 0], dz[:, 0]
        ds = -rs - rz - dz / w
        if mg:
            a_aff = min(_step_to_boundary(s, ds), _step_to_boundary(z, dz))
            mu_aff = float((s + a_aff * ds) @ (z + a_aff * dz) / mg)
            sigma = (mu_aff / mu) ** 3
            rc = -s * z + sigma * mu - ds * dz
            rz = -rs - rc / z
            dx, dy, dz = newton(qp, rk, dk, w, rx[:, None], ry[:, None], rz[:, None])
            dx, dy, dz = dx[:, 0], dy[:, 0], dz[:, 0]
            ds = -rs - rz - dz / w
            alpha = min(1.0, 0.99 * min(_step_to_boundary(s, ds), _step_to_boundary(z, dz)))
        else:
            alpha = 1.0
        x += alpha * dx
        y += alpha * dy
        z += alpha * dz
        s += alpha * ds
    return dict(x=x, y=y, z=z, s=s, iterations=it, converged=converged, history=hist)
