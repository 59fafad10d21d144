"""Exact optimum of the standard-form LTV MPC QP (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The problem (the standard form of Sec. III, with C = I, costs on x_1..x_N and
u_0..u_{N-1}, and the wrench sets of Sec. II-B):

    min  sum_{k=0}^{N-1} 1/2 (x_{k+1}-r_k)^T Q (x_{k+1}-r_k)
                         + 1/2 (u_k-r^u_k)^T R (u_k-r^u_k)
    s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,  x_0 given
         stance contact: G_c (f, tau) <= h_c   (eleven rows, see projection)
         swing contact:  (f, tau) = 0

R > 0 makes it strictly convex and u = 0 is feasible, so the minimiser is
unique.  This module computes it by its plain definition, in four steps:

 1. condense: eliminate the states with the dynamics, X = Gamma U + c, giving
    a dense QP  min 1/2 U^T H U + g^T U  s.t.  G U <= h  over the stance
    inputs (swing inputs are fixed to 0 and dropped);
 2. a primal-dual interior point with Mehrotra's predictor-corrector on that
    dense QP, run to a duality measure near FP64 rounding;
 3. polish: take the rows whose multiplier exceeds their slack as active,
    solve the equality-constrained QP on them exactly (null-space method),
    recover nonnegative multipliers by NNLS, and correct the active set if
    the result is infeasible or a multiplier must be negative;
 4. certify: primal feasibility, stationarity and multiplier signs to near
    FP64 rounding; an uncertified result raises instead of being returned.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.optimize

from .projection import wrench_rows

NX, NU = 13, 12


def n_contacts(p):
    """Contacts per stage of a problem (2: the feet; 4: feet and hands), from
    its contact schedule [N, contacts]; every contact contributes six inputs."""
    return int(np.shape(p["contact"])[-1])


class NotCertified(RuntimeError):
    pass


def condense(p):
    """X = Gam @ U + c for X = (x_1..x_N), U = (u_0..u_{N-1}) stacked."""
    N = p["N"]
    nu = 6 * n_contacts(p)
    Gam = np.zeros((N * NX, N * nu))
    c = np.zeros(N * NX)
    row = np.zeros((NX, N * nu))
    xc = p["x0"].copy()
    for k in range(N):
        xc = p["A"][k] @ xc + p["e"][k]
        row = p["A"][k] @ row
        row[:, k * nu:(k + 1) * nu] += p["B"][k]
        Gam[k * NX:(k + 1) * NX] = row
        c[k * NX:(k + 1) * NX] = xc
    return Gam, c


def rollout(p, u):
    """States x_0..x_N of the dynamics driven by u [N, 6 contacts]."""
    N = p["N"]
    x = np.zeros((N + 1, NX))
    x[0] = p["x0"]
    for k in range(N):
        x[k + 1] = p["A"][k] @ x[k] + p["B"][k] @ u[k] + p["e"][k]
    return x


def costates(p, x):
    """Adjoint p_{k+1} (returned at index k) of the Lagrangian
    L = cost + sum p_{k+1}^T (A_k x_k + B_k u_k + e_k - x_{k+1}) + ...,
    from grad_{x_{k+1}} L = 0:  p_{k+1} = Q (x_{k+1}-r_k) + A_{k+1}^T p_{k+2}."""
    N = p["N"]
    lam = np.zeros((N, NX))
    nxt = np.zeros(NX)
    for k in range(N - 1, -1, -1):
        lam[k] = p["Q"] * (x[k + 1] - p["x_ref"][k])
        if k + 1 < N:
            lam[k] += p["A"][k + 1].T @ nxt
        nxt = lam[k]
    return lam


def cost(p, u, x=None):
    if x is None:
        x = rollout(p, u)
    dx = x[1:] - p["x_ref"]
    du = u - p["u_ref"]
    return 0.5 * np.sum(dx * dx * p["Q"]) + 0.5 * np.sum(du * du * p["R"])


def dense_qp(p):
    """Condensed QP over the stance inputs.

    Returns H, g, G, h, free (indices into the stacked U) and rows, a list of
    (stage, contact, row-within-contact) for each row of G.
    """
    N = p["N"]
    Gam, c = condense(p)
    qv = np.tile(p["Q"], N)
    rv = np.tile(p["R"], N)
    r = p["x_ref"].reshape(-1)
    ru = p["u_ref"].reshape(-1)
    H = Gam.T @ (qv[:, None] * Gam) + np.diag(rv)
    g = Gam.T @ (qv * (c - r)) - rv * ru
    nc = n_contacts(p)
    nu = 6 * nc
    free = []
    for k in range(N):
        for i in range(nc):
            if p["contact"][k][i]:
                free.extend(range(k * nu + 6 * i, k * nu + 6 * i + 6))
    free = np.array(free, dtype=np.int64)
    col = {int(f): j for j, f in enumerate(free)}
    Gc, hc = wrench_rows(p["mu"], p["fz_max"], p["tau_max"])
    Grows, hrows, rows = [], [], []
    for k in range(N):
        for i in range(nc):
            if not p["contact"][k][i]:
                continue
            base = k * nu + 6 * i
            for j in range(11):
                gr = np.zeros(len(free))
                for t in range(6):
                    gr[col[base + t]] = Gc[j, t]
                Grows.append(gr)
                hrows.append(hc[j])
                rows.append((k, i, j))
    G = np.array(Grows, dtype=np.float64).reshape(len(Grows), len(free))
    h = np.array(hrows, dtype=np.float64)
    Hf = H[np.ix_(free, free)]
    gf = g[free]
    return Hf, gf, G, h, free, rows


def interior_point(H, g, G, h, maxit=200):
    """Mehrotra predictor-corrector primal-dual interior point for
    min 1/2 x^T H x + g^T x  s.t.  G x <= h   (slack s, multiplier z)."""
    n, m = len(g), len(h)
    x = np.linalg.solve(H, -g) if n else np.zeros(0)
    if m == 0:
        return x, np.zeros(0), np.zeros(0)
    s = np.maximum(h - G @ x, 1.0)
    z = np.ones(m)
    hs = 1.0 + np.max(np.abs(h))
    gs = 1.0 + np.max(np.abs(g))
    for _ in range(maxit):
        rd = H @ x + g + G.T @ z
        rp = G @ x + s - h
        mu = s @ z / m
        if (np.max(np.abs(rd)) <= 1e-12 * gs and np.max(np.abs(rp)) <= 1e-12 * hs
                and mu <= 1e-13 * hs):
            break
        w = z / s
        try:
            L = scipy.linalg.cho_factor(H + G.T @ (w[:, None] * G))
        except np.linalg.LinAlgError:
            break       # the polish below finishes from here

        def newton(rc):
            rhs = -rd - G.T @ ((-rc + z * rp) / s)
            dx = scipy.linalg.cho_solve(L, rhs)
            ds = -rp - G @ dx
            dz = (-rc - z * ds) / s
            return dx, ds, dz

        def max_step(v, dv):
            neg = dv < 0
            return min(1.0, np.min(-v[neg] / dv[neg])) if np.any(neg) else 1.0

        dxa, dsa, dza = newton(s * z)
        aa = min(max_step(s, dsa), max_step(z, dza))
        mu_aff = (s + aa * dsa) @ (z + aa * dza) / m
        sigma = (mu_aff / mu) ** 3
        dx, ds, dz = newton(s * z + dsa * dza - sigma * mu)
        a = min(1.0, 0.99 * min(max_step(s, ds), max_step(z, dz)))
        x = x + a * dx
        s = s + a * ds
        z = z + a * dz
    return x, s, z


def equality_qp(H, g, Ga, ha):
    """min 1/2 x^T H x + g^T x  s.t.  Ga x = ha  by the null-space method
    (rank-revealing SVD, so dependent rows such as the pyramid apex are
    fine).  Returns None if the rows are inconsistent."""
    n = len(g)
    if Ga.shape[0] == 0:
        return np.linalg.solve(H, -g)
    U, S, Vt = np.linalg.svd(Ga)
    r = int(np.sum(S > 1e-10 * S[0]))
    x0 = Vt[:r].T @ ((U[:, :r].T @ ha) / S[:r])
    if np.max(np.abs(Ga @ x0 - ha)) > 1e-9 * (1.0 + np.max(np.abs(ha))):
        return None
    Z = Vt[r:].T
    if Z.shape[1] == 0:
        return x0
    w = np.linalg.solve(Z.T @ H @ Z, -Z.T @ (g + H @ x0))
    return x0 + Z @ w


def _certify(H, g, G, h, x, active, feas_scale):
    """Returns (ok, z, measures) for candidate x and active rows."""
    grad = H @ x + g
    z = np.zeros(len(h))
    if len(active):
        za, _ = scipy.optimize.nnls(G[active].T, -grad, maxiter=50 * len(active) + 100)
        z[active] = za
    stat_res = grad + G.T @ z
    stat = np.max(np.abs(stat_res)) / (1.0 + np.max(np.abs(grad)) + np.max(np.abs(g)))
    feas = max(0.0, np.max(G @ x - h)) / feas_scale if len(h) else 0.0
    slack = h - G @ x
    comp = np.max(z * np.maximum(slack, 0.0)) / (1.0 + np.max(z) * feas_scale) if len(h) else 0.0
    ok = stat <= 1e-9 and feas <= 1e-11 and comp <= 1e-11
    return ok, z, dict(stat=stat, feas=feas, comp=comp)


def solve_dense(H, g, G, h, feas_scale, max_passes=60):
    """Optimum of the dense QP with certificate; raises NotCertified."""
    x, s, z = interior_point(H, g, G, h)
    active = [i for i in range(len(h)) if z[i] > s[i]]
    for _ in range(max_passes):
        xa = equality_qp(H, g, G[active], h[active])
        if xa is None:          # inconsistent rows: drop the newest
            active = active[:-1]
            continue
        viol = G @ xa - h if len(h) else np.zeros(0)
        if len(h) and np.max(viol) > 1e-11 * feas_scale:
            active = sorted(set(active) | {int(np.argmax(viol))})
            continue
        ok, zz, meas = _certify(H, g, G, h, xa, active, feas_scale)
        if ok:
            return xa, zz, meas
        # a multiplier must go negative: drop the row whose unsigned
        # least-squares multiplier is most negative
        grad = H @ xa + g
        zl, *_ = np.linalg.lstsq(G[active].T, -grad, rcond=None)
        active = [a for j, a in enumerate(active) if j != int(np.argmin(zl))]
    raise NotCertified("active-set polish did not certify")


def solve(p):
    """Certified optimum of one problem (dict from mpcgen.problem_fp64).

    Returns dict with u [N, 6 nc], x [N+1,13], lam [N,13] (costate of
    x_{k+1}), mu [N, nc, 11] (row multipliers, 0 for swing; nc contacts per
    stage), cost and the certificate.
    """
    N = p["N"]
    H, g, G, h, free, rows = dense_qp(p)
    fs = max(1.0, float(p["weight"]))
    nc = n_contacts(p)
    U = np.zeros(N * 6 * nc)
    meas = dict(stat=0.0, feas=0.0, comp=0.0)
    z = np.zeros(len(h))
    if len(free):
        Uf, z, meas = solve_dense(H, g, G, h, fs)
        U[free] = Uf
    u = U.reshape(N, 6 * nc)
    x = rollout(p, u)
    mu = np.zeros((N, nc, 11))
    for (k, i, j), zz in zip(rows, z):
        mu[k, i, j] = zz
    return dict(u=u, x=x, lam=costates(p, x), mu=mu, cost=cost(p, u, x), cert=meas)


def solve_batch(batch, indices=None):
    """Oracle solutions for problems of a generator batch (list of dicts)."""
    from mpcgen import problem_fp64
    if indices is None:
        indices = range(len(batch["N"]))
    return [solve(problem_fp64(batch, int(b))) for b in indices]
