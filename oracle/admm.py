"""The paper's parallel-in-horizon ADMM in FP64 (iterate-level reference).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. III: velocity-form lifting xi_k = (x_k, u_{k-1}) with
Abar_k = [[A_k, B_k], [0, I]], Bbar_k = [B_k; I], ebar_k = (e_k, 0); the
splitting z_{k+1} = xi_{k+1}, v_k = Bbar_k du_k with z in the dynamics; the
scaled augmented Lagrangian with duals (theta, beta, lambda); cached
J_k = (Bbar^T Bbar)^{-1} Bbar^T and
H_k = (Qbar_k + rho I + [k < N-1] rho Abar_{k+1}^T Abar_{k+1})^{-1};
and the three stage-parallel closed-form block updates.  Readings where the
printed text disagrees with its own derivation (each update re-derived as the
exact minimiser of the augmented Lagrangian):
  * the dynamics residual inside the xi-update uses ebar_{k+1};
  * the second penalty term of the Lagrangian uses Bbar_k;
  * the stage-k set constrains z_{k+1} = (x_{k+1}, u_k).

Additions the paper leaves to its references (readings, stated as such):
  * block-constant input scaling u = S_k ut, S_k constant on each contact's
    force triple (m g / stance count) and moment triple (tau_max), so the
    projection stays Euclidean (optimum unchanged, iterates not);
  * fast ADMM with restart (Goldstein, O'Donoghue, Setzer, Baraniuk 2014,
    the restart variant) on (z, v) and the duals, with
    c = |y - yhat|^2 + |dz|^2 + |dv|^2 + |dz - dv|^2;
  * zero initial iterates, fixed iteration count.

Array slot k holds xi_{k+1}, z_{k+1}, v_k, theta_k, beta_k, lambda_k, du_k.
"""
from __future__ import annotations

import numpy as np

from .projection import project_input
from .qp import n_contacts, rollout

NX = 13


def input_scale(p, scaling=True):
    """Diagonal S_k [N, 6 contacts] of the block-constant input scaling."""
    N = p["N"]
    nc = n_contacts(p)
    S = np.ones((N, 6 * nc))
    if not scaling:
        return S
    for k in range(N):
        ns = max(1, int(np.sum(p["contact"][k])))
        for i in range(nc):
            S[k, 6 * i:6 * i + 3] = p["weight"] / ns
            S[k, 6 * i + 3:6 * i + 6] = p["tau_max"]
    return S


def setup(p, rho, scaling=True):
    N = p["N"]
    NU = 6 * n_contacts(p)
    NL = NX + NU
    S = input_scale(p, scaling)
    Bt = p["B"] * S[:, None, :]
    Ab = np.zeros((N, NL, NL))
    Ab[:, :NX, :NX] = p["A"]
    Ab[:, :NX, NX:] = Bt
    Ab[:, NX:, NX:] = np.eye(NU)
    Bb = np.zeros((N, NL, NU))
    Bb[:, :NX] = Bt
    Bb[:, NX:] = np.eye(NU)
    eb = np.zeros((N, NL))
    eb[:, :NX] = p["e"]
    Rt = p["R"][None, :] * S * S
    Qb = np.zeros((N, NL))
    Qb[:, :NX] = p["Q"]
    Qb[:, NX:] = Rt
    qb = np.zeros((N, NL))
    qb[:, :NX] = p["Q"] * p["x_ref"]
    qb[:, NX:] = Rt * (p["u_ref"] / S)
    J = np.zeros((N, NU, NL))
    H = np.zeros((N, NL, NL))
    for k in range(N):
        J[k] = np.linalg.solve(Bb[k].T @ Bb[k], Bb[k].T)
        M = np.diag(Qb[k]) + rho * np.eye(NL)
        if k < N - 1:
            M = M + rho * Ab[k + 1].T @ Ab[k + 1]
        H[k] = np.linalg.inv(M)
    xi0 = np.concatenate([p["x0"], p["u_prev"] / S[0]])
    return dict(S=S, Ab=Ab, Bb=Bb, eb=eb, J=J, H=H, qb=qb, xi0=xi0, rho=rho)


def _project(p, S, y):
    """Proj onto Xbar_k = R^13 x U_k, in scaled input coordinates."""
    z = y.copy()
    for k in range(p["N"]):
        u = y[k, NX:] * S[k]
        z[k, NX:] = project_input(u, p["contact"][k], p["mu"], p["fz_max"],
                                  p["tau_max"]) / S[k]
    return z


def iterate(p, c, st):
    """One sweep of the three block updates from the extrapolated iterates
    st = dict(z, v, th, be, la) (the 'hat' values).  Returns the new iterates
    and the block-1 outputs (xi, du)."""
    N, rho = p["N"], c["rho"]
    NL = c["H"].shape[1]
    Ab, Bb, eb, H, J, qb = c["Ab"], c["Bb"], c["eb"], c["H"], c["J"], c["qb"]
    z, v, th, be, la = st["z"], st["v"], st["th"], st["be"], st["la"]
    # block 1
    du = np.einsum("kij,kj->ki", J, v - be)
    h = qb + rho * (z - th)
    for k in range(N - 1):
        y = z[k + 1] - v[k + 1] - eb[k + 1] + la[k + 1]
        h[k] += rho * Ab[k + 1].T @ y
    xi = np.einsum("kij,kj->ki", H, h)
    # block 2: xi_k of the same sweep (xi_0 fixed)
    prev = np.vstack([c["xi0"][None], xi[:-1]])
    s = np.einsum("kij,kj->ki", Ab, prev)
    b = np.einsum("kij,kj->ki", Bb, du)
    gam = b + be - s - eb + la
    gtil = xi + th + s + eb - la
    zn = _project(p, c["S"], (2.0 * gtil + gam) / 3.0)
    vn = 0.5 * (zn + gam)
    # block 3
    thn = th + xi - zn
    ben = be + b - vn
    lan = la + zn - s - vn - eb
    return dict(z=zn, v=vn, th=thn, be=ben, la=lan), dict(xi=xi, du=du, s=s, b=b)


def _combo(st):
    return st["z"], st["v"], np.concatenate([st["th"], st["be"], st["la"]], axis=1)


def solve(p, iters=100, rho=1.0, scaling=True, accel=True, eta=0.999,
          history=False):
    """Run the ADMM for a fixed number of sweeps from zero iterates.

    Returns dict with u [N, 6 contacts] (unscaled input of z), x (rollout of u), the
    final iterates, the multiplier estimates lam_x = -rho lambda_x (costate
    of x_{k+1}) and mu_u = rho S^{-1} (theta - lambda)_u (= G^T mu), the
    number of restarts and, when ``history`` is set, the iterates after every
    sweep.
    """
    N = p["N"]
    c = setup(p, rho, scaling)
    zero = np.zeros((N, c["H"].shape[1]))
    cur = dict(z=zero.copy(), v=zero.copy(), th=zero.copy(), be=zero.copy(), la=zero.copy())
    prev = {k: v.copy() for k, v in cur.items()}
    hat = {k: v.copy() for k, v in cur.items()}
    alpha, c_prev = 1.0, np.inf
    restarts = 0
    hist = []
    for _ in range(iters):
        new, aux = iterate(p, c, hat)
        if accel:
            zh, vh, yh = _combo(hat)
            zn, vn, yn = _combo(new)
            dz, dv = zn - zh, vn - vh
            cm = np.sum((yn - yh) ** 2) + np.sum(dz ** 2) + np.sum(dv ** 2) + np.sum((dz - dv) ** 2)
            if cm < eta * c_prev:
                a_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * alpha * alpha))
                f = (alpha - 1.0) / a_next
                hat = {k: new[k] + f * (new[k] - cur[k]) for k in new}
                alpha, c_prev = a_next, cm
            else:
                restarts += 1
                hat = {k: cur[k].copy() for k in cur}
                alpha, c_prev = 1.0, c_prev / eta
            prev, cur = cur, new
        else:
            prev, cur = cur, new
            hat = cur
        if history:
            hist.append({k: v.copy() for k, v in cur.items()})
    S = c["S"]
    u = cur["z"][:, NX:] * S
    x = rollout(p, u)
    out = dict(u=u, x=x, iterates=cur, restarts=restarts, setup=c,
               lam_x=-rho * cur["la"][:, :NX],
               gmu=rho * (cur["th"][:, NX:] - cur["la"][:, NX:]) / S)
    if history:
        out["history"] = hist
    return out
