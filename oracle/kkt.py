"""Accuracy measures for a candidate solution (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states no accuracy measure; these are the ones every result is
reported with.  For one problem with force scale m g (``weight``):

  rel-err   |u - u*|_2 / max(|u*|_2, m g)   and   |x - x*|_2 / max(|x*|_2, 1)
  r_dyn     max_k |x_{k+1} - A_k x_k - B_k u_k - e_k|_inf
                  / (1 + max(|x_{k+1}|, |A_k x_k|, |B_k u_k|)_inf)
  r_ineq    max over stance rows of [G u - h]_+ / (m g), and |u| / (m g) on
            swing contacts
  r_stat    |(grad_x L, grad_u L)|_inf / (1 + the largest term norm), with
            grad_u L = R (u_k - r^u_k) + B_k^T p_{k+1} + G_k^T mu_k (stance
            components) and grad_{x_{k+1}} L = Q (x_{k+1} - r_k) - p_{k+1}
            + A_{k+1}^T p_{k+2}
  r_comp    max_i mu_i [h_i - G_i u]_+ / (1 + |mu|_inf m g)
  r_sign    max_i [-mu_i]_+ / (1 + the largest term norm of r_stat): the
            multipliers of inequality rows must be nonnegative
  KKT       max(r_dyn, r_ineq, r_stat, r_comp, r_sign)

When no multipliers are given, the costates come from the adjoint recursion
on x and each stance contact's row multipliers from a nonnegative least-squares
fit of its input gradient on the rows whose slack is below ``act_tol`` m g.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize

from .projection import wrench_rows
from .qp import costates, n_contacts

NX, NU = 13, 12


def rel_err(u, u_star, x, x_star, weight):
    eu = np.linalg.norm(u - u_star) / max(np.linalg.norm(u_star), float(weight))
    ex = np.linalg.norm(x - x_star) / max(np.linalg.norm(x_star), 1.0)
    return eu, ex


def residuals(p, u, x, lam=None, mu=None, act_tol=1e-7):
    N = p["N"]
    mg = float(p["weight"])
    u = np.asarray(u, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    A, B, e = p["A"], p["B"], p["e"]
    Gc, hc = wrench_rows(p["mu"], p["fz_max"], p["tau_max"])

    r_dyn = abs(x[0] - p["x0"]).max() / (1.0 + abs(p["x0"]).max())
    for k in range(N):
        ax = A[k] @ x[k]
        bu = B[k] @ u[k]
        d = x[k + 1] - ax - bu - e[k]
        den = 1.0 + max(abs(x[k + 1]).max(), abs(ax).max(), abs(bu).max())
        r_dyn = max(r_dyn, abs(d).max() / den)

    if lam is None:
        lam = costates(p, x)
    nc = n_contacts(p)
    r_ineq = 0.0
    grad_u = np.zeros((N, 6 * nc))
    terms = [0.0]
    for k in range(N):
        ru = p["R"] * (u[k] - p["u_ref"][k])
        bl = B[k].T @ lam[k]
        grad_u[k] = ru + bl
        for i in range(nc):
            sl = slice(6 * i, 6 * i + 6)
            if p["contact"][k][i]:
                terms += [abs(ru[sl]).max(), abs(bl[sl]).max()]
                r_ineq = max(r_ineq, max(0.0, (Gc @ u[k, sl] - hc).max()) / mg)
            else:
                r_ineq = max(r_ineq, abs(u[k, sl]).max() / mg)

    if mu is None:
        mu = np.zeros((N, nc, 11))
        for k in range(N):
            for i in range(nc):
                if not p["contact"][k][i]:
                    continue
                sl = slice(6 * i, 6 * i + 6)
                slack = hc - Gc @ u[k, sl]
                act = np.where(slack <= act_tol * mg)[0]
                if len(act):
                    m_a, _ = scipy.optimize.nnls(Gc[act].T, -grad_u[k, sl])
                    mu[k, i, act] = m_a

    r_comp = 0.0
    mu_max = float(np.max(mu)) if mu.size else 0.0
    stat = 0.0
    for k in range(N):
        for i in range(nc):
            if not p["contact"][k][i]:
                continue
            sl = slice(6 * i, 6 * i + 6)
            gm = Gc.T @ mu[k, i]
            terms.append(abs(gm).max())
            stat = max(stat, abs(grad_u[k, sl] + gm).max())
            slack = np.maximum(hc - Gc @ u[k, sl], 0.0)
            r_comp = max(r_comp, (mu[k, i] * slack).max() / (1.0 + mu_max * mg))
        gx = p["Q"] * (x[k + 1] - p["x_ref"][k]) - lam[k]
        qx = abs(p["Q"] * (x[k + 1] - p["x_ref"][k])).max()
        terms += [qx, abs(lam[k]).max()]
        if k + 1 < N:
            al = A[k + 1].T @ lam[k + 1]
            gx = gx + al
            terms.append(abs(al).max())
        stat = max(stat, abs(gx).max())
    r_stat = stat / (1.0 + max(terms))
    neg = 0.0
    for k in range(N):
        for i in range(nc):
            if p["contact"][k][i]:
                neg = max(neg, float(np.max(-mu[k, i])))
    r_sign = max(0.0, neg) / (1.0 + max(terms))
    out = dict(r_dyn=r_dyn, r_ineq=r_ineq, r_stat=r_stat, r_comp=r_comp, r_sign=r_sign)
    out["kkt"] = max(out.values())
    return out
