"""Euclidean projection onto the per-contact wrench set (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The wrench set of a stance contact (Sec. II-B: friction pyramid, normal-force
bound and a moment box) is

    F = { f : f_x - mu f_z <= 0, -f_x - mu f_z <= 0,
              f_y - mu f_z <= 0, -f_y - mu f_z <= 0, f_z <= fz_max }
    T = [-tau_max, tau_max]^3

and a swing contact has the set {0}.  The projection onto the lifted set
X_k x U_k that the z-update applies (Sec. III) is the identity on the state
part and this projection on each contact's input part.

The force projection is computed by its definition: the projection of y onto a
polytope is the projection onto the affine hull of the face that contains it,
so enumerating every subset of the five rows, projecting onto the subset's
affine set, keeping the feasible results and taking the nearest gives it.
Slow and plain on purpose.
"""
from __future__ import annotations

import itertools

import numpy as np


def force_rows(mu, fz_max):
    """Rows (G, h) of G f <= h for one stance contact's force (3-vector)."""
    G = np.array([[1.0, 0.0, -mu],
                  [-1.0, 0.0, -mu],
                  [0.0, 1.0, -mu],
                  [0.0, -1.0, -mu],
                  [0.0, 0.0, 1.0]])
    h = np.array([0.0, 0.0, 0.0, 0.0, fz_max])
    return G, h


def moment_rows(tau_max):
    G = np.vstack([np.eye(3), -np.eye(3)])
    h = np.full(6, tau_max)
    return G, h


def wrench_rows(mu, fz_max, tau_max):
    """All 11 rows (G, h) of one stance contact over (f, tau) in R^6."""
    Gf, hf = force_rows(mu, fz_max)
    Gt, ht = moment_rows(tau_max)
    G = np.zeros((11, 6))
    G[:5, :3] = Gf
    G[5:, 3:] = Gt
    return G, np.concatenate([hf, ht])


def _affine_projection(y, Ga, ha):
    """Projection of y onto {f : Ga f = ha} (None if inconsistent)."""
    if Ga.shape[0] == 0:
        return y.copy()
    # minimum-norm correction d with Ga (y + d) = ha
    d, *_ = np.linalg.lstsq(Ga, ha - Ga @ y, rcond=None)
    f = y + d
    if np.max(np.abs(Ga @ f - ha)) > 1e-9 * (1.0 + np.max(np.abs(ha))):
        return None
    return f


def project_force(y, mu, fz_max):
    """Nearest point of the truncated friction pyramid to y (3-vector)."""
    G, h = force_rows(mu, fz_max)
    scale = 1.0 + np.max(np.abs(y)) + fz_max
    best, best_d = None, np.inf
    for r in range(0, 6):
        for sub in itertools.combinations(range(5), r):
            sub = list(sub)
            f = _affine_projection(y, G[sub], h[sub])
            if f is None:
                continue
            if np.max(G @ f - h) > 1e-12 * scale:
                continue
            dist = np.sum((f - y) ** 2)
            if dist < best_d:
                best, best_d = f, dist
    return best


def project_contact(y, stance, mu, fz_max, tau_max):
    """Projection of one contact's 6-vector (f, tau) onto its wrench set."""
    if not stance:
        return np.zeros(6)
    out = np.empty(6)
    out[:3] = project_force(np.asarray(y[:3], dtype=np.float64), mu, fz_max)
    out[3:] = np.clip(y[3:], -tau_max, tau_max)
    return out


def project_input(u, contact_k, mu, fz_max, tau_max):
    """Projection of a stage input (6 entries per contact of contact_k) onto
    U_k."""
    out = np.empty(6 * len(contact_k))
    for i in range(len(contact_k)):
        out[6 * i:6 * i + 6] = project_contact(u[6 * i:6 * i + 6], bool(contact_k[i]),
                                               mu, fz_max, tau_max)
    return out
