"""Stage matrices A_k, B_k of the centroidal model from compact physics (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper obtains its state matrices along the planned contact sequence from
the discrete centroidal dynamics of Sec. II-A (CoM position, linear and angular
momentum; contact forces and moments entering through the lever arm p_{i,k} - c_k).
The workloads here use the same physics written as the 13-state single-rigid-
body form with gravity carried as a state (roll, pitch, yaw, CoM position,
world angular velocity, CoM velocity, gravity), discretised by forward Euler:

    angle rates      d(roll, pitch, yaw)/dt = R_z(psi_k)^T omega
    CoM              dp/dt = v
    angular          d omega/dt = I_w^{-1} sum_i ((p_{i,k} - c_k) x f_i + tau_i)
    linear           dv/dt = sum_i f_i / m + g_s e_z,      dg_s/dt = 0

with I_w = R_z(psi_k) diag(I_body) R_z(psi_k)^T the world-frame inertia at the
stage's yaw, and the bilinear lever arm linearised at the reference CoM
(c_k -> c_ref,k).  Then A_k = I + dt A_c(psi_k), B_k = dt B_c(psi_k, r_k).

Every entry is formed from its definition: each column of B_k is the state
derivative produced by one unit input (a unit force through the cross product
with the lever arm, a unit moment directly), mapped through the world-frame
inverse inertia obtained by inverting I_w; each column of A_k likewise from
one unit state.  No matrix shortcut (skew matrices, closed-form inverses) is
used, so the construction can be checked against an independent one.
"""
from __future__ import annotations

import numpy as np

NX, NU, NC = 13, 12, 2


def rot_z(psi):
    c, s = np.cos(psi), np.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def state_derivative(x, u, psi, c_ref, feet, mass, inertia):
    """Continuous-time derivative of the 13-state model at state x and input u
    (both 1-D), with the lever arms taken from c_ref (the linearisation of
    Sec. II-A's (p_{i,k} - c_k) x f at the reference CoM)."""
    Rz = rot_z(psi)
    Iw = Rz @ np.diag(inertia) @ Rz.T
    omega = x[6:9]
    vel = x[9:12]
    g_s = x[12]
    wrench_moment = np.zeros(3)
    force = np.zeros(3)
    for i in range(NC):
        f = u[6 * i:6 * i + 3]
        tau = u[6 * i + 3:6 * i + 6]
        wrench_moment += np.cross(feet[i] - c_ref, f) + tau
        force += f
    d = np.zeros(NX)
    d[0:3] = Rz.T @ omega
    d[3:6] = vel
    d[6:9] = np.linalg.solve(Iw, wrench_moment)
    d[9:12] = force / mass
    d[11] += g_s
    return d


def stage_matrices(psi, c_ref, feet, mass, inertia, dt):
    """A_k, B_k of one stage: A = I + dt A_c, B = dt B_c, with the columns of
    A_c and B_c the derivatives produced by unit states and unit inputs (the
    model is linear in (x, u) once the lever arm is fixed)."""
    A = np.eye(NX)
    B = np.zeros((NX, NU))
    zx, zu = np.zeros(NX), np.zeros(NU)
    for j in range(NX):
        ej = np.zeros(NX)
        ej[j] = 1.0
        A[:, j] += dt * state_derivative(ej, zu, psi, c_ref, feet, mass, inertia)
    for j in range(NU):
        ej = np.zeros(NU)
        ej[j] = 1.0
        B[:, j] = dt * state_derivative(zx, ej, psi, c_ref, feet, mass, inertia)
    return A, B


def horizon_matrices(yaw, c_ref, feet, mass, inertia, dt, N):
    """A [n][13][13], B [n][13][12] for one problem: stage k < N from
    stage_matrices(yaw[k], c_ref[k], feet[k], ...); padding stages k >= N get
    A = I, B = 0.

    yaw [n], c_ref [n][3] (reference CoM at stage k), feet [n][2][3] (contact
    positions at stage k), mass, inertia [3] (body-frame principal moments), dt."""
    n = len(yaw)
    A = np.tile(np.eye(NX), (n, 1, 1))
    B = np.zeros((n, NX, NU))
    for k in range(N):
        A[k], B[k] = stage_matrices(float(yaw[k]), np.asarray(c_ref[k], float),
                                    np.asarray(feet[k], float), float(mass),
                                    np.asarray(inertia, float), float(dt))
    return A, B


# --------------------------------------------------------------------------
# The paper's own model: 9 centroidal states (CoM c, linear momentum l_G,
# angular momentum about the CoM k_G), Sec. II-A, its three discrete updates
#   c_{k+1}   = c_k + dt l_k / m
#   l_{k+1}   = l_k + dt (m g + sum_i f_i)
#   k_{k+1}   = k_k + dt sum_i ((p_{i,k} - c_k) x f_i + tau_i)
# with the lever arm taken at the reference CoM (the bilinear c_k x f_i
# linearised at c_ref,k).  Gravity enters through the affine term e_k.  The
# 13-slot state layout of the solver holds (c, l_G, k_G) in slots 0..8; slots
# 9..12 are inert (A = I, B = 0, e = 0), so with zero initial value, zero
# reference and any positive weight they add nothing to the cost and the
# optimum of the 9-state problem is unchanged.

GRAV = np.array([0.0, 0.0, -9.81])


def momentum_next(x, u, c_ref, feet, mass, dt):
    """x_{k+1} of the paper's discrete centroidal dynamics (embedded layout)."""
    c, l, kg = x[0:3], x[3:6], x[6:9]
    force = np.zeros(3)
    moment = np.zeros(3)
    for i in range(NC):
        f = u[6 * i:6 * i + 3]
        tau = u[6 * i + 3:6 * i + 6]
        force += f
        moment += np.cross(feet[i] - c_ref, f) + tau
    out = np.array(x, dtype=np.float64)
    out[0:3] = c + dt * l / mass
    out[3:6] = l + dt * (mass * GRAV + force)
    out[6:9] = kg + dt * moment
    return out


def momentum_stage_matrices(c_ref, feet, mass, dt):
    """A_k, B_k, e_k of one stage: e = the image of the zero state and input,
    each column of A and B the image of one unit state or input minus e."""
    zx, zu = np.zeros(NX), np.zeros(NU)
    e = momentum_next(zx, zu, c_ref, feet, mass, dt)
    A = np.zeros((NX, NX))
    B = np.zeros((NX, NU))
    for j in range(NX):
        ej = np.zeros(NX)
        ej[j] = 1.0
        A[:, j] = momentum_next(ej, zu, c_ref, feet, mass, dt) - e
    for j in range(NU):
        ej = np.zeros(NU)
        ej[j] = 1.0
        B[:, j] = momentum_next(zx, ej, c_ref, feet, mass, dt) - e
    return A, B, e


def momentum_horizon_matrices(c_ref, feet, mass, dt, N):
    """A [n][13][13], B [n][13][12], e [n][13] of the momentum model; padding
    stages k >= N get A = I, B = 0, e = 0."""
    n = len(c_ref)
    A = np.tile(np.eye(NX), (n, 1, 1))
    B = np.zeros((n, NX, NU))
    e = np.zeros((n, NX))
    for k in range(N):
        A[k], B[k], e[k] = momentum_stage_matrices(np.asarray(c_ref[k], float),
                                                   np.asarray(feet[k], float), float(mass),
                                                   float(dt))
    return A, B, e
