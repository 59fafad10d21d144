"""Pins of the dynamics oracle (oracle/dynamics.py): the stage matrices built
from compact physics must agree with the paper's discrete centroidal dynamics
(Sec. II-A: the CoM, linear-momentum and angular-momentum updates), with
rigid-body mechanics worked in the body frame, and with the workload
generator's independent construction."""
import numpy as np
import pytest

import mpcgen
from oracle import dynamics

G = 9.81


def _random_stage(rng):
    psi = rng.uniform(-np.pi, np.pi)
    c_ref = np.array([rng.normal(0, 0.3), rng.normal(0, 0.3), 0.8 + rng.normal(0, 0.05)])
    feet = np.array([[rng.normal(0, 0.2), 0.1 + rng.normal(0, 0.1), rng.normal(0, 0.05)],
                     [rng.normal(0, 0.2), -0.1 + rng.normal(0, 0.1), rng.normal(0, 0.05)]])
    mass = rng.uniform(30, 60)
    inertia = rng.uniform(1, 4, 3)
    dt = rng.uniform(0.02, 0.05)
    return psi, c_ref, feet, mass, inertia, dt


@pytest.mark.parametrize("seed", range(6))
def test_momentum_updates_of_the_paper(seed):
    """x_{k+1} = A x + B u reproduces the paper's discrete updates: CoM
    c + dt l / m, linear momentum l + dt (m g + sum f), angular momentum about
    the CoM k + dt sum ((p_i - c) x f_i + tau_i), with l = m v and k = I_w omega
    (the lever arm at the reference CoM)."""
    rng = np.random.default_rng([11, seed])
    psi, c_ref, feet, m, inertia, dt = _random_stage(rng)
    A, B = dynamics.stage_matrices(psi, c_ref, feet, m, inertia, dt)
    x = rng.normal(0, 1, 13)
    x[12] = -G
    u = rng.normal(0, 50, 12)
    x1 = A @ x + B @ u
    Rz = dynamics.rot_z(psi)
    Iw = Rz @ np.diag(inertia) @ Rz.T
    c, v, w = x[3:6], x[9:12], x[6:9]
    f = [u[0:3], u[6:9]]
    tau = [u[3:6], u[9:12]]
    assert np.allclose(x1[3:6], c + dt * (m * v) / m, atol=1e-12)
    l1 = m * v + dt * (m * np.array([0, 0, -G]) + f[0] + f[1])
    assert np.allclose(m * x1[9:12], l1, atol=1e-9)
    k1 = Iw @ w + dt * sum(np.cross(feet[i] - c_ref, f[i]) + tau[i] for i in range(2))
    assert np.allclose(Iw @ x1[6:9], k1, atol=1e-9)
    assert x1[12] == x[12]


@pytest.mark.parametrize("seed", range(6))
def test_angular_rows_match_body_frame_euler(seed):
    """The angular-acceleration rows equal Euler's equation solved in the body
    frame (torque rotated into the body, divided by the principal moments,
    rotated back), so the world-frame inertia R diag(I) R^T is not transposed."""
    rng = np.random.default_rng([12, seed])
    psi, c_ref, feet, m, inertia, dt = _random_stage(rng)
    _, B = dynamics.stage_matrices(psi, c_ref, feet, m, inertia, dt)
    u = rng.normal(0, 50, 12)
    torque = sum(np.cross(feet[i] - c_ref, u[6 * i:6 * i + 3]) + u[6 * i + 3:6 * i + 6]
                 for i in range(2))
    Rz = dynamics.rot_z(psi)
    wdot = Rz @ ((Rz.T @ torque) / inertia)
    assert np.allclose(B[6:9] @ u / dt, wdot, rtol=1e-12, atol=1e-12)
    assert np.all(B[0:6] == 0) and np.all(B[12] == 0)


def test_angle_rates_and_gravity():
    """Yaw rate from a world z spin; roll rate from a spin about the body x
    axis; free fall from the gravity state."""
    psi = 0.7
    A, _ = dynamics.stage_matrices(psi, np.zeros(3), np.zeros((2, 3)), 40.0,
                                   np.array([1.0, 2.0, 3.0]), 0.1)
    x = np.zeros(13)
    x[6:9] = [0, 0, 1.0]
    assert np.allclose((A @ x - x)[0:3] / 0.1, [0, 0, 1.0])
    x[6:9] = dynamics.rot_z(psi) @ np.array([1.0, 0, 0])
    assert np.allclose((A @ x - x)[0:3] / 0.1, [1.0, 0, 0])
    x = np.zeros(13)
    x[12] = -G
    x1 = A @ x
    assert np.isclose(x1[11], -G * 0.1) and np.allclose(x1[3:6], 0)


@pytest.mark.parametrize("config", ["small_b64_n10", "uneven_b16384"])
def test_agrees_with_generator_construction(config):
    """The generator builds the same matrices another way (skew matrices,
    matrix inverse, constant yaw over the horizon); both must agree."""
    batch = mpcgen.make_batch(config, indices=range(5), as_float32=False)
    for b in range(5):
        N = int(batch["N"][b])
        A, B = dynamics.horizon_matrices(batch["yaw_k"][b], batch["c_ref"][b], batch["feet"][b],
                                         batch["mass"][b], batch["inertia"][b], batch["dt"][b], N)
        assert np.allclose(A, batch["A"][b], rtol=0, atol=1e-13)
        assert np.allclose(B, batch["B"][b], rtol=0, atol=1e-13)


# ---------------------------------------------- the paper's momentum model

@pytest.mark.parametrize("seed", range(6))
def test_momentum_model_equations(seed):
    """A x + B u + e reproduces the three discrete updates of Sec. II-A written
    out directly, and the inert slots 9..12 keep their values."""
    rng = np.random.default_rng([13, seed])
    _, c_ref, feet, m, _, dt = _random_stage(rng)
    A, B, e = dynamics.momentum_stage_matrices(c_ref, feet, m, dt)
    x = rng.normal(0, 1, 13)
    u = rng.normal(0, 50, 12)
    x1 = A @ x + B @ u + e
    c, l, kg = x[0:3], x[3:6], x[6:9]
    f = [u[0:3], u[6:9]]
    tau = [u[3:6], u[9:12]]
    assert np.allclose(x1[0:3], c + dt * l / m, atol=1e-12)
    assert np.allclose(x1[3:6], l + dt * (m * np.array([0, 0, -G]) + f[0] + f[1]), atol=1e-9)
    kk = kg + dt * sum(np.cross(feet[i] - c_ref, f[i]) + tau[i] for i in range(2))
    assert np.allclose(x1[6:9], kk, atol=1e-9)
    assert np.array_equal(x1[9:13], x[9:13])
    # gravity only through the affine term: e = (0, dt m g, 0, inert zeros)
    assert np.allclose(e, np.r_[0, 0, 0, 0, 0, -dt * m * G, np.zeros(7)], atol=1e-12)


def test_momentum_model_agrees_with_generator_construction():
    batch = mpcgen.make_batch("plain_b4096_n20", indices=range(4), as_float32=False,
                              model="momentum")
    for b in range(4):
        N = int(batch["N"][b])
        A, B, e = dynamics.momentum_horizon_matrices(batch["c_ref"][b], batch["feet"][b],
                                                     batch["mass"][b], batch["dt"][b], N)
        assert np.allclose(A, batch["A"][b], rtol=0, atol=1e-13)
        assert np.allclose(B, batch["B"][b], rtol=0, atol=1e-13)
        assert np.allclose(e, batch["e"][b], rtol=0, atol=1e-12)


def test_momentum_embedding_leaves_the_optimum_unchanged():
    """The inert slots start at zero, are never driven and have zero reference:
    the optimum does not depend on their weights (so it is the optimum of the
    9-state problem), they stay zero, and the result is certified."""
    from oracle import kkt, qp
    batch = mpcgen.make_batch("plain_b4096_n20", indices=[0, 1], model="momentum")
    for b in range(2):
        p = mpcgen.problem_fp64(batch, b)
        ref = qp.solve(p)
        assert np.all(ref["x"][:, 9:13] == 0)
        p2 = dict(p)
        p2["Q"] = p["Q"].copy()
        p2["Q"][9:13] = 123.0
        alt = qp.solve(p2)
        assert np.allclose(alt["u"], ref["u"], rtol=0, atol=1e-9 * np.abs(ref["u"]).max())
        assert kkt.residuals(p, ref["u"], ref["x"])["kkt"] <= 1e-9
        # gravity is carried: the optimum supports the weight on average
        fz = ref["u"][:, [2, 8]].sum(axis=1)
        assert abs(fz.mean() - p["weight"]) < 0.5 * p["weight"]
