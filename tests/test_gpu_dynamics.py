"""On-device stage matrices from compact physics (pinmpc_build_dynamics)
against the dynamics oracle, and a solve from compact physics against the
QP oracle, through the C ABI.

Bar for the matrices: the kernel works in FP32.  An entry of A is 0, 1, dt, or
1 + dt cos / dt sin of the yaw: FP32 rounding of cos/sin (a few ulp) and of the
sum, below 4e-7 absolute for |A| <= 1.1.  An entry of the angular rows of B is
dt times a sum of three products of the inverse world inertia (itself from
cos^2, sin^2 and 1/I, about ten roundings) with the lever arm (a difference of
two positions): relative error below 2e-6 of the largest entry of its 3 x 3
block; the linear rows dt / m round once.  Padding stages are exact.
"""
import numpy as np
import pytest

import mpcgen
from oracle import dynamics, kkt, qp
from gpu_common import ACT_TOL_FP32, TOL_ERR, TOL_KKT

pytestmark = pytest.mark.gpu

PHYS = ("N", "yaw_k", "c_ref", "feet", "mass", "inertia", "dt")


def _turning(batch, seed):
    """Per-stage yaw (a turn at a random rate) and footholds that move along
    the horizon, so every stage has its own matrices."""
    rng = np.random.default_rng([seed, 99])
    out = dict(batch)
    Bn, n = batch["yaw_k"].shape
    rate = rng.uniform(-1.5, 1.5, Bn)
    dt = batch["dt"].astype(np.float64)
    k = np.arange(n)
    valid = k[None, :] < batch["N"][:, None]
    yaw = batch["yaw_k"].astype(np.float64) + rate[:, None] * dt[:, None] * k[None, :]
    out["yaw_k"] = np.where(valid, yaw, 0.0).astype(np.float32)
    step = rng.normal(0.0, 0.05, (Bn, n, 2, 3)).cumsum(axis=1)
    out["feet"] = np.where(valid[:, :, None, None], batch["feet"] + step, 0.0).astype(np.float32)
    return out


def _build(phys):
    import torch
    from paper_2606_05687_amd import binding
    dev = {k: torch.from_numpy(np.ascontiguousarray(phys[k])).cuda() for k in PHYS}
    A, B, _ = binding.build_dynamics(dev)
    torch.cuda.synchronize()
    return A.cpu().numpy(), B.cpu().numpy()


def _oracle(phys, b):
    f = {k: np.asarray(phys[k][b], dtype=np.float64) for k in PHYS if k != "N"}
    return dynamics.horizon_matrices(f["yaw_k"], f["c_ref"], f["feet"], f["mass"],
                                     f["inertia"], f["dt"], int(phys["N"][b]))


def _check(phys, A, B, idx):
    for b in idx:
        Ar, Br = _oracle(phys, b)
        N = int(phys["N"][b])
        assert np.all(np.abs(A[b, :N] - Ar[:N]) <= 4e-7), b
        for k in range(N):
            for r0 in range(6, 12, 3):
                for c0 in range(0, 12, 3):
                    blk = Br[k, r0:r0 + 3, c0:c0 + 3]
                    err = np.abs(B[b, k, r0:r0 + 3, c0:c0 + 3] - blk).max()
                    assert err <= 2e-6 * max(np.abs(blk).max(), 1e-30), (b, k, r0, c0, err)
            assert np.all(B[b, k, :6] == 0) and np.all(B[b, k, 12] == 0)
        assert np.array_equal(A[b, N:], np.tile(np.eye(13, dtype=np.float32), (A.shape[1] - N, 1, 1)))
        assert np.all(B[b, N:] == 0)


def test_dynamics_match_oracle_ragged():
    """Uneven horizons padded to 60 and a stage count that is not a multiple
    of the kernel's stages per block (37 x 60): every problem compared."""
    batch = mpcgen.make_batch("uneven_b16384", indices=range(37), n_max=60)
    phys = _turning(batch, 3)
    A, B = _build(phys)
    _check(phys, A, B, range(37))


def test_dynamics_full_size_sampled_and_generator_agreement():
    """4096 x 20 in one launch: sampled problems against the oracle; with the
    generator's constant yaw the kernel reproduces the generator's own
    matrices to the same bar."""
    batch = mpcgen.make_batch("plain_b4096_n20")
    A, B = _build(batch)
    _check(batch, A, B, range(0, 4096, 97))
    assert np.all(np.abs(A - batch["A"]) <= 4e-7)
    turned = _turning(batch, 2)
    A2, B2 = _build(turned)
    _check(turned, A2, B2, range(5, 4096, 211))


def test_dynamics_empty_and_bad_arguments():
    import ctypes
    from paper_2606_05687_amd import binding
    lib = binding.load()
    ph = binding.Physics()
    ph.batch, ph.n_max = 0, 20
    assert lib.pinmpc_build_dynamics(ctypes.byref(ph), None, None, None, None) == 0
    ph.batch = 4
    assert lib.pinmpc_build_dynamics(ctypes.byref(ph), None, None, None, None) == -1
    ph.n_max = 65
    assert lib.pinmpc_build_dynamics(ctypes.byref(ph), None, None, None, None) == -1
    ph.n_max, ph.model = 20, 2
    assert lib.pinmpc_build_dynamics(ctypes.byref(ph), None, None, None, None) == -1


def test_solve_from_compact_physics_matches_oracle():
    """The step before the path and the path: matrices built on the device
    from compact physics (turning, moving footholds), then solved; the oracle
    solves the same problem with its own FP64 matrices."""
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch("plain_b4096_n20", indices=range(48))
    phys = _turning(batch, 5)
    dev = binding.to_device(batch)
    pdev = {k: torch.from_numpy(np.ascontiguousarray(phys[k])).cuda() for k in PHYS}
    binding.build_dynamics(pdev, dev["A"], dev["B"])
    solver = binding.Solver(0, iters=3, refine_passes=12, first_passes=0)
    try:
        out = solver.solve(dev)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        solver.close()
    assert (got["status"] == 0).all()
    for b in range(0, 48, 3):
        p = mpcgen.problem_fp64(batch, b)
        Ar, Br = _oracle(phys, b)
        p["A"], p["B"] = Ar[:p["N"]], Br[:p["N"]]
        ref = qp.solve(p)
        N = p["N"]
        u = got["u"][b, :N].astype(np.float64)
        x = got["x"][b, :N + 1].astype(np.float64)
        eu, ex = kkt.rel_err(u, ref["u"], x, ref["x"], p["weight"])
        assert eu <= TOL_ERR and ex <= TOL_ERR, (b, eu, ex)
        # the solve certified its own (FP32-built) problem; against the FP64
        # matrices the dynamics residual carries the matrices' rounding
        r = kkt.residuals(p, u, x, act_tol=ACT_TOL_FP32)
        assert r["r_stat"] <= TOL_KKT and r["r_ineq"] <= TOL_KKT, (b, r)


# ------------------------------------------- the paper's 9-state momentum model

def test_momentum_model_matches_oracle():
    """Model 1 (the 9-state momentum model of Sec. II-A embedded in the
    13-slot layout) against the oracle: A and the linear-momentum rows of B
    are dt / m or dt, rounded once (4e-7 for entries <= 1.1); the angular rows
    dt [r]_x, a difference of two positions times dt (2e-6 of the block's
    largest entry); e_k = -dt m g on l_z, one rounding of a product of three
    (1e-6 relative); padding exact."""
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch("uneven_b16384", indices=range(37), n_max=60)
    phys = _turning(batch, 4)
    dev = {k: torch.from_numpy(np.ascontiguousarray(phys[k])).cuda() for k in PHYS}
    A, B, e = binding.build_dynamics(dev, model="momentum")
    torch.cuda.synchronize()
    A, B, e = A.cpu().numpy(), B.cpu().numpy(), e.cpu().numpy()
    for b in range(37):
        N = int(phys["N"][b])
        Ar, Br, er = dynamics.momentum_horizon_matrices(
            phys["c_ref"][b].astype(np.float64), phys["feet"][b].astype(np.float64),
            float(phys["mass"][b]), float(phys["dt"][b]), N)
        assert np.all(np.abs(A[b] - Ar) <= 4e-7), b
        for k in range(N):
            for r0, c0 in ((3, 0), (3, 6), (6, 0), (6, 3), (6, 6), (6, 9)):
                blk = Br[k, r0:r0 + 3, c0:c0 + 3]
                err = np.abs(B[b, k, r0:r0 + 3, c0:c0 + 3] - blk).max()
                assert err <= 2e-6 * max(np.abs(blk).max(), 1e-30), (b, k, r0, c0, err)
            assert np.all(B[b, k, :3] == 0) and np.all(B[b, k, 9:] == 0)
        assert np.all(np.abs(e[b] - er) <= 1e-6 * np.abs(er).max()), b
        assert np.all(B[b, N:] == 0) and np.all(e[b, N:] == 0)


def test_solve_momentum_model_matches_oracle():
    """The paper's own model solved end to end: matrices and the gravity term
    e_k built on the device, the solve, against the oracle on its own FP64
    matrices; the inert slots stay zero."""
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch("plain_b4096_n20", indices=range(40), model="momentum")
    dev = binding.to_device(batch)
    pdev = {k: torch.from_numpy(np.ascontiguousarray(batch[k])).cuda() for k in PHYS}
    binding.build_dynamics(pdev, dev["A"], dev["B"], dev["e"], model="momentum")
    solver = binding.Solver(0, iters=3, refine_passes=12, first_passes=0)
    try:
        out = solver.solve(dev)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        solver.close()
    assert (got["status"] == 0).all(), got["status"]
    assert np.all(got["x"][:, :, 9:13] == 0)
    for b in range(0, 40, 3):
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        Ar, Br, er = dynamics.momentum_horizon_matrices(p["c_ref"], p["feet"], p["mass"],
                                                        p["dt"], N)
        p["A"], p["B"], p["e"] = Ar[:N], Br[:N], er[:N]
        ref = qp.solve(p)
        u = got["u"][b, :N].astype(np.float64)
        x = got["x"][b, :N + 1].astype(np.float64)
        eu, ex = kkt.rel_err(u, ref["u"], x, ref["x"], p["weight"])
        assert eu <= TOL_ERR and ex <= TOL_ERR, (b, eu, ex)
