"""Synthetic batches of linear time-varying centroidal MPC problems.

Every problem is drawn from its own substream ``default_rng([seed, index])``, so
any subset of a batch is reproducible on its own and independent of the batch
size.  Values are generated in float64 and then rounded to float32; the rounded
arrays are the problem as stored, and both the FP64 oracle and the GPU solver
solve exactly that rounded problem (the oracle upcasts it).

Model (single-rigid-body centroidal dynamics, forward Euler; the paper's
discrete centroidal dynamics of Sec. II-A written in the 13-state form with
gravity carried as a state):

    x = (roll, pitch, yaw, p (3), omega (3), v (3), g_s)      13 states
    u = per contact i in {0, 1}: (f_i (3), tau_i (3))          12 inputs
        (model "hands": contacts 2, 3 are the hands, 24 inputs)
    A_k = I + dt * A_c(yaw),   B_k = dt * B_c(yaw, r_{i,k}, m, I_body)
    r_{i,k} = p_i - c_ref,k  (foot position minus reference CoM at stage k)

The standard-form problem (Sec. III) that results is

    min  sum_k 1/2 |x_{k+1} - x_ref[k]|_Q^2 + 1/2 |u_k - u_ref[k]|_R^2
    s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,   x_0 given,
         stance contact: |f_x|, |f_y| <= mu f_z, f_z <= fz_max, |tau_j| <= tau_max
         swing contact:  f = 0, tau = 0.
"""
from __future__ import annotations

import math

import numpy as np

NX = 13          # state dimension
NU = 12          # input dimension: 2 contacts x (force 3 + moment 3)
NC = 2           # contacts
GRAVITY = 9.81
COM_HEIGHT = 0.8
GAIT_PERIOD = 0.4
FOOT_HALF_WIDTH = 0.10

# Workloads.  ``horizons`` is the set the per-problem horizon is drawn from
# uniformly; ``duty`` None draws the stance fraction per problem from
# U(0.35, 0.65) (flight, single and double support all occur).
CONFIGS = {
    "small_b64_n10": dict(batch=64, horizons=(10,), dt=0.04, duty=0.5,
                          mu=(0.4, 0.8), push=0.0, payload=0.0, seed=1),
    "plain_b4096_n20": dict(batch=4096, horizons=(20,), dt=0.03, duty=0.6,
                            mu=(0.3, 0.9), push=0.5, payload=0.0, seed=2),
    "uneven_b16384": dict(batch=16384, horizons=(10, 20, 30, 40, 60), dt=0.03,
                          duty=None, mu=(0.3, 0.9), push=0.5, payload=0.0,
                          seed=3),
    "precision_b16384_n30": dict(batch=16384, horizons=(30,), dt=0.03,
                                 duty=0.6, mu=(0.3, 0.9), push=0.5,
                                 payload=0.0, seed=4),
    # long single horizons at small batch (horizon split across workgroups)
    "long_b64_n400": dict(batch=64, horizons=(100, 200, 400), dt=0.03, duty=0.6,
                          mu=(0.3, 0.9), push=0.5, payload=0.0, seed=6),
    "serving_tick": dict(batch=32768, horizons=tuple(range(10, 61)), dt=0.03,
                         duty=None, mu=(0.3, 0.9), push=0.5, payload=10.0,
                         seed=5),
    # loco-manipulation: both feet and both hands as contacts (24 inputs)
    "hands_b4096_n20": dict(batch=4096, horizons=(20,), dt=0.03, duty=0.6,
                            mu=(0.3, 0.9), push=0.5, payload=10.0, seed=7,
                            model="hands"),
}

# Hands (model "hands"): nominal position relative to the CoM in the heading
# frame, and the contact frame of a hand: its local z axis (the normal of the
# wrench set's pyramid) points backwards along the heading, so a pushing hand
# takes the reaction of the pushed object as a normal force, and its local x
# axis points up.  Hand inputs are expressed in that frame.
HAND_NOMINAL = ((0.35, 0.20, 0.25), (0.35, -0.20, 0.25))
HAND_FRAME = np.array([[0.0, 0.0, -1.0],
                       [0.0, 1.0, 0.0],
                       [1.0, 0.0, 0.0]])


def _cfg(config):
    if isinstance(config, str):
        return dict(CONFIGS[config])
    return dict(config)


def _draw(cfg, seed, idx):
    """Per-problem scalar draws, in a fixed order from one substream."""
    rng = np.random.default_rng([int(seed), int(idx)])
    d = {}
    d["mass"] = rng.uniform(30.0, 60.0)
    d["inertia"] = rng.uniform(1.0, 4.0, 3)
    d["yaw"] = rng.uniform(-math.pi, math.pi)
    d["vx"] = rng.uniform(-1.0, 1.0)
    lo, hi = cfg["mu"]
    d["mu"] = lo + (hi - lo) * rng.uniform(0.0, 1.0)
    d["phase"] = rng.uniform(0.0, 1.0)
    d["q"] = rng.uniform(1.0, 100.0, NX)
    d["foot_off"] = rng.normal(0.0, 0.1, (NC, 3))
    d["push"] = cfg["push"] * rng.normal(0.0, 1.0, 3)
    duty = rng.uniform(0.35, 0.65)
    d["duty"] = duty if cfg["duty"] is None else cfg["duty"]
    hz = cfg["horizons"]
    d["N"] = int(hz[int(rng.integers(0, len(hz)))])
    d["mass"] += cfg["payload"] * rng.uniform(0.0, 1.0)
    return d


def _rotz(psi):
    c, s = np.cos(psi), np.sin(psi)
    R = np.zeros(psi.shape + (3, 3))
    R[..., 0, 0] = c
    R[..., 0, 1] = -s
    R[..., 1, 0] = s
    R[..., 1, 1] = c
    R[..., 2, 2] = 1.0
    return R


def _skew(r):
    S = np.zeros(r.shape[:-1] + (3, 3))
    S[..., 0, 1] = -r[..., 2]
    S[..., 0, 2] = r[..., 1]
    S[..., 1, 0] = r[..., 2]
    S[..., 1, 2] = -r[..., 0]
    S[..., 2, 0] = -r[..., 1]
    S[..., 2, 1] = r[..., 0]
    return S


def _draw_hands(seed, idx):
    """Per-problem draws of the hand contacts (model "hands"), from a substream
    of their own: position offsets N(0, 0.05) m per hand, the phase and the
    fraction U(0.5, 1) of the push cycle (twice the gait period) the hands are
    in contact, and each hand's reference normal force U(40, 120) N (the
    pushing-force reference of loco-manipulation)."""
    rng = np.random.default_rng([int(seed), int(idx), 11])
    return dict(off=rng.normal(0.0, 0.05, (2, 3)), phase=rng.uniform(0.0, 1.0),
                duty=rng.uniform(0.5, 1.0), push=rng.uniform(40.0, 120.0, 2))


def _draw_offsets(seed, idx, n, N, mass, nc=NC):
    """Nonzero affine terms of one problem, from a substream of its own (so the
    draws of ``_draw`` and every workload without offsets are unchanged):

      e_k     per-stage disturbance of the dynamics, different at every stage
              (angles and positions N(0, 2e-3), angular and linear velocity
              N(0, 0.02), gravity state N(0, 1e-3))
      u_ref   input reference: each contact's force (N(0, 20), N(0, 20),
              m g / 2 + N(0, 30)) and moment N(0, 5)^3, at every stage
              (swing stages included: their inputs are fixed to 0 anyway)
      u_prev  input before stage 0: forces N(0, 50), moments N(0, 5)
    """
    rng = np.random.default_rng([int(seed), int(idx), 7])
    sd = np.array([2e-3] * 6 + [0.02] * 6 + [1e-3])
    e = rng.normal(0.0, 1.0, (n, NX)) * sd
    ur = np.zeros((n, 6 * nc))
    up = np.zeros(6 * nc)
    for i in range(nc):
        ur[:, 6 * i:6 * i + 3] = rng.normal(0.0, 1.0, (n, 3)) * np.array([20.0, 20.0, 30.0])
        ur[:, 6 * i + 2] += 0.5 * mass * GRAVITY
        ur[:, 6 * i + 3:6 * i + 6] = rng.normal(0.0, 5.0, (n, 3))
        up[6 * i:6 * i + 3] = rng.normal(0.0, 50.0, 3)
        up[6 * i + 3:6 * i + 6] = rng.normal(0.0, 5.0, 3)
    e[N:] = 0.0
    ur[N:] = 0.0
    return e, ur, up


def make_batch(config, indices=None, batch=None, seed=None, n_max=None,
               dt=None, as_float32=True, offsets=False, model=None):
    """Build a batch of problems.

    config   name in CONFIGS or a dict with the same keys
    indices  problem indices to draw (default range(batch))
    n_max    padded horizon (default: the largest drawn horizon)
    offsets  draw nonzero e_k, u_ref and u_prev (``_draw_offsets``); without
             it all three are zero, as in the paper's workloads
    model    "srb": the 13-state single-rigid-body form above; "momentum": the
             paper's 9-state centroidal model (CoM, linear momentum, angular
             momentum about the CoM; Sec. II-A) in slots 0..8 of the same
             13-slot layout, slots 9..12 inert (A = I, B = 0, e = 0, x0 = 0,
             reference 0, weight 1), gravity in e_k = (0, dt m g, 0); the same
             draws, the weights carried over (Q_v / m^2 on l, Q_omega / I^2 on
             k), the lever arm at the reference CoM; "hands": the 13-state
             form with four contacts, the feet (0, 1) and the hands (2, 3):
             a hand sits at the reference CoM plus its nominal offset (turned
             by the yaw) plus its drawn offset, its force and moment are in
             its contact frame (HAND_FRAME turned by the yaw), both hands are
             in contact on the same push cycle, its input reference is its
             drawn normal force while in contact, and its force weight in R is
             1e-3 (the moments keep 1e-5); default: the config's model, else
             "srb"

    Returns a dict of arrays (float32 unless ``as_float32`` is False):
      N [B] int32, A [B,n,13,13], B [B,n,13,m], e [B,n,13], x0 [B,13],
      u_prev [B,m], x_ref [B,n,13] (reference for x_{k+1}), u_ref [B,n,m],
      Q [B,13], R [B,m] (diagonals), contact [B,n,c] uint8 (1 = stance) with
      c contacts and m = 6 c inputs (c = 4 for "hands", else 2),
      mu [B], fz_max [B], tau_max [B], weight [B] (m g, the force scale),
      and the compact physics of A and B: yaw_k [B,n], c_ref [B,n,3], feet
      [B,n,2,3], mass [B], inertia [B,3], dt [B].
    Stages k >= N[b] are padding: A = I, B = 0, e = 0, references 0, swing.
    """
    cfg = _cfg(config)
    if model is None:
        model = cfg.get("model", "srb")
    if seed is None:
        seed = cfg["seed"]
    if dt is None:
        dt = cfg["dt"]
    if indices is None:
        indices = np.arange(cfg["batch"] if batch is None else batch)
    indices = np.asarray(indices, dtype=np.int64)
    Bn = len(indices)
    draws = [_draw(cfg, seed, i) for i in indices]
    Nh = np.array([d["N"] for d in draws], dtype=np.int32)
    if n_max is None:
        n_max = int(Nh.max()) if Bn else int(max(cfg["horizons"]))
    if Bn and int(Nh.max()) > n_max:
        raise ValueError("n_max smaller than a drawn horizon")
    n = n_max

    if Bn == 0:
        return _empty(n, 4 if model == "hands" else NC)

    def col(key):
        return np.array([d[key] for d in draws], dtype=np.float64)

    mass = col("mass")
    inertia = col("inertia")
    yaw = col("yaw")
    vx = col("vx")
    mu = col("mu")
    phase = col("phase")
    q = col("q")
    foot_off = col("foot_off")
    push = col("push")
    duty = col("duty")

    Rz = _rotz(yaw)                                            # [B,3,3]
    Iw = Rz @ (inertia[:, :, None] * np.swapaxes(Rz, 1, 2))      # R diag(I) R^T
    Iw_inv = np.linalg.inv(Iw)
    vel_w = Rz @ np.array([1.0, 0.0, 0.0]) * vx[:, None]        # [B,3]
    c0 = np.array([0.0, 0.0, COM_HEIGHT])
    kk = np.arange(n + 1, dtype=np.float64)
    c_ref = c0[None, None, :] + kk[None, :, None] * dt * vel_w[:, None, :]  # [B,n+1,3]

    side = np.array([FOOT_HALF_WIDTH, -FOOT_HALF_WIDTH])
    feet = np.zeros((Bn, NC, 3))
    for i in range(NC):
        feet[:, i, :] = (Rz @ np.array([0.0, side[i], 0.0])) + foot_off[:, i, :]
        feet[:, i, 2] = foot_off[:, i, 2]

    # continuous-time A_c and the forward-Euler A_k (identical over k: the yaw
    # linearisation point is the constant reference yaw)
    Ac = np.zeros((Bn, NX, NX))
    Ac[:, 0:3, 6:9] = np.swapaxes(Rz, 1, 2)
    Ac[:, 3:6, 9:12] = np.eye(3)
    Ac[:, 11, 12] = 1.0
    A1 = np.eye(NX)[None] + dt * Ac                              # [B,13,13]

    stage = np.arange(n)
    valid = stage[None, :] < Nh[:, None]                         # [B,n]
    A = np.where(valid[:, :, None, None], A1[:, None], np.eye(NX)[None, None])

    Bm = np.zeros((Bn, n, NX, NU))
    for i in range(NC):
        r = feet[:, None, i, :] - c_ref[:, :n, :]                # [B,n,3]
        Bm[:, :, 6:9, 6 * i:6 * i + 3] = Iw_inv[:, None] @ _skew(r)
        Bm[:, :, 6:9, 6 * i + 3:6 * i + 6] = Iw_inv[:, None]
        Bm[:, :, 9:12, 6 * i:6 * i + 3] = np.eye(3)[None, None] / mass[:, None, None, None]
    Bm *= dt
    Bm[~valid] = 0.0

    # reference state at stage j (time j*dt); x_ref[k] is the target of x_{k+1}
    xr = np.zeros((Bn, n + 1, NX))
    xr[:, :, 2] = yaw[:, None]
    xr[:, :, 3:6] = c_ref
    xr[:, :, 9:12] = vel_w[:, None, :]
    xr[:, :, 12] = -GRAVITY
    x_ref = xr[:, 1:, :].copy()
    x_ref[~valid] = 0.0
    x0 = xr[:, 0, :].copy()
    x0[:, 9:12] += push

    ph = phase[:, None, None] + stage[None, :, None] * dt / GAIT_PERIOD \
        + np.arange(NC)[None, None, :] / NC
    frac = ph - np.floor(ph)
    contact = (frac < duty[:, None, None]) & valid[:, :, None]

    out = {
        "N": Nh,
        "A": A,
        "B": Bm,
        "e": np.zeros((Bn, n, NX)),
        "x0": x0,
        "u_prev": np.zeros((Bn, NU)),
        "x_ref": x_ref,
        "u_ref": np.zeros((Bn, n, NU)),
        "Q": q,
        "R": np.full((Bn, NU), 1e-5),
        "contact": contact.astype(np.uint8),
        "mu": mu,
        "fz_max": np.full(Bn, 1000.0),
        "tau_max": np.full(Bn, 50.0),
        "weight": mass * GRAVITY,
        # the compact physics the matrices above are built from (the input of
        # an on-device construction): yaw, reference CoM and contact positions
        # per stage (zero on padding), mass, principal moments, time step
        "yaw_k": np.where(valid, yaw[:, None], 0.0),
        "c_ref": np.where(valid[:, :, None], c_ref[:, :n, :], 0.0),
        "feet": np.where(valid[:, :, None, None], feet[:, None, :, :], 0.0),
        "mass": mass,
        "inertia": inertia,
        "dt": np.full(Bn, float(dt)),
    }
    if model == "momentum":
        if offsets:
            raise ValueError("offsets are drawn for the single-rigid-body layout only")
        Am = np.tile(np.eye(NX), (Bn, n, 1, 1))
        Am[:, :, 0:3, 3:6] = (dt / mass)[:, None, None, None] * np.eye(3)
        Bq = np.zeros((Bn, n, NX, NU))
        for i in range(NC):
            r = feet[:, None, i, :] - c_ref[:, :n, :]
            Bq[:, :, 3:6, 6 * i:6 * i + 3] = dt * np.eye(3)
            Bq[:, :, 6:9, 6 * i:6 * i + 3] = dt * _skew(r)
            Bq[:, :, 6:9, 6 * i + 3:6 * i + 6] = dt * np.eye(3)
        eq = np.zeros((Bn, n, NX))
        eq[:, :, 5] = -dt * mass[:, None] * GRAVITY
        Am[~valid] = np.eye(NX)
        Bq[~valid] = 0.0
        eq[~valid] = 0.0
        xq0 = np.zeros((Bn, NX))
        xq0[:, 0:3] = out["x0"][:, 3:6]
        xq0[:, 3:6] = mass[:, None] * out["x0"][:, 9:12]
        xqr = np.zeros((Bn, n, NX))
        xqr[:, :, 0:3] = out["x_ref"][:, :, 3:6]
        xqr[:, :, 3:6] = mass[:, None, None] * out["x_ref"][:, :, 9:12]
        xqr[~valid] = 0.0
        qq = np.ones((Bn, NX))
        qq[:, 0:3] = q[:, 3:6]
        qq[:, 3:6] = q[:, 9:12] / mass[:, None] ** 2
        qq[:, 6:9] = q[:, 6:9] / inertia.mean(axis=1)[:, None] ** 2
        out.update(A=Am, B=Bq, e=eq, x0=xq0, x_ref=xqr, Q=qq)
    elif model == "hands":
        hd = [_draw_hands(seed, i) for i in indices]
        Bh = np.zeros((Bn, n, NX, 6 * 4))
        Bh[..., :NU] = Bm
        ch = np.zeros((Bn, n, 4), dtype=bool)
        ch[..., :NC] = contact
        urh = np.zeros((Bn, n, 6 * 4))
        Rh = np.full((Bn, 6 * 4), 1e-5)
        hoff = np.array([d["off"] for d in hd])                     # [B,2,3]
        hph = np.array([d["phase"] for d in hd])
        hdu = np.array([d["duty"] for d in hd])
        hpush = np.array([d["push"] for d in hd])                   # [B,2]
        frame = Rz @ HAND_FRAME                                      # [B,3,3]
        hfr = hph[:, None] + stage[None, :] * dt / (2.0 * GAIT_PERIOD)
        hcon = ((hfr - np.floor(hfr)) < hdu[:, None]) & valid         # [B,n]
        for h in range(2):
            i = NC + h
            r = (Rz @ np.array(HAND_NOMINAL[h])) + hoff[:, h, :]      # [B,3]
            Bh[:, :, 6:9, 6 * i:6 * i + 3] = (Iw_inv @ _skew(r) @ frame)[:, None]
            Bh[:, :, 6:9, 6 * i + 3:6 * i + 6] = (Iw_inv @ frame)[:, None]
            Bh[:, :, 9:12, 6 * i:6 * i + 3] = (frame / mass[:, None, None])[:, None]
            ch[..., i] = hcon
            urh[:, :, 6 * i + 2] = np.where(hcon, hpush[:, h, None], 0.0)
            Rh[:, 6 * i:6 * i + 3] = 1e-3
        Bh[:, :, :, NU:] *= dt
        Bh[~valid] = 0.0
        out.update(B=Bh, contact=ch.astype(np.uint8), u_ref=urh, R=Rh,
                   u_prev=np.zeros((Bn, 6 * 4)))
    elif model != "srb":
        raise ValueError(f"unknown model {model!r}")
    if offsets:
        nc = out["contact"].shape[2]
        for j, idx in enumerate(indices):
            e, ur, up = _draw_offsets(seed, idx, n, int(Nh[j]), mass[j], nc)
            out["e"][j] = e
            out["u_ref"][j] = ur if model != "hands" else ur + out["u_ref"][j]
            out["u_prev"][j] = up
    if as_float32:
        for k, v in out.items():
            if v.dtype == np.float64:
                out[k] = np.ascontiguousarray(v.astype(np.float32))
    for k, v in out.items():
        out[k] = np.ascontiguousarray(v)
    return out


def _empty(n, nc=NC):
    f = np.float32
    nu = 6 * nc
    return {
        "N": np.zeros(0, np.int32), "A": np.zeros((0, n, NX, NX), f),
        "B": np.zeros((0, n, NX, nu), f), "e": np.zeros((0, n, NX), f),
        "x0": np.zeros((0, NX), f), "u_prev": np.zeros((0, nu), f),
        "x_ref": np.zeros((0, n, NX), f), "u_ref": np.zeros((0, n, nu), f),
        "Q": np.zeros((0, NX), f), "R": np.zeros((0, nu), f),
        "contact": np.zeros((0, n, nc), np.uint8), "mu": np.zeros(0, f),
        "fz_max": np.zeros(0, f), "tau_max": np.zeros(0, f),
        "weight": np.zeros(0, f), "yaw_k": np.zeros((0, n), f),
        "c_ref": np.zeros((0, n, 3), f), "feet": np.zeros((0, n, NC, 3), f),
        "mass": np.zeros(0, f), "inertia": np.zeros((0, 3), f), "dt": np.zeros(0, f),
    }


def problem_slice(batch, idx):
    """Sub-batch with the problems ``idx`` (array of positions)."""
    idx = np.asarray(idx)
    return {k: np.ascontiguousarray(v[idx]) for k, v in batch.items()}


def problem_fp64(batch, b):
    """Problem ``b`` of a batch, trimmed to its own horizon, as float64."""
    N = int(batch["N"][b])
    p = {"N": N}
    for k, v in batch.items():
        if k == "N":
            continue
        a = v[b]
        if a.ndim >= 1 and k in ("A", "B", "e", "x_ref", "u_ref", "contact"):
            a = a[:N]
        p[k] = a.astype(np.float64) if k != "contact" else a.astype(bool)
    return p
