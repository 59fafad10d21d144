"""The associative scan of the refinement's backward recursion, in plain
numpy (CPU): the chunk summaries and their combination, written from the
same formulas the GPU path uses, checked against a dense solve of the
equality-constrained LQ problem each active-set pass solves (all stages'
KKT system at once, no recursion), for several chunkings, including chunks
of one stage and the whole horizon in one chunk.

Problem of one pass (the faces fixed):
  min sum_k 1/2 (x_{k+1} - r_k)^T Q (x_{k+1} - r_k) + 1/2 (u_k - ur_k)^T R (u_k - ur_k)
  s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,  u_k = c_k + P_k w_k  (P_k a projector).
"""
import numpy as np
import pytest

NX, NU = 13, 12


def _problem(rng, N):
    A = [np.eye(NX) + 0.05 * rng.standard_normal((NX, NX)) for _ in range(N)]
    B = [0.1 * rng.standard_normal((NX, NU)) for _ in range(N)]
    e = [0.1 * rng.standard_normal(NX) for _ in range(N)]
    r = [rng.standard_normal(NX) for _ in range(N)]
    ur = [rng.standard_normal(NU) for _ in range(N)]
    Q = np.diag(rng.uniform(1, 100, NX))
    R = np.diag(rng.uniform(1e-3, 1, NU))
    P, c = [], []
    for _ in range(N):
        Pk = np.zeros((NU, NU))
        for i in range(2):
            rank = int(rng.integers(0, 7))
            if rank:
                q, _ = np.linalg.qr(rng.standard_normal((6, rank)))
                Pk[6 * i:6 * i + 6, 6 * i:6 * i + 6] = q @ q.T
        P.append(Pk)
        c.append((np.eye(NU) - Pk) @ rng.standard_normal(NU))   # a point off the face's span
    x0 = rng.standard_normal(NX)
    return dict(A=A, B=B, e=e, r=r, ur=ur, Q=Q, R=R, P=P, c=c, x0=x0, N=N)


def _dense(p):
    """The pass's QP solved at once: unknowns w_0..w_{N-1} (u_k = c_k + P_k w_k),
    states eliminated by the dynamics; a least-squares solve of the normal
    equations (P_k singular: the minimum-norm w gives the unique u)."""
    N = p["N"]
    # x_{k+1} = F_k x0 + sum_j G_kj w_j + h_k
    F = np.eye(NX)
    h = np.zeros(NX)
    G = []
    Hq, hq, Fx = [], [], []
    rows = []
    for k in range(N):
        F = p["A"][k] @ F
        h = p["A"][k] @ h + p["B"][k] @ p["c"][k] + p["e"][k]
        rows = [p["A"][k] @ g for g in rows] + [p["B"][k] @ p["P"][k]]
        G.append(np.hstack(rows + [np.zeros((NX, NU * (N - k - 1)))]))
        Fx.append(F @ p["x0"] + h)
    L = np.sqrt(np.diag(p["Q"]))
    M, v = [], []
    for k in range(N):   # state residuals sqrt(Q) (x_{k+1} - r_k)
        M.append(L[:, None] * G[k])
        v.append(-L * (Fx[k] - p["r"][k]))
    Lr = np.sqrt(np.diag(p["R"]))
    for k in range(N):   # input residuals sqrt(R) (c_k + P_k w_k - ur_k)
        row = np.zeros((NU, NU * N))
        row[:, NU * k:NU * (k + 1)] = Lr[:, None] * p["P"][k]
        M.append(row)
        v.append(-Lr * (p["c"][k] - p["ur"][k]))
    w = np.linalg.lstsq(np.vstack(M), np.concatenate(v), rcond=None)[0]
    return np.array([p["c"][k] + p["P"][k] @ w[NU * k:NU * (k + 1)] for k in range(N)])


def _step(p, k, S, s):
    """One stage of the backward recursion (value of x_{k+1} excluding its
    own cost: W = S + Q), returning the stage's gains and the new value."""
    Q, R, P, A, B = p["Q"], p["R"], p["P"][k], p["A"][k], p["B"][k]
    W = S + Q
    Bp = B @ P
    d = B @ p["c"][k] + p["e"][k]
    q = -Q @ p["r"][k]
    H = P @ R @ P + Bp.T @ W @ Bp + (np.eye(NU) - P)
    Hwx = Bp.T @ W @ A
    hw = P @ R @ (p["c"][k] - p["ur"][k]) + Bp.T @ (W @ d + q + s)
    Hi = np.linalg.inv(H)
    K, kap = -Hi @ Hwx, -Hi @ hw
    S2 = A.T @ W @ A + Hwx.T @ K
    s2 = A.T @ (W @ d + q + s) + Hwx.T @ kap
    return 0.5 * (S2 + S2.T), s2, K, kap, Hi, Bp, d


def _summary(p, k0, k1):
    """Chunk summary from a zero value at x_{k1} (S = -Q, s = -q there):
    closed-loop affine map (A_E, b_E), reachability term C_E, value (S_E, s_E)."""
    S, s = -p["Q"].copy(), p["Q"] @ p["r"][k1 - 1]
    AE, bE, CE = np.eye(NX), np.zeros(NX), np.zeros((NX, NX))
    for k in range(k1 - 1, k0 - 1, -1):
        S, s, K, kap, Hi, Bp, d = _step(p, k, S, s)
        Z = AE @ Bp
        CE = CE + Z @ Hi @ Z.T
        bE = AE @ (d + Bp @ kap) + bE
        AE = AE @ (p["A"][k] + Bp @ K)
    return AE, bE, CE, S, s


def _combine(p, E, S, s, k1):
    """Value at x_{k0} of a chunk with summary E for the value (S, s) at x_{k1}."""
    AE, bE, CE, SE, sE = E
    J = S + p["Q"]
    eta = -(s - p["Q"] @ p["r"][k1 - 1])
    G = np.linalg.inv(np.linalg.inv(J) + CE)
    u = (np.eye(NX) - G @ CE) @ (eta - J @ bE)
    S0 = AE.T @ G @ AE + SE
    return 0.5 * (S0 + S0.T), sE - AE.T @ u


def _scan_solve(p, W):
    """u of the pass by the chunked scan: summaries, boundary values from the
    last chunk back, each chunk's ordinary recursion, then the rollout."""
    N = p["N"]
    b = [(w * N) // W for w in range(W + 1)]
    E = [None] + [_summary(p, b[w], b[w + 1]) for w in range(1, W)]
    V = [None] * W
    S, s = np.zeros((NX, NX)), np.zeros(NX)
    V[W - 1] = (S, s)
    for w in range(W - 1, 0, -1):
        S, s = _combine(p, E[w], S, s, b[w + 1])
        V[w - 1] = (S, s)
    K, kap = [None] * N, [None] * N
    for w in range(W):
        S, s = V[w]
        for k in range(b[w + 1] - 1, b[w] - 1, -1):
            S, s, K[k], kap[k], _, _, _ = _step(p, k, S, s)
    x = p["x0"].copy()
    u = []
    for k in range(N):
        uk = p["c"][k] + p["P"][k] @ (K[k] @ x + kap[k])
        u.append(uk)
        x = p["A"][k] @ x + p["B"][k] @ uk + p["e"][k]
    return np.array(u)


@pytest.mark.parametrize("N,chunks", [(20, (1, 2, 4, 5, 20)), (13, (1, 3, 13)), (40, (8,))])
def test_chunked_scan_solves_the_pass(N, chunks):
    rng = np.random.default_rng(100 + N)
    p = _problem(rng, N)
    ref = _dense(p)
    scale = np.abs(ref).max()
    for W in chunks:
        u = _scan_solve(p, W)
        assert np.abs(u - ref).max() <= 1e-7 * scale, (N, W, np.abs(u - ref).max() / scale)


def test_summary_combination_is_associative():
    """Combining two adjacent chunk summaries' values in either grouping gives
    the same value at the first chunk's start."""
    rng = np.random.default_rng(7)
    p = _problem(rng, 12)
    S, s = np.zeros((NX, NX)), np.zeros(NX)
    # ((E[0:4] E[4:8]) E[8:12]) applied right to left versus E[0:8] as one chunk then E[8:12]
    Sa, sa = _combine(p, _summary(p, 8, 12), S, s, 12)
    Sb, sb = _combine(p, _summary(p, 4, 8), Sa, sa, 8)
    Sc, sc = _combine(p, _summary(p, 0, 4), Sb, sb, 4)
    Sd, sd = _combine(p, _summary(p, 0, 8), Sa, sa, 8)
    assert np.allclose(Sc, Sd, rtol=1e-10, atol=1e-9 * np.abs(Sd).max())
    assert np.allclose(sc, sd, rtol=1e-10, atol=1e-9 * np.abs(sd).max())
