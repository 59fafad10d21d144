"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies the oracle into a scratch folder, plants one mistake in the
copy (never in the oracle itself), and runs the pins that must catch it
against the copy in a subprocess: at least one of them has to fail.  The
mistakes are the ones the affine terms of Sec. III make easy to write and
that zero e_k, u_ref and u_prev could not reveal:

  * the dynamics residual inside the xi-update indexed with ebar_k instead of
    ebar_{k+1};
  * the sign of the R r^u term of the condensed linear cost flipped;
  * the e_k term dropped from the condensed state trajectory;
  * complementarity measured without the row multiplier;
  * feasibility measured, or the wrench rows built, for the two feet only
    when the hands are contacts too;

and, in the stage matrices built from compact physics (Sec. II-A), the
world-frame inertia rotated the wrong way, the lever-arm cross product
reversed, and the angle rates taken through R_z instead of R_z^T; in the
landmark reward (Sec. II-C), the landmark offsets without their leading 1, the
confidence weights dropped, and the target tick counted in MPC steps instead
of ticks.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("admm-ebar-index", "oracle/admm.py",
     "y = z[k + 1] - v[k + 1] - eb[k + 1] + la[k + 1]",
     "y = z[k + 1] - v[k + 1] - eb[k] + la[k + 1]",
     "block1 and offsets"),
    ("qp-uref-sign", "oracle/qp.py",
     "g = Gam.T @ (qv * (c - r)) - rv * ru",
     "g = Gam.T @ (qv * (c - r)) + rv * ru",
     "(riccati or closed_form) and offsets"),
    ("qp-drop-e", "oracle/qp.py",
     "xc = p[\"A\"][k] @ xc + p[\"e\"][k]",
     "xc = p[\"A\"][k] @ xc",
     "riccati and offsets"),
    ("kkt-comp-without-multiplier", "oracle/kkt.py",
     "r_comp = max(r_comp, (mu[k, i] * slack).max() / (1.0 + mu_max * mg))",
     "r_comp = max(r_comp, (0.0 * mu[k, i] * slack).max() / (1.0 + mu_max * mg))",
     "complementarity"),
    ("kkt-ineq-feet-only", "oracle/kkt.py",
     "grad_u[k] = ru + bl\n        for i in range(nc):",
     "grad_u[k] = ru + bl\n        for i in range(2):",
     "hands"),
    ("qp-hand-rows-dropped", "oracle/qp.py",
     "    for k in range(N):\n        for i in range(nc):\n            if not p[\"contact\"][k][i]:",
     "    for k in range(N):\n        for i in range(2):\n            if not p[\"contact\"][k][i]:",
     "hands or hand"),
    ("dyn-inertia-rotation", "oracle/dynamics.py",
     "Iw = Rz @ np.diag(inertia) @ Rz.T",
     "Iw = Rz.T @ np.diag(inertia) @ Rz",
     "tests/test_oracle_dynamics.py"),
    ("dyn-cross-order", "oracle/dynamics.py",
     "wrench_moment += np.cross(feet[i] - c_ref, f) + tau",
     "wrench_moment += np.cross(f, feet[i] - c_ref) + tau",
     "tests/test_oracle_dynamics.py"),
    ("dyn-angle-rate-rotation", "oracle/dynamics.py",
     "d[0:3] = Rz.T @ omega",
     "d[0:3] = Rz @ omega",
     "tests/test_oracle_dynamics.py"),
    ("lm-offset-base", "oracle/landmarks.py",
     "return [1 + math.floor(Fraction(l, n_landmarks - 1) * (N - 1)) for l in range(n_landmarks)]",
     "return [math.floor(Fraction(l, n_landmarks - 1) * (N - 1)) for l in range(n_landmarks)]",
     "tests/test_oracle_landmarks.py"),
    ("lm-alpha-dropped", "oracle/landmarks.py",
     "total += alpha[l] * float(e @ (np.asarray(qc, dtype=np.float64) * e)) / sigma ** 2",
     "total += float(e @ (np.asarray(qc, dtype=np.float64) * e)) / sigma ** 2",
     "tests/test_oracle_landmarks.py"),
    ("lm-target-in-steps", "oracle/landmarks.py",
     "self.table[(env, step + n * self.d, l)]",
     "self.table[(env, step + n, l)]",
     "tests/test_oracle_landmarks.py"),
]


@pytest.mark.parametrize("name,path,old,new,select", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_oracle_mistake_fails_a_pin(tmp_path, name, path, old, new, select):
    for d in ("oracle", "mpcgen", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path / "pytest.ini")
    src = (tmp_path / path).read_text()
    assert src.count(old) == 1, f"mutation site of {name} not found"
    (tmp_path / path).write_text(src.replace(old, new))
    if select.startswith("tests/"):
        target = [select]                 # a whole pin file
    else:
        target = ["tests/test_oracle_pins.py", "-k", select]
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *target]
    r = subprocess.run(cmd, cwd=tmp_path, capture_output=True, text=True, timeout=600)
    tail = r.stdout[-2000:]
    assert "passed" in tail or "failed" in tail, tail + r.stderr[-2000:]
    assert r.returncode == 1 and "failed" in tail, f"no pin caught {name}:\n{tail}"
