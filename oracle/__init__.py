"""FP64 CPU oracle for the batched centroidal MPC solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library;
the only common input is the seeded workload generator (``mpcgen``), which
holds none of the solver's arithmetic.

Modules
  qp          exact optimum of the standard-form QP (Sec. III): dense
              condensed QP, Mehrotra interior point, active-set polish and a
              KKT certificate.  The result every GPU solve is compared with.
  admm        the paper's parallel-in-horizon ADMM (Sec. III, the three-block
              update with cached J_k, H_k) in FP64, optionally with block-
              constant input scaling and fast ADMM with restart.  Iterate-level
              reference only: its iterates at a fixed iteration count are not
              pinned by the paper (rho, restart constant and initial iterate
              are not given), so iterate parity is "parity unpinned".
  projection  Euclidean projection onto the stage wrench set.
  kkt         the accuracy measures (solution error, normalised KKT
              residuals) applied to any candidate solution.
  landmarks   the landmark guidance reward of Sec. II-C (landmark offsets, the
              store of predicted CoM landmarks, the reward).
  dynamics    the stage matrices A_k, B_k of the centroidal model (Sec. II-A)
              from compact physics (yaw, reference CoM, contact positions,
              mass, inertia, time step), each column from its definition.
"""
from . import projection, qp, admm, kkt, dynamics, landmarks  # noqa: F401
