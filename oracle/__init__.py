"""Plain FP64 CPU oracle of the alternating-minimisation (AM) trajectory optimiser.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_2011_04240_amd``)
and imports nothing from it; random inputs come in as arguments.

Paper: Rastgar et al., "GPU Accelerated Convex Approximations for Fast
Multi-Agent Trajectory Optimization" (arXiv 2011.04240).

Modules
  basis  -- trajectory parametrisation P, P-dot, P-ddot, eq. (param), Sec. III-B
  kkt    -- boundary matrix A, collision matrix A_fc (eq. A_f), the KKT matrix
            of eq. (kkt_step_x) and its inverse (Remarks 1-2)
  am     -- Algorithm 1: initialisation, steps (step_x_3d)-(lag_update),
            residual bookkeeping

Pinned by tests/test_oracle_*.py (closed forms, brute force, invariances).
The trajectories on colliding scenes themselves have no published values:
beyond the invariants and sub-step pins, that part is "parity unpinned".
"""
