"""FP64 CPU oracle for the batched scalarised value-iteration path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or run it; the library
and its Python binding never do.  It shares no code with the HIP path: it
reads the raw agent / task data produced by ``workloads`` and builds its own
product models.

Modules (each function cites the passage of Robinson & Su, "Multi-Objective
Task Assignment and Multiagent Planning with Hybrid GPU-CPU Acceleration",
that it follows):
  product   agent x DFA product MDPs with done_j and the two reward columns
  vi        scalarised value iteration (Alg. 3) and its stage-ordered form,
            policy extraction, policy evaluation (Alg. 4), exact evaluation
            by a sparse solve
  geometry  M-norm projections of Alg. 1 (inner and outer approximation)
  alg       Alg. 2 (supporting hyperplane: VI, assignment, evaluation) and
            Alg. 1 (point-oriented Pareto computation)
  mlp       FP64 reference of the learned weight proposer (not in the paper)
  centralised  the team MDP of the decentralised model (Def. teamMDP), small
            instances only, as an independent check of Alg. 2

Parity unpinned: the literal pre-sink probability reward (``presink_literal``)
and the trajectory-dependent policy rule (``policy_rule="paper"``) are kept as
options for the record only; nothing pins them.
"""
from . import product, vi, geometry, alg, mlp, centralised  # noqa: F401
