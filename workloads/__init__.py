"""Seeded synthetic inputs: grid-world agent MDPs, task DFAs, labellings,
weight vectors and threshold points.

This package draws random numbers and lays out raw problem data only.  It holds
none of the method's arithmetic (no product construction, no value iteration,
no assignment, no geometry); both the HIP library's callers and the CPU oracle
consume what it produces.
"""
from .gridworld import (  # noqa: F401
    Agent, Task, Workload, make_workload, make_agent, make_task_dfa,
    dirichlet_weights, workload_seed, worked_example, tiny_workload,
)
