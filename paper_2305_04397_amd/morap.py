"""ctypes binding of libmorap (include/morap.h): the same entry points with
numpy arrays in and out.  Argument marshalling only: every step runs in the
library.  Importing this module loads the in-tree libmorap.so and fails
loudly when it is missing (build it with ``python -m
paper_2305_04397_amd.build``).

libmorap links the system ROCm HIP runtime.  PyTorch wheels bundle their own
runtime with the same soname; whichever loads first serves the whole process,
so import this module before torch when both are used.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmorap.so")

OK, E_INVALID, E_OOM, E_NOT_CONVERGED, E_IMPROPER, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
FEASIBLE, INFEASIBLE, UNDECIDED = 1, 0, 2
_NAMES = {E_INVALID: "INVALID", E_OOM: "OOM", E_NOT_CONVERGED: "NOT_CONVERGED", E_IMPROPER: "IMPROPER",
          E_HIP: "HIP", E_UNSUPPORTED: "UNSUPPORTED", E_STATE: "STATE"}


class MorapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_04397_amd.build`")
    return C.CDLL(LIB_PATH)


lib = _load()

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class Agent(C.Structure):
    _fields_ = [("n_states", C.c_int32), ("n_actions", C.c_int32), ("init", C.c_int32),
                ("sa_ptr", _p), ("succ", _p), ("prob", _p), ("cost", _p)]


class Dfa(C.Structure):
    _fields_ = [("n_locs", C.c_int32), ("n_letters", C.c_int32), ("q0", C.c_int32),
                ("delta", _p), ("accepting", _p)]


class Model(C.Structure):
    _fields_ = [("agent", C.c_int32), ("task", C.c_int32), ("n_states", C.c_int32), ("n_rows", C.c_int32),
                ("nnz", C.c_int32), ("init", C.c_int32), ("state_row", _p), ("row_ptr", _p), ("col", _p),
                ("prob", _p), ("rew", _p), ("to_done", _p)]


class ViOpts(C.Structure):
    _fields_ = [("eps_vi", C.c_double), ("eps_eval", C.c_double), ("tau", C.c_double),
                ("precision", C.c_int32), ("max_sweeps", C.c_int32), ("check_every", C.c_int32),
                ("schedule", C.c_int32), ("use_graph", C.c_int32), ("time_kernels", C.c_int32),
                ("eval_start", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("backups", C.c_int64), ("sweeps", C.c_int64), ("max_pair_sweeps", C.c_int64),
                ("eval_sweeps", C.c_int64), ("polish_sweeps", C.c_int64), ("rank_rounds", C.c_int64),
                ("floor_stops", C.c_int64), ("bytes", C.c_double), ("ms_vi", C.c_double),
                ("ms_eval", C.c_double), ("ms_total", C.c_double), ("ms_sweep_kernel", C.c_double),
                ("sweep_launches", C.c_int64), ("bytes_refine", C.c_double),
                ("ms_sweep_kernel_refine", C.c_double), ("sweep_launches_refine", C.c_int64),
                ("variant", C.c_int32), ("variant_refine", C.c_int32), ("sweeps_tail", C.c_int64),
                ("sweep_launches_tail", C.c_int64), ("bytes_tail", C.c_double),
                ("ms_sweep_kernel_tail", C.c_double), ("variant_tail", C.c_int32), ("reserved", C.c_int32),
                ("refine_pairs", C.c_int64), ("refine_columns", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class QueryOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int32), ("verification_only", C.c_int32),
                ("use_proposer", C.c_int32), ("keep_trace", C.c_int32), ("warm_start", C.c_int32),
                ("proposer_passes", C.c_int32), ("vi", ViOpts)]


class QueryResult(C.Structure):
    _fields_ = [("verdict", C.c_int32), ("iterations", C.c_int32), ("fallback", C.c_int32),
                ("reserved", C.c_int32), ("gap", C.c_double), ("ms", C.c_double), ("backups", C.c_int64),
                ("t_up", _p), ("t_down", _p), ("lam", _p), ("trace_w", _p), ("trace_r", _p), ("trace_f", _p),
                ("latency_ms", C.c_double)]


class TrainOpts(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("seed", C.c_uint64)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_ctxp = _p
_sig("morap_create", C.c_int, C.POINTER(_p), C.c_int, _p)
_sig("morap_destroy", C.c_int, _ctxp)
_sig("morap_last_error", C.c_char_p, _ctxp)
_sig("morap_set_memory_budget", C.c_int, _ctxp, C.c_int64, _p)
_sig("morap_build_products", C.c_int, _ctxp, C.POINTER(Agent), C.c_int, C.POINTER(Dfa), C.c_int, C.POINTER(_p))
_sig("morap_load_models", C.c_int, _ctxp, C.POINTER(Model), C.c_int, C.c_int, C.c_int)
_sig("morap_model_info", C.c_int, _ctxp, C.c_int, _p)
_sig("morap_get_model", C.c_int, _ctxp, C.c_int, _p, _p, _p, _p, _p, _p, _p)
_sig("morap_default_opts", None, C.POINTER(ViOpts))
_sig("morap_solve", C.c_int, _ctxp, _p, C.c_int, C.POINTER(ViOpts), _p, C.POINTER(Stats))
_sig("morap_solve_staged", C.c_int, _ctxp, _p, C.c_int, C.POINTER(ViOpts), _p, C.POINTER(Stats))
_sig("morap_evaluate", C.c_int, _ctxp, _p, C.c_int, C.POINTER(ViOpts), _p, C.POINTER(Stats))
_sig("morap_assign", C.c_int, _ctxp, _p, C.c_int, _p)
_sig("morap_assign_host", C.c_int, _p, C.c_int, C.c_int, C.c_int, _p)
_sig("morap_product_host", C.c_int, C.POINTER(Agent), C.POINTER(Dfa), _p, _p, _p, _p, _p, _p, _p, _p, _p)
_sig("morap_team_model_host", C.c_int, C.POINTER(Agent), C.c_int, C.POINTER(Dfa), C.c_int, C.POINTER(_p), _p, _p,
     _p, _p, _p, _p, _p, _p)
_sig("morap_team_model_mo_host", C.c_int, C.POINTER(Agent), C.c_int, C.POINTER(Dfa), C.c_int, C.POINTER(_p), _p,
     _p, _p, _p, _p, _p, _p, _p)
_sig("morap_load_team_model", C.c_int, _ctxp, C.c_int, C.c_int, C.POINTER(Model), _p)
_sig("morap_support", C.c_int, _ctxp, _p, C.c_int, C.POINTER(ViOpts), _p, _p, _p, C.POINTER(Stats))
_sig("morap_get_policy", C.c_int, _ctxp, C.c_int, C.c_int, _p)
_sig("morap_get_stats", C.c_int, _ctxp, C.POINTER(Stats))
_sig("morap_reset_stats", C.c_int, _ctxp)
_sig("morap_get_values", C.c_int, _ctxp, C.c_int, C.c_int, _p)
_sig("morap_query", C.c_int, _ctxp, _p, _p, C.POINTER(QueryOpts), C.POINTER(QueryResult))
_sig("morap_query_batch", C.c_int, _ctxp, _p, _p, C.c_int, _p, C.POINTER(QueryOpts), C.POINTER(QueryResult))
_sig("morap_synthesize", C.c_int, _ctxp, _p, _p, _p, C.c_int, C.POINTER(ViOpts), _p, _p, _p, _p)
_sig("morap_project_inner", C.c_int, _p, C.c_int, C.c_int, _p, _p, _p, _p)
_sig("morap_project_outer", C.c_int, _p, _p, C.c_int, C.c_int, _p, _p, _p)
_sig("morap_set_features", C.c_int, _ctxp, _p, C.c_int)
_sig("morap_proposer_target", C.c_int, _p, _p, _p, C.c_int, _p, _p)
_sig("morap_proposer_init", C.c_int, _ctxp, C.c_int, C.c_int, C.c_uint64)
_sig("morap_proposer_num_params", C.c_int64, _ctxp)
_sig("morap_proposer_get_params", C.c_int, _ctxp, _p)
_sig("morap_proposer_set_params", C.c_int, _ctxp, _p)
_sig("morap_proposer_set_input_norm", C.c_int, _ctxp, _p, _p)
_sig("morap_proposer_infer", C.c_int, _ctxp, _p, C.c_int, _p)
_sig("morap_proposer_infer_noalloc", C.c_int, _ctxp, _p, C.c_int, _p)
_sig("morap_proposer_step", C.c_int, _ctxp, _p, _p, C.c_int, C.POINTER(TrainOpts), C.c_int, _p, _p)
_sig("morap_proposer_train", C.c_int, _ctxp, _p, _p, C.c_int, C.POINTER(TrainOpts), _p)
_sig("morap_proposer_save", C.c_int, _ctxp, C.c_char_p)
_sig("morap_proposer_load", C.c_int, _ctxp, C.c_char_p)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_p)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Options:
    """Mirror of morap_vi_opts."""
    eps_vi: float = 1e-6
    eps_eval: Optional[float] = None
    tau: float = 1e-9
    precision: str = "f32"
    max_sweeps: int = 1_000_000
    check_every: int = 32
    schedule: int = 0
    use_graph: bool = True
    time_kernels: bool = False
    eval_from_values: bool = False   # Alg. 4 starts from the solve's scalarised values

    def to_c(self) -> ViOpts:
        o = ViOpts()
        o.eps_vi = self.eps_vi
        o.eps_eval = self.eps_vi if self.eps_eval is None else self.eps_eval
        o.tau = self.tau
        o.precision = F32 if self.precision == "f32" else F64
        o.max_sweeps = self.max_sweeps
        o.check_every = self.check_every
        o.schedule = self.schedule
        o.use_graph = 1 if self.use_graph else 0
        o.time_kernels = 1 if self.time_kernels else 0
        o.eval_start = 1 if self.eval_from_values else 0
        return o


def proposer_target(t, t_down, w_last, M=None) -> np.ndarray:
    """morap_proposer_target: the weight vector a query should have started
    from (host, no context)."""
    t, t_down, w_last = _c(t, np.float64), _c(t_down, np.float64), _c(w_last, np.float64)
    Mc = None if M is None else _c(M, np.float64)
    out = np.zeros(t.size)
    rc = lib.morap_proposer_target(_ptr(t), _ptr(t_down), _ptr(w_last), t.size, _ptr(Mc), _ptr(out))
    if rc != 0:
        raise MorapError(rc, "morap_proposer_target failed")
    return out


def product_host(agent, task, letters) -> dict:
    """One agent x task product built on the host, no context (the layout of
    ``Context.get_model``)."""
    arrs = [_c(agent.sa_ptr, np.int32), _c(agent.succ, np.int32), _c(agent.prob, np.float64),
            _c(agent.cost, np.float64)]
    a = Agent(agent.n_states, agent.n_actions, agent.init, *[_ptr(x) for x in arrs])
    tarrs = [_c(task.delta, np.int32), _c(task.accepting, np.uint8)]
    t = Dfa(task.n_locs, task.n_letters, task.q0, *[_ptr(x) for x in tarrs])
    lets = _c(letters, np.int32)
    sizes = np.zeros(4, np.int32)
    rc = lib.morap_product_host(C.byref(a), C.byref(t), _ptr(lets), _ptr(sizes), *([None] * 7))
    if rc:
        raise MorapError(rc, "product construction failed")
    S, R, N, init = (int(v) for v in sizes)
    out = {"state_row": np.zeros(S + 1, np.int32), "row_ptr": np.zeros(R + 1, np.int32),
           "col": np.zeros(N, np.int32), "prob": np.zeros(N), "rew": np.zeros((R, 2)),
           "to_done": np.zeros(R, np.uint8), "states": np.zeros((S, 2), np.int32), "init": init}
    rc = lib.morap_product_host(C.byref(a), C.byref(t), _ptr(lets), _ptr(sizes),
                                *[_ptr(out[k]) for k in ("state_row", "row_ptr", "col", "prob", "rew", "to_done",
                                                         "states")])
    if rc:
        raise MorapError(rc, "product construction failed")
    return out


def team_model_host(workload, w) -> dict:
    """The team MDP of ``workload`` (|I| = |J|) scalarised for the weight
    vector w, as one single-objective model for ``Context.load_models`` (a
    1 x 1 problem solved with the weight row (1, 0))."""
    n = workload.n_agents
    keep = []
    agents = (Agent * n)()
    for i, a in enumerate(workload.agents):
        arrs = [_c(a.sa_ptr, np.int32), _c(a.succ, np.int32), _c(a.prob, np.float64), _c(a.cost, np.float64)]
        keep += arrs
        agents[i] = Agent(a.n_states, a.n_actions, a.init, *[_ptr(x) for x in arrs])
    tasks = (Dfa * workload.n_tasks)()
    for j, t in enumerate(workload.tasks):
        arrs = [_c(t.delta, np.int32), _c(t.accepting, np.uint8)]
        keep += arrs
        tasks[j] = Dfa(t.n_locs, t.n_letters, t.q0, *[_ptr(x) for x in arrs])
    lets = (_p * (n * workload.n_tasks))()
    for i in range(n):
        for j in range(workload.n_tasks):
            arr = _c(workload.letters[i][j], np.int32)
            keep.append(arr)
            lets[i * workload.n_tasks + j] = arr.ctypes.data
    wv = _c(w, np.float64)
    sizes = np.zeros(4, np.int32)
    nJ = workload.n_tasks
    rc = lib.morap_team_model_host(agents, n, tasks, nJ, lets, _ptr(wv), _ptr(sizes), *([None] * 6))
    if rc:
        raise MorapError(rc, "team MDP construction failed")
    S, R, N, init = (int(v) for v in sizes)
    out = {"state_row": np.zeros(S + 1, np.int32), "row_ptr": np.zeros(R + 1, np.int32),
           "col": np.zeros(N, np.int32), "prob": np.zeros(N), "rew": np.zeros((R, 2)),
           "to_done": np.zeros(R, np.uint8), "init": init}
    rc = lib.morap_team_model_host(agents, n, tasks, nJ, lets, _ptr(wv), _ptr(sizes),
                                   *[_ptr(out[k]) for k in ("state_row", "row_ptr", "col", "prob", "rew", "to_done")])
    if rc:
        raise MorapError(rc, "team MDP construction failed")
    return out


def team_model_mo_host(workload) -> dict:
    """The team MDP of ``workload`` (|I| = |J|) with its d = 2n objectives
    (Def. teamMDP), for ``Context.load_team_model``: rew [R, 2] = (-cost,
    acceptance mass) and obj [R, 2] the objective each belongs to."""
    n = workload.n_agents
    keep = []
    agents = (Agent * n)()
    for i, a in enumerate(workload.agents):
        arrs = [_c(a.sa_ptr, np.int32), _c(a.succ, np.int32), _c(a.prob, np.float64), _c(a.cost, np.float64)]
        keep += arrs
        agents[i] = Agent(a.n_states, a.n_actions, a.init, *[_ptr(x) for x in arrs])
    tasks = (Dfa * workload.n_tasks)()
    for j, t in enumerate(workload.tasks):
        arrs = [_c(t.delta, np.int32), _c(t.accepting, np.uint8)]
        keep += arrs
        tasks[j] = Dfa(t.n_locs, t.n_letters, t.q0, *[_ptr(x) for x in arrs])
    nJ = workload.n_tasks
    lets = (_p * (n * nJ))()
    for i in range(n):
        for j in range(nJ):
            arr = _c(workload.letters[i][j], np.int32)
            keep.append(arr)
            lets[i * nJ + j] = arr.ctypes.data
    sizes = np.zeros(4, np.int32)
    rc = lib.morap_team_model_mo_host(agents, n, tasks, nJ, lets, _ptr(sizes), *([None] * 7))
    if rc:
        raise MorapError(rc, "team MDP construction failed")
    S, R, N, init = (int(v) for v in sizes)
    out = {"state_row": np.zeros(S + 1, np.int32), "row_ptr": np.zeros(R + 1, np.int32),
           "col": np.zeros(N, np.int32), "prob": np.zeros(N), "rew": np.zeros((R, 2)),
           "obj": np.zeros((R, 2), np.int32), "to_done": np.zeros(R, np.uint8), "init": init}
    rc = lib.morap_team_model_mo_host(agents, n, tasks, nJ, lets, _ptr(sizes),
                                      *[_ptr(out[k]) for k in ("state_row", "row_ptr", "col", "prob", "rew", "obj",
                                                               "to_done")])
    if rc:
        raise MorapError(rc, "team MDP construction failed")
    return out


def assign_host(c):
    """Alg. 2's assignment on the host, no context: c [K, nI, nJ] -> the
    agent of each task, [K, nJ]."""
    c = np.asarray(c, dtype=np.float64)
    c = _c(c[None] if c.ndim == 2 else c, np.float64)
    K, nI, nJ = c.shape
    out = np.zeros((K, nJ), np.int32)
    rc = lib.morap_assign_host(_ptr(c), nI, nJ, K, _ptr(out))
    if rc:
        raise MorapError(rc, "assignment failed")
    return out


def project_inner(Phi, t, M=None):
    """Alg. 1 inner projection (host): returns (x, lam)."""
    Phi = _c(np.atleast_2d(Phi), np.float64)
    t = _c(t, np.float64)
    m, d = Phi.shape
    x = np.zeros(d)
    lam = np.zeros(m)
    Mc = None if M is None else _c(M, np.float64)
    rc = lib.morap_project_inner(_ptr(Phi), m, d, _ptr(t), _ptr(Mc), _ptr(x), _ptr(lam))
    if rc:
        raise MorapError(rc, "inner projection failed")
    return x, lam


def project_outer(W, R, t, M=None):
    """Alg. 1 outer projection (host)."""
    W = _c(np.atleast_2d(W), np.float64)
    R = _c(np.atleast_2d(R), np.float64)
    t = _c(t, np.float64)
    n, d = W.shape
    z = np.zeros(d)
    Mc = None if M is None else _c(M, np.float64)
    rc = lib.morap_project_outer(_ptr(W), _ptr(R), n, d, _ptr(t), _ptr(Mc), _ptr(z))
    if rc:
        raise MorapError(rc, "outer projection failed")
    return z


class Context:
    """One morap_ctx (one HIP device, one stream)."""

    def __init__(self, device: int = 0, stream=None):
        h = _p()
        handle = None
        if stream is not None:
            handle = _p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        rc = lib.morap_create(C.byref(h), device, handle)
        if rc:
            raise MorapError(rc, f"morap_create(device={device}) failed")
        self._h = h
        self.nI = self.nJ = 0
        self.team = False
        self._keep = []

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc:
            msg = lib.morap_last_error(self._h)
            raise MorapError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_h", None):
            lib.morap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def d(self) -> int:
        return self.nI + self.nJ

    # -- models ------------------------------------------------------------
    def build_products(self, workload):
        """Build every agent-task product of a ``workloads.Workload``."""
        keep = []
        nI, nJ = workload.n_agents, workload.n_tasks
        agents = (Agent * nI)()
        for i, a in enumerate(workload.agents):
            arrs = [_c(a.sa_ptr, np.int32), _c(a.succ, np.int32), _c(a.prob, np.float64), _c(a.cost, np.float64)]
            keep += arrs
            agents[i] = Agent(a.n_states, a.n_actions, a.init, *[_ptr(x) for x in arrs])
        tasks = (Dfa * nJ)()
        for j, t in enumerate(workload.tasks):
            arrs = [_c(t.delta, np.int32), _c(t.accepting, np.uint8)]
            keep += arrs
            tasks[j] = Dfa(t.n_locs, t.n_letters, t.q0, *[_ptr(x) for x in arrs])
        lets = (_p * (nI * nJ))()
        for i in range(nI):
            for j in range(nJ):
                arr = _c(workload.letters[i][j], np.int32)
                keep.append(arr)
                lets[i * nJ + j] = arr.ctypes.data
        self._check(lib.morap_build_products(self._h, agents, nI, tasks, nJ, lets), "morap_build_products")
        self.nI, self.nJ = nI, nJ
        self.team = False

    def load_models(self, models: Sequence[dict], n_agents: int, n_tasks: int):
        """models[m]: dict with state_row, row_ptr, col, prob, rew [R,2], to_done, init."""
        keep = []
        arr = (Model * len(models))()
        for m, md in enumerate(models):
            a = [_c(md["state_row"], np.int32), _c(md["row_ptr"], np.int32), _c(md["col"], np.int32),
                 _c(md["prob"], np.float64), _c(md["rew"], np.float64), _c(md["to_done"], np.uint8)]
            keep += a
            S = len(a[0]) - 1
            arr[m] = Model(m // n_tasks, m % n_tasks, S, len(a[1]) - 1, len(a[2]), int(md["init"]),
                           *[_ptr(x) for x in a])
        self._check(lib.morap_load_models(self._h, arr, len(models), n_agents, n_tasks), "morap_load_models")
        self.nI, self.nJ = n_agents, n_tasks
        self.team = False

    def load_team_model(self, model: dict, n_agents: int, n_tasks: int):
        """A team MDP with its d = n_agents + n_tasks objectives (from
        ``team_model_mo_host``): solve takes W [K, d] and returns c [K] (the
        value at the initial state), support returns r [K, d]."""
        a = [_c(model["state_row"], np.int32), _c(model["row_ptr"], np.int32), _c(model["col"], np.int32),
             _c(model["prob"], np.float64), _c(model["rew"], np.float64), _c(model["to_done"], np.uint8)]
        obj = _c(model["obj"], np.int32)
        md = Model(0, 0, len(a[0]) - 1, len(a[1]) - 1, len(a[2]), int(model["init"]), *[_ptr(x) for x in a])
        self._check(lib.morap_load_team_model(self._h, n_agents, n_tasks, C.byref(md), _ptr(obj)),
                    "morap_load_team_model")
        self.nI, self.nJ = n_agents, n_tasks
        self.team = True

    def _c_shape(self, K):
        return (K,) if self.team else (K, self.nI, self.nJ)

    def model_info(self, m: int) -> dict:
        s = np.zeros(5, np.int32)
        self._check(lib.morap_model_info(self._h, m, _ptr(s)), "morap_model_info")
        return {"n_states": int(s[0]), "n_rows": int(s[1]), "nnz": int(s[2]), "init": int(s[3]),
                "total_states": int(s[4])}

    def get_model(self, m: int) -> dict:
        info = self.model_info(m)
        S, R, N = info["n_states"], info["n_rows"], info["nnz"]
        out = {"state_row": np.zeros(S + 1, np.int32), "row_ptr": np.zeros(R + 1, np.int32),
               "col": np.zeros(N, np.int32), "prob": np.zeros(N), "rew": np.zeros((R, 2)),
               "to_done": np.zeros(R, np.uint8), "states": np.zeros((S, 2), np.int32), "init": info["init"]}
        self._check(lib.morap_get_model(self._h, m, *[_ptr(out[k]) for k in
                                                     ("state_row", "row_ptr", "col", "prob", "rew", "to_done",
                                                      "states")]), "morap_get_model")
        return out

    # -- Alg. 2 / 3 / 4 ----------------------------------------------------
    def solve(self, W, opts: Options = Options()):
        W = _c(np.atleast_2d(W), np.float64)
        K = W.shape[0]
        c = np.zeros(self._c_shape(K))
        st = Stats()
        o = opts.to_c()
        self._check(lib.morap_solve(self._h, _ptr(W), K, C.byref(o), _ptr(c), C.byref(st)), "morap_solve")
        return c, st.as_dict()

    def solve_staged(self, W, opts: Options = Options(precision="f64")):
        """morap_solve with stages retiring inside the iteration (FP64)."""
        W = _c(np.atleast_2d(W), np.float64)
        K = W.shape[0]
        c = np.zeros(self._c_shape(K))
        st = Stats()
        o = opts.to_c()
        self._check(lib.morap_solve_staged(self._h, _ptr(W), K, C.byref(o), _ptr(c), C.byref(st)),
                    "morap_solve_staged")
        return c, st.as_dict()

    def evaluate(self, assign, opts: Options = Options(), K: int = None):
        """assign [K, nJ]; on a team model None (give K)."""
        A = None if assign is None else _c(np.atleast_2d(assign), np.int32)
        K = A.shape[0] if A is not None else int(K)
        r = np.zeros((K, self.d))
        st = Stats()
        o = opts.to_c()
        self._check(lib.morap_evaluate(self._h, _ptr(A) if A is not None else None, K, C.byref(o), _ptr(r),
                                       C.byref(st)), "morap_evaluate")
        return r, st.as_dict()

    def assign(self, c):
        c = _c(c, np.float64).reshape(-1, self.nI, self.nJ)
        out = np.zeros((c.shape[0], self.nJ), np.int32)
        self._check(lib.morap_assign(self._h, _ptr(c), c.shape[0], _ptr(out)), "morap_assign")
        return out

    def support(self, W, opts: Options = Options()):
        W = _c(np.atleast_2d(W), np.float64)
        K = W.shape[0]
        r = np.zeros((K, self.d))
        A = np.zeros((K, self.nJ), np.int32)
        c = np.zeros(self._c_shape(K))
        st = Stats()
        o = opts.to_c()
        self._check(lib.morap_support(self._h, _ptr(W), K, C.byref(o), _ptr(r), _ptr(A), _ptr(c), C.byref(st)),
                    "morap_support")
        return r, A, c, st.as_dict()

    def stats(self) -> dict:
        st = Stats()
        self._check(lib.morap_get_stats(self._h, C.byref(st)), "morap_get_stats")
        return st.as_dict()

    def reset_stats(self):
        self._check(lib.morap_reset_stats(self._h), "morap_reset_stats")

    def get_policy(self, k: int, j: int, n_states: int) -> np.ndarray:
        mu = np.zeros(n_states, np.int8)
        self._check(lib.morap_get_policy(self._h, k, j, _ptr(mu)), "morap_get_policy")
        return mu

    def get_values(self, k: int, m: int) -> np.ndarray:
        x = np.zeros(self.model_info(m)["n_states"])
        self._check(lib.morap_get_values(self._h, k, m, _ptr(x)), "morap_get_values")
        return x

    # -- Alg. 1 ------------------------------------------------------------
    def query_batch(self, T, M=None, eps: float = 1e-3, max_iter: int = 64, opts: Options = Options(),
                    verification_only: bool = False, use_proposer: bool = False, trace: bool = False,
                    W0=None, warm_start: bool = True, proposer_passes: int = 1):
        T = _c(np.atleast_2d(T), np.float64)
        Q, d = T.shape
        W0c = None if W0 is None else _c(np.atleast_2d(W0), np.float64)
        qo = QueryOpts()
        qo.eps, qo.max_iter = eps, max_iter
        qo.verification_only = int(verification_only)
        qo.use_proposer = int(use_proposer)
        qo.keep_trace = int(trace)
        qo.warm_start = int(warm_start)
        qo.proposer_passes = int(proposer_passes)
        qo.vi = opts.to_c()
        res = (QueryResult * Q)()
        bufs = []
        for q in range(Q):
            b = {"t_up": np.zeros(d), "t_down": np.zeros(d), "lam": np.zeros(max_iter),
                 "trace_w": np.zeros((max_iter, d)), "trace_r": np.zeros((max_iter, d)),
                 "trace_f": np.zeros((max_iter, self.nJ), np.int32)}
            bufs.append(b)
            for k, v in b.items():
                setattr(res[q], k, _ptr(v))
        Mc = None if M is None else _c(M, np.float64)
        self._check(lib.morap_query_batch(self._h, _ptr(T), _ptr(W0c), Q, _ptr(Mc), C.byref(qo), res),
                    "morap_query_batch")
        out = []
        for q in range(Q):
            n = res[q].iterations
            out.append({"verdict": res[q].verdict, "iterations": n, "fallback": res[q].fallback,
                        "gap": res[q].gap, "ms": res[q].ms, "latency_ms": res[q].latency_ms,
                        "backups": res[q].backups,
                        "t_up": bufs[q]["t_up"], "t_down": bufs[q]["t_down"], "lam": bufs[q]["lam"][:n],
                        "W": bufs[q]["trace_w"][:n], "R": bufs[q]["trace_r"][:n], "F": bufs[q]["trace_f"][:n]})
        return out

    def query(self, t, M=None, **kw) -> dict:
        return self.query_batch(np.atleast_2d(t), M, **kw)[0]

    def synthesize(self, q: dict, opts: Options = Options()) -> dict:
        """morap_synthesize on a traced query result (its W, F and lam): the
        picked passes, their points, the random assignment matrix [|I|][|J|]
        and the scheduler of every task in every picked pass (model
        (F[pass][j], j))."""
        W = _c(q["W"], np.float64)
        F = _c(q["F"], np.int32)
        v = _c(q["lam"], np.float64)
        n = W.shape[0]
        npk = C.c_int32(0)
        picked = np.zeros(n, np.int32)
        R = np.zeros((n, self.d))
        mat = np.zeros((self.nI, self.nJ))
        o = opts.to_c()
        self._check(lib.morap_synthesize(self._h, _ptr(W), _ptr(F), _ptr(v), n, C.byref(o), C.byref(npk),
                                         _ptr(picked), _ptr(R), _ptr(mat)), "morap_synthesize")
        m = npk.value
        picked = picked[:m]
        sched = [[self.get_policy(k, j, self.model_info(int(F[p, j]) * self.nJ + j)["n_states"])
                  for j in range(self.nJ)] for k, p in enumerate(picked)]
        return {"picked": picked, "v": v[picked], "F": F[picked], "R": R[:m], "matrix": mat,
                "schedulers": sched}

    # -- proposer ----------------------------------------------------------
    def set_features(self, phi):
        phi = _c(phi, np.float64)
        self._check(lib.morap_set_features(self._h, _ptr(phi), len(phi)), "morap_set_features")

    def proposer_num_params(self) -> int:
        return int(lib.morap_proposer_num_params(self._h))

    def set_memory_budget(self, nbytes: int) -> int:
        """Device memory budget in bytes (0 = none); returns the bytes held."""
        used = C.c_int64()
        self._check(lib.morap_set_memory_budget(self._h, int(nbytes), C.byref(used)), "morap_set_memory_budget")
        return int(used.value)

    def proposer_init(self, n_in: int, d: int, seed: int = 0):
        self._check(lib.morap_proposer_init(self._h, n_in, d, seed), "morap_proposer_init")

    def proposer_params(self) -> np.ndarray:
        n = lib.morap_proposer_num_params(self._h)
        out = np.zeros(n, np.float32)
        self._check(lib.morap_proposer_get_params(self._h, _ptr(out)), "morap_proposer_get_params")
        return out

    def proposer_set_params(self, flat):
        flat = _c(flat, np.float32)
        self._check(lib.morap_proposer_set_params(self._h, _ptr(flat)), "morap_proposer_set_params")

    def proposer_set_input_norm(self, mu, sd):
        mu, sd = _c(mu, np.float32), _c(sd, np.float32)
        self._check(lib.morap_proposer_set_input_norm(self._h, _ptr(mu), _ptr(sd)),
                    "morap_proposer_set_input_norm")

    def proposer_infer(self, X, d: int) -> np.ndarray:
        X = _c(np.atleast_2d(X), np.float32)
        out = np.zeros((X.shape[0], d), np.float32)
        self._check(lib.morap_proposer_infer(self._h, _ptr(X), X.shape[0], _ptr(out)), "morap_proposer_infer")
        return out

    def proposer_infer_noalloc(self, x_dev: int, n: int, w_dev: int):
        """morap_proposer_infer_noalloc on device pointers (integers); enqueued
        on the context's stream, not waited for."""
        self._check(lib.morap_proposer_infer_noalloc(self._h, C.c_void_p(x_dev), n, C.c_void_p(w_dev)),
                    "morap_proposer_infer_noalloc")

    @staticmethod
    def _topts(batch=4096, epochs=1, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, seed=0) -> TrainOpts:
        return TrainOpts(batch, epochs, lr, beta1, beta2, adam_eps, seed)

    def proposer_step(self, X, T, apply: bool = False, with_grads: bool = True, **kw):
        X = _c(np.atleast_2d(X), np.float32)
        T = _c(np.atleast_2d(T), np.float32)
        loss = np.zeros(1, np.float32)
        grads = np.zeros(lib.morap_proposer_num_params(self._h), np.float32) if with_grads else None
        o = self._topts(**kw)
        self._check(lib.morap_proposer_step(self._h, _ptr(X), _ptr(T), X.shape[0], C.byref(o), int(apply),
                                            _ptr(loss), _ptr(grads)), "morap_proposer_step")
        return float(loss[0]), grads

    def proposer_train(self, X, T, **kw) -> np.ndarray:
        X = _c(np.atleast_2d(X), np.float32)
        T = _c(np.atleast_2d(T), np.float32)
        o = self._topts(**kw)
        losses = np.zeros(o.epochs, np.float32)
        self._check(lib.morap_proposer_train(self._h, _ptr(X), _ptr(T), X.shape[0], C.byref(o), _ptr(losses)),
                    "morap_proposer_train")
        return losses

    def proposer_save(self, path: str):
        self._check(lib.morap_proposer_save(self._h, path.encode()), "morap_proposer_save")

    def proposer_load(self, path: str):
        self._check(lib.morap_proposer_load(self._h, path.encode()), "morap_proposer_load")
