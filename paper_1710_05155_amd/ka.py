"""Thin ctypes binding of libka (include/ka.h).  Argument marshalling only: every step of
the sweep runs in the library's HIP kernels; torch is used, if at all, only to hand over a
HIP stream.  Importing this module does not touch the GPU; loading the library does not
either.  There is no fallback: if libka.so is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# KA_LIB names another build of libka (for example one with the host code under sanitizers)
LIB_PATH = os.environ.get("KA_LIB") or os.path.join(PKG, "libka.so")

KA_OK = 0
KA_EINVAL = -1
KA_ENOMEM = -2
KA_EDEVICE = -3
KA_ESTATE = -4
KA_OPT_PATH = 1
KA_OPT_TIMING = 2
KA_OPT_NOISE = 3
KA_OPT_PLANE_STREAMS = 4
KA_OPT_TAIL = 5
KA_OPT_PLANE_GROUPS = 6

# Every symbol include/ka.h declares.
SYMBOLS = (
    "ka_graph_lattice", "ka_graph_rrg", "ka_graph_layered", "ka_graph_from_adjacency", "ka_graph_info",
    "ka_graph_export", "ka_graph_free", "ka_footprint", "ka_init", "ka_init_k", "ka_sweep",
    "ka_observe", "ka_observe_pairs", "ka_run", "ka_get_state", "ka_set_state", "ka_sim_info", "ka_set_option",
    "ka_timing", "ka_sim_path", "ka_free", "ka_last_error",
    "ka_batch_create", "ka_batch_add", "ka_batch_run", "ka_batch_steps_left", "ka_batch_poll",
    "ka_batch_wait_all", "ka_batch_set_option", "ka_batch_info", "ka_batch_free",
    "ka_server_create", "ka_server_submit", "ka_server_poll", "ka_server_result", "ka_server_take_sim", "ka_server_release",
    "ka_server_wait_idle", "ka_server_stats", "ka_server_free", "ka_probe_valu",
    "ka_particles", "ka_derived", "ka_g4", "ka_observe_noalloc",
)


class JobDesc(ctypes.Structure):
    """ka_job_desc (include/ka.h)."""
    _fields_ = [
        ("graph", ctypes.c_void_p),
        ("m", ctypes.c_int),
        ("rho", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("n_replicas", ctypes.c_int),
        ("n_sweeps", ctypes.c_int64),
        ("obs_times", ctypes.c_void_p),
        ("n_obs", ctypes.c_int),
        ("keep_sim", ctypes.c_int),
    ]


KA_BOPT_AUTOTUNE = 1
KA_BOPT_BLOCK = 2
KA_BOPT_GRAPH_STEPS = 4
KA_BOPT_CACHE_BUDGET = 5
KA_BOPT_SOLO_BYTES = 6


class KaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libka error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libka.so (built in-tree by build.py); raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KaError(KA_EDEVICE, f"{LIB_PATH} is not built (run paper_1710_05155_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    I = ctypes.c_int
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    D = ctypes.c_double
    sig = {
        "ka_graph_lattice": ([I, I, PP], I),
        "ka_graph_rrg": ([I64, I, U64, PP], I),
        "ka_graph_layered": ([I, I, I, U64, PP], I),
        "ka_graph_from_adjacency": ([I64, I, P, PP], I),
        "ka_graph_info": ([P, P, P, P, P], I),
        "ka_graph_export": ([P, P, P, P, P], I),
        "ka_graph_free": ([P], None),
        "ka_footprint": ([P, I, P], I),
        "ka_init": ([P, I, D, U64, I, P, PP], I),
        "ka_init_k": ([P, I, I64, U64, I, P, PP], I),
        "ka_sweep": ([P, I64], I),
        "ka_observe": ([P, P, P, P, P], I),
        "ka_observe_noalloc": ([P, P, P, P, P], I),
        "ka_run": ([P, P, I, P, P, P], I),
        "ka_observe_pairs": ([P, I, P, P, P], I),
        "ka_get_state": ([P, P, P, P, P], I),
        "ka_set_state": ([P, P, P, P, I64], I),
        "ka_sim_info": ([P, P, P, P, P, P, P], I),
        "ka_set_option": ([P, I, I64], I),
        "ka_timing": ([P, P, P, P], I),
        "ka_sim_path": ([P, P], I),
        "ka_free": ([P], None),
        "ka_last_error": ([], ctypes.c_char_p),
        "ka_batch_create": ([I, P, PP], I),
        "ka_batch_add": ([P, P, I64, P], I),
        "ka_batch_run": ([P, I64], I),
        "ka_batch_steps_left": ([P, P], I),
        "ka_batch_poll": ([P, P, I, P], I),
        "ka_batch_wait_all": ([P], I),
        "ka_batch_set_option": ([P, I, I64], I),
        "ka_batch_info": ([P, P, P, P, P], I),
        "ka_batch_free": ([P], None),
        "ka_server_create": ([ctypes.c_size_t, I, P, PP], I),
        "ka_server_submit": ([P, ctypes.POINTER(JobDesc), P], I),
        "ka_server_poll": ([P, P, I, P], I),
        "ka_server_result": ([P, I64, P, P, P, P, P], I),
        "ka_server_take_sim": ([P, I64, PP], I),
        "ka_server_release": ([P, I64], I),
        "ka_server_wait_idle": ([P], I),
        "ka_server_stats": ([P, P, P, P, P], I),
        "ka_server_free": ([P], None),
        "ka_probe_valu": ([I, I, I, P, P, P], I),
        "ka_particles": ([I64, D, P], I),
        "ka_derived": ([I64, I64, I, I, P, P, P, P, P], I),
        "ka_g4": ([I64, I64, I, I, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != KA_OK:
        msg = load().ka_last_error()
        raise KaError(rc, msg.decode() if msg else "")


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Graph:
    """Owning handle of a ka_graph."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        N = ctypes.c_int64()
        z = ctypes.c_int()
        E = ctypes.c_int64()
        C = ctypes.c_int()
        _check(load().ka_graph_info(self._h, ctypes.byref(N), ctypes.byref(z), ctypes.byref(E),
                                    ctypes.byref(C)))
        self.N, self.z, self.E, self.C = N.value, z.value, E.value, C.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ka_graph_free(self._h)
            self._h = None


class Sim:
    """Owning handle of a ka_sim."""

    def __init__(self, handle: ctypes.c_void_p, graph: Graph, stream):
        self._h = handle
        self.graph = graph
        self.stream = stream
        N = ctypes.c_int64()
        R = ctypes.c_int()
        K = ctypes.c_int64()
        m = ctypes.c_int()
        t = ctypes.c_int64()
        C = ctypes.c_int()
        _check(load().ka_sim_info(self._h, ctypes.byref(N), ctypes.byref(R), ctypes.byref(K),
                                  ctypes.byref(m), ctypes.byref(t), ctypes.byref(C)))
        self.N, self.R, self.K, self.m, self.C = N.value, R.value, K.value, m.value, C.value

    @property
    def handle(self):
        return self._h

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        _check(load().ka_sim_info(self._h, None, None, None, None, ctypes.byref(t), None))
        return t.value

    def free(self):
        if self._h and _lib is not None:
            _lib.ka_free(self._h)
        self._h = None

    def __del__(self):
        self.free()


# ------------------------------------------------------------------------------ graphs
def ka_graph_lattice(d: int, L: int) -> Graph:
    h = ctypes.c_void_p()
    _check(load().ka_graph_lattice(d, L, ctypes.byref(h)))
    return Graph(h)


def ka_graph_rrg(N: int, z: int, graph_seed: int) -> Graph:
    h = ctypes.c_void_p()
    _check(load().ka_graph_rrg(N, z, graph_seed, ctypes.byref(h)))
    return Graph(h)


def ka_graph_layered(d: int, L: int, M: int, graph_seed: int) -> Graph:
    h = ctypes.c_void_p()
    _check(load().ka_graph_layered(d, L, M, graph_seed, ctypes.byref(h)))
    return Graph(h)


def ka_graph_from_adjacency(adj) -> Graph:
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    N, z = adj.shape
    h = ctypes.c_void_p()
    _check(load().ka_graph_from_adjacency(N, z, _ptr(adj), ctypes.byref(h)))
    return Graph(h)


def ka_graph_info(g: Graph):
    return g.N, g.z, g.E, g.C


def ka_graph_export(g: Graph):
    adj = np.empty((g.N, g.z), dtype=np.int32)
    eu = np.empty(g.E, dtype=np.int32)
    ev = np.empty(g.E, dtype=np.int32)
    ec = np.empty(g.E, dtype=np.int32)
    _check(load().ka_graph_export(g.handle, _ptr(adj), _ptr(eu), _ptr(ev), _ptr(ec)))
    return adj, eu, ev, ec


def ka_footprint(g: Graph, n_replicas: int) -> int:
    out = ctypes.c_size_t()
    _check(load().ka_footprint(g.handle, n_replicas, ctypes.byref(out)))
    return int(out.value)


# ------------------------------------------------------------------------------ sims
def ka_init(g: Graph, m: int, rho: float, seed: int, n_replicas: int, stream=None) -> Sim:
    h = ctypes.c_void_p()
    _check(load().ka_init(g.handle, m, float(rho), seed, n_replicas, _stream_handle(stream),
                          ctypes.byref(h)))
    return Sim(h, g, stream)


def ka_init_k(g: Graph, m: int, K: int, seed: int, n_replicas: int, stream=None) -> Sim:
    h = ctypes.c_void_p()
    _check(load().ka_init_k(g.handle, m, int(K), seed, n_replicas, _stream_handle(stream),
                            ctypes.byref(h)))
    return Sim(h, g, stream)


def ka_sweep(s: Sim, n_sweeps: int) -> None:
    _check(load().ka_sweep(s.handle, int(n_sweeps)))


def ka_observe(s: Sim):
    t = ctypes.c_int64()
    dens = np.empty(s.R, dtype=np.int64)
    ov = np.empty(s.R, dtype=np.int64)
    pers = np.empty(s.R, dtype=np.int64)
    _check(load().ka_observe(s.handle, ctypes.byref(t), _ptr(dens), _ptr(ov), _ptr(pers)))
    return t.value, dens, ov, pers


def ka_observe_noalloc(s: Sim):
    """ka_observe through the library's fixed device scratch (no device allocation)."""
    t = ctypes.c_int64()
    dens = np.empty(s.R, dtype=np.int64)
    ov = np.empty(s.R, dtype=np.int64)
    pers = np.empty(s.R, dtype=np.int64)
    _check(load().ka_observe_noalloc(s.handle, ctypes.byref(t), _ptr(dens), _ptr(ov), _ptr(pers)))
    return t.value, dens, ov, pers


def ka_observe_pairs(s: Sim, r2_max: int):
    """Four-point sums per shell r2 = 0..r2_max: (S2, S11, count), int64 arrays."""
    S2 = np.empty(r2_max + 1, dtype=np.int64)
    S11 = np.empty(r2_max + 1, dtype=np.int64)
    cnt = np.empty(r2_max + 1, dtype=np.int64)
    _check(load().ka_observe_pairs(s.handle, int(r2_max), _ptr(S2), _ptr(S11), _ptr(cnt)))
    return S2, S11, cnt


def ka_run(s: Sim, obs_times):
    times = np.ascontiguousarray(np.asarray(obs_times, dtype=np.int64))
    n = times.shape[0]
    dens = np.empty((n, s.R), dtype=np.int64)
    ov = np.empty((n, s.R), dtype=np.int64)
    pers = np.empty((n, s.R), dtype=np.int64)
    _check(load().ka_run(s.handle, _ptr(times), n, _ptr(dens), _ptr(ov), _ptr(pers)))
    return dens, ov, pers


def ka_get_state(s: Sim, n: bool = True, n0: bool = True, f: bool = True):
    """(n, n0, f, t) in the canonical [W][N] layout; an array not asked for comes back as None."""
    W = s.R // 64
    arrs = [np.empty((W, s.N), dtype=np.uint64) if want else None for want in (n, n0, f)]
    t = ctypes.c_int64()
    ptrs = [_ptr(a) if a is not None else None for a in arrs]
    _check(load().ka_get_state(s.handle, ptrs[0], ptrs[1], ptrs[2], ctypes.byref(t)))
    return arrs[0], arrs[1], arrs[2], t.value


def ka_set_state(s: Sim, n, n0, f, t: int) -> None:
    W = s.R // 64
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(W, s.N)) for a in (n, n0, f)]
    _check(load().ka_set_state(s.handle, _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), int(t)))


def ka_set_option(s: Sim, option: int, value: int) -> None:
    _check(load().ka_set_option(s.handle, option, int(value)))


def ka_timing(s: Sim):
    launches = ctypes.c_int64()
    timed = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().ka_timing(s.handle, ctypes.byref(launches), ctypes.byref(timed), ctypes.byref(ms)))
    return launches.value, timed.value, ms.value


def ka_sim_path(s: Sim) -> int:
    p = ctypes.c_int()
    _check(load().ka_sim_path(s.handle, ctypes.byref(p)))
    return p.value


def ka_free(s: Sim) -> None:
    s.free()


def ka_last_error() -> str:
    msg = load().ka_last_error()
    return msg.decode() if msg else ""


# ------------------------------------------------------------------------------ batches
class Batch:
    """Owning handle of a ka_batch.  Members are Sim objects; the batch keeps them alive."""

    def __init__(self, handle, stream):
        self._h = handle
        self.stream = stream
        self.members = {}

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h and _lib is not None:
            _lib.ka_batch_free(self._h)
        self._h = None
        self.members = {}

    def __del__(self):
        self.free()


def ka_batch_create(capacity: int, stream=None) -> Batch:
    h = ctypes.c_void_p()
    _check(load().ka_batch_create(int(capacity), _stream_handle(stream), ctypes.byref(h)))
    return Batch(h, stream)


def ka_batch_add(b: Batch, s: Sim, n_sweeps: int) -> int:
    slot = ctypes.c_int()
    _check(load().ka_batch_add(b.handle, s.handle, int(n_sweeps), ctypes.byref(slot)))
    b.members[slot.value] = s
    return slot.value


def ka_batch_run(b: Batch, n_steps: int) -> None:
    _check(load().ka_batch_run(b.handle, int(n_steps)))


def ka_batch_steps_left(b: Batch) -> int:
    v = ctypes.c_int64()
    _check(load().ka_batch_steps_left(b.handle, ctypes.byref(v)))
    return v.value


def ka_batch_poll(b: Batch) -> list:
    """Slots whose members finished on the device (now detached)."""
    cap = max(1, len(b.members))
    slots = np.empty(cap, dtype=np.int32)
    n = ctypes.c_int()
    _check(load().ka_batch_poll(b.handle, _ptr(slots), cap, ctypes.byref(n)))
    out = [int(x) for x in slots[: n.value]]
    for k in out:
        b.members.pop(k, None)
    return out


def ka_batch_wait_all(b: Batch) -> None:
    _check(load().ka_batch_wait_all(b.handle))
    b.members = {}


def ka_batch_set_option(b: Batch, option: int, value: int) -> None:
    _check(load().ka_batch_set_option(b.handle, option, int(value)))


def ka_batch_info(b: Batch):
    step = ctypes.c_int64()
    members = ctypes.c_int()
    block = ctypes.c_int()
    tiles = ctypes.c_int()
    _check(load().ka_batch_info(b.handle, ctypes.byref(step), ctypes.byref(members), ctypes.byref(block),
                                ctypes.byref(tiles)))
    return step.value, members.value, block.value, tiles.value


def ka_batch_free(b: Batch) -> None:
    b.free()


# ------------------------------------------------------------------------------ serving
class Server:
    """Owning handle of a ka_server.  Keeps the graphs of queued jobs alive."""

    def __init__(self, handle, stream):
        self._h = handle
        self.stream = stream
        self.jobs = {}   # id -> (graph, n_obs, R)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h and _lib is not None:
            _lib.ka_server_free(self._h)
        self._h = None

    def __del__(self):
        self.free()


def ka_server_create(device_budget: int, max_active: int, stream=None) -> Server:
    h = ctypes.c_void_p()
    _check(load().ka_server_create(int(device_budget), int(max_active), _stream_handle(stream), ctypes.byref(h)))
    return Server(h, stream)


def ka_server_submit(sv: Server, graph: Graph, m: int, rho: float, seed: int, n_replicas: int,
                     n_sweeps: int, obs_times=None, keep_sim: bool = False) -> int:
    obs = None if obs_times is None else np.ascontiguousarray(np.asarray(obs_times, dtype=np.int64))
    d = JobDesc(graph.handle, int(m), float(rho), int(seed), int(n_replicas), int(n_sweeps),
                _ptr(obs) if obs is not None else None, 0 if obs is None else int(obs.shape[0]),
                1 if keep_sim else 0)
    jid = ctypes.c_int64()
    _check(load().ka_server_submit(sv.handle, ctypes.byref(d), ctypes.byref(jid)))
    sv.jobs[jid.value] = (graph, 1 if obs is None else int(obs.shape[0]), int(n_replicas))
    return jid.value


def ka_server_poll(sv: Server, max_ids: int = 4096) -> list:
    ids = np.empty(max_ids, dtype=np.int64)
    n = ctypes.c_int()
    _check(load().ka_server_poll(sv.handle, _ptr(ids), max_ids, ctypes.byref(n)))
    return [int(x) for x in ids[: n.value]]


def ka_server_result(sv: Server, job_id: int):
    info = sv.jobs.get(int(job_id))
    if info is None:   # not submitted here, or released: the library reports the error
        _check(load().ka_server_result(sv.handle, int(job_id), None, None, None, None, None))
        raise KaError(KA_ESTATE, f"job {job_id} is unknown")
    _, n_obs, R = info
    dens = np.empty((n_obs, R), dtype=np.int64)
    ov = np.empty((n_obs, R), dtype=np.int64)
    pers = np.empty((n_obs, R), dtype=np.int64)
    wait = ctypes.c_double()
    lat = ctypes.c_double()
    _check(load().ka_server_result(sv.handle, int(job_id), _ptr(dens), _ptr(ov), _ptr(pers), ctypes.byref(wait),
                                   ctypes.byref(lat)))
    return {"density": dens, "overlap": ov, "persistence": pers, "wait_s": wait.value, "latency_s": lat.value}


def ka_server_take_sim(sv: Server, job_id: int) -> Sim:
    h = ctypes.c_void_p()
    _check(load().ka_server_take_sim(sv.handle, int(job_id), ctypes.byref(h)))
    return Sim(h, sv.jobs[job_id][0], None)   # the sim now has a stream of its own


def ka_server_release(sv: Server, job_id: int) -> None:
    """Forget a completed job (its results and, if not taken, its kept sim)."""
    _check(load().ka_server_release(sv.handle, int(job_id)))
    sv.jobs.pop(int(job_id), None)


def ka_server_wait_idle(sv: Server) -> None:
    _check(load().ka_server_wait_idle(sv.handle))


def ka_server_stats(sv: Server):
    done = ctypes.c_int64()
    att = ctypes.c_double()
    peak = ctypes.c_int()
    pbytes = ctypes.c_size_t()
    _check(load().ka_server_stats(sv.handle, ctypes.byref(done), ctypes.byref(att), ctypes.byref(peak),
                                  ctypes.byref(pbytes)))
    return {"jobs_done": done.value, "attempts": att.value, "peak_active": peak.value, "peak_bytes": pbytes.value}


def ka_server_free(sv: Server) -> None:
    sv.free()


# ------------------------------------------------------------------------------ calibration
def ka_probe_valu(kind: int, iters: int = 20000, blocks: int = 4096, stream=None):
    """(wave instructions/s, lane operations/s) of register-only VALU chains: kind 0 =
    v_xor_b32, kind 1 = v_mad_u64_u32."""
    ips = ctypes.c_double()
    lops = ctypes.c_double()
    rc = load().ka_probe_valu(int(kind), int(iters), int(blocks), _stream_handle(stream), ctypes.byref(ips),
                              ctypes.byref(lops))
    if rc != KA_OK:
        raise KaError(rc, "ka_probe_valu failed")
    return ips.value, lops.value


# ------------------------------------------------------------------------------ host-side quantities
def ka_particles(N: int, rho: float) -> int:
    """Particle number the library uses for density rho (ka_particles)."""
    K = ctypes.c_int64()
    _check(load().ka_particles(int(N), float(rho), ctypes.byref(K)))
    return K.value


def ka_derived(N: int, K: int, overlap, persistence=None):
    """(C, chi4, P) per row of the [n_rows, R] counts (ka_derived); P is None without
    persistence."""
    ov = np.ascontiguousarray(np.atleast_2d(np.asarray(overlap, dtype=np.int64)))
    rows, R = ov.shape
    pe = None
    if persistence is not None:
        pe = np.ascontiguousarray(np.atleast_2d(np.asarray(persistence, dtype=np.int64)))
        assert pe.shape == ov.shape
    C = np.empty(rows)
    chi4 = np.empty(rows)
    P = np.empty(rows) if pe is not None else None
    _check(load().ka_derived(int(N), int(K), R, rows, _ptr(ov), _ptr(pe), _ptr(C), _ptr(chi4), _ptr(P)))
    return C, chi4, P


def ka_g4(N: int, K: int, n_replicas: int, S2, S11):
    """g4 per shell from the sums of ka_observe_pairs (ka_g4)."""
    a = np.ascontiguousarray(np.asarray(S2, dtype=np.int64))
    b = np.ascontiguousarray(np.asarray(S11, dtype=np.int64))
    assert a.shape == b.shape and a.ndim == 1
    out = np.empty(a.shape[0])
    _check(load().ka_g4(int(N), int(K), int(n_replicas), a.shape[0], _ptr(a), _ptr(b), _ptr(out)))
    return out


from .workloads import log_time_grid  # noqa: E402,F401  (observation grid recipe)
