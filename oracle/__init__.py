"""CPU oracle for the EDFFS priority-based hybrid parallel GA (arXiv 1903.10741).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
statement of what the GPU path computes: the C library ``ffs_oracle.c``
(decoder, GA, rescheduling, Philox), the pure-Python event-list decoder
``eventlist.py`` (a second decoder written independently, used to pin the
first) and the invariant validator ``validate.py``. Only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg may import it. It shares no
code with the GPU library and imports nothing from it: instances come in as
any object with the instance fields (duck typing) and results go out as
numpy arrays and dicts.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

OK = 0
E_INVAL = -1
E_INFEASIBLE = -2


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class _Instance(ctypes.Structure):
    _fields_ = [
        ("n_jobs", ctypes.c_int32), ("n_stages", ctypes.c_int32), ("o_max", ctypes.c_int32),
        ("n_machines", _i32p), ("proc", _i32p), ("power", _i32p),
        ("release", _i32p), ("due", _i32p),
        ("q_max", ctypes.c_int32), ("wt", ctypes.c_int32), ("rs", ctypes.c_int32),
        ("first_stage", _i32p), ("ready", _i32p), ("machine_free", _i32p),
        ("n_running", ctypes.c_int32), ("running", _i32p),
        ("frozen_tardiness", ctypes.c_int64), ("frozen_cmax", ctypes.c_int32),
        ("n_active", ctypes.c_int32), ("active", _i32p),
        ("decode_rules", ctypes.c_int32),
        ("n_fixed", ctypes.c_int32), ("fixed", _i32p),
    ]


RULE_FIFO = 1        # decode variant: each stage in order of the previous stage's completion
RULE_POWER_ECT = 2   # decode variant: machine of earliest completion after the power push-right


class _GaParams(ctypes.Structure):
    _fields_ = [
        ("islands", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
        ("pc", ctypes.c_uint32), ("pm", ctypes.c_uint32),
        ("mig_interval", ctypes.c_int32), ("mig_k", ctypes.c_int32),
        ("encoding", ctypes.c_int32),
    ]


class _ReschedOut(ctypes.Structure):
    _fields_ = [
        ("proc", _i32p), ("power", _i32p),
        ("release", _i32p), ("due", _i32p), ("first_stage", _i32p), ("ready", _i32p),
        ("machine_free", _i32p), ("running", _i32p), ("active", _i32p),
        ("n_jobs", ctypes.c_int32), ("n_running", ctypes.c_int32), ("n_active", ctypes.c_int32),
        ("frozen_tardiness", ctypes.c_int64), ("frozen_cmax", ctypes.c_int32),
        ("fixed", _i32p), ("n_fixed", ctypes.c_int32),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # FFS_ORACLE_LIB: another build of the oracle (the planted-mistake test loads
    # deliberately broken copies this way); by default the library built here.
    path = os.environ.get("FFS_ORACLE_LIB") or _build.LIB
    src = os.path.join(_HERE, "ffs_oracle.c")
    if path == _build.LIB and (not os.path.exists(path)
                               or os.path.getmtime(path) < os.path.getmtime(src)):
        _build.build()
    lib = ctypes.CDLL(path)
    lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_philox4x64_10.restype = None
    lib.orc_horizon_bound.argtypes = [ctypes.POINTER(_Instance)]
    lib.orc_horizon_bound.restype = ctypes.c_int64
    lib.orc_decode.argtypes = [ctypes.POINTER(_Instance), _i32p, _i64p, _i32p, _i32p, _i64p]
    lib.orc_decode_pop.argtypes = [ctypes.POINTER(_Instance), _i32p, ctypes.c_int32, _i64p,
                                   _i64p, ctypes.c_int32]
    lib.orc_decode_ops.argtypes = [ctypes.POINTER(_Instance), ctypes.c_int32, _i32p, _i64p,
                                   _i32p, _i32p]
    lib.orc_ga_init.argtypes = [ctypes.POINTER(_Instance), ctypes.POINTER(_GaParams),
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                _i32p, _i64p, _i32p, _i64p, ctypes.c_int32]
    lib.orc_ga_generation.argtypes = [ctypes.POINTER(_Instance), ctypes.POINTER(_GaParams),
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_int32, _i32p, _i64p, _i32p, _i64p,
                                      _i32p, _i64p, _i32p, _i64p, _u8p, ctypes.c_int32]
    lib.orc_ga_breed.argtypes = [ctypes.POINTER(_Instance), ctypes.POINTER(_GaParams),
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _i32p, _i64p, _i32p, _u8p]
    lib.orc_ga_finish.argtypes = [ctypes.POINTER(_Instance), ctypes.POINTER(_GaParams),
                                  ctypes.c_int32, _i32p, _i64p, _i32p, _i64p, _i32p, _i64p, _u8p,
                                  ctypes.c_int32]
    lib.orc_crossover.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.orc_crossover.restype = None
    lib.orc_crossover_xy.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.orc_crossover_xy.restype = None
    lib.orc_xy_ops.argtypes = [ctypes.POINTER(_Instance)]
    lib.orc_xy_ops.restype = ctypes.c_int32
    lib.orc_xy_order.argtypes = [ctypes.POINTER(_Instance), _i32p, _i32p]
    lib.orc_decode_xy.argtypes = [ctypes.POINTER(_Instance), _i32p, _i64p, _i32p, _i32p, _i64p]
    lib.orc_decode_xy_pop.argtypes = [ctypes.POINTER(_Instance), _i32p, ctypes.c_int32, _i64p,
                                      _i64p, ctypes.c_int32]
    lib.orc_correct.argtypes = [ctypes.c_int32, _i32p]
    lib.orc_correct.restype = None
    lib.orc_mutate.argtypes = [ctypes.c_int32, _i32p, ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_mutate.restype = None
    lib.orc_reschedule.argtypes = [ctypes.POINTER(_Instance), _i32p, _i32p, ctypes.c_int32,
                                   ctypes.c_int32, _i32p, _i32p, _i32p, _i32p,
                                   ctypes.POINTER(_ReschedOut)]
    lib.orc_reschedule_static.argtypes = lib.orc_reschedule.argtypes
    lib.orc_emax.argtypes = [_i64p, ctypes.c_int32]
    lib.orc_emax.restype = ctypes.c_int64
    lib.orc_ga_generation_scheme.argtypes = [
        ctypes.POINTER(_Instance), ctypes.POINTER(_GaParams), ctypes.c_int32, ctypes.c_int64,
        ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, _i32p, _i64p, _i32p,
        _i64p, _i32p, _i64p, _i32p, _i64p, ctypes.c_int32]
    for f in ("orc_decode", "orc_decode_pop", "orc_decode_ops", "orc_ga_init",
              "orc_ga_generation", "orc_ga_breed", "orc_ga_finish", "orc_reschedule",
              "orc_reschedule_static", "orc_ga_generation_scheme",
              "orc_xy_order", "orc_decode_xy", "orc_decode_xy_pop"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _arr(x, dtype=np.int32):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def _ptr(a, t=_i32p):
    return a.ctypes.data_as(t)


class _Pinned:
    """An oracle instance struct plus the numpy arrays it points into."""

    def __init__(self, inst):
        g = int(inst.n_stages)
        om = int(inst.o_max)
        n = int(inst.n_jobs)
        self.keep = {
            "n_machines": _arr(inst.n_machines).reshape(g),
            "proc": _arr(inst.proc).reshape(n, g, om) if n else np.zeros((0, g, om), np.int32),
            "power": _arr(inst.power).reshape(n, g, om) if n else np.zeros((0, g, om), np.int32),
            "release": _arr(inst.release).reshape(n),
            "due": _arr(inst.due).reshape(n),
            "first_stage": _arr(inst.first_stage).reshape(n),
            "ready": _arr(inst.ready).reshape(n),
            "machine_free": _arr(inst.machine_free).reshape(g, om),
            "running": _arr(inst.running).reshape(-1, 2) if len(inst.running) else np.zeros((1, 2), np.int32),
            "active": _arr(inst.active).reshape(-1) if len(inst.active) else np.zeros(1, np.int32),
        }
        fixed = np.asarray(getattr(inst, "fixed", np.zeros((0, 3), np.int32))).reshape(-1, 3)
        self.keep["fixed"] = _arr(fixed) if len(fixed) else np.zeros((1, 3), np.int32)
        k = self.keep
        self.s = _Instance(
            n, g, om, _ptr(k["n_machines"]), _ptr(k["proc"]), _ptr(k["power"]),
            _ptr(k["release"]), _ptr(k["due"]), int(inst.q_max), int(inst.wt), int(inst.rs),
            _ptr(k["first_stage"]), _ptr(k["ready"]), _ptr(k["machine_free"]),
            int(len(inst.running)), _ptr(k["running"]), int(inst.frozen_tardiness),
            int(inst.frozen_cmax), int(len(inst.active)), _ptr(k["active"]),
            int(getattr(inst, "decode_rules", 0)), int(len(fixed)), _ptr(k["fixed"]))
        self.n_active = int(len(inst.active))
        self.n_jobs = n
        self.g = g

    def ref(self):
        return ctypes.byref(self.s)


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def philox4x64_10(counter, key):
    """Philox4x64-10 block at `counter` (4 x uint64) under `key` (2 x uint64)."""
    lib = _load()
    c = _arr(counter, np.uint64)
    k = _arr(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib.orc_philox4x64_10(_ptr(c, _u64p), _ptr(k, _u64p), _ptr(out, _u64p))
    return out


def horizon_bound(inst):
    p = _Pinned(inst)
    return int(_load().orc_horizon_bound(p.ref()))


def decode(inst, prio, want_schedule=False, want_work=False):
    """Decode one priority vector. Returns obj, or (obj, start, mach, work)."""
    lib = _load()
    p = _Pinned(inst)
    pr = _arr(prio).reshape(-1)
    if pr.size != p.n_active:
        raise ValueError("priority vector length != n_active")
    if pr.size == 0:
        pr = np.zeros(1, np.int32)
    obj = np.zeros(1, np.int64)
    work = np.zeros(1, np.int64)
    start = np.full((p.n_jobs, p.g), -1, np.int32) if want_schedule else None
    mach = np.full((p.n_jobs, p.g), -1, np.int32) if want_schedule else None
    rc = lib.orc_decode(p.ref(), _ptr(pr), _ptr(obj, _i64p),
                        _ptr(start) if want_schedule else None,
                        _ptr(mach) if want_schedule else None, _ptr(work, _i64p))
    _check(rc, "orc_decode")
    if want_schedule or want_work:
        return int(obj[0]), start, mach, int(work[0])
    return int(obj[0])


def decode_pop(inst, prio, n_threads=1, want_work=False):
    lib = _load()
    p = _Pinned(inst)
    pr = _arr(prio)
    pop = pr.shape[0]
    pr = pr.reshape(pop, p.n_active)
    buf = pr if pr.size else np.zeros(1, np.int32)
    obj = np.zeros(max(pop, 1), np.int64)
    work = np.zeros(max(pop, 1), np.int64)
    rc = lib.orc_decode_pop(p.ref(), _ptr(buf), pop, _ptr(obj, _i64p), _ptr(work, _i64p),
                            int(n_threads))
    _check(rc, "orc_decode_pop")
    if want_work:
        return obj[:pop], work[:pop]
    return obj[:pop]


def decode_ops(inst, ops, start=None, mach=None):
    """Place ops [(job, stage, machine or -1)] in order. Returns (obj, start, mach).

    start/mach may carry the schedule of frozen ops; decoded entries are written.
    """
    lib = _load()
    p = _Pinned(inst)
    o = _arr(ops).reshape(-1, 3)
    st = _arr(start).copy() if start is not None else np.full((p.n_jobs, p.g), -1, np.int32)
    mc = _arr(mach).copy() if mach is not None else np.full((p.n_jobs, p.g), -1, np.int32)
    obj = np.zeros(1, np.int64)
    rc = lib.orc_decode_ops(p.ref(), o.shape[0], _ptr(o if o.size else np.zeros(3, np.int32)),
                            _ptr(obj, _i64p), _ptr(st), _ptr(mc))
    _check(rc, "orc_decode_ops")
    return int(obj[0]), st, mc


def xy_ops(inst):
    """R: operations not frozen at RS (genes per matrix of an X/Y chromosome)."""
    return int(_load().orc_xy_ops(_Pinned(inst).ref()))


def xy_order(inst, y):
    """Assignment order Z (Algorithm 1, greedy) from priority genes y[R]: [R, 2] (job, stage)."""
    lib = _load()
    p = _Pinned(inst)
    R = int(lib.orc_xy_ops(p.ref()))
    yy = _arr(y).reshape(R) if R else np.zeros(1, np.int32)
    out = np.zeros((max(R, 1), 2), np.int32)
    _check(lib.orc_xy_order(p.ref(), _ptr(yy), _ptr(out)), "orc_xy_order")
    return out[:R]


def decode_xy(inst, genes, want_schedule=False, want_work=False):
    """Decode one X/Y chromosome genes[2R]. Returns obj, or (obj, start, mach, work)."""
    lib = _load()
    p = _Pinned(inst)
    R = int(lib.orc_xy_ops(p.ref()))
    gv = _arr(genes).reshape(-1)
    if gv.size != 2 * R:
        raise ValueError("X/Y chromosome length != 2R")
    if gv.size == 0:
        gv = np.zeros(2, np.int32)
    obj = np.zeros(1, np.int64)
    work = np.zeros(1, np.int64)
    start = np.full((p.n_jobs, p.g), -1, np.int32) if want_schedule else None
    mach = np.full((p.n_jobs, p.g), -1, np.int32) if want_schedule else None
    rc = lib.orc_decode_xy(p.ref(), _ptr(gv), _ptr(obj, _i64p),
                           _ptr(start) if want_schedule else None,
                           _ptr(mach) if want_schedule else None, _ptr(work, _i64p))
    _check(rc, "orc_decode_xy")
    if want_schedule or want_work:
        return int(obj[0]), start, mach, int(work[0])
    return int(obj[0])


def decode_xy_pop(inst, genes, n_threads=1, want_work=False):
    lib = _load()
    p = _Pinned(inst)
    R = int(lib.orc_xy_ops(p.ref()))
    gv = _arr(genes)
    pop = gv.shape[0]
    gv = gv.reshape(pop, 2 * R)
    buf = gv if gv.size else np.zeros(1, np.int32)
    obj = np.zeros(max(pop, 1), np.int64)
    work = np.zeros(max(pop, 1), np.int64)
    rc = lib.orc_decode_xy_pop(p.ref(), _ptr(buf), pop, _ptr(obj, _i64p), _ptr(work, _i64p),
                               int(n_threads))
    _check(rc, "orc_decode_xy_pop")
    if want_work:
        return obj[:pop], work[:pop]
    return obj[:pop]


def _gp(ga):
    return _GaParams(int(ga.islands), int(ga.rows), int(ga.cols), int(ga.pc), int(ga.pm),
                     int(ga.mig_interval), int(ga.mig_k), int(getattr(ga, "encoding", 0)))


def _chrom_len(p, gp):
    """Genes per chromosome: n_active (job priorities) or 2R (X/Y)."""
    return 2 * int(_load().orc_xy_ops(p.ref())) if gp.encoding == 1 else p.n_active


def ga_init(inst, ga, seed, shop, event, n_threads=1):
    """Generation 0. Returns dict(prio, obj, elite, elite_obj)."""
    lib = _load()
    p = _Pinned(inst)
    gp = _gp(ga)
    pop = gp.islands * gp.rows * gp.cols
    L = _chrom_len(p, gp)
    n = max(L, 1)
    prio = np.zeros((pop, n), np.int32)
    obj = np.zeros(pop, np.int64)
    elite = np.zeros((gp.islands, n), np.int32)
    elite_obj = np.zeros(gp.islands, np.int64)
    rc = lib.orc_ga_init(p.ref(), ctypes.byref(gp), seed, shop, event, _ptr(prio),
                         _ptr(obj, _i64p), _ptr(elite), _ptr(elite_obj, _i64p), int(n_threads))
    _check(rc, "orc_ga_init")
    return {"prio": prio[:, :L].copy(), "obj": obj, "elite": elite[:, :L].copy(),
            "elite_obj": elite_obj}


def ga_generation(inst, ga, seed, shop, event, gen, state, island_sel=None, n_threads=1):
    """One generation from `state` (dict as returned by ga_init). Returns a new dict.

    With island_sel (bool array over islands) only those islands are valid in the result.
    """
    lib = _load()
    p = _Pinned(inst)
    gp = _gp(ga)
    pop = gp.islands * gp.rows * gp.cols
    n = _chrom_len(p, gp)
    nn = max(n, 1)

    def padded(a, rows):
        a = _arr(a).reshape(rows, n)
        if n == 0:
            return np.zeros((rows, 1), np.int32)
        return a

    prio_in = padded(state["prio"], pop)
    elite_in = padded(state["elite"], gp.islands)
    obj_in = _arr(state["obj"], np.int64).reshape(pop)
    eobj_in = _arr(state["elite_obj"], np.int64).reshape(gp.islands)
    prio_out = np.zeros((pop, nn), np.int32)
    obj_out = np.zeros(pop, np.int64)
    elite_out = np.zeros((gp.islands, nn), np.int32)
    eobj_out = np.zeros(gp.islands, np.int64)
    sel = None
    if island_sel is not None:
        sel = _arr(island_sel, np.uint8).reshape(gp.islands)
    rc = lib.orc_ga_generation(p.ref(), ctypes.byref(gp), seed, shop, event, gen,
                               _ptr(prio_in), _ptr(obj_in, _i64p), _ptr(elite_in),
                               _ptr(eobj_in, _i64p), _ptr(prio_out), _ptr(obj_out, _i64p),
                               _ptr(elite_out), _ptr(eobj_out, _i64p),
                               _ptr(sel, _u8p) if sel is not None else None, int(n_threads))
    _check(rc, "orc_ga_generation")
    return {"prio": prio_out[:, :n].copy(), "obj": obj_out, "elite": elite_out[:, :n].copy(),
            "elite_obj": eobj_out}


def ga_breed(inst, ga, seed, shop, event, gen, variant, state):
    """Selection, crossover and mutation of generation `gen` with the draws of
    `variant` (0 = the plain generation's). Returns the children [pop, n]."""
    lib = _load()
    p = _Pinned(inst)
    gp = _gp(ga)
    pop = gp.islands * gp.rows * gp.cols
    n = _chrom_len(p, gp)
    nn = max(n, 1)
    prio_in = _arr(state["prio"]).reshape(pop, n) if n else np.zeros((pop, 1), np.int32)
    obj_in = _arr(state["obj"], np.int64).reshape(pop)
    out = np.zeros((pop, nn), np.int32)
    rc = lib.orc_ga_breed(p.ref(), ctypes.byref(gp), seed, shop, event, gen, int(variant),
                          _ptr(prio_in), _ptr(obj_in, _i64p), _ptr(out), None)
    _check(rc, "orc_ga_breed")
    return out[:, :n].copy()


def ga_finish(inst, ga, gen, children, state, n_threads=1):
    """Decode `children` (the bred generation `gen`), then replacement and
    migration against `state`'s elites. Returns the new state dict."""
    lib = _load()
    p = _Pinned(inst)
    gp = _gp(ga)
    pop = gp.islands * gp.rows * gp.cols
    n = _chrom_len(p, gp)
    nn = max(n, 1)
    prio = np.zeros((pop, nn), np.int32)
    prio[:, :n] = _arr(children).reshape(pop, n)
    obj = np.zeros(pop, np.int64)
    elite_in = np.zeros((gp.islands, nn), np.int32)
    elite_in[:, :n] = _arr(state["elite"]).reshape(gp.islands, n)
    eobj_in = _arr(state["elite_obj"], np.int64).reshape(gp.islands)
    elite_out = np.zeros((gp.islands, nn), np.int32)
    eobj_out = np.zeros(gp.islands, np.int64)
    rc = lib.orc_ga_finish(p.ref(), ctypes.byref(gp), gen, _ptr(prio), _ptr(obj, _i64p),
                           _ptr(elite_in), _ptr(eobj_in, _i64p), _ptr(elite_out),
                           _ptr(eobj_out, _i64p), None, int(n_threads))
    _check(rc, "orc_ga_finish")
    return {"prio": prio[:, :n].copy(), "obj": obj, "elite": elite_out[:, :n].copy(),
            "elite_obj": eobj_out}


def ga_run(inst, ga, seed, shop, event, generations, n_threads=1):
    """Generation 0 then `generations` more. Returns the final state dict."""
    st = ga_init(inst, ga, seed, shop, event, n_threads)
    for k in range(1, generations + 1):
        st = ga_generation(inst, ga, seed, shop, event, k, st, n_threads=n_threads)
    return st


GA_CLASSICAL = 1   # the classical GA of Section 5.2 (roulette wheel, random pairing)
GA_CELLULAR = 2    # the cellular GA of Section 5.2 (neighbourhood parents, replace if better)


def emax(obj):
    """E_max of eq. (13): 10^a, the least a >= 1 with every objective below it."""
    o = _arr(obj, np.int64)
    return int(_load().orc_emax(_ptr(o, _i64p), int(o.size)))


def ga_generation_scheme(inst, ga, scheme, e_max, seed, shop, event, gen, state, n_threads=1):
    """One generation of the classical (GA_CLASSICAL) or cellular (GA_CELLULAR) GA
    on job-priority vectors (one population, ga.islands == 1). Returns a new state."""
    lib = _load()
    p = _Pinned(inst)
    gp = _gp(ga)
    pop = gp.rows * gp.cols
    n = max(p.n_active, 1)
    prio_in = _arr(state["prio"]).reshape(pop, -1)
    if prio_in.shape[1] == 0:
        prio_in = np.zeros((pop, 1), np.int32)
    elite_in = _arr(state["elite"]).reshape(1, -1)
    if elite_in.shape[1] == 0:
        elite_in = np.zeros((1, 1), np.int32)
    obj_in = _arr(state["obj"], np.int64)
    eobj_in = _arr(state["elite_obj"], np.int64)
    prio = np.zeros((pop, n), np.int32)
    obj = np.zeros(pop, np.int64)
    elite = np.zeros((1, n), np.int32)
    eobj = np.zeros(1, np.int64)
    rc = lib.orc_ga_generation_scheme(p.ref(), ctypes.byref(gp), int(scheme), int(e_max), seed,
                                      shop, event, gen, _ptr(prio_in), _ptr(obj_in, _i64p),
                                      _ptr(elite_in), _ptr(eobj_in, _i64p), _ptr(prio),
                                      _ptr(obj, _i64p), _ptr(elite), _ptr(eobj, _i64p),
                                      int(n_threads))
    _check(rc, "orc_ga_generation_scheme")
    L = p.n_active
    return {"prio": prio[:, :L].copy(), "obj": obj, "elite": elite[:, :L].copy(),
            "elite_obj": eobj}


def ga_run_scheme(inst, ga, scheme, seed, shop, event, generations, n_threads=1):
    """Generation 0 (ga_init) and `generations` generations of a comparison GA;
    the state carries e_max (eq. (13), from generation 0)."""
    st = ga_init(inst, ga, seed, shop, event, n_threads)
    e = emax(st["obj"])
    for g in range(1, generations + 1):
        st = ga_generation_scheme(inst, ga, scheme, e, seed, shop, event, g, st, n_threads)
    st["e_max"] = e
    return st


def ga_best(state):
    """Event result: the best elite, ties to the lowest island."""
    i = int(np.argmin(state["elite_obj"]))
    return state["elite"][i].copy(), int(state["elite_obj"][i])


def crossover_xy(a, b, cut):
    """X/Y crossover of genes[2R] pairs (Fig. 11): both matrices at `cut`, Y corrected."""
    lib = _load()
    a = _arr(a)
    b = _arr(b)
    ca = np.zeros_like(a)
    cb = np.zeros_like(b)
    lib.orc_crossover_xy(int(a.size // 2), _ptr(a), _ptr(b), int(cut), _ptr(ca), _ptr(cb))
    return ca, cb


def crossover(a, b, cut):
    lib = _load()
    a = _arr(a)
    b = _arr(b)
    ca = np.zeros_like(a)
    cb = np.zeros_like(b)
    lib.orc_crossover(a.size, _ptr(a), _ptr(b), int(cut), _ptr(ca), _ptr(cb))
    return ca, cb


def correct(v):
    lib = _load()
    v = _arr(v).copy()
    lib.orc_correct(v.size, _ptr(v))
    return v


def mutate(v, w1, w2):
    """Swap mutation driven by two 64-bit draws (positions from their high words)."""
    lib = _load()
    v = _arr(v).copy()
    lib.orc_mutate(v.size, _ptr(v), int(w1), int(w2))
    return v


def reschedule(prev, plan_start, plan_mach, rs, new_proc, new_power, new_release, new_due,
               static=False):
    """Freeze the executed plan at rs and append new jobs. Returns a dict of instance fields.
    static=True: the traditional static approach (orc_reschedule_static): the whole plan
    of the known jobs stays in place and the arrivals go after each stage's planned ops."""
    lib = _load()
    p = _Pinned(prev)
    g = p.g
    om = int(prev.o_max)
    n_new = int(len(new_release))
    n = p.n_jobs + n_new
    nproc = _arr(new_proc).reshape(n_new, g, om) if n_new else np.zeros((1, g, om), np.int32)
    npow = _arr(new_power).reshape(n_new, g, om) if n_new else np.zeros((1, g, om), np.int32)
    nrel = _arr(new_release).reshape(n_new) if n_new else np.zeros(1, np.int32)
    ndue = _arr(new_due).reshape(n_new) if n_new else np.zeros(1, np.int32)
    ps = _arr(plan_start).reshape(p.n_jobs, g) if p.n_jobs else np.zeros((1, g), np.int32)
    pm = _arr(plan_mach).reshape(p.n_jobs, g) if p.n_jobs else np.zeros((1, g), np.int32)
    cap = max(1, g * om)
    bufs = {
        "proc": np.zeros((max(n, 1), g, om), np.int32),
        "power": np.zeros((max(n, 1), g, om), np.int32),
        "release": np.zeros(max(n, 1), np.int32), "due": np.zeros(max(n, 1), np.int32),
        "first_stage": np.zeros(max(n, 1), np.int32), "ready": np.zeros(max(n, 1), np.int32),
        "machine_free": np.zeros((g, om), np.int32), "running": np.zeros((cap, 2), np.int32),
        "active": np.zeros(max(n, 1), np.int32),
        "fixed": np.zeros((max(p.n_jobs * g, 1), 3), np.int32),
    }
    out = _ReschedOut(*[_ptr(bufs[k]) for k in ("proc", "power", "release", "due", "first_stage",
                                                 "ready", "machine_free", "running", "active")],
                      0, 0, 0, 0, 0, _ptr(bufs["fixed"]), 0)
    fn = lib.orc_reschedule_static if static else lib.orc_reschedule
    rc = fn(p.ref(), _ptr(ps), _ptr(pm), int(rs), n_new, _ptr(nproc), _ptr(npow),
            _ptr(nrel), _ptr(ndue), ctypes.byref(out))
    _check(rc, "orc_reschedule_static" if static else "orc_reschedule")
    return {
        "n_jobs": n, "n_stages": g, "o_max": om, "n_machines": _arr(prev.n_machines).copy(),
        "proc": bufs["proc"][:n].copy(), "power": bufs["power"][:n].copy(),
        "release": bufs["release"][:n].copy(), "due": bufs["due"][:n].copy(),
        "q_max": int(prev.q_max), "wt": int(prev.wt), "rs": int(rs),
        "first_stage": bufs["first_stage"][:n].copy(), "ready": bufs["ready"][:n].copy(),
        "machine_free": bufs["machine_free"].copy(),
        "running": bufs["running"][:out.n_running].copy(),
        "frozen_tardiness": int(out.frozen_tardiness), "frozen_cmax": int(out.frozen_cmax),
        "active": bufs["active"][:out.n_active].copy(),
        "fixed": bufs["fixed"][:out.n_fixed].copy(),
    }


def run_events(initial, arrivals, ga, generations, seed, shop=0, n_threads=1, events=None,
               static=False):
    """The predictive-reactive loop (Section 4.1) on the oracle: for each event,
    run the GA (generation 0 then `generations`), execute the best elite's
    plan until the next arrival, freeze and reschedule. Returns one dict per
    event: best_obj, best_prio, the instance dict and the plan after the event.
    static=True: each arrival is handled by the traditional static approach
    instead (reschedule(..., static=True))."""
    inst = initial
    g = int(initial.n_stages)
    plan_s = np.full((int(initial.n_jobs), g), -1, np.int32)
    plan_m = np.full((int(initial.n_jobs), g), -1, np.int32)
    out = []
    n_events = 1 + len(arrivals) if events is None else events
    for e in range(n_events):
        st = ga_run(inst, ga, seed, shop, e, generations, n_threads)
        prio, obj = ga_best(st)
        dec = decode_xy if getattr(ga, "encoding", 0) == 1 else decode
        obj2, s, m, _ = dec(inst, prio, want_schedule=True)
        assert obj2 == obj
        for j in np.asarray(inst.active):
            f = int(np.asarray(inst.first_stage)[j])
            plan_s[j, f:] = s[j, f:]
            plan_m[j, f:] = m[j, f:]
        out.append({"best_obj": obj, "best_prio": prio, "instance": inst,
                     "plan_start": plan_s.copy(), "plan_mach": plan_m.copy()})
        if e + 1 < n_events and e < len(arrivals):
            a = arrivals[e]
            nxt = reschedule(inst, plan_s, plan_m, a.rs, a.proc, a.power, a.release, a.due,
                             static=static)
            k = len(a.release)
            plan_s = np.vstack([plan_s, np.full((k, g), -1, np.int32)])
            plan_m = np.vstack([plan_m, np.full((k, g), -1, np.int32)])
            inst = _Fields(nxt)
            inst.decode_rules = int(getattr(initial, "decode_rules", 0))
    return out


class _Fields:
    """Attribute access to an instance dict."""

    def __init__(self, d):
        self.__dict__.update(d)
