"""Python binding of libffsga.so (include/ffsga.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels. torch supplies device memory (int32/int64/uint8 tensors on cuda)
and the stream (``torch.cuda.current_stream()``). The library must be built
(``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffsga.so")

FFS_OK = 0
FFS_E_INVAL = -1
FFS_E_INFEASIBLE = -2
FFS_E_WORKSPACE = -3
FFS_E_DEVICE = -4
FFS_E_UNSUPPORTED = -5
FFS_PREPARE_WORKSPACE = 256
FFS_DECODE_SCRATCH_BYTES = 16 << 20
FFS_LDS_AUTO = -1
FFS_GA_HYBRID, FFS_GA_CLASSICAL, FFS_GA_CELLULAR = 0, 1, 2

TIMING_DECODE, TIMING_GENERATION, TIMING_REPLACE, TIMING_OVERFLOW = 0, 1, 2, 3
TIMING_BATCH, TIMING_SCREENED = 4, 5
TIMING_STEP = 6  # whole ga_step calls, counted in generations

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p


class FfsInstance(ctypes.Structure):
    _fields_ = [
        ("n_jobs", ctypes.c_int32), ("n_stages", ctypes.c_int32), ("o_max", ctypes.c_int32),
        ("n_machines", _vp), ("proc", _vp), ("power", _vp), ("release", _vp), ("due", _vp),
        ("q_max", ctypes.c_int32), ("wt", ctypes.c_int32), ("rs", ctypes.c_int32),
        ("first_stage", _vp), ("ready", _vp), ("machine_free", _vp),
        ("n_running", ctypes.c_int32), ("running", _vp),
        ("frozen_tardiness", ctypes.c_int64), ("frozen_cmax", ctypes.c_int32),
        ("n_active", ctypes.c_int32), ("active", _vp),
        ("horizon", ctypes.c_int32), ("n_ops", ctypes.c_int32), ("decode_rules", ctypes.c_int32),
        ("n_fixed", ctypes.c_int32), ("fixed", _vp),
    ]


RULE_FIFO = 1        # FFS_RULE_FIFO: each stage in order of the previous stage's completion
RULE_POWER_ECT = 2   # FFS_RULE_POWER_ECT: machine of earliest completion after the push-right


class FfsGaParams(ctypes.Structure):
    _fields_ = [
        ("islands", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
        ("pc", ctypes.c_uint32), ("pm", ctypes.c_uint32),
        ("mig_interval", ctypes.c_int32), ("mig_k", ctypes.c_int32),
        ("lds_slots", ctypes.c_int32), ("encoding", ctypes.c_int32), ("scheme", ctypes.c_int32),
    ]


class FfsGa(ctypes.Structure):
    _fields_ = [
        ("params", FfsGaParams),
        ("n_genes", ctypes.c_int32), ("pop", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("shop", ctypes.c_uint64),
        ("event", ctypes.c_int32), ("generation", ctypes.c_int32), ("cur", ctypes.c_int32),
        ("lds_slots", ctypes.c_int32), ("n_jobs", ctypes.c_int32), ("horizon", ctypes.c_int32),
        ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t),
        ("prio", _vp * 2), ("obj", _vp * 2), ("elite", _vp), ("elite_obj", _vp),
        ("island_groups", ctypes.c_int32), ("narrow_lds", ctypes.c_int32),
    ]


class FfsGaView(ctypes.Structure):
    _fields_ = [("prio", _vp), ("obj", _vp), ("elite", _vp), ("elite_obj", _vp), ("work", _vp),
                ("e_max", _vp), ("overflows", _vp)]


_P = ctypes.POINTER
_lib.ffs_prepare.argtypes = [_P(FfsInstance), _vp, ctypes.c_size_t, _vp]
_lib.ffs_decode_workspace_size.argtypes = [_P(FfsInstance), ctypes.c_int32, ctypes.c_int32]
_lib.ffs_decode_workspace_size.restype = ctypes.c_size_t
_lib.ffs_decode.argtypes = [_P(FfsInstance), _vp, ctypes.c_int32, _vp, _vp, _vp, _vp,
                            ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
_lib.ffs_decode_xy.argtypes = [_P(FfsInstance), _vp, ctypes.c_int32, _vp, _vp, _vp, _vp,
                               ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
_lib.ffs_decode_noalloc.argtypes = [_P(FfsInstance), _vp, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                    ctypes.c_int32, _vp]
_lib.ffs_status.argtypes = [_vp, _vp]
_lib.ffs_ga_workspace_size.argtypes = [_P(FfsInstance), _P(FfsGaParams)]
_lib.ffs_ga_workspace_size.restype = ctypes.c_size_t
_lib.ga_init.argtypes = [_P(FfsGa), _P(FfsInstance), _P(FfsGaParams), ctypes.c_uint64,
                         ctypes.c_uint64, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
_lib.ga_step.argtypes = [_P(FfsGa), _P(FfsInstance), ctypes.c_int32, _vp]
_lib.ga_set_island_groups.argtypes = [ctypes.c_int32]
_lib.ga_best.argtypes = [_P(FfsGa), _vp, _vp, _vp]
_lib.ga_view.argtypes = [_P(FfsGa), _P(FfsGaView)]
_lib.ffs_reschedule_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.ffs_reschedule_workspace_size.restype = ctypes.c_size_t
_lib.reschedule.argtypes = [_P(FfsInstance), _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                            _vp, _vp, _P(FfsInstance), _vp, ctypes.c_size_t, _vp]
_lib.reschedule_static.argtypes = _lib.reschedule.argtypes
_lib.ffs_timing_enable.argtypes = [ctypes.c_int32]
_lib.ffs_timing_every.argtypes = [ctypes.c_int32]
_lib.ffs_timing_read.argtypes = [ctypes.c_int32, _P(ctypes.c_double), _P(ctypes.c_int64)]
_lib.ffs_strerror.argtypes = [ctypes.c_int]
_lib.ffs_strerror.restype = ctypes.c_char_p
_lib.ffs_build_id.argtypes = []
_lib.ffs_build_id.restype = ctypes.c_char_p
for _f in ("ffs_prepare", "ffs_decode", "ffs_decode_noalloc", "ffs_decode_xy", "ffs_status", "ga_init", "ga_step",
           "ga_set_island_groups", "ga_best", "ga_view",
           "reschedule", "reschedule_static", "ffs_timing_enable", "ffs_timing_every",
           "ffs_timing_read"):
    getattr(_lib, _f).restype = ctypes.c_int


class FfsError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {ffs_strerror(code)} ({code})")
        self.code = code


def ffs_strerror(code):
    return _lib.ffs_strerror(int(code)).decode()


def ffs_build_id():
    """Hash of the HIP source and ABI header the loaded library was built from."""
    return _lib.ffs_build_id().decode()


def _check(rc, what):
    if rc != FFS_OK:
        raise FfsError(rc, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    """Device address of a tensor (None -> NULL)."""
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _i32(x, device):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32)).to(device)


class DeviceInstance:
    """An ffs_instance whose arrays live in torch cuda tensors."""

    def __init__(self, s: FfsInstance, tensors: dict):
        self.s = s
        self.t = tensors
        _make_group_streams(tensors["proc"].device)

    @classmethod
    def from_host(cls, inst, device="cuda", prepare=True, workspace=None):
        g, om, n = int(inst.n_stages), int(inst.o_max), int(inst.n_jobs)
        t = {
            "n_machines": _i32(inst.n_machines, device),
            "proc": _i32(np.asarray(inst.proc).reshape(n, g, om), device),
            "power": _i32(np.asarray(inst.power).reshape(n, g, om), device),
            "release": _i32(inst.release, device), "due": _i32(inst.due, device),
            "first_stage": _i32(inst.first_stage, device), "ready": _i32(inst.ready, device),
            "machine_free": _i32(np.asarray(inst.machine_free).reshape(g, om), device),
            "running": _i32(np.asarray(inst.running).reshape(-1, 2), device),
            "active": _i32(inst.active, device),
            "fixed": _i32(np.asarray(getattr(inst, "fixed", np.zeros((0, 3)))).reshape(-1, 3),
                          device),
        }
        s = FfsInstance(
            n, g, om, _dptr(t["n_machines"]), _dptr(t["proc"]), _dptr(t["power"]),
            _dptr(t["release"]), _dptr(t["due"]), int(inst.q_max), int(inst.wt), int(inst.rs),
            _dptr(t["first_stage"]), _dptr(t["ready"]), _dptr(t["machine_free"]),
            int(len(inst.running)), _dptr(t["running"]), int(inst.frozen_tardiness),
            int(inst.frozen_cmax), int(len(inst.active)), _dptr(t["active"]), 0, 0,
            int(getattr(inst, "decode_rules", 0)), int(t["fixed"].shape[0]),
            _dptr(t["fixed"]) if t["fixed"].numel() else None)
        d = cls(s, t)
        if prepare:
            d.prepare(workspace)
        return d

    @property
    def n_active(self):
        return int(self.s.n_active)

    @property
    def horizon(self):
        return int(self.s.horizon)

    @property
    def n_ops(self):
        """Unfrozen operations R (genes per matrix of an X/Y chromosome)."""
        return int(self.s.n_ops)

    def prepare(self, workspace=None):
        ws = workspace if workspace is not None else torch.empty(
            FFS_PREPARE_WORKSPACE, dtype=torch.uint8, device=self.t["proc"].device)
        _check(_lib.ffs_prepare(ctypes.byref(self.s), _dptr(ws), ws.numel(), _stream()),
               "ffs_prepare")

    def to_host(self) -> dict:
        """Instance fields as numpy arrays and ints (for checks and tests)."""
        s = self.s
        out = {k: v.cpu().numpy() for k, v in self.t.items() if not k.startswith("_")}
        out["running"] = out["running"][:s.n_running].reshape(-1, 2)
        out["active"] = out["active"][:s.n_active]
        out["fixed"] = out["fixed"].reshape(-1, 3)[:s.n_fixed]
        for k in ("n_jobs", "n_stages", "o_max", "q_max", "wt", "rs", "frozen_tardiness",
                  "frozen_cmax", "horizon", "n_ops", "decode_rules"):
            out[k] = int(getattr(s, k))
        n = out["n_jobs"]
        for k in ("proc", "power"):
            out[k] = out[k][:n]
        for k in ("release", "due", "first_stage", "ready"):
            out[k] = out[k][:n]
        return out


def _decode_outputs(dinst, prio, want_schedule, want_work, start=None, mach=None):
    s = dinst.s
    dev = dinst.t["proc"].device
    prio = prio.to(device=dev, dtype=torch.int32).contiguous()
    pop = int(prio.shape[0]) if prio.dim() == 2 else 1
    obj = torch.empty(pop, dtype=torch.int64, device=dev)
    work = None
    if start is not None or mach is not None:
        # caller-owned plan arrays: decoded ops are written, frozen entries kept
        shape = (pop * s.n_jobs * s.n_stages,)
        for t in (start, mach):
            if (t is None or t.dtype != torch.int32 or not t.is_contiguous() or t.device != dev
                    or tuple(t.reshape(-1).shape) != shape):
                raise ValueError("start/mach must both be contiguous int32 [pop][n_jobs][g] "
                                 "tensors on the instance's device")
    elif want_schedule:
        start = torch.full((pop, s.n_jobs, s.n_stages), -1, dtype=torch.int32, device=dev)
        mach = torch.full((pop, s.n_jobs, s.n_stages), -1, dtype=torch.int32, device=dev)
    if want_work:
        work = torch.empty(pop, dtype=torch.int64, device=dev)
    return prio, pop, obj, start, mach, work


def ffs_decode(dinst: DeviceInstance, prio: torch.Tensor, lds_slots: int = 0,
               want_schedule: bool = False, want_work: bool = False, workspace=None,
               xy: bool = False, start_out: torch.Tensor = None, mach_out: torch.Tensor = None):
    """Decode prio [pop, n_active] (int32, cuda), or with xy=True X/Y chromosomes
    [pop, 2 * n_ops] (ffs_decode_xy). Returns obj (int64 [pop]) or a dict.
    start_out/mach_out: caller-owned [pop][n_jobs][g] plan arrays that receive the
    decoded ops' start times and machines in place (frozen entries untouched)."""
    s = dinst.s
    dev = dinst.t["proc"].device
    want_schedule = want_schedule or start_out is not None
    prio, pop, obj, start, mach, work = _decode_outputs(dinst, prio, want_schedule, want_work,
                                                        start_out, mach_out)
    need = _lib.ffs_decode_workspace_size(ctypes.byref(s), pop, int(lds_slots))
    if need == 0:
        raise FfsError(FFS_E_INVAL, "ffs_decode_workspace_size")
    ws = workspace if workspace is not None and workspace.numel() >= need else torch.empty(
        need, dtype=torch.uint8, device=dev)
    fn = _lib.ffs_decode_xy if xy else _lib.ffs_decode
    _check(fn(ctypes.byref(s), _dptr(prio), pop, _dptr(obj), _dptr(start), _dptr(mach),
              _dptr(work), int(lds_slots), _dptr(ws), ws.numel(), _stream()),
           "ffs_decode_xy" if xy else "ffs_decode")
    _check(_lib.ffs_status(_dptr(ws), _stream()), "ffs_decode (device status)")
    if want_schedule or want_work:
        return {"obj": obj, "start": start, "mach": mach, "work": work}
    return obj


def ffs_decode_noalloc(dinst: DeviceInstance, prio: torch.Tensor, lds_slots: int = 0,
                       want_schedule: bool = False, want_work: bool = False):
    """ffs_decode on the library's own per-GPU scratch buffer (no workspace argument).
    Output tensors are allocated here, as for ffs_decode; the call itself allocates nothing."""
    s = dinst.s
    prio, pop, obj, start, mach, work = _decode_outputs(dinst, prio, want_schedule, want_work)
    _check(_lib.ffs_decode_noalloc(ctypes.byref(s), _dptr(prio), pop, _dptr(obj), _dptr(start),
                                   _dptr(mach), _dptr(work), int(lds_slots), _stream()),
           "ffs_decode_noalloc")
    if want_schedule or want_work:
        return {"obj": obj, "start": start, "mach": mach, "work": work}
    return obj


@dataclass
class GaConfig:
    islands: int
    rows: int
    cols: int
    pc: int
    pm: int
    mig_interval: int = 10
    mig_k: int = 1
    lds_slots: int = 0
    encoding: int = 0   # 0: one priority per job; 1: X/Y matrices (2 * n_ops genes)
    scheme: int = 0     # FFS_GA_HYBRID, FFS_GA_CLASSICAL or FFS_GA_CELLULAR

    @classmethod
    def of(cls, ga, lds_slots=0, encoding=None, scheme=0):
        enc = getattr(ga, "encoding", 0) if encoding is None else encoding
        return cls(ga.islands, ga.rows, ga.cols, ga.pc, ga.pm, ga.mig_interval, ga.mig_k, lds_slots,
                   enc, scheme)

    def c(self):
        return FfsGaParams(self.islands, self.rows, self.cols, self.pc, self.pm, self.mig_interval,
                           self.mig_k, self.lds_slots, self.encoding, self.scheme)


class GA:
    """One event's island GA on the device (ga_init / ga_step / ga_best / ga_view)."""

    def __init__(self, dinst: DeviceInstance, cfg: GaConfig, seed: int, shop: int, event: int,
                 workspace=None):
        self.dinst = dinst
        self.cfg = cfg
        self.p = cfg.c()
        self.ga = FfsGa()
        dev = dinst.t["proc"].device
        need = _lib.ffs_ga_workspace_size(ctypes.byref(dinst.s), ctypes.byref(self.p))
        if need == 0:
            raise FfsError(FFS_E_INVAL, "ffs_ga_workspace_size")
        self.ws = workspace if workspace is not None and workspace.numel() >= need else torch.empty(
            need, dtype=torch.uint8, device=dev)
        _check(_lib.ga_init(ctypes.byref(self.ga), ctypes.byref(dinst.s), ctypes.byref(self.p),
                            int(seed), int(shop), int(event), _dptr(self.ws), self.ws.numel(),
                            _stream()), "ga_init")

    @property
    def generation(self):
        return int(self.ga.generation)

    def step(self, n_generations=1):
        _check(_lib.ga_step(ctypes.byref(self.ga), ctypes.byref(self.dinst.s), int(n_generations),
                            _stream()), "ga_step")

    def step_screened(self, model: "Surrogate", table: torch.Tensor, variants: int = 4,
                      n_generations: int = 1, scores: torch.Tensor = None,
                      choice: torch.Tensor = None):
        """Screened generations (ga_step_screened): `variants` candidates per cell,
        the lowest surrogate score kept and decoded exactly."""
        _check(_lib.ga_step_screened(ctypes.byref(self.ga), ctypes.byref(self.dinst.s),
                                     ctypes.byref(model.s), _dptr(table), int(variants),
                                     int(n_generations), _dptr(scores), _dptr(choice), _stream()),
               "ga_step_screened")

    def status(self):
        _check(_lib.ffs_status(_dptr(self.ws), _stream()), "ga (device status)")

    def best(self):
        n = max(int(self.ga.n_genes), 1)
        dev = self.ws.device
        prio = torch.empty(n, dtype=torch.int32, device=dev)
        obj = torch.empty(1, dtype=torch.int64, device=dev)
        _check(_lib.ga_best(ctypes.byref(self.ga), _dptr(prio), _dptr(obj), _stream()), "ga_best")
        return prio[: self.ga.n_genes], obj

    def _slice(self, ptr, count, dtype):
        off = ptr - self.ws.data_ptr()
        size = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off: off + count * size].view(dtype)

    def view(self):
        """Tensors viewing the live state: prio [pop, n], obj [pop], elite [I, n], elite_obj [I]."""
        v = FfsGaView()
        _check(_lib.ga_view(ctypes.byref(self.ga), ctypes.byref(v)), "ga_view")
        pop, n, isl = int(self.ga.pop), int(self.ga.n_genes), self.cfg.islands
        return {
            "prio": self._slice(v.prio, pop * n, torch.int32).view(pop, n),
            "obj": self._slice(v.obj, pop, torch.int64),
            "elite": self._slice(v.elite, isl * n, torch.int32).view(isl, n),
            "elite_obj": self._slice(v.elite_obj, isl, torch.int64),
            "work": self._slice(v.work, 1, torch.int64),
        }

    def overflows(self):
        """Decodes since ga_init redone off chip (their schedule outgrew the on-chip slots)."""
        v = FfsGaView()
        _check(_lib.ga_view(ctypes.byref(self.ga), ctypes.byref(v)), "ga_view")
        return int(self._slice(v.overflows, 1, torch.int64).item())

    def e_max(self):
        """E_max of eq. (13) set by ga_init for FFS_GA_CLASSICAL (0 otherwise)."""
        v = FfsGaView()
        _check(_lib.ga_view(ctypes.byref(self.ga), ctypes.byref(v)), "ga_view")
        return int(self._slice(v.e_max, 1, torch.int64).item())


def reschedule(prev: DeviceInstance, plan_start: torch.Tensor, plan_mach: torch.Tensor, arrival,
               workspace=None, static=False) -> DeviceInstance:
    """Freeze `prev`'s executed plan at arrival.rs, append the arrival's jobs.
    static=True: the traditional static approach (reschedule_static)."""
    s = prev.s
    dev = prev.t["proc"].device
    g, om = int(s.n_stages), int(s.o_max)
    n_new = int(len(arrival.release))
    n = int(s.n_jobs) + n_new
    t = {
        "n_machines": prev.t["n_machines"],
        "proc": torch.empty((max(n, 1), g, om), dtype=torch.int32, device=dev),
        "power": torch.empty((max(n, 1), g, om), dtype=torch.int32, device=dev),
        "release": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "due": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "first_stage": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "ready": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "machine_free": torch.empty((g, om), dtype=torch.int32, device=dev),
        "running": torch.empty((max(g * om, 1), 2), dtype=torch.int32, device=dev),
        "active": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "fixed": torch.empty((max(int(s.n_jobs) * g, 1), 3), dtype=torch.int32, device=dev),
    }
    nxt = FfsInstance()
    for k in ("n_machines", "proc", "power", "release", "due", "first_stage", "ready",
              "machine_free", "running", "active", "fixed"):
        setattr(nxt, k, t[k].data_ptr())
    new = {
        "proc": _i32(np.asarray(arrival.proc).reshape(n_new, g, om), dev),
        "power": _i32(np.asarray(arrival.power).reshape(n_new, g, om), dev),
        "release": _i32(arrival.release, dev), "due": _i32(arrival.due, dev),
    }
    need = _lib.ffs_reschedule_workspace_size(int(s.n_jobs), n_new)
    ws = workspace if workspace is not None and workspace.numel() >= need else torch.empty(
        need, dtype=torch.uint8, device=dev)
    ps = plan_start.to(device=dev, dtype=torch.int32).contiguous()
    pm = plan_mach.to(device=dev, dtype=torch.int32).contiguous()
    fn = _lib.reschedule_static if static else _lib.reschedule
    _check(fn(ctypes.byref(s), _dptr(ps), _dptr(pm), int(arrival.rs), n_new,
              _dptr(new["proc"]), _dptr(new["power"]), _dptr(new["release"]),
              _dptr(new["due"]), ctypes.byref(nxt), _dptr(ws), ws.numel(), _stream()),
           "reschedule_static" if static else "reschedule")
    t["_new"] = new
    return DeviceInstance(nxt, t)


def timing_enable(on=True, families=None, every=1):
    """Time kernel launches with HIP events: every family, or only those listed;
    events on one launch in `every` of each (timing_read counts those)."""
    mask = 0 if not on else (-1 if families is None else sum(1 << int(f) for f in families))
    _check(_lib.ffs_timing_every(int(every)), "ffs_timing_every")
    _check(_lib.ffs_timing_enable(mask), "ffs_timing_enable")


_island_groups = 0        # the value last given to ga_set_island_groups
_group_stream_devices = set()


def set_island_groups(groups):
    """ga_set_island_groups: island groups ga_step runs on streams of their own
    (0: the library's default of 4; 1: one stream). Also creates the current
    device's group streams."""
    global _island_groups
    _check(_lib.ga_set_island_groups(int(groups)), "ga_set_island_groups")
    _island_groups = int(groups)
    if _island_groups != 1:
        _group_stream_devices.add(torch.cuda.current_device())


def _make_group_streams(device):
    """Create `device`'s island-group streams with the first instance placed on it:
    before the streams of a Batch, so that they get hardware queues of their own."""
    idx = torch.device(device).index
    if idx is None:
        idx = torch.cuda.current_device()
    if _island_groups == 1 or idx in _group_stream_devices:
        return
    with torch.cuda.device(idx):
        _check(_lib.ga_set_island_groups(_island_groups), "ga_set_island_groups")
    _group_stream_devices.add(idx)


def timing_read(family):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.ffs_timing_read(int(family), ctypes.byref(ms), ctypes.byref(n)), "ffs_timing_read")
    return float(ms.value), int(n.value)


def exported_symbols():
    """Names declared in include/ffsga.h that the loaded library exports."""
    names = []
    for name in ("ffs_prepare", "ffs_decode_workspace_size", "ffs_decode", "ffs_decode_noalloc",
                 "ffs_decode_xy",
                 "ffs_status",
                 "ffs_ga_workspace_size", "ga_init", "ga_step", "ga_set_island_groups", "ga_best",
                 "ga_view",
                 "ffs_reschedule_workspace_size", "reschedule", "reschedule_static",
                 "ffs_timing_enable",
                 "ffs_timing_every", "ffs_timing_read", "ffs_strerror", "ffs_build_id", "ffs_batch_workspace_size",
                 "ga_batch_create", "ga_batch_set", "ga_batch_clear", "ga_batch_step",
                 "ga_batch_best", "ga_batch_view", "ga_batch_destroy", "sg_refresh",
                 "sg_features", "sg_table_workspace_size", "sg_score_table", "sg_score",
                 "sg_train_workspace_size", "sg_train_step", "ga_step_screened", "sg_targets"):
        if hasattr(_lib, name):
            names.append(name)
    return names


# --------------------------------------------------------------------------
# Batched GA (ga_batch_*).
# --------------------------------------------------------------------------
FFS_SCHEDULE_CHROMOSOME = 0
FFS_SCHEDULE_ISLAND = 1
FFS_BATCH_MAX_SLOTS = 4096
FFS_BATCH_MAX_CLASSES = 4


class FfsBatchParams(ctypes.Structure):
    _fields_ = [
        ("n_slots", ctypes.c_int32), ("max_jobs", ctypes.c_int32), ("max_genes", ctypes.c_int32),
        ("max_stages", ctypes.c_int32), ("o_max", ctypes.c_int32), ("max_horizon", ctypes.c_int32),
        ("ga", FfsGaParams), ("schedule", ctypes.c_int32), ("blocks", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("profile_classes", ctypes.c_int32),
    ]


class FfsBatch(ctypes.Structure):
    _fields_ = [
        ("params", FfsBatchParams),
        ("pop", ctypes.c_int32), ("lds_slots", ctypes.c_int32), ("blocks", ctypes.c_int32),
        ("omp", ctypes.c_int32),
        ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t),
        ("graph", _vp), ("graph_exec", _vp), ("graph_stream", _vp),
        ("active", ctypes.c_int32 * FFS_BATCH_MAX_SLOTS),
        ("generation", ctypes.c_int32 * FFS_BATCH_MAX_SLOTS),
        ("n_genes", ctypes.c_int32 * FFS_BATCH_MAX_SLOTS),
    ]


_lib.ffs_batch_workspace_size.argtypes = [_P(FfsBatchParams)]
_lib.ffs_batch_workspace_size.restype = ctypes.c_size_t
_lib.ga_batch_create.argtypes = [_P(FfsBatch), _P(FfsBatchParams), _vp, ctypes.c_size_t, _vp]
_lib.ga_batch_set.argtypes = [_P(FfsBatch), ctypes.c_int32, _P(FfsInstance), ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_int32, _vp]
_lib.ga_batch_clear.argtypes = [_P(FfsBatch), ctypes.c_int32, _vp]
_lib.ga_batch_step.argtypes = [_P(FfsBatch), ctypes.c_int32, _vp]
_lib.ga_batch_best.argtypes = [_P(FfsBatch), ctypes.c_int32, _vp, _vp, _vp]
_lib.ga_batch_view.argtypes = [_P(FfsBatch), ctypes.c_int32, _P(FfsGaView)]
_lib.ga_batch_destroy.argtypes = [_P(FfsBatch)]
for _f in ("ga_batch_create", "ga_batch_set", "ga_batch_clear", "ga_batch_step", "ga_batch_best",
           "ga_batch_view", "ga_batch_destroy"):
    getattr(_lib, _f).restype = ctypes.c_int


@dataclass
class BatchConfig:
    """Room and shape of a batch: every slot holds one instance of at most these sizes."""
    n_slots: int
    max_jobs: int
    max_genes: int
    max_stages: int
    o_max: int
    max_horizon: int
    ga: GaConfig
    schedule: int = FFS_SCHEDULE_CHROMOSOME
    blocks: int = 0
    use_graph: bool = False
    profile_classes: int = 1

    def c(self):
        return FfsBatchParams(self.n_slots, self.max_jobs, self.max_genes, self.max_stages,
                              self.o_max, self.max_horizon, self.ga.c(), self.schedule,
                              self.blocks, 1 if self.use_graph else 0, self.profile_classes)

    def workspace_bytes(self) -> int:
        """Device bytes a batch of this shape needs (ffs_batch_workspace_size)."""
        need = _lib.ffs_batch_workspace_size(ctypes.byref(self.c()))
        if need == 0:
            raise FfsError(FFS_E_INVAL, "ffs_batch_workspace_size")
        return int(need)


class Batch:
    """Slots of independent instances advanced together on one stream of their own."""

    def __init__(self, cfg: BatchConfig, device="cuda", workspace=None):
        self.cfg = cfg
        self.p = cfg.c()
        self.b = FfsBatch()
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.insts = {}
        need = _lib.ffs_batch_workspace_size(ctypes.byref(self.p))
        if need == 0:
            raise FfsError(FFS_E_INVAL, "ffs_batch_workspace_size")
        self.ws = workspace if workspace is not None and workspace.numel() >= need else torch.empty(
            need, dtype=torch.uint8, device=self.device)
        self._enter()
        _check(_lib.ga_batch_create(ctypes.byref(self.b), ctypes.byref(self.p), _dptr(self.ws),
                                    self.ws.numel(), _stream(self.stream)), "ga_batch_create")

    def _enter(self):
        # work queued on the caller's stream (uploads, tensors) happens first
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    @property
    def pop(self):
        return int(self.b.pop)

    def set(self, slot, dinst: DeviceInstance, seed, shop, event):
        self._enter()
        _check(_lib.ga_batch_set(ctypes.byref(self.b), int(slot), ctypes.byref(dinst.s), int(seed),
                                 int(shop), int(event), _stream(self.stream)), "ga_batch_set")
        self.insts[slot] = dinst
        self._leave()

    def clear(self, slot):
        self._enter()
        _check(_lib.ga_batch_clear(ctypes.byref(self.b), int(slot), _stream(self.stream)),
               "ga_batch_clear")
        self.insts.pop(slot, None)
        self._leave()

    def step(self, n_generations=1):
        self._enter()
        _check(_lib.ga_batch_step(ctypes.byref(self.b), int(n_generations), _stream(self.stream)),
               "ga_batch_step")
        self._leave()

    def generation(self, slot):
        return int(self.b.generation[slot])

    def best(self, slot):
        n = max(int(self.b.n_genes[slot]), 1)
        prio = torch.empty(n, dtype=torch.int32, device=self.device)
        obj = torch.empty(1, dtype=torch.int64, device=self.device)
        self._enter()
        _check(_lib.ga_batch_best(ctypes.byref(self.b), int(slot), _dptr(prio), _dptr(obj),
                                  _stream(self.stream)), "ga_batch_best")
        self._leave()
        return prio[: self.b.n_genes[slot]], obj

    def _slice(self, ptr, count, dtype):
        off = ptr - self.ws.data_ptr()
        size = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off: off + count * size].view(dtype)

    def view(self, slot):
        v = FfsGaView()
        _check(_lib.ga_batch_view(ctypes.byref(self.b), int(slot), ctypes.byref(v)), "ga_batch_view")
        pop, n, isl = self.pop, int(self.b.n_genes[slot]), self.cfg.ga.islands
        self._leave()
        return {
            "prio": self._slice(v.prio, pop * n, torch.int32).view(pop, n),
            "obj": self._slice(v.obj, pop, torch.int64),
            "elite": self._slice(v.elite, isl * n, torch.int32).view(isl, n),
            "elite_obj": self._slice(v.elite_obj, isl, torch.int64),
            "work": self._slice(v.work, 1, torch.int64),
        }

    def status(self):
        self.stream.synchronize()
        _check(_lib.ffs_status(_dptr(self.ws), _stream(self.stream)), "ga_batch (device status)")

    def destroy(self):
        _check(_lib.ga_batch_destroy(ctypes.byref(self.b)), "ga_batch_destroy")

    def __del__(self):
        try:
            _lib.ga_batch_destroy(ctypes.byref(self.b))
        except Exception:
            pass


# --------------------------------------------------------------------------
# Learned offspring pre-screen (include/ffs_surrogate.h).
# --------------------------------------------------------------------------
SG_HIDDEN = 256
SG_PARAMS = 4 * 256 + 256 + 256 * 256 + 256 + 256 + 1
SG_MAX_GENES = 256
SG_MAX_BATCH = 8192
SG_MAX_VARIANTS = 8


class FfsSurrogate(ctypes.Structure):
    _fields_ = [("theta", _vp), ("adam_m", _vp), ("adam_v", _vp), ("w2_bf16", _vp),
                ("w2t_bf16", _vp), ("step", ctypes.c_int32)]


_lib.sg_refresh.argtypes = [_P(FfsSurrogate), _vp]
_lib.sg_features.argtypes = [_P(FfsInstance), _vp, _vp, ctypes.c_size_t, _vp]
_lib.sg_table_workspace_size.argtypes = [ctypes.c_int32]
_lib.sg_table_workspace_size.restype = ctypes.c_size_t
_lib.sg_score_table.argtypes = [_P(FfsSurrogate), _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t,
                                _vp]
_lib.sg_score.argtypes = [_P(FfsSurrogate), _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]
_lib.sg_targets.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]
_lib.sg_train_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.sg_train_workspace_size.restype = ctypes.c_size_t
_lib.sg_train_step.argtypes = [_P(FfsSurrogate), _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                               ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.ga_step_screened.argtypes = [_P(FfsGa), _P(FfsInstance), _P(FfsSurrogate), _vp,
                                  ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
for _f in ("sg_refresh", "sg_features", "sg_score_table", "sg_score", "sg_train_step",
           "ga_step_screened", "sg_targets"):
    getattr(_lib, _f).restype = ctypes.c_int


class Surrogate:
    """The surrogate's parameters, Adam moments and bf16 copies of W2 on the device."""

    def __init__(self, theta, device="cuda"):
        t = torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float32)).to(device)
        if t.numel() != SG_PARAMS:
            raise FfsError(FFS_E_INVAL, f"surrogate needs {SG_PARAMS} parameters, got {t.numel()}")
        self.theta = t.contiguous()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.w2b = torch.empty(SG_HIDDEN * SG_HIDDEN, dtype=torch.int16, device=device)
        self.w2tb = torch.empty_like(self.w2b)
        self.s = FfsSurrogate(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                              self.w2b.data_ptr(), self.w2tb.data_ptr(), 0)
        _check(_lib.sg_refresh(ctypes.byref(self.s), _stream()), "sg_refresh")
        self._train_ws = None
        self._table_ws = None

    @property
    def step(self):
        return int(self.s.step)

    def features(self, dinst: DeviceInstance) -> torch.Tensor:
        dev = self.theta.device
        feats = torch.empty((max(dinst.n_active, 1), 4), dtype=torch.float32, device=dev)
        ws = torch.empty(FFS_PREPARE_WORKSPACE, dtype=torch.uint8, device=dev)
        _check(_lib.sg_features(ctypes.byref(dinst.s), _dptr(feats), _dptr(ws), ws.numel(),
                                _stream()), "sg_features")
        return feats

    def score_table(self, feats: torch.Tensor, n: int) -> torch.Tensor:
        need = _lib.sg_table_workspace_size(int(n))
        if need == 0:
            raise FfsError(FFS_E_INVAL, "sg_table_workspace_size")
        if self._table_ws is None or self._table_ws.numel() < need:
            self._table_ws = torch.empty(need, dtype=torch.uint8, device=self.theta.device)
        table = torch.empty((n, n), dtype=torch.float32, device=self.theta.device)
        _check(_lib.sg_score_table(ctypes.byref(self.s), _dptr(feats), int(n), _dptr(table),
                                   _dptr(self._table_ws), self._table_ws.numel(), _stream()),
               "sg_score_table")
        return table

    def score(self, table: torch.Tensor, prio: torch.Tensor) -> torch.Tensor:
        prio = prio.to(device=self.theta.device, dtype=torch.int32).contiguous()
        n = int(prio.shape[-1])
        count = int(prio.numel() // max(n, 1))
        y = torch.empty(count, dtype=torch.float32, device=self.theta.device)
        _check(_lib.sg_score(ctypes.byref(self.s), _dptr(table), n, _dptr(prio), count, _dptr(y),
                             _stream()), "sg_score")
        return y

    def targets(self, obj, group):
        """Training targets: ln obj standardised within groups of `group` (sg_targets)."""
        dev = self.theta.device
        obj = obj.to(device=dev, dtype=torch.int64).contiguous()
        t = torch.empty(obj.numel(), dtype=torch.float32, device=dev)
        ws = torch.empty(FFS_PREPARE_WORKSPACE, dtype=torch.uint8, device=dev)
        _check(_lib.sg_targets(_dptr(obj), obj.numel(), int(group), _dptr(t), _dptr(ws), ws.numel(),
                               _stream()), "sg_targets")
        _check(_lib.ffs_status(_dptr(ws), _stream()), "sg_targets (device status)")
        return t

    def train_step(self, feats, prio, target, lr, want_grad=False):
        """One Adam step; returns (loss tensor [1], gradient [SG_PARAMS] or None)."""
        dev = self.theta.device
        prio = prio.to(device=dev, dtype=torch.int32).contiguous()
        target = target.to(device=dev, dtype=torch.float32).contiguous()
        B, n = int(prio.shape[0]), int(prio.shape[1])
        need = _lib.sg_train_workspace_size(n, B)
        if need == 0:
            raise FfsError(FFS_E_INVAL, "sg_train_workspace_size")
        if self._train_ws is None or self._train_ws.numel() < need:
            self._train_ws = torch.empty(need, dtype=torch.uint8, device=dev)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        grad = torch.empty(SG_PARAMS, dtype=torch.float32, device=dev) if want_grad else None
        _check(_lib.sg_train_step(ctypes.byref(self.s), _dptr(feats), n, _dptr(prio), _dptr(target), B,
                                  float(lr), _dptr(loss), _dptr(grad), _dptr(self._train_ws),
                                  self._train_ws.numel(), _stream()), "sg_train_step")
        return loss, grad
