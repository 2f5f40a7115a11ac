"""ctypes binding of libawe.so (declarations in include/awe.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  PyTorch
supplies device memory (tensors) and the current HIP stream.  If the library is missing or
fails to load, every entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libawe.so")

AWE_OK = 0
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "CFL", 4: "GEOMETRY", 5: "WORKSPACE",
          6: "STATE", 7: "HIP", 8: "NONFINITE", 9: "INTERNAL"}
AWE_ERR_CFL, AWE_ERR_WORKSPACE, AWE_ERR_NONFINITE = 3, 5, 8
STORE_NONE, STORE_FULL, STORE_CHECKPOINT, STORE_AUTO, STORE_PROBED = 0, 1, 2, 3, 4
CHECK_INPUTS, CHECK_OUTPUTS, CHECK_LAUNCHES = 1, 2, 4
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2

EXPORTS = ["awe_plan_create", "awe_plan_workspace_size", "awe_plan_destroy", "awe_forward",
           "awe_backward", "awe_gradient", "awe_adjoint", "awe_born", "awe_reduce_workspace_size",
           "awe_residual", "awe_residual_noalloc", "awe_dot_f64", "awe_dot_f64d", "awe_checkpoint_schedule",
           "awe_plan_autotune", "awe_plan_get_tiles", "awe_plan_set_tiles", "awe_plan_set_tiles_dir",
           "awe_plan_set_fusion", "awe_plan_set_groups", "awe_profile_enable", "awe_profile_read", "awe_profile_disable",
           "awe_slowness2", "awe_velocity_gradient", "awe_patchy", "awe_patchy_vjp", "awe_status_string", "awe_last_error", "awe_version",
           "awe_storage_select", "awe_plan_get_storage", "awe_plan_set_checks", "awe_gradient_probed"]


FUSE_NONE, FUSE_FORWARD, FUSE_ADJOINT, FUSE_BOTH = 0, 1, 2, 3


class AweError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"awe status {STATUS.get(status, status)}: {message}")
        self.status = status


class AwePatchyConsts(ctypes.Structure):
    _fields_ = [("k_min", ctypes.c_double), ("k_brine", ctypes.c_double), ("k_co2", ctypes.c_double),
                ("rho_co2", ctypes.c_double), ("rho_brine", ctypes.c_double)]


class AweShot(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("m_offset", ctypes.c_int64), ("q_offset", ctypes.c_int64),
                ("d_offset", ctypes.c_int64), ("rec_offset", ctypes.c_int64),
                ("nrec", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("src", ctypes.c_double * 3)]


class AweProblem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nbl", ctypes.c_int32), ("h", ctypes.c_double),
                ("dt", ctypes.c_double), ("vmax", ctypes.c_double), ("damp_vref", ctypes.c_double),
                ("damp_R", ctypes.c_double), ("nshot", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("shots", ctypes.POINTER(AweShot)), ("rec_pos", ctypes.POINTER(ctypes.c_double))]


class AweStorage(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("nslots", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("budget_mib", ctypes.c_int32)]


_lib = None


def lib():
    """Load libawe.so once (raises OSError if it is missing: build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing; build it with `python -m paper_2304_05592_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int
    L.awe_plan_create.argtypes = [ctypes.POINTER(AweProblem), ctypes.POINTER(AweStorage), ctypes.POINTER(vp)]
    L.awe_plan_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.awe_plan_destroy.argtypes = [vp]
    L.awe_plan_destroy.restype = None
    L.awe_storage_select.argtypes = [ctypes.POINTER(AweProblem), ctypes.POINTER(AweStorage),
                                     ctypes.POINTER(AweStorage), ctypes.POINTER(sz)]
    L.awe_plan_get_storage.argtypes = [vp, ctypes.POINTER(AweStorage)]
    L.awe_plan_set_checks.argtypes = [vp, ctypes.c_int32]
    L.awe_forward.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp]
    L.awe_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.awe_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.awe_gradient_probed.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.awe_adjoint.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.awe_born.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.awe_reduce_workspace_size.argtypes = [i64]
    L.awe_reduce_workspace_size.restype = sz
    L.awe_residual.argtypes = [vp, vp, vp, i64, vp, vp, sz, vp]
    L.awe_residual_noalloc.argtypes = [vp, vp, vp, i64, vp, vp]
    L.awe_dot_f64.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    L.awe_dot_f64d.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    L.awe_checkpoint_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          i64, ctypes.POINTER(i64)]
    L.awe_plan_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, sz, vp,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    L.awe_plan_set_tiles.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.awe_plan_set_tiles_dir.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.awe_plan_get_tiles.argtypes = [vp, i32p, i32p, i32p]
    L.awe_plan_set_fusion.argtypes = [vp, ctypes.c_int32]
    L.awe_plan_set_groups.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.awe_slowness2.argtypes = [vp, vp, i64, vp]
    L.awe_velocity_gradient.argtypes = [vp, vp, vp, i64, vp]
    pc = ctypes.POINTER(AwePatchyConsts)
    L.awe_patchy.argtypes = [vp, vp, vp, vp, vp, vp, i64, pc, vp]
    L.awe_patchy_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, pc, vp]
    L.awe_profile_enable.argtypes = [vp, i64, ctypes.c_int32]
    L.awe_profile_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.awe_profile_disable.argtypes = [vp]
    L.awe_status_string.argtypes = [i32]
    L.awe_status_string.restype = ctypes.c_char_p
    L.awe_last_error.restype = ctypes.c_char_p
    L.awe_version.restype = ctypes.c_int
    for name in ("awe_plan_create", "awe_plan_workspace_size", "awe_forward", "awe_backward",
                 "awe_gradient", "awe_adjoint", "awe_born", "awe_residual", "awe_residual_noalloc",
                 "awe_dot_f64",
                 "awe_dot_f64d", "awe_checkpoint_schedule", "awe_plan_autotune", "awe_plan_get_tiles", "awe_plan_set_tiles",
                 "awe_plan_set_tiles_dir", "awe_plan_set_fusion", "awe_plan_set_groups", "awe_slowness2", "awe_velocity_gradient", "awe_patchy",
                 "awe_patchy_vjp", "awe_profile_enable",
                 "awe_profile_read", "awe_profile_disable", "awe_storage_select", "awe_plan_get_storage",
                 "awe_plan_set_checks", "awe_gradient_probed"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status: int):
    if status != AWE_OK:
        raise AweError(status, lib().awe_last_error().decode())


def checkpoint_schedule(nsteps: int, nslots: int) -> np.ndarray:
    """Action list (op, a, b) of the binomial reverse schedule (host only)."""
    L = lib()
    cnt = ctypes.c_int64(0)
    L.awe_checkpoint_schedule(nsteps, nslots, None, 0, ctypes.byref(cnt))
    buf = (ctypes.c_int32 * (3 * max(cnt.value, 1)))()
    check(L.awe_checkpoint_schedule(nsteps, nslots, buf, cnt.value, ctypes.byref(cnt)))
    return np.frombuffer(buf, dtype=np.int32, count=3 * cnt.value).reshape(-1, 3).copy()


# --------------------------------------------------------------------------------------
# survey description -> plan
# --------------------------------------------------------------------------------------
@dataclass
class ShotGeometry:
    """One shot: its model window index, samples and acquisition (metres, window coordinates)."""
    window: int
    nt: int
    src: Sequence[float]
    rec: np.ndarray


@dataclass
class Storage:
    """Wavefield storage of a plan.  STORE_AUTO: FULL if its workspace fits budget_mib MiB (0: 90 %
    of the device's free memory), else CHECKPOINT with the most slots that fit (at most nslots
    when nslots > 0).  STORE_PROBED: no wavefield, nslots probes (Plan.gradient_probed)."""
    mode: int = STORE_NONE
    nslots: int = 0
    prec: int = PREC_FP32
    budget_mib: int = 0

    def c(self):
        return AweStorage(int(self.mode), int(self.nslots), int(self.prec), int(self.budget_mib))


def select_storage(ndim, h, dt, nbl, vmax, windows, shots, storage: Storage, damp_vref=None, damp_R=1e-3):
    """(storage in effect, workspace bytes) that a plan of this survey would get, computed on the
    host without creating a plan (no device call unless AUTO with budget_mib = 0)."""
    prob, _, _cs, _rec = describe(ndim, h, dt, nbl, vmax, windows, shots, damp_vref, damp_R)
    st, out, nb = storage.c(), AweStorage(), ctypes.c_size_t(0)
    check(lib().awe_storage_select(ctypes.byref(prob), ctypes.byref(st), ctypes.byref(out), ctypes.byref(nb)))
    return Storage(out.mode, out.nslots, out.prec), nb.value


@dataclass
class Layout:
    """Element offsets of every window / shot in the packed m, q and d arrays."""
    windows: List[tuple]
    m_offset: List[int] = field(default_factory=list)
    q_offset: List[int] = field(default_factory=list)
    d_offset: List[int] = field(default_factory=list)
    m_size: int = 0
    q_size: int = 0
    d_size: int = 0


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def describe(ndim, h, dt, nbl, vmax, windows, shots, damp_vref=None, damp_R=1e-3):
    """The awe_problem of a survey (windows = computational-grid shapes, shots = ShotGeometry
    list) and the packed-array layout.  Returns (problem, layout, shot array, receiver rows);
    the last two must stay alive while the problem is used."""
    windows = [tuple(int(n) for n in w) for w in windows]
    lay = Layout(windows)
    off = 0
    for w in windows:
        lay.m_offset.append(off)
        off += int(np.prod(w))
    lay.m_size = off
    qo = do = 0
    recs = []
    cs = (AweShot * len(shots))()
    roff = 0
    for i, s in enumerate(shots):
        shape = windows[s.window]
        if ndim == 2:
            nz, nx = shape
            ny = 1
        else:
            nz, ny, nx = shape
        rec = np.asarray(s.rec, dtype=np.float64).reshape(-1, 3)
        cs[i].nx, cs[i].ny, cs[i].nz, cs[i].nt = nx, ny, nz, int(s.nt)
        cs[i].m_offset = lay.m_offset[s.window]
        cs[i].q_offset = qo
        cs[i].d_offset = do
        cs[i].rec_offset = roff
        cs[i].nrec = rec.shape[0]
        for a in range(3):
            cs[i].src[a] = float(s.src[a])
        lay.q_offset.append(qo)
        lay.d_offset.append(do)
        qo += int(s.nt)
        do += int(s.nt) * rec.shape[0]
        roff += rec.shape[0]
        recs.append(rec)
    lay.q_size, lay.d_size = qo, do
    rec_rows = np.ascontiguousarray(np.concatenate(recs, axis=0) if recs else np.zeros((1, 3)))
    prob = AweProblem()
    prob.ndim, prob.nbl, prob.h, prob.dt = ndim, int(nbl), float(h), float(dt)
    prob.vmax = float(vmax)
    prob.damp_vref = float(vmax if damp_vref is None else damp_vref)
    prob.damp_R = float(damp_R)
    prob.nshot = len(shots)
    prob.shots = ctypes.cast(cs, ctypes.POINTER(AweShot))
    prob.rec_pos = rec_rows.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return prob, lay, cs, rec_rows


class Plan:
    """A survey on one GPU: windows (computational-grid shapes) and shots.

    Arrays are packed flat: m / dm / g hold the windows back to back (C order), q / v the
    shots' wavelets, d / dd the shots' traces [nt][nrec].
    """

    def __init__(self, ndim: int, h: float, dt: float, nbl: int, vmax: float, windows,
                 shots: List[ShotGeometry], storage: Optional[Storage] = None,
                 damp_vref: Optional[float] = None, damp_R: float = 1e-3):
        L = lib()
        self.ndim, self.h, self.dt, self.nbl = ndim, float(h), float(dt), int(nbl)
        self.storage = storage or Storage()
        self.windows = [tuple(int(n) for n in w) for w in windows]
        self.shots = shots
        prob, self.layout, self._cshots, self._rec = describe(ndim, h, dt, nbl, vmax, self.windows, shots,
                                                             damp_vref, damp_R)
        st = self.storage.c()
        handle = ctypes.c_void_p()
        check(L.awe_plan_create(ctypes.byref(prob), ctypes.byref(st), ctypes.byref(handle)))
        self._h = handle
        sz = ctypes.c_size_t(0)
        check(L.awe_plan_workspace_size(self._h, ctypes.byref(sz)))
        self.ws_bytes = sz.value
        eff = AweStorage()
        check(L.awe_plan_get_storage(self._h, ctypes.byref(eff)))
        #: the storage in effect (AUTO resolved to FULL or CHECKPOINT)
        self.storage_in_effect = Storage(eff.mode, eff.nslots, eff.prec)
        if self.storage.mode == STORE_AUTO and eff.mode == STORE_CHECKPOINT:
            warnings.warn(f"AUTO storage: FULL storage does not fit the memory budget; the plan "
                          f"recomputes from CHECKPOINT storage with {eff.nslots} slots per shot "
                          f"({self.ws_bytes} bytes of workspace)", RuntimeWarning, stacklevel=2)

    def set_checks(self, flags: int):
        """Screen the inputs (CHECK_INPUTS: non-finite values -> NONFINITE, m above the vmax bound ->
        CFL) and / or the outputs (CHECK_OUTPUTS) of every later compute call, and / or check every
        launch's ranges against the plan's layout on the host (CHECK_LAUNCHES -> INTERNAL); 0
        turns it off.  Screening synchronises the stream."""
        check(lib().awe_plan_set_checks(self._h, int(flags)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().awe_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- memory helpers
    def workspace(self, device=None):
        """A fresh device workspace (uint8 tensor, 256-byte aligned view)."""
        import torch
        dev = torch.device("cuda") if device is None else device
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        shift = (-raw.data_ptr()) % 256
        return raw[shift:shift + self.ws_bytes]

    def pack(self, arrays, kind: str, device=None, dtype=None):
        """Pack per-window (kind 'm') / per-shot (kind 'q' or 'd') arrays into one device tensor."""
        import torch
        dtype = torch.float32 if dtype is None else dtype
        flat = np.concatenate([np.asarray(a, dtype=np.float64 if dtype == torch.float64 else np.float32).ravel()
                               for a in arrays])
        return torch.from_numpy(flat).to(torch.device("cuda") if device is None else device)

    def unpack(self, t, kind: str):
        """Split a packed tensor into per-window ('m') or per-shot ('q', 'd') numpy arrays."""
        a = t.detach().cpu().numpy()
        lay = self.layout
        out = []
        if kind == "m":
            for w, o in zip(self.windows, lay.m_offset):
                out.append(a[o:o + int(np.prod(w))].reshape(w))
        elif kind == "q":
            for s, o in zip(self.shots, lay.q_offset):
                out.append(a[o:o + s.nt])
        else:
            for s, o in zip(self.shots, lay.d_offset):
                nrec = np.asarray(s.rec).reshape(-1, 3).shape[0]
                out.append(a[o:o + s.nt * nrec].reshape(s.nt, nrec))
        return out

    # ---------------------------------------------------------------- tile autotuning
    def autotune(self, m, q, dd=None, probe_steps: int = 24, ws=None, stream=None):
        """Time the candidate launch shapes of each direction on these inputs and keep the
        fastest.  Returns ({'tz', 'ty', 'bz', 'fusion', 'adjoint': {'tz', 'ty', 'bz'}}, probe ms):
        the forward shape, the fusion mode and the adjoint shape."""
        ws = self.workspace(m.device) if ws is None else ws
        ch = (ctypes.c_int32 * 4)()
        ms = ctypes.c_double(0.0)
        check(lib().awe_plan_autotune(self._h, _ptr(m), _ptr(q), _ptr(dd), int(probe_steps), _ptr(ws),
                                      self.ws_bytes, _stream_ptr(stream), ch, ctypes.byref(ms)))
        return self.get_tiles(), ms.value

    def get_tiles(self):
        """{'tz', 'ty', 'bz', 'fusion', 'adjoint': {'tz', 'ty', 'bz'}}: the launch shapes in effect
        (forward solves and Born; adjoint steps) and the two-levels-per-launch mode."""
        fw, adj, fu = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)(), ctypes.c_int32(0)
        check(lib().awe_plan_get_tiles(self._h, fw, adj, ctypes.byref(fu)))
        return {"tz": fw[0], "ty": fw[1], "bz": fw[2], "fusion": fu.value,
                "adjoint": {"tz": adj[0], "ty": adj[1], "bz": adj[2]}}

    def set_tiles(self, tz: int = 32, ty: int = 8, bz: int = 0, dirs: int = 3):
        """Launch shape of the forward solves (dirs 1), the adjoint steps (2) or both (3)."""
        check(lib().awe_plan_set_tiles_dir(self._h, int(dirs), int(tz), int(ty), int(bz)))

    def set_fusion(self, mode):
        """Two time levels per launch (2D): mode bit 0 = forward solves, bit 1 = reverse sweeps
        (FUSE_FORWARD, FUSE_ADJOINT, FUSE_BOTH); True means both, False neither."""
        mode = (FUSE_BOTH if mode else FUSE_NONE) if isinstance(mode, bool) else int(mode)
        check(lib().awe_plan_set_fusion(self._h, mode))

    def set_groups(self, ngroups: int = 0) -> int:
        """Shot groups run one after the other (0: automatic, sized to the last-level cache);
        returns the number of groups in effect.  Results do not depend on the grouping."""
        n = ctypes.c_int32(0)
        check(lib().awe_plan_set_groups(self._h, int(ngroups), ctypes.byref(n)))
        return n.value

    # ---------------------------------------------------------------- kernel timing
    def profile_enable(self, max_launches: int, stride: int = 1):
        check(lib().awe_profile_enable(self._h, int(max_launches), int(stride)))

    def profile_read(self):
        """{class: (launches, total ms)} for classes 'forward', 'adjoint', 'born'."""
        counts = (ctypes.c_int64 * 3)()
        ms = (ctypes.c_double * 3)()
        check(lib().awe_profile_read(self._h, counts, ms))
        return {name: (counts[i], ms[i]) for i, name in enumerate(("forward", "adjoint", "born"))}

    def profile_disable(self):
        check(lib().awe_profile_disable(self._h))

    def _check(self, t, n, dtype, name):
        import torch
        if t is None:
            raise ValueError(f"{name} is required")
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor with >= {n} elements "
                             f"(got {t.dtype}, {tuple(t.shape)}, cuda={t.is_cuda})")
        return t

    # ---------------------------------------------------------------- operators
    def forward(self, m, q, d=None, keep=False, ws=None, stream=None):
        """d = F(m) q (packed traces).  keep=True stores the wavefield in ws for backward."""
        import torch
        lay = self.layout
        self._check(m, lay.m_size, torch.float32, "m")
        self._check(q, lay.q_size, torch.float32, "q")
        if d is None:
            d = torch.empty(lay.d_size, dtype=torch.float32, device=m.device)
        ws = self.workspace(m.device) if ws is None else ws
        check(lib().awe_forward(self._h, _ptr(m), _ptr(q), _ptr(d), int(bool(keep)), _ptr(ws),
                                self.ws_bytes, _stream_ptr(stream)))
        return d

    def backward(self, m, q, dd, g=True, v=False, ws=None, stream=None):
        """Reverse sweep after forward(keep=True): returns (g FP64 or None, v or None)."""
        import torch
        lay = self.layout
        self._check(dd, lay.d_size, torch.float32, "dd")
        gt = torch.empty(lay.m_size, dtype=torch.float64, device=dd.device) if g is True else \
            (None if g is None or g is False else g)
        vt = torch.empty(lay.q_size, dtype=torch.float32, device=dd.device) if v is True else \
            (None if v is None or v is False else v)
        if gt is not None:
            self._check(gt, lay.m_size, torch.float64, "g")
        if vt is not None:
            self._check(vt, lay.q_size, torch.float32, "v")
        check(lib().awe_backward(self._h, _ptr(m), _ptr(q), _ptr(dd), _ptr(gt), _ptr(vt), _ptr(ws),
                                 self.ws_bytes, _stream_ptr(stream)))
        return gt, vt

    def gradient(self, m, q, dd, v=False, d=False, ws=None, stream=None):
        """(g, v, d): g = J^T dd (FP64), v = F^T dd, d = F(m) q, in one forward + reverse sweep."""
        import torch
        lay = self.layout
        self._check(m, lay.m_size, torch.float32, "m")
        self._check(q, lay.q_size, torch.float32, "q")
        self._check(dd, lay.d_size, torch.float32, "dd")
        gt = torch.empty(lay.m_size, dtype=torch.float64, device=m.device)
        vt = torch.empty(lay.q_size, dtype=torch.float32, device=m.device) if v else None
        dt_ = torch.empty(lay.d_size, dtype=torch.float32, device=m.device) if d else None
        ws = self.workspace(m.device) if ws is None else ws
        check(lib().awe_gradient(self._h, _ptr(m), _ptr(q), _ptr(dd), _ptr(gt), _ptr(vt), _ptr(dt_),
                                 _ptr(ws), self.ws_bytes, _stream_ptr(stream)))
        return gt, vt, dt_

    def gradient_probed(self, m, q, dd, C, s, v=False, d=False, ws=None, stream=None):
        """(g, v, d) with g the probed estimate of J^T dd (plan storage STORE_PROBED, r probes):
        C float32 [r][max_nt] (column k weights local level k; a device tensor, or an array that
        is copied to the device), s the r weights.  See awe_gradient_probed."""
        import torch
        lay = self.layout
        r = self.storage.nslots
        max_nt = max(int(sh.nt) for sh in self.shots)
        self._check(m, lay.m_size, torch.float32, "m")
        self._check(q, lay.q_size, torch.float32, "q")
        self._check(dd, lay.d_size, torch.float32, "dd")
        if not isinstance(C, torch.Tensor):
            C = torch.from_numpy(np.ascontiguousarray(C, dtype=np.float32)).to(m.device)
        if tuple(C.shape) != (r, max_nt):
            raise ValueError(f"C must be [{r}][{max_nt}] (probes x largest nt), got {tuple(C.shape)}")
        self._check(C, r * max_nt, torch.float32, "C")
        sw = np.ascontiguousarray(s, dtype=np.float64)
        if sw.shape != (r,):
            raise ValueError(f"s must hold {r} weights")
        gt = torch.empty(lay.m_size, dtype=torch.float64, device=m.device)
        vt = torch.empty(lay.q_size, dtype=torch.float32, device=m.device) if v else None
        dt_ = torch.empty(lay.d_size, dtype=torch.float32, device=m.device) if d else None
        ws = self.workspace(m.device) if ws is None else ws
        check(lib().awe_gradient_probed(self._h, _ptr(m), _ptr(q), _ptr(dd), _ptr(C),
                                        sw.ctypes.data_as(ctypes.c_void_p), _ptr(gt), _ptr(vt), _ptr(dt_),
                                        _ptr(ws), self.ws_bytes, _stream_ptr(stream)))
        return gt, vt, dt_

    def adjoint(self, m, dd, v=None, ws=None, stream=None):
        """v = F(m)^T dd (packed per shot)."""
        import torch
        lay = self.layout
        self._check(m, lay.m_size, torch.float32, "m")
        self._check(dd, lay.d_size, torch.float32, "dd")
        if v is None:
            v = torch.empty(lay.q_size, dtype=torch.float32, device=m.device)
        ws = self.workspace(m.device) if ws is None else ws
        check(lib().awe_adjoint(self._h, _ptr(m), _ptr(dd), _ptr(v), _ptr(ws), self.ws_bytes,
                                _stream_ptr(stream)))
        return v

    def rtm(self, m, q, d, ws=None, stream=None):
        """Reverse-time migration image J(m, q)^T d of recorded data d (FP64, packed like m): the
        adjoint-state imaging condition applied to the data themselves, i.e. the gradient sweep
        with d in place of a residual (needs FULL or CHECKPOINT storage)."""
        return self.gradient(m, q, d, ws=ws, stream=stream)[0]

    def born(self, m, q, dm, dd=None, ws=None, stream=None):
        """dd = J(m, q) dm (packed traces)."""
        import torch
        lay = self.layout
        self._check(m, lay.m_size, torch.float32, "m")
        self._check(q, lay.q_size, torch.float32, "q")
        self._check(dm, lay.m_size, torch.float32, "dm")
        if dd is None:
            dd = torch.empty(lay.d_size, dtype=torch.float32, device=m.device)
        ws = self.workspace(m.device) if ws is None else ws
        check(lib().awe_born(self._h, _ptr(m), _ptr(q), _ptr(dm), _ptr(dd), _ptr(ws), self.ws_bytes,
                             _stream_ptr(stream)))
        return dd


def _reduce_ws(n, device):
    import torch
    nb = lib().awe_reduce_workspace_size(n)
    return torch.empty((nb + 7) // 8, dtype=torch.float64, device=device)


def residual(d_pred, d_obs, r=None, stream=None):
    """(r, loss): r = d_pred - d_obs and loss = 1/2 sum r^2 (FP64 device scalar)."""
    import torch
    n = d_pred.numel()
    if r is None:
        r = torch.empty_like(d_pred)
    loss = torch.empty(1, dtype=torch.float64, device=d_pred.device)
    ws = _reduce_ws(n, d_pred.device)
    check(lib().awe_residual(_ptr(d_pred), _ptr(d_obs), _ptr(r), n, _ptr(loss), _ptr(ws),
                             ws.numel() * 8, _stream_ptr(stream)))
    return r, loss


def residual_noalloc(d_pred, d_obs, r, loss, stream=None):
    """awe_residual_noalloc: r = d_pred - d_obs and loss[0] = 1/2 sum r^2 into the given tensors
    (r may be d_pred; loss may be None), using the library's static scratch instead of a
    workspace - nothing is allocated, so it can run where allocation is not allowed."""
    n = d_pred.numel()
    check(lib().awe_residual_noalloc(_ptr(d_pred), _ptr(d_obs), _ptr(r), n, _ptr(loss),
                                     _stream_ptr(stream)))
    return r, loss


def slowness2(v, m=None, stream=None):
    """m = 1/v^2 (float32 device tensors, computed in FP64 and rounded once)."""
    import torch
    if v.dtype != torch.float32 or not v.is_contiguous():
        raise TypeError("v must be a contiguous float32 tensor")
    m = torch.empty_like(v) if m is None else m
    check(lib().awe_slowness2(_ptr(v), _ptr(m), v.numel(), _stream_ptr(stream)))
    return m


def velocity_gradient(v, gm, gv=None, stream=None):
    """gv = -2 gm / v^3: the gradient with respect to the wavespeed v from the gradient with
    respect to m = 1/v^2 (float32 device tensors)."""
    import torch
    for t, n in ((v, "v"), (gm, "gm")):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{n} must be a contiguous float32 tensor")
    gv = torch.empty_like(v) if gv is None else gv
    check(lib().awe_velocity_gradient(_ptr(v), _ptr(gm), _ptr(gv), v.numel(), _stream_ptr(stream)))
    return gv


def _patchy_args(tensors, consts):
    import torch
    n = tensors[0][0].numel()
    for t, name in tensors:
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
            raise TypeError(f"{name} must be a contiguous float32 tensor of {n} values")
    c = None
    if consts is not None:
        c = ctypes.byref(AwePatchyConsts(consts["k_min"], consts["k_brine"], consts["k_co2"],
                                         consts["rho_co2"], consts["rho_brine"]))
    return n, c


def patchy(sw, vp, rho, phi, consts=None, stream=None):
    """Patchy-saturation rock physics: (vp_new, rho_new) from CO2 saturation sw, wavespeed vp
    (km/s), density rho (kg/m^3) and porosity phi (float32 device tensors of one size; FP64
    arithmetic).  consts: dict with k_min, k_brine, k_co2, rho_co2, rho_brine (None: the
    paper's values)."""
    import torch
    n, c = _patchy_args([(sw, "sw"), (vp, "vp"), (rho, "rho"), (phi, "phi")], consts)
    vp_new, rho_new = torch.empty_like(vp), torch.empty_like(rho)
    check(lib().awe_patchy(_ptr(sw), _ptr(vp), _ptr(rho), _ptr(phi), _ptr(vp_new), _ptr(rho_new), n, c,
                           _stream_ptr(stream)))
    return vp_new, rho_new


def patchy_vjp(sw, vp, rho, phi, g_vp, g_rho=None, consts=None, stream=None):
    """g_sw = g_vp dvp_new/dsw + g_rho drho_new/dsw (g_rho None: 0)."""
    import torch
    ts = [(sw, "sw"), (vp, "vp"), (rho, "rho"), (phi, "phi"), (g_vp, "g_vp")]
    if g_rho is not None:
        ts.append((g_rho, "g_rho"))
    n, c = _patchy_args(ts, consts)
    g_sw = torch.empty_like(sw)
    check(lib().awe_patchy_vjp(_ptr(sw), _ptr(vp), _ptr(rho), _ptr(phi), _ptr(g_vp),
                               None if g_rho is None else _ptr(g_rho), _ptr(g_sw), n, c,
                               _stream_ptr(stream)))
    return g_sw


def dot(a, b, stream=None):
    """sum a_i b_i accumulated in FP64 on the device (float32 or float64 inputs)."""
    import torch
    n = a.numel()
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    ws = _reduce_ws(n, a.device)
    fn = lib().awe_dot_f64d if a.dtype == torch.float64 else lib().awe_dot_f64
    check(fn(_ptr(a), _ptr(b), n, _ptr(out), _ptr(ws), ws.numel() * 8, _stream_ptr(stream)))
    return out
