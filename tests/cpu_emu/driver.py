"""Driver of the CPU build (`libawe_emu.so`): the library's C ABI on host arrays.

Runs inside a process that has the AddressSanitizer runtime preloaded (see `run`): every
workspace gets its gaps between sub-buffers poisoned, so an access of a kernel or of the
host code that leaves its own sub-buffer is reported with its stack.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2304_05592_amd import binding as B  # noqa: E402  (ctypes structs and problem layout)


class EmuLib:
    def __init__(self, path):
        L = ctypes.CDLL(path)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.awe_plan_create.argtypes = [ctypes.POINTER(B.AweProblem), ctypes.POINTER(B.AweStorage),
                                      ctypes.POINTER(vp)]
        L.awe_plan_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
        L.awe_plan_destroy.argtypes = [vp]
        L.awe_plan_destroy.restype = None
        L.awe_forward.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]
        L.awe_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.awe_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.awe_adjoint.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.awe_born.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        if hasattr(L, "awe_gradient_probed"):
            L.awe_gradient_probed.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        for name, args in (("awe_plan_set_tiles", [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
                           ("awe_plan_set_tiles_dir", [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.c_int32]),
                           ("awe_plan_set_fusion", [vp, ctypes.c_int32]),
                           ("awe_plan_set_checks", [vp, ctypes.c_int32]),
                           ("awe_plan_get_storage", [vp, ctypes.POINTER(B.AweStorage)]),
                           ("awe_plan_get_tiles", [vp] + [ctypes.POINTER(ctypes.c_int32)] * 3),
                           ("awe_plan_autotune", [vp, vp, vp, vp, ctypes.c_int32, vp, sz, vp,
                                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
                           ("awe_plan_set_groups", [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)])):
            if hasattr(L, name):
                getattr(L, name).argtypes = args
        L.awe_emu_subbuffers.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.awe_emu_subbuffers.restype = ctypes.c_int
        L.awe_last_error.restype = ctypes.c_char_p
        L.emu_launch_count.restype = ctypes.c_longlong
        self.L = L
        self.asan = None
        try:
            self.asan = getattr(ctypes.CDLL(None), "__asan_poison_memory_region")
            self.asan.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
        except AttributeError:
            pass

    def check(self, st):
        if st != 0:
            raise B.AweError(st, self.L.awe_last_error().decode())


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


_POISON = None


def _poison(addr, n):
    """Mark [addr, addr + n) as unaddressable for AddressSanitizer (no-op without it)."""
    global _POISON
    if _POISON is None:
        try:
            _POISON = getattr(ctypes.CDLL(None), "__asan_poison_memory_region")
            _POISON.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
        except AttributeError:
            _POISON = False
    if _POISON and n > 0:
        _POISON(ctypes.c_void_p(addr), n)


def _guarded(nbytes):
    """`_filled(nbytes)` as a 256-byte aligned view with EMU_ARRAY_GUARD poisoned bytes (or
    more) on both sides: an access that runs off the front or the end of an array the library
    is given, by any distance up to the guard, is reported.  On the GPU such an access lands in
    whatever the caching allocator placed next to the tensor, or in unmapped memory."""
    g = int(os.environ.get("EMU_ARRAY_GUARD", "0"))
    raw = _filled(nbytes + 2 * g + 256)
    off = g + (-(raw.ctypes.data + g)) % 256
    if g > 0:
        _poison(raw.ctypes.data, off)
        _poison(raw.ctypes.data + off + nbytes, raw.nbytes - off - nbytes)
    return raw[off:off + nbytes]


def _guarded_copy(a):
    a = np.ascontiguousarray(a)
    out = _guarded(a.nbytes).view(a.dtype)
    out[:] = a.ravel()
    return out


class EmuPlan:
    """The survey of `binding.Plan` on the CPU build; arrays are numpy (packed as there)."""

    def __init__(self, lib: EmuLib, wl, storage=None, shots=None):
        self.lib, self.L = lib, lib.L
        shots = range(wl.nshot) if shots is None else list(shots)
        self.geoms = [B.ShotGeometry(wl.shots[s].window, wl.shots[s].nt, wl.shots[s].src, wl.shots[s].rec)
                      for s in shots]
        windows = [wl.comp_shape(w) for w in range(wl.nwindow)]
        self.storage = storage or B.Storage()
        prob, self.layout, self._cs, self._rec = B.describe(wl.ndim, wl.h, wl.dt, wl.nbl, wl.vmax, windows,
                                                            self.geoms, wl.vmax)
        st = self.storage.c()
        h = ctypes.c_void_p()
        lib.check(self.L.awe_plan_create(ctypes.byref(prob), ctypes.byref(st), ctypes.byref(h)))
        self.h = h
        self.windows = windows
        self._ws = None

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.awe_plan_destroy(self.h)

    def ws_bytes(self):
        n = ctypes.c_size_t()
        self.lib.check(self.L.awe_plan_workspace_size(self.h, ctypes.byref(n)))
        return n.value

    def workspace(self):
        """A fresh 256-byte aligned workspace with the gaps between sub-buffers poisoned."""
        n = self.ws_bytes()
        ws = _guarded(n)
        cap = 4096
        buf = (ctypes.c_longlong * (2 * cap))()
        cnt = self.L.awe_emu_subbuffers(self.h, buf, cap)
        if self.lib.asan is not None:
            spans = sorted((buf[2 * i], buf[2 * i + 1]) for i in range(cnt))
            cur = 0
            for b, e in spans + [(n, n)]:
                if b > cur:
                    self.lib.asan(ctypes.c_void_p(ws.ctypes.data + cur), b - cur)
                cur = max(cur, e)
        return ws

    def set_tiles(self, tz=32, ty=8, bz=0, dirs=3):
        if dirs == 3:
            self.lib.check(self.L.awe_plan_set_tiles(self.h, tz, ty, bz))
        else:
            self.lib.check(self.L.awe_plan_set_tiles_dir(self.h, dirs, tz, ty, bz))

    def get_storage(self):
        out = B.AweStorage()
        self.lib.check(self.L.awe_plan_get_storage(self.h, ctypes.byref(out)))
        return B.Storage(out.mode, out.nslots, out.prec)

    def set_checks(self, flags):
        self.lib.check(self.L.awe_plan_set_checks(self.h, flags))

    def get_tiles(self):
        fw, adj, fu = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)(), ctypes.c_int32(0)
        self.lib.check(self.L.awe_plan_get_tiles(self.h, fw, adj, ctypes.byref(fu)))
        return tuple(fw), tuple(adj), fu.value

    def autotune(self, m, q, dd=None, probe_steps=4):
        ws = self.workspace()
        ch, ms = (ctypes.c_int32 * 4)(), ctypes.c_double(0.0)
        self.lib.check(self.L.awe_plan_autotune(self.h, _p(m), _p(q), _p(dd), probe_steps, _p(ws), ws.nbytes,
                                                None, ch, ctypes.byref(ms)))
        return self.get_tiles(), ms.value

    def set_groups(self, n):
        a = ctypes.c_int32()
        self.lib.check(self.L.awe_plan_set_groups(self.h, n, ctypes.byref(a)))
        return a.value

    def set_fusion(self, mode):
        self.lib.check(self.L.awe_plan_set_fusion(self.h, mode))

    def pack(self, arrays, dtype=np.float32):
        return _guarded_copy(np.concatenate([np.asarray(a, dtype=dtype).ravel() for a in arrays]))

    def gradient(self, m, q, dd, v=False, d=False, ws=None):
        lay = self.layout
        g = _guarded(lay.m_size * 8).view(np.float64)
        vv = _guarded(lay.q_size * 4).view(np.float32) if v else None
        dt = _guarded(lay.d_size * 4).view(np.float32) if d else None
        ws = self.workspace() if ws is None else ws
        self.lib.check(self.L.awe_gradient(self.h, _p(m), _p(q), _p(dd), _p(g), _p(vv), _p(dt), _p(ws),
                                           ws.nbytes, None))
        return g, vv, dt

    def gradient_probed(self, m, q, dd, C, s, v=False, d=False, ws=None):
        lay = self.layout
        g = _guarded(lay.m_size * 8).view(np.float64)
        vv = _guarded(lay.q_size * 4).view(np.float32) if v else None
        dt = _guarded(lay.d_size * 4).view(np.float32) if d else None
        ws = self.workspace() if ws is None else ws
        C = _guarded_copy(np.asarray(C, dtype=np.float32))
        s = _guarded_copy(np.asarray(s, dtype=np.float64))
        self.lib.check(self.L.awe_gradient_probed(self.h, _p(m), _p(q), _p(dd), _p(C), _p(s), _p(g), _p(vv),
                                                  _p(dt), _p(ws), ws.nbytes, None))
        return g, vv, dt

    def forward(self, m, q, ws=None):
        d = _guarded(self.layout.d_size * 4).view(np.float32)
        ws = self.workspace() if ws is None else ws
        self.lib.check(self.L.awe_forward(self.h, _p(m), _p(q), _p(d), 0, _p(ws), ws.nbytes, None))
        return d

    def adjoint(self, m, dd, ws=None):
        v = _guarded(self.layout.q_size * 4).view(np.float32)
        ws = self.workspace() if ws is None else ws
        self.lib.check(self.L.awe_adjoint(self.h, _p(m), _p(dd), _p(v), _p(ws), ws.nbytes, None))
        return v

    def born(self, m, q, dm, ws=None):
        dd = _guarded(self.layout.d_size * 4).view(np.float32)
        ws = self.workspace() if ws is None else ws
        self.lib.check(self.L.awe_born(self.h, _p(m), _p(q), _p(dm), _p(dd), _p(ws), ws.nbytes, None))
        return dd


def _filled(nbytes):
    """Bytes for a workspace or an output array. On the GPU both come from a caching allocator
    and hold whatever an earlier tensor left there; EMU_FILL makes that visible here: a byte
    value (e.g. 255: every float NaN, every int -1) or "random" (seeded by EMU_FILL_SEED)."""
    f = os.environ.get("EMU_FILL")
    if f is None:
        return np.zeros(nbytes, dtype=np.uint8)
    if f == "random":
        rng = np.random.default_rng(int(os.environ.get("EMU_FILL_SEED", "1")))
        return rng.integers(0, 256, nbytes, dtype=np.uint8)
    return np.full(nbytes, int(f, 0), dtype=np.uint8)


def run(script_args, so_path, env_extra=None, timeout=1800):
    """Run `python <script_args>` with the AddressSanitizer runtime preloaded; returns the
    completed process (stdout + stderr captured)."""
    from build_emu import asan_runtime  # noqa: WPS433
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1:detect_stack_use_after_return=0"
    env["AWE_EMU_SO"] = so_path
    env["PYTHONPATH"] = HERE + os.pathsep + ROOT
    if env_extra:
        env.update(env_extra)
    return subprocess.run([sys.executable] + list(script_args), env=env, capture_output=True, text=True,
                          timeout=timeout)
