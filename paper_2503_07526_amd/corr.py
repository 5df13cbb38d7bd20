"""ctypes binding of the correlator's C ABI (include/corr.h).

Argument marshalling only: every step of the per-step update, the k-space
density and the readout reduction runs in the library's HIP kernels.  PyTorch
supplies device memory (sample tensors) and streams.  If the library has not
been built the import fails; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime first, so one runtime serves both)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorr_gfx950.so")

CORR_OK, CORR_E_INVALID, CORR_E_OOM, CORR_E_DEVICE, CORR_E_STATE, CORR_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
DTYPES = {"f32": 1, "f64": 2, "cf32": 3, "cf64": 4}
ACCUMS = {"f64": 1, "kahan": 2, "f32": 3}
SOURCES = {"samples": 0, "rhok": 1, "currents": 2, "momentum": 3}
FLAG_GRAPH, FLAG_PER_GROUP, FLAG_TIMING, FLAG_DIRECT, FLAG_RHOK_VALU = 1, 2, 4, 8, 16
_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64, "cf32": torch.complex64,
                "cf64": torch.complex128}


class CorrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"corr error {code}: {msg}")
        self.code = code


class _GroupDesc(ctypes.Structure):
    _fields_ = [("n_channels", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("points", ctypes.c_int32), ("m", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("accum", ctypes.c_int32), ("source", ctypes.c_int32),
                ("update_every", ctypes.c_int32), ("pair", ctypes.c_int32),
                ("dt", ctypes.c_double), ("kvec", ctypes.POINTER(ctypes.c_int32)),
                ("n_atoms", ctypes.c_int64), ("box", ctypes.c_double),
                ("species", ctypes.POINTER(ctypes.c_int32)),
                ("masses", ctypes.POINTER(ctypes.c_double)), ("n_species", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_channels", ctypes.c_int32), ("chans_per_thread", ctypes.c_int32),
                ("lag_chunk", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("overlap_producers", ctypes.c_int32), ("fold_block", ctypes.c_int32),
                ("fold_threads", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class _ReadoutOpts(ctypes.Structure):
    _fields_ = [("ch_begin", ctypes.c_int64), ("ch_end", ctypes.c_int64),
                ("t_cut", ctypes.c_double), ("gk_kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("volume", ctypes.c_double),
                ("kB", ctypes.c_double), ("temperature", ctypes.c_double),
                ("slice_begin", ctypes.c_int64), ("slice_end", ctypes.c_int64)]


EXPORTS = ["corr_create", "corr_input_buffer", "corr_bind_input", "corr_push", "corr_push_steps",
           "corr_query", "corr_finalize", "corr_finalize_noalloc", "corr_sync", "corr_destroy",
           "corr_last_error", "corr_state_bytes", "corr_get_tuning", "corr_kernel_time",
           "corr_set_timing_stride", "corr_autotune", "corr_group_form"]

_lib = None


def lib():
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.corr_create.argtypes = [ctypes.POINTER(_GroupDesc), i32, i32, vp, ctypes.c_uint32,
                                  ctypes.POINTER(Tuning), ctypes.POINTER(vp)]
        L.corr_input_buffer.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.corr_bind_input.argtypes = [vp, i32, vp, sz]
        L.corr_push.argtypes = [vp, ctypes.POINTER(vp)]
        L.corr_push_steps.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
        L.corr_query.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.corr_finalize.argtypes = [vp, i32, ctypes.POINTER(_ReadoutOpts), ctypes.POINTER(i32),
                                    vp, vp, vp, vp, vp, vp]
        L.corr_finalize_noalloc.argtypes = L.corr_finalize.argtypes
        L.corr_sync.argtypes = [vp]
        L.corr_destroy.argtypes = [vp]
        L.corr_last_error.argtypes = [vp]
        L.corr_last_error.restype = ctypes.c_char_p
        L.corr_state_bytes.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.corr_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.corr_kernel_time.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(i64), i32]
        L.corr_set_timing_stride.argtypes = [vp, i32]
        L.corr_group_form.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.corr_autotune.argtypes = [ctypes.POINTER(_GroupDesc), i32, i32, vp, ctypes.c_uint32,
                                    ctypes.c_char_p, i64, i32, ctypes.POINTER(Tuning)]
        for name in EXPORTS:
            if name != "corr_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


@dataclass
class GroupDesc:
    """One channel group: b levels of p points, averaging m (Section 2.2)."""
    n_channels: int
    levels: int
    points: int
    m: int = 2
    dtype: str = "f32"
    accum: str = "f64"
    source: str = "samples"
    update_every: int = 1
    dt: float = 1.0
    kvec: np.ndarray | None = None
    n_atoms: int = 0
    box: float = 0.0
    pair: bool = False  # correlate (x, y) per channel: samples [2][n_channels]
    species: np.ndarray | None = None  # momentum: species id of every atom
    masses: np.ndarray | None = None   # momentum: mass of each species
    _kbuf: object = field(default=None, repr=False)
    _sbuf: object = field(default=None, repr=False)
    _mbuf: object = field(default=None, repr=False)

    def to_c(self) -> _GroupDesc:
        d = _GroupDesc()
        d.n_channels, d.levels, d.points, d.m = self.n_channels, self.levels, self.points, self.m
        d.dtype, d.accum, d.source = DTYPES[self.dtype], ACCUMS[self.accum], SOURCES[self.source]
        d.update_every, d.dt = self.update_every, self.dt
        d.pair = 1 if self.pair else 0
        if self.kvec is not None:
            self._kbuf = np.ascontiguousarray(self.kvec, dtype=np.int32)
            d.kvec = self._kbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_atoms, d.box = int(self.n_atoms), float(self.box)
        if self.species is not None:
            self._sbuf = np.ascontiguousarray(self.species, dtype=np.int32)
            d.species = self._sbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if self.masses is not None:
            self._mbuf = np.ascontiguousarray(self.masses, dtype=np.float64)
            d.masses = self._mbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.n_species = len(self._mbuf)
        return d

    @property
    def max_out(self) -> int:
        return self.points + (self.levels - 1) * (self.points - self.points // self.m)


def autotune(groups, device: int = 0, stream=None, graph=False, per_group=False, direct=False,
             cache_path: str | None = None, max_trial_channels: int = 0, force: bool = False,
             rhok_valu: bool = False):
    """Run (or read from the cache) the launch-shape autotuner; returns the tuning dict."""
    L = lib()
    groups = list(groups)
    descs = (_GroupDesc * len(groups))(*[g.to_c() for g in groups])
    st = stream if stream is not None else torch.cuda.current_stream(device)
    flags = (FLAG_GRAPH if graph else 0) | (FLAG_PER_GROUP if per_group else 0) | \
        (FLAG_DIRECT if direct else 0) | (FLAG_RHOK_VALU if rhok_valu else 0)
    t = Tuning()
    rc = L.corr_autotune(descs, len(groups), int(device), ctypes.c_void_p(st.cuda_stream), flags,
                         cache_path.encode() if cache_path else None, int(max_trial_channels),
                         int(force), ctypes.byref(t))
    if rc != CORR_OK:
        raise CorrError(rc, "autotune failed")
    return t.as_dict()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


class Correlator:
    """A context of channel groups on one GPU (wraps corr_create ... corr_destroy)."""

    def __init__(self, groups, device: int = 0, stream: torch.cuda.Stream | None = None,
                 graph: bool = False, per_group: bool = False, tuning: dict | None = None,
                 timing: bool = False, direct: bool = False, rhok_valu: bool = False):
        L = lib()
        self.groups = list(groups)
        descs = (_GroupDesc * len(self.groups))(*[g.to_c() for g in self.groups])
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        flags = (FLAG_GRAPH if graph else 0) | (FLAG_PER_GROUP if per_group else 0) | \
            (FLAG_TIMING if timing else 0) | (FLAG_DIRECT if direct else 0) | \
            (FLAG_RHOK_VALU if rhok_valu else 0)
        tn = Tuning(**tuning) if tuning else None
        h = ctypes.c_void_p()
        rc = L.corr_create(descs, len(self.groups), self.device,
                           ctypes.c_void_p(self.stream.cuda_stream), flags,
                           ctypes.byref(tn) if tn is not None else None, ctypes.byref(h))
        if rc != CORR_OK:
            raise CorrError(rc, L.corr_last_error(None).decode())
        self._h = h
        self._bound = {}

    # -------------------------------------------------------------- helpers
    def _check(self, rc):
        if rc != CORR_OK:
            raise CorrError(rc, lib().corr_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().corr_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ API
    def input_buffer(self, g: int):
        p = ctypes.c_void_p()
        n = ctypes.c_size_t()
        self._check(lib().corr_input_buffer(self._h, g, ctypes.byref(p), ctypes.byref(n)))
        return int(p.value or 0), int(n.value)

    def bind_input(self, g: int, tensor: torch.Tensor | None):
        """Make `tensor` (kept alive here) the buffer group g reads on NULL pushes."""
        if tensor is None:
            self._check(lib().corr_bind_input(self._h, g, None, 0))
            self._bound.pop(g, None)
            return
        assert tensor.is_cuda and tensor.is_contiguous()
        nbytes = tensor.numel() * tensor.element_size()
        self._check(lib().corr_bind_input(self._h, g, ctypes.c_void_p(tensor.data_ptr()), nbytes))
        self._bound[g] = tensor

    def push(self, samples=None):
        """samples: None (input buffers) or a list with one tensor (or None) per group."""
        if samples is None:
            self._check(lib().corr_push(self._h, None))
            return
        arr = (ctypes.c_void_p * len(self.groups))(*[_ptr(s) for s in samples])
        self._check(lib().corr_push(self._h, arr))

    def push_steps(self, histories):
        """Replay n consecutive steps: histories = one tensor per group with the
        steps along dim 0 ([n][...] with each row one push's input)."""
        hs = list(histories)
        n = int(hs[0].shape[0])
        for h in hs:
            assert h.is_cuda and h.shape[0] == n
        arr = (ctypes.c_void_p * len(hs))(*[h.data_ptr() for h in hs])
        st = (ctypes.c_int64 * len(hs))(*[h.stride(0) * h.element_size() for h in hs])
        self._check(lib().corr_push_steps(self._h, n, arr, st))

    def sync(self):
        self._check(lib().corr_sync(self._h))

    def n_pushes(self, g: int = 0) -> int:
        n = ctypes.c_int64()
        m = ctypes.c_int32()
        self._check(lib().corr_query(self._h, g, ctypes.byref(n), ctypes.byref(m)))
        return int(n.value)

    def state_bytes(self, g: int) -> int:
        n = ctypes.c_int64()
        self._check(lib().corr_state_bytes(self._h, g, ctypes.byref(n)))
        return int(n.value)

    def kernel_time(self, which: int = 0, reset: bool = False):
        """(summed milliseconds, count): which=0 the update kernels of each push
        (incl. flushes), which=1 the flush fold kernels only, which=2 the
        k-density producer launches (HIP events, on the timed pushes); which=3
        the flush fold kernels of every push, from the kernels' own device
        stamps."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().corr_kernel_time(self._h, int(which), ctypes.byref(ms), ctypes.byref(n),
                                           int(reset)))
        return float(ms.value), int(n.value)

    def set_timing_stride(self, stride: int) -> None:
        """Record the timing events on one push in `stride` only."""
        self._check(lib().corr_set_timing_stride(self._h, int(stride)))

    def group_form(self, g: int):
        """(form, block): 0 per-step, 1 block-deferred (block = T pushes), 2
        block-deferred window (block 64), 3 per-step window."""
        f = ctypes.c_int32()
        b = ctypes.c_int32()
        self._check(lib().corr_group_form(self._h, g, ctypes.byref(f), ctypes.byref(b)))
        return int(f.value), int(b.value)

    def tuning(self) -> dict:
        t = Tuning()
        self._check(lib().corr_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def finalize(self, g: int, ch=None, t_cut: float = 0.0, gk_kind: int = 0, volume=0.0,
                 kB=0.0, temperature=0.0, slice_=None, noalloc: bool = False):
        """Readout (Algorithm 2) of group g.  Returns a dict with t, c, count,
        gk_running, gk_at_cut and, if slice_=(b, e) is given, c_per_channel.
        noalloc=True calls corr_finalize_noalloc (no device allocation)."""
        gd = self.groups[g]
        nmax = gd.max_out
        cplx = gd.dtype in ("cf32", "cf64")
        o = _ReadoutOpts()
        if ch is not None:
            o.ch_begin, o.ch_end = int(ch[0]), int(ch[1])
        o.t_cut, o.gk_kind = float(t_cut), int(gk_kind)
        o.volume, o.kB, o.temperature = float(volume), float(kB), float(temperature)
        t = np.zeros(nmax)
        c = np.zeros((nmax, 2) if cplx else nmax)
        cnt = np.zeros(nmax, dtype=np.int64)
        run = np.zeros(nmax)
        at = ctypes.c_double()
        n_out = ctypes.c_int32()
        per = None
        if slice_ is not None:
            o.slice_begin, o.slice_end = int(slice_[0]), int(slice_[1])
            ns = o.slice_end - o.slice_begin
            per = np.zeros((ns, nmax, 2) if cplx else (ns, nmax))
        P = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        fn = lib().corr_finalize_noalloc if noalloc else lib().corr_finalize
        self._check(fn(self._h, g, ctypes.byref(o), ctypes.byref(n_out), P(t), P(c), P(cnt),
                       P(run), ctypes.byref(at), P(per)))
        n = int(n_out.value)
        res = {"t": t[:n], "count": cnt[:n], "gk_running": run[:n], "gk_at_cut": float(at.value)}
        if cplx:
            res["c"] = c[:n, 0] + 1j * c[:n, 1]
        else:
            res["c"] = c[:n]
        if per is not None:
            # the library writes [slice][n_out] (complex: [slice][n_out][2]) contiguously
            ns = per.shape[0]
            if cplx:
                flat = per.reshape(-1)[: ns * n * 2].reshape(ns, n, 2)
                res["c_per_channel"] = flat[:, :, 0] + 1j * flat[:, :, 1]
            else:
                res["c_per_channel"] = per.reshape(-1)[: ns * n].reshape(ns, n)
        return res
