"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Stand-ins for the molecular-dynamics observables of the paper's workloads:
independent Ornstein-Uhlenbeck (OU) series for atom-velocity components and
for the global stress / heat-flux components, and atom positions (uniform in
a cubic box plus a small OU displacement) for the k-space density.  The paper
correlates velocities, stress and heat flux produced by DL_POLY; no MD data is
used here.

This module holds none of the correlator's arithmetic.  ``synth_cpu.c`` and
``synth_gpu.hip`` implement one counter-based generator (SplitMix64 output
function on a counter, Irwin-Hall innovations, explicit-fma OU recursion) and
are bit-identical, so any channel of any step can be regenerated on the CPU.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
CPU_LIB = os.path.join(_HERE, "libsynth_cpu.so")
GPU_LIB = os.path.join(_HERE, "libsynth_gpu.so")
GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-mcode-object-version=5", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=off"]


def build_cpu() -> str:
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-Wall", "-o", CPU_LIB, os.path.join(_HERE, "synth_cpu.c"), "-lm"])
    return CPU_LIB


def build_gpu() -> str:
    subprocess.check_call(["/opt/rocm/bin/hipcc"] + HIP_FLAGS +
                          ["-o", GPU_LIB, os.path.join(_HERE, "synth_gpu.hip")])
    return GPU_LIB


def build() -> None:
    build_cpu()
    build_gpu()


_cpu = None
_gpu = None


def cpu():
    global _cpu
    if _cpu is None:
        if not os.path.exists(CPU_LIB):
            build_cpu()
        L = ctypes.CDLL(CPU_LIB)
        u64, i64, i32, f32, f64, vp = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_float, ctypes.c_double, ctypes.c_void_p)
        L.synth_key.restype = u64
        L.synth_key.argtypes = [u64, u64]
        L.synth_bits.restype = u64
        L.synth_bits.argtypes = [u64, u64, u64, u64]
        L.synth_ou_f32.argtypes = [u64, i64, vp, i32, vp, vp, f32, i64, i64, vp, vp]
        L.synth_ou_f64.argtypes = [u64, i64, vp, i32, vp, vp, f64, i64, i64, vp, vp]
        L.synth_positions.argtypes = [u64, i64, vp, f32, f32, f32, i64, i64, vp, vp]
        L.synth_uniform_f64.argtypes = [u64, i64, u64, vp]
        _cpu = L
    return _cpu


def gpu():
    """The GPU generator library (import torch before calling: one HIP runtime)."""
    global _gpu
    if _gpu is None:
        if not os.path.exists(GPU_LIB):
            raise RuntimeError(f"{GPU_LIB} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(GPU_LIB)
        u64, i64, i32, f32, f64, vp = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_float, ctypes.c_double, ctypes.c_void_p)
        L.synth_gpu_ou_f32.argtypes = [u64, i64, i32, vp, vp, f32, i64, i64, vp, vp, i64, vp]
        L.synth_gpu_ou_f64.argtypes = [u64, i64, i32, vp, vp, f64, i64, i64, vp, vp, i64, vp]
        L.synth_gpu_positions.argtypes = [u64, i64, vp, f32, f32, f32, i64, i64, vp, vp, i64, vp]
        for f in (L.synth_gpu_ou_f32, L.synth_gpu_ou_f64, L.synth_gpu_positions):
            f.restype = i32
        _gpu = L
    return _gpu


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def key(seed: int, stream: int) -> int:
    return int(cpu().synth_key(seed & MASK64, stream & MASK64))


def uniform(seed: int, stream: int, n: int, word: int = 0) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    cpu().synth_uniform_f64(key(seed, stream), int(n), int(word), _p(out))
    return out


# ---------------------------------------------------------------- OU tables
def ou_coeffs(tau, sigma=1.0, dtype=np.float32):
    """Per-entry OU coefficients a = round(exp(-1/tau)), b = round(sigma sqrt(1 - a^2)),
    computed in double on the host, rounded to `dtype`."""
    tau = np.asarray(tau, dtype=np.float64)
    a = np.exp(-1.0 / tau).astype(dtype)
    b = (float(sigma) * np.sqrt(1.0 - a.astype(np.float64) ** 2)).astype(dtype)
    return np.atleast_1d(a), np.atleast_1d(b)


def ou_tau_table(seed: int, stream: int, n_atoms: int, tau_lo: float, tau_hi: float):
    """tau per atom, uniform in [tau_lo, tau_hi] (all components of an atom share it)."""
    if tau_lo == tau_hi:
        return np.full(int(n_atoms), float(tau_lo))
    u = uniform(seed, stream + 0x7A0, n_atoms)
    return tau_lo + (tau_hi - tau_lo) * u


def stationary_variance(a, b):
    """Exact stationary variance of x' = a x + b xi (unit-variance xi) for the
    rounded coefficients: b^2 / (1 - a^2)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return b * b / (1.0 - a * a)


class OUSpec:
    """A block of n channels of OU series; channel c uses coefficients of entry c // comps."""

    def __init__(self, seed, stream, n, comps, a, b, sigma, dtype):
        self.seed, self.stream, self.n, self.comps = int(seed), int(stream), int(n), int(comps)
        self.dtype = np.dtype(dtype)
        self.a = np.ascontiguousarray(a, dtype=self.dtype)
        self.b = np.ascontiguousarray(b, dtype=self.dtype)
        self.sigma = float(sigma)
        self.key = key(self.seed, self.stream)
        assert self.a.shape[0] * self.comps >= self.n

    @staticmethod
    def make(seed, stream, n, *, comps=1, tau=50.0, tau_hi=None, sigma=1.0, dtype=np.float32):
        n_ent = -(-int(n) // int(comps))
        if tau_hi is None:
            taus = np.full(n_ent, float(tau))
        else:
            taus = ou_tau_table(seed, stream, n_ent, float(tau), float(tau_hi))
        a, b = ou_coeffs(taus, sigma, dtype)
        return OUSpec(seed, stream, n, comps, a, b, sigma, dtype)

    def series(self, t_begin: int, n_steps: int, state=None, channels=None):
        """CPU twin: returns (out[n_steps][n_sel], new_state)."""
        chan = None if channels is None else np.ascontiguousarray(channels, dtype=np.int64)
        n_sel = self.n if chan is None else chan.shape[0]
        st = np.zeros(n_sel, dtype=self.dtype) if state is None else np.array(state,
                                                                              dtype=self.dtype)
        out = np.empty((int(n_steps), n_sel), dtype=self.dtype)
        if self.dtype == np.float32:
            cpu().synth_ou_f32(self.key, n_sel, _p(chan), self.comps, _p(self.a), _p(self.b),
                               self.sigma, int(t_begin), int(n_steps), _p(st), _p(out))
        else:
            cpu().synth_ou_f64(self.key, n_sel, _p(chan), self.comps, _p(self.a), _p(self.b),
                               self.sigma, int(t_begin), int(n_steps), _p(st), _p(out))
        return out, st


class GpuOU:
    """Device-side generator for an OUSpec (torch tensors for memory and stream)."""

    def __init__(self, spec: OUSpec, device="cuda"):
        import torch
        self.spec = spec
        tdt = torch.float32 if spec.dtype == np.float32 else torch.float64
        self.a = torch.from_numpy(spec.a).to(device)
        self.b = torch.from_numpy(spec.b).to(device)
        self.state = torch.zeros(spec.n, dtype=tdt, device=device)
        self.t = 0
        self.tdt = tdt

    def fill(self, out, n_steps: int, stream=None):
        """Write the next n_steps steps into out[n_steps][>=n] (row stride out.stride(0))."""
        import torch
        s = self.spec
        st = torch.cuda.current_stream() if stream is None else stream
        assert out.dtype == self.tdt and out.is_contiguous() or out.stride(1) == 1
        assert out.shape[0] >= n_steps and out.shape[1] >= s.n
        fn = gpu().synth_gpu_ou_f32 if s.dtype == np.float32 else gpu().synth_gpu_ou_f64
        rc = fn(s.key, s.n, s.comps, ctypes.c_void_p(self.a.data_ptr()),
                ctypes.c_void_p(self.b.data_ptr()), s.sigma, self.t, int(n_steps),
                ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                int(out.stride(0)), ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"synth GPU launch failed: hip error {rc}")
        self.t += int(n_steps)


# -------------------------------------------------------------- positions
class PositionSpec:
    """N atoms uniform in [0, L)^3 plus an OU displacement per component."""

    def __init__(self, seed, stream, n_atoms, box=100.0, sigma_d=0.1, tau_d=50.0):
        self.seed, self.stream, self.n_atoms, self.box = int(seed), int(stream), int(n_atoms), \
            float(box)
        u = np.stack([uniform(seed, stream + 0x500 + q, n_atoms) for q in range(3)])
        self.r0 = np.ascontiguousarray((box * u).astype(np.float32))  # [3][N]
        a, b = ou_coeffs(np.array([tau_d]), sigma_d, np.float32)
        self.a_d, self.b_d, self.sigma_d = float(a[0]), float(b[0]), float(np.float32(sigma_d))
        self.key = key(seed, stream)

    def series(self, t_begin, n_steps, d_state=None):
        n3 = 3 * self.n_atoms
        st = np.zeros(n3, dtype=np.float32) if d_state is None else np.array(d_state,
                                                                           dtype=np.float32)
        out = np.empty((int(n_steps), 3, self.n_atoms), dtype=np.float32)
        cpu().synth_positions(self.key, self.n_atoms, _p(self.r0), self.a_d, self.b_d,
                              self.sigma_d, int(t_begin), int(n_steps), _p(st), _p(out))
        return out, st


class GpuPositions:
    def __init__(self, spec: PositionSpec, device="cuda"):
        import torch
        self.spec = spec
        self.r0 = torch.from_numpy(spec.r0).to(device)
        self.d = torch.zeros(3 * spec.n_atoms, dtype=torch.float32, device=device)
        self.t = 0

    def fill(self, out, n_steps: int, stream=None):
        import torch
        s = self.spec
        st = torch.cuda.current_stream() if stream is None else stream
        rc = gpu().synth_gpu_positions(s.key, s.n_atoms, ctypes.c_void_p(self.r0.data_ptr()),
                                       s.a_d, s.b_d, s.sigma_d, self.t, int(n_steps),
                                       ctypes.c_void_p(self.d.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), int(out.stride(0)),
                                       ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"synth GPU launch failed: hip error {rc}")
        self.t += int(n_steps)


# ---------------------------------------------------------------- k-vectors
def kvectors(n_k: int = 2048, nmax: int = 12) -> np.ndarray:
    """Integer lattice vectors n (k = 2 pi n / L) with 0 < |n| <= nmax in the half
    space whose first non-zero component is positive, sorted by (|n|^2, n
    lexicographically); the first n_k of them.  Half of each +-n pair suffices
    because n(-k) is the conjugate of n(k) for real positions."""
    pts = []
    r = range(-nmax, nmax + 1)
    for x in r:
        for y in r:
            for z in r:
                n2 = x * x + y * y + z * z
                if n2 == 0 or n2 > nmax * nmax:
                    continue
                first = x if x != 0 else (y if y != 0 else z)
                if first > 0:
                    pts.append((n2, x, y, z))
    pts.sort()
    if n_k > len(pts):
        raise ValueError(f"only {len(pts)} half-space lattice vectors with |n| <= {nmax}")
    return np.array([p[1:] for p in pts[:n_k]], dtype=np.int32)
