"""Shared helpers of the GPU parity tests (the HIP library vs the CPU oracle)."""
from __future__ import annotations

import numpy as np

import oracle
import synth

# Gate tolerances on max |C_gpu - C_oracle| / |C_oracle(0)| (per group mean and
# per sampled channel), by (sample dtype, accumulator).  FP64 accumulators:
# 1e-6; compensated FP32: 1e-5; all-double paths: rounding-order level.
TOL = {
    ("f64", "f64"): 1e-12,
    ("cf64", "f64"): 1e-12,
    ("f32", "f64"): 1e-6,
    ("cf32", "f64"): 1e-6,
    ("f32", "kahan"): 1e-5,
    ("cf32", "kahan"): 1e-5,
    ("f32", "f32"): 1e-3,
    ("cf32", "f32"): 1e-3,
}

NP_DTYPE = {"f32": np.float32, "f64": np.float64, "cf32": np.complex64, "cf64": np.complex128}


def say(msg: str) -> None:
    print(msg, flush=True)


def ou_inputs(seed, stream, n, S, dtype, tau=20.0, tau_hi=200.0, sigma=1.0):
    """[S][n] samples of the requested dtype (complex: two independent OU series)."""
    real = np.float32 if dtype in ("f32", "cf32") else np.float64
    spec = synth.OUSpec.make(seed, stream, n, comps=1, tau=tau, tau_hi=tau_hi, sigma=sigma,
                             dtype=real)
    x, _ = spec.series(0, S)
    if dtype in ("cf32", "cf64"):
        spec2 = synth.OUSpec.make(seed, stream + 1000, n, comps=1, tau=tau, tau_hi=tau_hi,
                                  sigma=sigma, dtype=real)
        y, _ = spec2.series(0, S)
        out = np.empty((S, n), dtype=NP_DTYPE[dtype])
        out.real = x
        out.imag = y
        return out
    return x


def oracle_run(x, levels, points, m):
    """Run the FP64 oracle on [S][n] samples."""
    cplx = np.iscomplexobj(x)
    o = oracle.OracleCorrelator(x.shape[1], levels, points, m, complex_=cplx)
    for row in x:
        o.push(row.astype(np.complex128) if cplx else row.astype(np.float64))
    return o


def gate(res, o, tol, scale=1.0, slice_=None, label=""):
    """Compare a finalize() result with the oracle: times and counts exact,
    values within tol relative to |C(0)|; returns the measured error."""
    t, c, n = o.readout()
    assert np.array_equal(res["t"], t), f"{label}: lag times differ"
    assert np.array_equal(res["count"], n), f"{label}: counts differ"
    if len(t) == 0:
        return 0.0
    ref = c * scale
    c0 = abs(ref[0]) if abs(ref[0]) > 0 else np.max(np.abs(ref))
    err = float(np.max(np.abs(res["c"] - ref)) / c0)
    assert err <= tol, f"{label}: group max |dC|/|C(0)| = {err:.3e} > {tol:.1e}"
    if slice_ is not None:
        b, e = slice_
        for i, ch in enumerate(range(b, e)):
            _, cc, _ = o.readout(ch, ch + 1)
            refc = cc * scale
            c0c = abs(refc[0]) if abs(refc[0]) > 0 else max(np.max(np.abs(refc)), 1e-300)
            errc = float(np.max(np.abs(res["c_per_channel"][i] - refc)) / c0c)
            assert errc <= tol, f"{label}: channel {ch} max |dC|/|C(0)| = {errc:.3e} > {tol:.1e}"
            err = max(err, errc)
    return err
