"""Pins of the oracle's longitudinal / transverse currents (Section "Currents",
Eqs. long-current and trans-current; readings R19, R20 of oracle/corr_oracle.c)
against facts the definition fixes, independent of the function's own formula:
a one-point cluster, the reduction to the k-space density (a separate oracle
function) when every velocity equals khat, the length of the current vector,
linearity in the velocities, inversion symmetry and the basis itself."""
import numpy as np
import pytest

import oracle


def _rand(seed, n, box):
    rng = np.random.default_rng(seed)
    pos = (rng.random((3, n)) * box).astype(np.float32)
    vel = rng.standard_normal((3, n)).astype(np.float32)
    return pos, vel


def test_one_point_cluster_k_along_axes():
    """All N atoms at r0 with velocity v: J = N v exp(i k.r0).  For k along z
    the components are (z, x, y) -- the paper's C_L from the z component and
    C_T from x and y; for k along x they are (x, y, z)."""
    N, box = 7, 10.0
    r0 = np.array([1.25, -2.5, 3.75], dtype=np.float32)
    v = np.array([0.5, -1.5, 2.0], dtype=np.float32)
    pos = np.repeat(r0[:, None], N, axis=1)
    vel = np.repeat(v[:, None], N, axis=1)
    kv = np.array([[0, 0, 3], [2, 0, 0], [0, -1, 0]], dtype=np.int32)
    out = oracle.currents(pos, vel, kv, box)
    vx, vy, vz = (float(c) for c in v)
    # k along z: khat = z, a = x, e1 = x, e2 = z cross x = y
    # k along x: khat = x, a = y, e1 = y, e2 = x cross y = z
    # k along -y: khat = -y, a = x, e1 = x, e2 = (-y) cross x = z
    comps = [(vz, vx, vy), (vx, vy, vz), (-vy, vx, vz)]
    for q in range(3):
        ph = np.exp(1j * 2 * np.pi * (kv[q].astype(np.float64) @ r0.astype(np.float64)) / box)
        np.testing.assert_allclose(out[q], N * ph * np.array(comps[q]), rtol=1e-12, atol=1e-12)


def test_velocity_along_khat_gives_density_and_no_transverse_part():
    """v_j = khat for every atom: khat . J = n(k) (the oracle's separate
    k-density sum) and both transverse components vanish."""
    N, box = 500, 20.0
    pos, _ = _rand(1, N, box)
    kv = np.array([[1, 2, -3], [0, 4, 1], [5, 0, 0], [2, -2, 1]], dtype=np.int32)
    for q in range(len(kv)):
        khat = kv[q] / np.linalg.norm(kv[q])
        vel = np.repeat(khat.astype(np.float32)[:, None], N, axis=1)
        out = oracle.currents(pos, vel, kv[q:q + 1], box)[0]
        # velocities were rounded to float: project the rounded vector
        vr = vel[:, 0].astype(np.float64)
        n_k = oracle.rhok(pos, kv[q:q + 1], box)[0]
        basis = oracle.current_basis(kv[q])
        np.testing.assert_allclose(out, (basis @ vr) * n_k, rtol=1e-10, atol=1e-9 * N)
        assert abs(out[1]) < 1e-6 * N and abs(out[2]) < 1e-6 * N


def test_constant_velocity_length():
    """A common velocity v: |J|^2 = |v|^2 |n(k)|^2, and the basis is
    orthonormal, so the squared components add up to it."""
    N, box = 300, 15.0
    pos, _ = _rand(2, N, box)
    v = np.array([0.3, -1.1, 0.7], dtype=np.float32)
    vel = np.repeat(v[:, None], N, axis=1)
    kv = np.array([[1, 1, 1], [3, -2, 0], [0, 0, 5], [4, 1, -2]], dtype=np.int32)
    out = oracle.currents(pos, vel, kv, box)
    n_k = oracle.rhok(pos, kv, box)
    lhs = np.sum(np.abs(out) ** 2, axis=1)
    rhs = float(v.astype(np.float64) @ v.astype(np.float64)) * np.abs(n_k) ** 2
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)


def test_linear_in_velocity_and_inversion():
    N, box = 200, 12.0
    pos, v1 = _rand(3, N, box)
    _, v2 = _rand(4, N, box)
    kv = np.array([[1, 0, 2], [-2, 3, 1], [0, 1, 0]], dtype=np.int32)
    a = oracle.currents(pos, v1, kv, box)
    b = oracle.currents(pos, v2, kv, box)
    ab = oracle.currents(pos, (v1.astype(np.float64) + v2).astype(np.float32), kv, box)
    # v1 + v2 rounds to float; compare at that rounding
    assert np.max(np.abs(ab - (a + b))) < 1e-5 * np.max(np.abs(a) + np.abs(b))
    # r -> -r, v -> -v: J -> -conj(J) (same basis)
    inv = oracle.currents(-pos, -v1, kv, box)
    np.testing.assert_allclose(inv, -np.conj(a), rtol=1e-12, atol=1e-10)


def test_basis_properties():
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = rng.integers(-12, 13, 3)
        if not n.any():
            continue
        B = oracle.current_basis(n)
        np.testing.assert_allclose(B @ B.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(B) > 0
        np.testing.assert_allclose(B[0], n / np.linalg.norm(n), atol=1e-15)


def test_zero_vector_rejected():
    pos, vel = _rand(6, 4, 5.0)
    with pytest.raises(ValueError):
        oracle.currents(pos, vel, np.zeros((1, 3), np.int32), 5.0)
