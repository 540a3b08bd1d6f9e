"""Pins of the oracle's element: shape functions, quadrature, element stiffness.

Section 2.1 (20-node serendipity element, full integration).  The pins are properties the
mathematics fixes, not re-typed formulas: partition of unity, Kronecker property, exact
reproduction of complete quadratics, exactness of the 3x3x3 rule, and the rank of the
fully integrated element stiffness (6 rigid-body modes only).
"""
import itertools

import numpy as np
import pytest

from oracle import element as E
from oracle import material as M
from oracle.mesh import reference_nodes

rng = np.random.default_rng(0)


def test_shape_partition_of_unity_and_kronecker():
    p = rng.uniform(-1, 1, (50, 3))
    N, dN = E.shape(p)
    assert np.allclose(N.sum(1), 1.0, atol=1e-14)
    assert np.allclose(dN.sum(1), 0.0, atol=1e-13)
    Nn, _ = E.shape(reference_nodes())
    assert np.allclose(Nn, np.eye(20), atol=1e-15)


def test_shape_reproduces_complete_quadratics():
    ref = reference_nodes()
    p = rng.uniform(-1, 1, (40, 3))
    N, dN = E.shape(p)
    monos = [(a, b, c) for a in range(3) for b in range(3) for c in range(3) if a + b + c <= 2]
    for (a, b, c) in monos:
        f = lambda q: q[:, 0] ** a * q[:, 1] ** b * q[:, 2] ** c
        assert np.allclose(N @ f(ref), f(p), atol=1e-13)
        # gradient of the interpolant equals the gradient of the monomial
        g = np.stack([a * p[:, 0] ** max(a - 1, 0) * p[:, 1] ** b * p[:, 2] ** c,
                      b * p[:, 0] ** a * p[:, 1] ** max(b - 1, 0) * p[:, 2] ** c,
                      c * p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** max(c - 1, 0)], 1)
        assert np.allclose(np.einsum("qa,a->q", dN[:, :, 0], f(ref)), g[:, 0], atol=1e-12)
        assert np.allclose(np.einsum("qa,a->q", dN[:, :, 2], f(ref)), g[:, 2], atol=1e-12)


def test_gauss_rule_exact_to_degree_five_per_axis():
    pts, w = E.gauss_hex(3)
    for a, b, c in itertools.product(range(6), repeat=3):
        exact = np.prod([0.0 if k % 2 else 2.0 / (k + 1) for k in (a, b, c)])
        num = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        assert abs(num - exact) < 1e-14
    # degree 6 is not integrated exactly: the rule is the 3-point one, not a higher one
    assert abs(np.sum(w * pts[:, 0] ** 6) - 4 * 2.0 / 7) > 1e-3


def _distorted_element(affine=False):
    ref = reference_nodes()
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.9, 0.15], [-0.05, 0.1, 0.4]])
    X = ref @ A.T + np.array([0.3, -0.2, 0.1])
    if not affine:
        X = X + 0.04 * rng.standard_normal(X.shape)
    return X, A


def test_volume_of_affine_hex():
    X, A = _distorted_element(affine=True)
    gp = E.gauss_point_data(X[None])
    vol = np.sum(gp["detJ"] * gp["w"])
    assert abs(vol - 8 * abs(np.linalg.det(A))) < 1e-13


def _ply_C():
    from workloads import PLY
    return M.orthotropic_stiffness(**PLY)


def test_element_stiffness_symmetric_psd_rank54_full_integration():
    X, _ = _distorted_element()
    K = E.element_stiffness(X[None], _ply_C()[None], np.array([30.0]))[0]
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    tol = 1e-10 * ev[-1]
    assert ev[0] > -tol
    assert np.sum(np.abs(ev) < tol) == 6
    assert ev[6] > 1e-6 * ev[-1]


def test_reduced_integration_has_spurious_modes():
    """A 2x2x2 rule leaves extra zero-energy modes: this pins 'full' integration."""
    X, _ = _distorted_element()
    K = E.element_stiffness(X[None], _ply_C()[None], np.array([0.0]), nq=2)[0]
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-9 * ev[-1]) > 6


def test_rigid_body_modes_in_element_null_space():
    X, _ = _distorted_element()
    K = E.element_stiffness(X[None], _ply_C()[None], np.array([-45.0]))[0]
    for r in _rbm(X):
        assert np.linalg.norm(K @ r) <= 1e-12 * np.linalg.norm(K) * np.linalg.norm(r)


def _rbm(X):
    out = []
    for c in range(3):
        t = np.zeros_like(X)
        t[:, c] = 1
        out.append(t.ravel())
    for axis in np.eye(3):
        out.append(np.cross(axis, X).ravel())
    return out


def test_face_load_sums_to_traction_times_area():
    X, A = _distorted_element(affine=True)
    t0 = np.array([0.7, -0.2, 1.1])
    f = E.face_load(X[None], 1.0, lambda x, n: np.broadcast_to(t0, x.shape).copy())[0]
    area = 4 * np.linalg.norm(np.cross(A[:, 1], A[:, 2]))
    assert np.allclose(f.reshape(20, 3).sum(0), t0 * area, rtol=1e-13)
    # only the 8 nodes of the xi = +1 face are loaded
    ref = reference_nodes()
    off = ref[:, 0] != 1
    assert np.all(f.reshape(20, 3)[off] == 0)
