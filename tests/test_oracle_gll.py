"""Pins of the GLL basis: closed forms, exactness, summation by parts."""
import numpy as np
import pytest

from oracle.gll import RefElement, diff_matrix, gll


def test_closed_forms():
    x, w = gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = gll(3)
    s = 1 / np.sqrt(5)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = gll(4)
    s = np.sqrt(3 / 7)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1], atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_quadrature_exact_to_2p_minus_1(p):
    x, w = gll(p)
    for k in range(2 * p):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    # and not exact at degree 2p (GLL has degree of exactness 2p-1)
    k = 2 * p
    assert abs(np.dot(w, x ** k) - 2 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [2, 3, 4])
def test_derivative_exact_and_sbp(p):
    x, w = gll(p)
    D = diff_matrix(x)
    for k in range(p + 1):
        dk = k * x ** (k - 1) if k > 0 else 0 * x
        assert np.max(np.abs(D @ x ** k - dk)) < 1e-12
    B = np.zeros((p + 1, p + 1))
    B[0, 0], B[-1, -1] = -1, 1
    Wm = np.diag(w)
    assert np.max(np.abs(Wm @ D + D.T @ Wm - B)) < 1e-14


def test_tensor_derivatives():
    ref = RefElement(3, 3)
    x = ref.x1
    X = [x[ref.idx[a]] for a in range(3)]
    f = X[0] ** 2 * X[1] ** 3 * X[2]
    grads = [2 * X[0] * X[1] ** 3 * X[2], 3 * X[0] ** 2 * X[1] ** 2 * X[2], X[0] ** 2 * X[1] ** 3]
    for a in range(3):
        assert np.max(np.abs(ref.Dr[a] @ f - grads[a])) < 1e-12
    assert abs(ref.W.sum() - 8.0) < 1e-14
    assert len(ref.faces) == 6 and all(len(fc[2]) == 16 for fc in ref.faces)
