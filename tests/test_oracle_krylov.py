"""Pins for the oracle's Lanczos exponential (Sec. II.A.2, TDVP-PS local integrator)."""

import numpy as np
import pytest
import scipy.linalg

from inputs import random_complex
from oracle.krylov import expm_lanczos, exp_tridiag_e1


def _herm(n, seed, scale=1.0):
    A = random_complex((n, n), seed)
    return scale * 0.5 * (A + A.conj().T)


@pytest.mark.parametrize("n,z", [(6, -0.7j), (12, 1.3j), (20, -2.0j), (9, -0.4)])
def test_full_dimension_is_exact(n, z):
    A = _herm(n, n)
    x = random_complex(n, 100 + n)
    y = expm_lanczos(lambda v: A @ v, x, z, kmax=n)
    ref = scipy.linalg.expm(z * A) @ x
    assert np.abs(y - ref).max() < 1e-12 * np.linalg.norm(x)


def test_truncated_space_converges_for_small_norm():
    A = _herm(200, 3, scale=0.05)
    x = random_complex(200, 4)
    y = expm_lanczos(lambda v: A @ v, x, -1j, kmax=20)
    ref = scipy.linalg.expm(-1j * A) @ x
    assert np.abs(y - ref).max() < 1e-12 * np.linalg.norm(x)


def test_breakdown_on_invariant_subspace():
    # x in a 3-dimensional invariant subspace: the space stops growing at k = 3
    lam = np.array([0.3, -1.1, 2.0, 5.0, 7.0])
    Q = np.linalg.qr(random_complex((5, 5), 9))[0]
    A = Q @ np.diag(lam) @ Q.conj().T
    x = Q[:, :3] @ np.array([1.0, 0.5j, -0.2])
    info = {}
    y = expm_lanczos(lambda v: A @ v, x, -0.8j, kmax=5, info=info)
    assert info["k"] == 3
    ref = scipy.linalg.expm(-0.8j * A) @ x
    assert np.abs(y - ref).max() < 1e-13


def test_tolerance_stop_estimate():
    A = _herm(300, 5, scale=0.02)
    x = random_complex(300, 6)
    info = {}
    y = expm_lanczos(lambda v: A @ v, x, -1j, kmax=40, tol=1e-10, info=info)
    ref = scipy.linalg.expm(-1j * A) @ x
    assert info["k"] < 40
    assert np.abs(y - ref).max() < 1e-9 * np.linalg.norm(x)


def test_zero_vector():
    y = expm_lanczos(lambda v: v, np.zeros(4, complex), -1j)
    assert np.all(y == 0)


def test_exp_tridiag_against_expm():
    a = np.array([0.1, -0.4, 0.9, 0.2])
    b = np.array([0.5, 0.3, 0.7])
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    c = exp_tridiag_e1(a, b, -1.7j)
    assert np.abs(c - scipy.linalg.expm(-1.7j * T)[:, 0]).max() < 1e-14


def test_unitarity_preserves_norm():
    A = _herm(64, 8, 0.1)
    x = random_complex(64, 10)
    y = expm_lanczos(lambda v: A @ v, x, -3j, kmax=30)
    assert np.linalg.norm(y) == pytest.approx(np.linalg.norm(x), rel=1e-13)
