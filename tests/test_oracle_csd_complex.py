"""Pins of the complex CSD oracle (``oracle.csd_complex``), CPU.

Each pin is fixed by something other than the oracle itself:
* inputs built from known unitary factors and angles (the decomposition is
  then known: angles to 10 n u, reconstruction and unitarity to rounding);
* brute force on tiny n: the angles are arccos of the singular values of A1
  (arcsin of those of A2 above pi/4);
* LAPACK's complete CSD (scipy.linalg.cossin) of a Haar unitary 2n x 2n
  matrix, a different algorithm;
* a real input gives the real oracle's angles;
* the swap symmetry theta(A2, A1) = pi/2 - theta(A1, A2) reversed (Remark (i),
  read as pi/2 - theta);
* a rank-deficient partial isometry (Theorem 2.1) keeps the rank and the
  angles of its nonzero part (Algorithm 3).
A transpose in place of a conjugate transpose anywhere fails the first pin.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import csd as O
from oracle import csd_complex as OC

U = 2.0 ** -53


def _unitary(n, rng):
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    return Q * (d / np.abs(d))


def _pair(n, seed, zero=0):
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(0.0, np.pi / 2, n))
    c, s = np.cos(th), np.sin(th)
    z = rng.choice(n, size=zero, replace=False) if zero else np.array([], dtype=int)
    c[z] = 0.0
    s[z] = 0.0
    U1, U2, V1 = (_unitary(n, rng) for _ in range(3))
    return (U1 * c) @ V1.conj().T, (U2 * s) @ V1.conj().T, np.sort(np.delete(th, z))


def _check(A1, A2, o, tol=1e-13):
    r = o["rank"]
    U1, U2, V1, th = o["U1"], o["U2"], o["V1"], o["theta"]
    assert np.all(np.diff(th) >= 0)
    R1 = (U1 * np.cos(th)) @ V1.conj().T - A1
    R2 = (U2 * np.sin(th)) @ V1.conj().T - A2
    A = np.vstack([A1, A2])
    assert np.linalg.norm(np.vstack([R1, R2]), 2) <= tol * max(1.0, np.linalg.norm(A, 2))
    for X in (U1, U2, V1):
        assert np.linalg.norm(X.conj().T @ X - np.eye(r), 2) <= tol


@pytest.mark.parametrize("n,seed", [(1, 1), (5, 2), (40, 3), (130, 4)])
def test_known_factors(n, seed):
    A1, A2, th = _pair(n, seed)
    assert np.abs(A1.imag).max() > 0.1  # really complex
    o = OC.csd(A1, A2)
    assert o["rank"] == n
    assert np.max(np.abs(o["theta"] - th)) <= 10 * n * U
    _check(A1, A2, o)


@pytest.mark.parametrize("n,seed", [(2, 5), (3, 6), (6, 7)])
def test_brute_force_singular_values(n, seed):
    A1, A2, _ = _pair(n, seed)
    o = OC.csd(A1, A2)
    c = np.sort(np.linalg.svd(A1, compute_uv=False))[::-1]   # cos theta, descending
    s = np.sort(np.linalg.svd(A2, compute_uv=False))          # sin theta, ascending
    th_c, th_s = np.arccos(np.clip(c, -1, 1)), np.arcsin(np.clip(s, -1, 1))
    ref = np.where(th_c < np.pi / 4, th_c, th_s)
    assert np.max(np.abs(o["theta"] - ref)) <= 1e-13


@pytest.mark.parametrize("n,seed", [(8, 8), (64, 9)])
def test_lapack_complete_csd(n, seed):
    Q = _unitary(2 * n, np.random.default_rng(seed))
    u, cs, vdh = scipy.linalg.cossin(Q, p=n, q=n)
    # the upper-left block of the middle factor is diag(cos theta)
    c = np.clip(np.real(np.diag(cs[:n, :n])), -1, 1)
    ref = np.sort(np.arccos(c))
    o = OC.csd(Q[:n, :n], Q[n:, :n])
    assert np.max(np.abs(o["theta"] - ref)) <= 10 * n * U


def test_real_input_matches_real_oracle():
    rng = np.random.default_rng(10)
    G = rng.standard_normal((60, 30))
    Qr, _ = np.linalg.qr(G)
    A1, A2 = Qr[:30], Qr[30:]
    o = OC.csd(A1.astype(np.complex128), A2.astype(np.complex128))
    r = O.csd(A1, A2)
    assert np.max(np.abs(o["theta"] - r["theta"])) <= 10 * 30 * U


def test_swap_symmetry():
    A1, A2, _ = _pair(25, 11)
    a = OC.csd(A1, A2)["theta"]
    b = OC.csd(A2, A1)["theta"]
    assert np.max(np.abs(b - (np.pi / 2 - a[::-1]))) <= 10 * 25 * U


@pytest.mark.parametrize("n,k,seed", [(20, 5, 12), (64, 16, 13)])
def test_rank_deficient(n, k, seed):
    A1, A2, th = _pair(n, seed, zero=k)
    o = OC.csd(A1, A2)
    assert o["rank"] == n - k
    assert np.max(np.abs(o["theta"] - th)) <= 10 * n * U
    _check(A1, A2, o)
