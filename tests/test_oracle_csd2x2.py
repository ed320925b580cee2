"""Pins of the complete 2 x 2 CSD oracle (``oracle.csd2x2``, Remark (viii) of Sec. 3), CPU.

* Inputs built from known factors: A = diag(U1, U2) [C -S; S C] diag(V1, V2)^T
  with Haar factors and known angles; the oracle's angles equal the known ones,
  and its factors reproduce A and are orthogonal.
* V2 agrees with the known V2 column by column up to sign where the angles
  are distinct (the CSD fixes each column up to sign then).
* LAPACK's complete CS decomposition (scipy.linalg.cossin with p = q = n, a
  different algorithm) gives the same angles on Haar orthogonal matrices.
* n = 1: A is a 2 x 2 rotation (or reflection) and theta is its angle.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import csd2x2 as C2
from paper_1804_09002_amd import workloads as WL

U = 2.0 ** -53


def _known(n, seed):
    rng = np.random.default_rng(seed)
    th = WL.angles_uniform(n, rng)
    U1, U2, V1, V2 = (WL.haar(n, rng) for _ in range(4))
    return C2.reconstruct2x2(U1, U2, V1, V2, th), (U1, U2, V1, V2, th)


@pytest.mark.parametrize("n,seed", [(5, 1), (40, 2), (120, 3)])
def test_known_factors(n, seed):
    A, (U1, U2, V1, V2, th) = _known(n, seed)
    assert np.linalg.norm(A.T @ A - np.eye(2 * n)) <= 1e-13
    r = C2.csd2x2(A)
    assert np.max(np.abs(r["theta"] - th)) <= 10 * n * U
    Ah = C2.reconstruct2x2(r["U1"], r["U2"], r["V1"], r["V2"], r["theta"])
    assert np.linalg.norm(Ah - A, 2) <= 100 * n * U
    for X in (r["U1"], r["U2"], r["V1"], r["V2"]):
        assert np.linalg.norm(X.T @ X - np.eye(n), 2) <= 100 * n * U
    # distinct angles: each column of V2 is the known one up to sign
    dots = np.abs(np.sum(r["V2"] * V2, axis=0))
    assert np.all(np.abs(dots - 1.0) <= 1e-8)


@pytest.mark.parametrize("n,seed", [(8, 4), (60, 5)])
def test_against_lapack_cossin(n, seed):
    A = WL.haar(2 * n, np.random.default_rng(seed))
    r = C2.csd2x2(A)
    _, cs, _ = scipy.linalg.cossin(A, p=n, q=n)
    th_lapack = np.sort(np.arctan2(np.diag(cs[n:, :n]), np.diag(cs[:n, :n])))
    assert np.max(np.abs(r["theta"] - th_lapack)) <= 1e-12
    Ah = C2.reconstruct2x2(r["U1"], r["U2"], r["V1"], r["V2"], r["theta"])
    assert np.linalg.norm(Ah - A, 2) <= 100 * n * U


@pytest.mark.parametrize("phi", [0.3, 1.2])
def test_n1_rotation(phi):
    c, s = np.cos(phi), np.sin(phi)
    A = np.array([[c, -s], [s, c]])
    r = C2.csd2x2(A)
    assert abs(r["theta"][0] - phi) <= 1e-15
    Ah = C2.reconstruct2x2(r["U1"], r["U2"], r["V1"], r["V2"], r["theta"])
    assert np.linalg.norm(Ah - A) <= 1e-15
