"""Closed-form gradients for the CSD (oracle, test infrastructure).

With A1 = U1 C V1^T, A2 = U2 S V1^T (C = diag(c), S = diag(s), distinct angles):

* angles: theta_i = atan2(s_i, c_i) with dc_i = u1_i^T dA1 v_i and
  ds_i = u2_i^T dA2 v_i (first-order perturbation of the diagonal of
  V1^T H_i V1 that gives C and S in Algorithm 1), so
      d theta_i / d A1 = -s_i u1_i v_i^T,   d theta_i / d A2 = c_i u2_i v_i^T;
* polar factor W = U V^T of A = U Sigma V^T: for E = U^T dA V,
  dW = U [(E - E^T) / (sigma_j + sigma_k)] V^T, so
      grad_A <G, W> = U [(M - M^T) / (sigma_j + sigma_k)] V^T,  M = U^T G V.

The loss of the differentiation workload is
    L = sum_i g_i theta_i + <G1, W1> + <G2, W2>.
These formulas are pinned against central finite differences of the oracle CSD.
"""
from __future__ import annotations

import numpy as np


def polar_grad(U, sig, V, G):
    M = U.T @ G @ V
    den = sig[:, None] + sig[None, :]
    return U @ ((M - M.T) / den) @ V.T


def csd_loss_grad(U1, U2, V1, theta, g, G1, G2):
    """Gradient of L = g.theta + <G1, W1> + <G2, W2> with respect to (A1, A2)."""
    c = np.cos(theta)
    s = np.sin(theta)
    gA1 = -(U1 * (g * s)) @ V1.T
    gA2 = (U2 * (g * c)) @ V1.T
    if G1 is not None:
        gA1 = gA1 + polar_grad(U1, c, V1, G1)
    if G2 is not None:
        gA2 = gA2 + polar_grad(U2, s, V1, G2)
    return gA1, gA2


def csd_loss(U1, U2, V1, theta, W1, W2, g, G1, G2):
    val = float(np.dot(g, theta))
    if G1 is not None:
        val += float(np.sum(G1 * W1))
    if G2 is not None:
        val += float(np.sum(G2 * W2))
    return val
