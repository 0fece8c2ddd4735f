"""O(n^2) brute-force Cox quantities straight from the definitions of Section 5.3.

Written independently of the oracle: no sorting, no cumulative sums.  The risk
set indicator is a dense n x n matrix R[i, j] = 1(y_j >= y_i) (ties included,
Breslow), and P has entries pi_ij = 1(y_i >= y_j) w_i / W_j, exactly as the
dense program of Section 5.3 builds pi_ind and pi.  Used on n <= 2000 only.
"""
import numpy as np


def risk_matrix(y):
    y = np.asarray(y, np.float64)
    return (y[None, :] >= y[:, None]).astype(np.float64)  # [i, j] = 1(y_j >= y_i)


def loglik(eta, y, delta):
    """L = sum_i delta_i (eta_i - log sum_{j: y_j >= y_i} exp(eta_j))."""
    eta = np.asarray(eta, np.float64)
    d = np.asarray(delta, np.float64)
    W = risk_matrix(y) @ np.exp(eta)
    return float(np.sum(d * (eta - np.log(W))))


def residual(eta, y, delta):
    """r = (I - P) delta with pi_ij = 1(y_i >= y_j) w_i / W_j."""
    eta = np.asarray(eta, np.float64)
    d = np.asarray(delta, np.float64)
    w = np.exp(eta)
    R = risk_matrix(y)
    W = R @ w                        # W_j
    Pi = R.T * w[:, None] / W[None, :]  # [i, j] = 1(y_i >= y_j) w_i / W_j
    return d - Pi @ d


def hessian_eta(eta, y, delta):
    """-d^2 L / d eta^2 = sum_j delta_j (diag(p_j) - p_j p_j') with p_j the
    risk-set softmax of subject j's event."""
    eta = np.asarray(eta, np.float64)
    d = np.asarray(delta, np.float64)
    w = np.exp(eta)
    R = risk_matrix(y)
    H = np.zeros((len(w), len(w)))
    for j in np.nonzero(d)[0]:
        pj = R[j] * w / (R[j] @ w)
        H += d[j] * (np.diag(pj) - np.outer(pj, pj))
    return H


def objective(X, beta, y, delta, lam):
    """f = -L(X'beta) + lam ||beta||_1 with X given as (p, n)."""
    return -loglik(X.T @ beta, y, delta) + lam * np.abs(beta).sum()


def gradient(X, beta, y, delta):
    """dL/dbeta = X r (X given as (p, n))."""
    return X @ residual(X.T @ beta, y, delta)
