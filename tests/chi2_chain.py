"""FP64 reference of the chi-square gradient through the operator, and the
scales its float32 GPU evaluation is compared under (test helpers).

The chain is render -> S = A Z (Sec. 3, Eq. (6)) -> chi-square -> A^T dS ->
renderer gradient.  Its float32 GPU evaluation differs from the FP64 chain by
(i) the image error, |dS_i| <= ~1.1e-5 S_i (every term of A Z is >= 0; the
scene is float32 too), which moves the residual r_i = K S_i - D_i by
K |dS_i|, and (ii) the adjoint's error, <= 1e-5 (|A|^T |2 K r / var|)_j.
Both are bounded by 1.1e-5 (|A|^T w)_j with w_i = 2K (|r_i| + K S_i) / var_i,
so gradient component k is within 1.1e-5 sum_j |dZ_j/dtheta_k| (|A|^T w)_j of
the FP64 chain.
"""
import numpy as np

import oracle as O


def loss(A, N, S, rmax, theta, counts, var, K):
    r = K * (A @ O.render_disk(N, S, rmax, theta)) - counts
    return float(np.sum(r * r / var))


def loss_and_grad(A, N, S, rmax, theta, counts, var, K):
    """FP64 chi-square and its gradient through the oracle chain."""
    Z = O.render_disk(N, S, rmax, theta)
    r = K * (A @ Z) - counts
    L = float(np.sum(r * r / var))
    return L, O.render_disk_grad(N, S, rmax, theta, A.T @ (2.0 * K * r / var))


def jacobian_abs(N, S, rmax, theta):
    """|dZ_j/dtheta_k| (5 x N^2) by central differences of the oracle renderer
    (used only as a tolerance scale)."""
    th = np.asarray(theta, dtype=np.float64)
    J = np.empty((5, N * N))
    for k in range(5):
        h = 1e-6 * max(abs(th[k]), 1e-3)
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        J[k] = np.abs(O.render_disk(N, S, rmax, tp) - O.render_disk(N, S, rmax, tm)) / (2 * h)
    return J


def gradient_scales(A, N, S, rmax, theta, counts, var, K):
    """Per-component scales: the rigorous one, sum_j |J_kj| (|A|^T w)_j with
    w = 2K(|r| + K S)/var, and the chain evaluated on |r| alone."""
    Sref = A @ O.render_disk(N, S, rmax, theta)
    r = K * Sref - counts
    J = jacobian_abs(N, S, rmax, theta)
    absA = np.abs(A)
    w = 2.0 * K * (np.abs(r) + K * np.abs(Sref)) / var
    wr = 2.0 * K * np.abs(r) / var
    return J @ (absA.T @ w), J @ (absA.T @ wr)


def central_differences(A, N, S, rmax, theta, counts, var, K, rel=1e-5):
    """Per-parameter FP64 central differences of the oracle loss."""
    th = np.asarray(theta, dtype=np.float64)
    out = np.empty(5)
    for k in range(5):
        h = rel * abs(th[k])
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        out[k] = (loss(A, N, S, rmax, tp, counts, var, K) -
                  loss(A, N, S, rmax, tm, counts, var, K)) / (2 * h)
    return out
