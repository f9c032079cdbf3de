"""Checks of returned eigenpairs against a dense Hermitian matrix (test helper, numpy only).

For Ritz pairs (theta_i, q_i) with orthonormal q_i and residual matrix R = H Q - Q Theta:
  - the theta_i lie within ||R||_2 of k distinct eigenvalues of H (Kahan's theorem for
    Hermitian matrices); if no eigenvalue outside the wanted set comes within ||R||_2 of any
    theta_i, the matched eigenvalues are exactly the wanted ones;
  - the sine of the largest angle between span Q and the exact wanted eigenspace is at most
    ||R||_2 / delta, delta the distance from the theta_i to the unwanted eigenvalues
    (Davis and Kahan's sin-theta theorem).
"""
import numpy as np


def check_smallest_abs_pairs(H, theta, Q, xi=None, tight=True):
    """H dense Hermitian (N x N), theta (k,) Ritz values, Q (k, N) rows orthonormal.  Returns
    (||R||_2, sin angle, delta).  With xi, each pair must meet ||H q - theta q|| <= xi |theta|.
    With tight, asserts that the pairs are the k smallest |lambda| (matching and sin-theta)."""
    k = len(theta)
    Qc = Q.T
    assert np.allclose(Q.conj() @ Qc, np.eye(k), atol=1e-10), "returned vectors are not orthonormal"
    R = H @ Qc - Qc * theta[None, :]
    res = np.linalg.norm(R, axis=0)
    if xi is not None:
        assert np.all(res <= xi * np.abs(theta) * (1 + 1e-6) + 1e-13), (res / np.abs(theta)).max()
    r2 = np.linalg.norm(R, 2)
    w, E = np.linalg.eigh(H)
    order = np.argsort(np.abs(w), kind="stable")
    want, rest = order[:k], order[k:]
    delta = np.min(np.abs(theta[:, None] - w[rest][None, :])) if rest.size else np.inf
    # sine of the largest angle: the norm of Q's component outside the wanted eigenspace
    # (computed directly; sqrt(1 - cos^2) would floor at sqrt(2 eps))
    sin = np.linalg.norm(E[:, rest].conj().T @ Qc, 2) if rest.size else 0.0
    if tight:
        # no unwanted eigenvalue within ||R|| of a returned value: the matches are the wanted ones
        assert delta > r2, (delta, r2)
        assert np.max(np.abs(np.sort(theta) - np.sort(w[want]))) <= r2 * (1 + 1e-9) + 1e-13
        assert sin <= r2 / delta * (1 + 1e-9) + 1e-12, (sin, r2, delta)
    return r2, sin, delta
