"""Pins for the per-pair PSD projection used by projected Newton
(Sec. III-C): P is the Frobenius-nearest PSD matrix, V max(L, 0) V^T."""
import numpy as np
import pytest

import oracle as O


def _sym(rng, n, scale=1.0):
    A = rng.normal(size=(n, n)) * scale
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n", [2, 3, 6, 9, 12])
def test_projection_invariants(n):
    rng = np.random.default_rng(n)
    for _ in range(30):
        H = _sym(rng, n, 10 ** rng.uniform(-3, 6))
        P, sweeps = O.project_psd(H)
        nrm = np.linalg.norm(H)
        assert sweeps < 30
        assert np.abs(P - P.T).max() <= 1e-14 * nrm
        lam = np.linalg.eigvalsh(H)
        assert np.linalg.eigvalsh(P).min() >= -1e-14 * nrm
        assert np.linalg.eigvalsh(H - P).max() <= 1e-13 * nrm
        assert np.linalg.norm(H - P) ** 2 == pytest.approx((np.minimum(lam, 0) ** 2).sum(), rel=1e-10, abs=1e-26 * nrm ** 2)
        P2, _ = O.project_psd(P)
        assert np.abs(P2 - P).max() <= 1e-13 * nrm
        # the same matrix from a library eigensolver
        w, V = np.linalg.eigh(H)
        ref = (V * np.maximum(w, 0)) @ V.T
        assert np.linalg.norm(P - ref) <= 1e-13 * nrm


def test_psd_input_is_unchanged():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(12, 7))
    H = A @ A.T
    P, _ = O.project_psd(H)
    assert np.abs(P - H).max() <= 1e-13 * np.linalg.norm(H)


def test_diagonal_and_rank_one():
    d = np.array([3.0, -2.0, 0.0, 1e-3, -1e5, 7.0])
    P, _ = O.project_psd(np.diag(d))
    assert np.array_equal(P, np.diag(np.maximum(d, 0)))
    rng = np.random.default_rng(1)
    g = rng.normal(size=12)
    for a in [2.5, -2.5]:
        P, _ = O.project_psd(a * np.outer(g, g))
        assert np.abs(P - max(a, 0) * np.outer(g, g)).max() <= 1e-13 * abs(a) * (g @ g)


def test_pair_hessians_project_like_library():
    """Projected pair Hessians from the barrier (PT and EE)."""
    from tests.test_oracle_barrier import _close_pair
    rng = np.random.default_rng(4)
    for kind in (0, 1):
        for _ in range(10):
            x12 = _close_pair(rng, kind, 1e-3)
            st, t, s, e, g, H = O.pair_eval(kind, x12, 1e-3, 1e3)
            P, _ = O.project_psd(H)
            w, V = np.linalg.eigh(H)
            ref = (V * np.maximum(w, 0)) @ V.T
            assert np.linalg.norm(P - ref) <= 1e-12 * np.linalg.norm(H)
