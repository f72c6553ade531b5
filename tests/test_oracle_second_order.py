"""Pins of the second-order oracle (AIRGA's solves, proportional damping).

Independent routes to the same numbers: the companion first-order
linearisation of the second-order model solved densely, the modal closed form
of a symmetric model, the exact inverse that a full pattern gives, and the
scaling relation between the second-order factors and first-order ones.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import chain, job
from oracle import second_order as so
from paper_2003_12759_amd.workloads import make_second_order


def _model(n, seed, symmetric=False, density=0.12):
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=density, random_state=rng, format="csr")
    R.data = rng.standard_normal(R.nnz)
    if symmetric:
        R = (R + R.T) * 0.5
    # K: a positive diagonal shift keeps K (and A(s) for s >= 0) well conditioned
    K = (R + sp.diags(8.0 + rng.uniform(0, 1, n))).tocsr()
    K.sort_indices()
    m = rng.uniform(1.0, 2.0, n)
    F = rng.standard_normal((n, 2))
    C = rng.standard_normal((n, 2))
    return K, m, F, C


def test_direct_matches_the_companion_linearisation():
    """With z = [x'; x], M x'' + D x' + K x = F u is E2 z' = A2 z + [F; 0] u,
    E2 = diag(M, I), A2 = [[-D, -K], [I, 0]]: (s E2 - A2)^{-1} [F; 0] has x in
    its lower half, and (s E2 - A2)^{-T} [0; C] has A(s)^{-T} C in its upper
    half.  Moments: the right-hand sides -M X_{j-1} and -M Y_{j-1} go in the
    same places."""
    n, alpha, beta = 40, 0.3, 0.02
    K, m, F, C = _model(n, 3)
    pts, nmom = [0.7, 3.0, -0.4], 3
    X, Y = so.direct(m, K, alpha, beta, F, C, pts, nmom)
    M = np.diag(m)
    Kd = K.toarray()
    D = alpha * M + beta * Kd
    I, Z = np.eye(n), np.zeros((n, n))
    E2 = np.block([[M, Z], [Z, I]])
    A2 = np.block([[-D, -Kd], [I, Z]])
    for i, s in enumerate(pts):
        L = s * E2 - A2
        x, y = F, C
        for j in range(nmom):
            rx = x if j == 0 else -(M @ x)
            ry = y if j == 0 else -(M @ y)
            x = np.linalg.solve(L, np.vstack([rx, np.zeros_like(rx)]))[n:]
            y = np.linalg.solve(L.T, np.vstack([np.zeros_like(ry), ry]))[:n]
            k = (j * len(pts) + i) * 2
            assert np.allclose(X[:, k:k + 2], x, rtol=1e-10, atol=1e-12 * abs(x).max())
            assert np.allclose(Y[:, k:k + 2], y, rtol=1e-10, atol=1e-12 * abs(y).max())


def test_direct_matches_the_modal_closed_form():
    """Symmetric K, K Phi = M Phi Lambda with Phi^T M Phi = I: A(s) =
    Phi^{-T} diag(d) Phi^{-1}, d = s^2 + s (alpha + beta lambda) + lambda, so
    X_j = (-1)^j Phi d^{-(j+1)} Phi^T F (and Y_j with C)."""
    n, alpha, beta = 30, 0.05, 5e-3
    K, m, F, C = _model(n, 5, symmetric=True)
    lam, Phi = sla.eigh(K.toarray(), np.diag(m))
    pts, nmom = [1.0, 4.0, 11.0], 3
    X, Y = so.direct(m, K, alpha, beta, F, C, pts, nmom)
    for i, s in enumerate(pts):
        d = s * s + s * (alpha + beta * lam) + lam
        for j in range(nmom):
            g = (-1.0) ** j * d ** (-(j + 1))
            x = Phi @ (g[:, None] * (Phi.T @ F))
            y = Phi @ (g[:, None] * (Phi.T @ C))
            k = (j * len(pts) + i) * 2
            assert np.allclose(X[:, k:k + 2], x, rtol=1e-9, atol=1e-11 * abs(x).max())
            assert np.allclose(Y[:, k:k + 2], y, rtol=1e-9, atol=1e-11 * abs(y).max())


def test_matrix_is_s2M_plus_sD_plus_K_on_the_pattern():
    n, alpha, beta, s = 25, 0.2, 0.01, 2.5
    K, m, _, _ = _model(n, 7)
    K = K.tolil()
    K[3, 3] = 0.0  # a row without a stored diagonal in K
    K = K.tocsr()
    K.eliminate_zeros()
    A = so.matrix(m, K, alpha, beta, s)
    M = np.diag(m)
    ref = s * s * M + s * (alpha * M + beta * K.toarray()) + K.toarray()
    assert np.allclose(A.toarray(), ref, rtol=1e-14, atol=1e-14)
    # pattern: K's plus the full diagonal
    P = (K.toarray() != 0) | np.eye(n, dtype=bool)
    got = np.zeros((n, n), dtype=bool)
    Ac = A.tocoo()
    got[Ac.row, Ac.col] = True
    assert np.array_equal(got, P)


def test_full_pattern_chains_are_the_exact_inverses():
    """With a full pattern the SPAI of A(s_1) is A(s_1)^{-1} and every update
    is A(s_i)^{-1} A(s_{i-1}), so each chain of Algorithm 4 (horizontal and
    vertical links) multiplies out to A(s_i)^{-1}."""
    n, alpha, beta = 10, 0.1, 0.02
    rng = np.random.default_rng(11)
    K = sp.csr_matrix(rng.standard_normal((n, n)) + 8.0 * np.eye(n))
    m = rng.uniform(1.0, 2.0, n)
    rounds = [[0.5, 2.0, 6.0], [0.6, 2.5, 5.0]]
    fs, chains = so.factors(m, K, alpha, beta, rounds)
    for z, pts in enumerate(rounds):
        for i, s in enumerate(pts):
            assert len(chains[z][i]) == i + z + 1
            P = chain.apply(fs, chains[z][i], np.eye(n))
            Ainv = np.linalg.inv(so.matrix(m, K, alpha, beta, s).toarray())
            assert np.allclose(P, Ainv, rtol=1e-9, atol=1e-11 * abs(Ainv).max())


def test_second_order_chains_are_scaled_first_order_chains():
    """A(s) = c (sigma M + K) with c = 1 + beta s, sigma = (s^2 + alpha s) / c:
    the SPAI of c A1 is SPAI(A1) / c and min ||c' A1' - c A1 Q|| is solved by
    (c'/c) Q1, so on a sparse pattern each second-order chain equals the
    first-order chain at sigma(s_i) (E = M, A = -K) divided by c(s_i)."""
    n, alpha, beta = 40, 0.3, 0.02
    K, m, _, _ = _model(n, 13)
    rounds = [[0.5, 2.0, 6.0], [0.6, 2.5, 5.0]]
    fs, chains = so.factors(m, K, alpha, beta, rounds)
    c = lambda s: 1.0 + beta * s
    sig = [[(s * s + alpha * s) / c(s) for s in pts] for pts in rounds]
    specs1, chains1 = chain.schedule(sig)
    fs1 = job.build_factors((-K).tocsr(), m, specs1)
    assert chains1 == chains
    for z, pts in enumerate(rounds):
        for i, s in enumerate(pts):
            P2 = chain.apply(fs, chains[z][i], np.eye(n))
            P1 = chain.apply(fs1, chains1[z][i], np.eye(n))
            assert np.allclose(P2, P1 / c(s), rtol=1e-10, atol=1e-13 * abs(P1).max())


def test_preconditioned_solve_matches_direct():
    """Lines 4 and 10 by BiCG with the reused chains over two rounds: every
    moment meets its own system to 1e-10 and agrees with the sparse LU."""
    w = make_second_order(N=6, nround=2, npoint=3, unit_io=False)
    nmom = 2
    out = so.solve(w.m, w.K, w.alpha, w.beta, w.F, w.C, w.rounds, nmom=nmom)
    for z, pts in enumerate(w.rounds):
        X, Y, stats = out[z]
        Xd, Yd = so.direct(w.m, w.K, w.alpha, w.beta, w.F, w.C, pts, nmom)
        assert all(st.status == "ok" for st in stats)
        for i, s in enumerate(pts):
            A = so.matrix(w.m, w.K, w.alpha, w.beta, s).tocsr()
            for j in range(nmom):
                k = j * len(pts) + i
                b = w.F[:, 0] if j == 0 else -(w.m * X[:, k - len(pts)])
                cc = w.C[:, 0] if j == 0 else -(w.m * Y[:, k - len(pts)])
                assert np.linalg.norm(b - A @ X[:, k]) <= 1e-10 * np.linalg.norm(b)
                assert np.linalg.norm(cc - A.T @ Y[:, k]) <= 1e-10 * np.linalg.norm(cc)
                cond = np.linalg.cond(A.toarray())
                assert np.linalg.norm(X[:, k] - Xd[:, k]) <= 4e-10 * cond * np.linalg.norm(Xd[:, k])


def test_reduction_interpolates_at_the_points_and_is_exact_on_a_full_basis():
    """Galerkin with V spanning A(s_i)^{-1} F interpolates H(s) = C^T A(s)^{-1} F at
    every s_i (and only there, in general); a complete basis reproduces H
    everywhere; and V^T D V = alpha M^ + beta K^."""
    n, alpha, beta = 40, 0.3, 0.02
    K, m, F, C = _model(n, 17)
    pts = [0.5, 2.0, 5.0]
    X, _ = so.direct(m, K, alpha, beta, F, C, pts)
    Mh, Dh, Kh, Fh, Ch = so.reduce(m, K, alpha, beta, F, C, X)
    assert np.allclose(Dh, alpha * Mh + beta * Kh, rtol=1e-12, atol=1e-12 * abs(Kh).max())
    for s in pts:
        full = so.full_transfer(m, K, alpha, beta, F, C, s)
        red = so.transfer(Mh, Dh, Kh, Fh, Ch, s)
        assert abs(red - full).max() <= 1e-10 * abs(full).max(), s
    off = so.full_transfer(m, K, alpha, beta, F, C, 1.1)
    assert abs(so.transfer(Mh, Dh, Kh, Fh, Ch, 1.1) - off).max() > 1e-8 * abs(off).max()
    full_basis = so.reduce(m, K, alpha, beta, F, C, np.eye(n))
    for s in (0.3, 1.1, 7.0):
        full = so.full_transfer(m, K, alpha, beta, F, C, s)
        assert abs(so.transfer(*full_basis, s) - full).max() <= 1e-10 * abs(full).max()
