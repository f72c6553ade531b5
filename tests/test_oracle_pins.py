"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one oracle function against brute force, a closed form from
the paper or from linear algebra, or a textbook special case, chosen so that
a dropped term, a wrong sign, index or shift, or a transposed operand fails.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import bicg, chain, gmres, irka, job, pattern, projection, spai
from oracle.precision import round_storage
from paper_2003_12759_amd.workloads import laplacian_5pt, make_workload


def _rand_sparse(n, density, seed, symmetric_pattern=False):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    M.data = rng.standard_normal(M.nnz)
    if symmetric_pattern:
        P = (abs(M) + abs(M.T)).tocsr()
        P.data = rng.standard_normal(P.nnz)
        M = P
    M = M + sp.diags(-5.0 - rng.uniform(0, 1, n))  # A with a stable-ish diagonal
    M = M.tocsr()
    M.sort_indices()
    return M


def test_pattern_matches_dense_bruteforce():
    A = _rand_sparse(30, 0.08, 1)
    S = pattern.pattern(A)
    D = (A.toarray() != 0) | np.eye(30, dtype=bool)
    assert np.array_equal(S.toarray() != 0, D)
    for k in range(30):
        J = pattern.column_support(S, k)
        assert np.array_equal(J, np.nonzero(D[:, k])[0])
        I = pattern.shadow_rows(S, J)
        assert np.array_equal(I, np.nonzero(D[:, J].any(axis=1))[0])


@pytest.mark.parametrize("sigma", [0.5, 7.0])
def test_spai_column_equals_bruteforce_least_squares(sigma):
    """eq. gen-precond-par: column k minimises ||e_k - A_s p|| over supp(p) = J_k,
    solved here over all n rows (no restriction to I_k)."""
    n = 40
    A = _rand_sparse(n, 0.1, 2)
    e = np.random.default_rng(3).uniform(1, 2, n)
    As = sigma * np.diag(e) - A.toarray()
    P = spai.spai(A, e, sigma).toarray()
    S = pattern.pattern(A).toarray() != 0
    for k in range(n):
        J = np.nonzero(S[:, k])[0]
        ek = np.zeros(n)
        ek[k] = 1.0
        pbf, *_ = np.linalg.lstsq(As[:, J], ek, rcond=None)
        assert np.allclose(P[J, k], pbf, rtol=1e-12, atol=1e-14)
        assert np.all(P[~S[:, k], k] == 0.0)
        # normal equations: the residual is orthogonal to the allowed columns
        res = ek - As[:, J] @ P[J, k]
        assert np.linalg.norm(As[:, J].T @ res) <= 1e-13 * np.linalg.norm(As[:, J]) ** 2


def test_spai_full_pattern_is_exact_inverse():
    """With a full pattern the Frobenius minimiser of ||I - A P|| is A^{-1}."""
    n = 12
    rng = np.random.default_rng(4)
    Ad = rng.standard_normal((n, n)) - 6 * np.eye(n)
    A = sp.csr_matrix(Ad)
    e = rng.uniform(1, 2, n)
    sigma = 2.5
    P = spai.spai(A, e, sigma).toarray()
    assert np.allclose(P, np.linalg.inv(sigma * np.diag(e) - Ad), rtol=1e-11, atol=1e-13)


def test_update_full_pattern_closed_form_appendix_b():
    """Appendix B: A_i = A_{i-1}(I + (s_i - s_{i-1}) A_{i-1}^{-1} E), so the exact
    update is Q_i = (I + (s_i - s_{i-1}) A_{i-1}^{-1} E)^{-1} = A_i^{-1} A_{i-1}."""
    n = 10
    rng = np.random.default_rng(5)
    Ad = rng.standard_normal((n, n)) - 6 * np.eye(n)
    A = sp.csr_matrix(Ad)
    e = rng.uniform(1, 2, n)
    s0, s1 = 1.5, 4.0
    Q = spai.update(A, e, s0, s1).toarray()
    E = np.diag(e)
    Aprev = s0 * E - Ad
    Anew = s1 * E - Ad
    assert np.allclose(Q, np.linalg.solve(Anew, Aprev), rtol=1e-11, atol=1e-13)
    Qb = np.linalg.inv(np.eye(n) + (s1 - s0) * np.linalg.solve(Aprev, E))
    assert np.allclose(Q, Qb, rtol=1e-10, atol=1e-12)


def test_update_column_equals_bruteforce_least_squares():
    n = 36
    A = _rand_sparse(n, 0.1, 6)
    e = np.random.default_rng(7).uniform(1, 2, n)
    s0, s1 = 3.0, 0.7  # a decreasing step: the shift difference is negative
    Q = spai.update(A, e, s0, s1).toarray()
    Aprev = s0 * np.diag(e) - A.toarray()
    Anew = s1 * np.diag(e) - A.toarray()
    S = pattern.pattern(A).toarray() != 0
    for k in range(n):
        J = np.nonzero(S[:, k])[0]
        qbf, *_ = np.linalg.lstsq(Anew[:, J], Aprev[:, k], rcond=None)
        assert np.allclose(Q[J, k], qbf, rtol=1e-12, atol=1e-14)


def test_update_static_pattern_identity():
    """With E diagonal and k in J_k: Q_i = I - (s_i - s_{i-1}) SPAI_J(A_i) E exactly
    (the update's right-hand side A_{i-1} e_k = A_i e_k - (s_i - s_{i-1}) e_kk e_k)."""
    A = laplacian_5pt(7)
    n = A.shape[0]
    e = np.random.default_rng(8).uniform(1, 2, n)
    s0, s1 = 2.0, 9.0
    Q = spai.update(A, e, s0, s1).toarray()
    P = spai.spai(A, e, s1).toarray()
    expect = np.eye(n) - (s1 - s0) * P @ np.diag(e)
    assert np.max(np.abs(Q - expect)) <= 1e-13 * np.max(np.abs(Q))


def test_schedule_follows_algorithm4():
    rounds = [[1.0, 2.0, 3.0], [1.1, 2.1, 3.1], [1.2, 2.2, 3.2]]
    specs, chains = chain.schedule(rounds)
    assert specs == [
        ("spai", 1.0), ("update", 1.0, 2.0), ("update", 2.0, 3.0),
        ("update", 1.0, 1.1), ("update", 1.1, 2.1), ("update", 2.1, 3.1),
        ("update", 1.1, 1.2), ("update", 1.2, 2.2), ("update", 2.2, 3.2),
    ]
    # P_1^(1); Q_2^(1) P_1^(1); Q_3^(1) Q_2^(1) P_1^(1)  (first applied listed first)
    assert chains[0] == [[0], [0, 1], [0, 1, 2]]
    # Q_1^(2) P_1^(1); Q_2^(2) Q_1^(2) P_1^(1); ...
    assert chains[1] == [[0, 3], [0, 3, 4], [0, 3, 4, 5]]
    assert chains[2] == [[0, 3, 6], [0, 3, 6, 7], [0, 3, 6, 7, 8]]
    for z in range(3):
        for i in range(3):
            assert len(chains[z][i]) == (i + 1) + (z + 1) - 1


def test_anchored_schedule_for_serving():
    """Anchors 1, 10, 100 (log-spaced over [1, 100]); each request's chain is
    the anchor prefix up to its nearest anchor in log(sigma) plus one update."""
    a = chain.anchor_shifts(3, 1.0, 100.0)
    assert a[0] == 1.0 and abs(a[1] - 10.0) < 1e-14 and abs(a[2] - 100.0) < 1e-12
    a = [1.0, 10.0, 100.0]
    assert chain.schedule_anchored(a, 2.0) == [("spai", 1.0), ("update", 1.0, 2.0)]
    assert chain.schedule_anchored(a, 5.0) == [("spai", 1.0), ("update", 1.0, 10.0),
                                               ("update", 10.0, 5.0)]
    assert chain.schedule_anchored(a, 1e4) == [("spai", 1.0), ("update", 1.0, 10.0),
                                               ("update", 10.0, 100.0), ("update", 100.0, 1e4)]
    # log-distance tie between 1 and 10 (sigma = sqrt(10)): the first anchor
    assert chain.schedule_anchored([1.0, 100.0], 10.0)[0:1] == [("spai", 1.0)]
    assert len(chain.schedule_anchored([1.0, 100.0], 10.0)) == 2
    assert chain.anchor_shifts(1, 3.0, 3.0) == [3.0]


def test_comparator_schedules():
    rounds = [[1.0, 2.0, 3.0], [1.1, 2.1, 3.1]]
    specs, chains = chain.schedule_direct(rounds)
    assert specs == [("spai", 1.0), ("spai", 2.0), ("spai", 3.0),
                     ("spai", 1.1), ("spai", 2.1), ("spai", 3.1)]
    assert chains == [[[0], [1], [2]], [[3], [4], [5]]]
    specs, chains = chain.schedule_first(rounds)
    assert specs == [("spai", 1.0), ("update", 1.0, 2.0), ("update", 1.0, 3.0),
                     ("spai", 1.1), ("update", 1.1, 2.1), ("update", 1.1, 3.1)]
    assert chains == [[[0], [0, 1], [0, 2]], [[3], [3, 4], [3, 5]]]


def test_first_approach_full_pattern_is_exact_inverse():
    """Table 2, first approach: with a full pattern Q_i = A_i^{-1} A_1, so the
    chain [P_1, Q_i] applies Q_i P_1 = A_i^{-1} exactly."""
    n = 10
    rng = np.random.default_rng(12)
    Ad = rng.standard_normal((n, n)) - 6 * np.eye(n)
    A = sp.csr_matrix(Ad)
    e = rng.uniform(1, 2, n)
    sig = [1.5, 4.0, 0.5]
    specs, chains = chain.schedule_first([sig])
    fs = job.build_factors(A, e, specs)
    v = rng.standard_normal(n)
    for i, s in enumerate(sig):
        want = np.linalg.solve(s * np.diag(e) - Ad, v)
        got = chain.apply(fs, chains[0][i], v)
        assert np.allclose(got, want, rtol=1e-10, atol=1e-12)


def test_chain_apply_matches_formed_product():
    n = 25
    fs = [_rand_sparse(n, 0.15, 20 + k) for k in range(4)]
    v = np.random.default_rng(9).standard_normal(n)
    ch = [2, 0, 3]
    dense = fs[3].toarray() @ fs[0].toarray() @ fs[2].toarray()
    assert np.allclose(chain.apply(fs, ch, v), dense @ v, rtol=1e-13, atol=1e-13)
    assert np.allclose(chain.apply_transpose(fs, ch, v), dense.T @ v, rtol=1e-13, atol=1e-13)


def test_chain_apply_rows_match_the_whole_apply():
    """Sampled rows of a chain product (row vectors pushed through the
    factors) against the whole apply, both directions, on a chain with a
    repeated factor."""
    rng = np.random.default_rng(17)
    n = 60
    mats = []
    for _ in range(3):
        M = sp.random(n, n, density=0.08, random_state=rng, format="csr")
        M.data = rng.standard_normal(M.nnz)
        mats.append((M + sp.identity(n)).tocsr())
    ch = [0, 1, 2, 1, 0]
    v = rng.standard_normal(n)
    rows = [0, 7, 31, 59]
    whole = chain.apply(mats, ch, v)
    whole_t = chain.apply_transpose(mats, ch, v)
    dense = np.eye(n)
    for f in ch:
        dense = mats[f].toarray() @ dense
    scale = np.abs(dense) @ np.abs(v)
    scale_t = np.abs(dense.T) @ np.abs(v)
    got = chain.apply_rows(mats, ch, v, rows)
    got_t = chain.apply_rows(mats, ch, v, rows, transpose=True)
    assert np.all(np.abs(got - whole[rows]) <= 1e-13 * scale[rows])
    assert np.all(np.abs(got_t - whole_t[rows]) <= 1e-13 * scale_t[rows])


def test_chain_apply_f32_exact_when_every_pass_is_representable():
    """Small-integer factors and input: every pass result is an FP32 number,
    so the FP32 apply equals the FP64 apply bit for bit (both directions)."""
    n = 20
    rng = np.random.default_rng(31)
    fs = []
    for k in range(3):
        F = sp.random(n, n, density=0.2, random_state=rng, format="csr")
        F.data = rng.integers(-3, 4, F.nnz).astype(np.float64)
        fs.append((F + sp.eye(n)).tocsr())
    v = rng.integers(-5, 6, n).astype(np.float64)
    ch = [1, 2, 0]
    assert np.array_equal(chain.apply(fs, ch, v, "f32"), chain.apply(fs, ch, v))
    assert np.array_equal(chain.apply_transpose(fs, ch, v, "f32"), chain.apply_transpose(fs, ch, v))


def test_chain_apply_f32_rounds_input_each_pass_and_output():
    """Hand-worked cases: 1 + 2^-30 is not an FP32 number and rounds to 1.
    A difference of two such values scaled by 2^30 exposes where rounding
    happens: at the input, after each pass, and after the last pass."""
    t = 2.0 ** -30
    I2 = sp.identity(2, format="csr")
    D = sp.csr_matrix(sp.diags([1.0 + t, 1.0]))
    K = sp.csr_matrix(np.array([[2.0 ** 30, -(2.0 ** 30)], [0.0, 1.0]]))
    # input rounding: [1 + t, 1] -> [1, 1]
    v = np.array([1.0 + t, 1.0])
    assert np.array_equal(chain.apply([I2, K], [0, 1], v, "f32"), [0.0, 1.0])
    assert np.array_equal(chain.apply([I2, K], [0, 1], v), [1.0, 1.0])
    # rounding after an intermediate pass: D [1, 1] = [1 + t, 1] -> [1, 1]
    one = np.array([1.0, 1.0])
    assert np.array_equal(chain.apply([D, K], [0, 1], one, "f32"), [0.0, 1.0])
    assert np.array_equal(chain.apply([D, K], [0, 1], one), [1.0, 1.0])
    # and in the transposed chain, which applies K^T first and D^T last
    KT = sp.csr_matrix(K.toarray().T)
    assert np.array_equal(chain.apply_transpose([D, KT], [1, 0], one, "f32"), [0.0, 1.0])
    # rounding of the last pass
    assert np.array_equal(chain.apply([D], [0], one, "f32"), [1.0, 1.0])
    assert chain.apply([D], [0], one)[0] == 1.0 + t


def test_chain_apply_f32_error_bound():
    """Random factors: each pass adds at most one FP32 rounding (relative
    2^-24) on top of the propagated error, so the gap to the FP64 apply is
    bounded by |F_k| applied to the previous bound plus 2^-24 |result|."""
    n = 40
    fs = [_rand_sparse(n, 0.1, 40 + k) for k in range(3)]
    v = np.random.default_rng(41).standard_normal(n)
    ch = [0, 1, 2]
    u = 2.0 ** -24
    got = chain.apply(fs, ch, v, "f32")
    exact = chain.apply(fs, ch, v)
    t = np.asarray(v, dtype=np.float64)
    bound = u * np.abs(t)
    for f in ch:
        t = fs[f] @ t
        bound = abs(fs[f]) @ bound + u * (np.abs(t) + abs(fs[f]) @ bound) + 1e-300
    assert np.all(np.abs(got - exact) <= bound * 1.0001)
    assert np.all(got.astype(np.float32).astype(np.float64) == got)
    assert np.max(np.abs(got - exact)) > 0.0  # the rounding is really there


@pytest.mark.parametrize("apply_prec", ["f64", "f32"])
def test_bicg_matches_dense_lu_on_laplace2d_n2025(apply_prec):
    """All six shifts of the 45x45 workload, SPAI chain, tolerance 1e-10:
    true residuals pass and ||x - x_LU|| <= ||A_s^{-1}|| (||r|| + rounding).
    With an FP32-applied preconditioner the FP64 recurrences and the
    true-residual refinement still reach the same bound."""
    w = make_workload(0)
    out = job.run(w.A, w.e, w.B, w.C, w.rounds, prec="f64", tol=1e-10, project=False,
                  apply_prec=apply_prec)
    Ad = w.A.toarray()
    for i, s in enumerate(w.rounds[0]):
        st = out["rounds"][0]["stats"][i]
        assert st.status == "ok" and st.relres_primal <= 1e-10 and st.relres_dual <= 1e-10
        M = s * np.diag(w.e) - Ad
        x = np.linalg.solve(M, w.B[:, 0])
        y = np.linalg.solve(M.T, w.C[:, 0])
        smin = np.linalg.eigvalsh(M)[0]  # M symmetric positive definite here
        bound_x = (st.relres_primal * np.linalg.norm(w.B) + 1e-13 * np.linalg.norm(w.B)) / smin
        bound_y = (st.relres_dual * np.linalg.norm(w.C) + 1e-13 * np.linalg.norm(w.C)) / smin
        assert np.linalg.norm(out["rounds"][0]["X"][:, i] - x) <= bound_x
        assert np.linalg.norm(out["rounds"][0]["Y"][:, i] - y) <= bound_y
        assert np.linalg.norm(out["rounds"][0]["X"][:, i] - x) <= 1e-8 * np.linalg.norm(x)


@pytest.mark.parametrize("policy", ["reuse", "direct", "first"])
def test_bicg_nonsymmetric_three_rounds_vs_sparse_lu(policy):
    w = make_workload(1, N=8, nshift=4, nrounds=3)
    out = job.run(w.A, w.e, w.B, w.C, w.rounds, prec="f64", tol=1e-10, project=False,
                  policy=policy)
    for z, sig in enumerate(w.rounds):
        for i, s in enumerate(sig):
            st = out["rounds"][z]["stats"][i]
            assert st.status == "ok"
            M = (s * sp.diags(w.e) - w.A).tocsc()
            lu = spla.splu(M)
            x = lu.solve(w.B[:, 0])
            y = lu.solve(w.C[:, 0].copy(), trans="T")
            assert np.linalg.norm(out["rounds"][z]["X"][:, i] - x) <= 1e-8 * np.linalg.norm(x)
            assert np.linalg.norm(out["rounds"][z]["Y"][:, i] - y) <= 1e-8 * np.linalg.norm(y)


def _textbook_cg(M, b, k):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    for _ in range(k):
        Mp = M @ p
        a = rr / (p @ Mp)
        x = x + a * p
        r = r - a * Mp
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def test_bicg_reduces_to_cg_for_symmetric_systems():
    """Symmetric A_s, c = b, no preconditioner: the BiCG iterates are the CG iterates
    and the shadow iterate equals the primal one."""
    A = laplacian_5pt(6)
    n = A.shape[0]
    e = np.ones(n)
    M = (3.0 * sp.identity(n) - A).tocsr()
    b = np.random.default_rng(10).standard_normal(n)
    for k in (1, 4, 9):
        res = bicg.solve(lambda v: M @ v, lambda v: M.T @ v, b, b.copy(), tol=0.0,
                         maxit=k, max_restarts=0)
        xcg = _textbook_cg(M, b, k)
        assert res.iters == k
        assert np.allclose(res.x, xcg, rtol=1e-12, atol=1e-14 * np.linalg.norm(xcg))
        assert np.allclose(res.y, res.x, rtol=1e-13, atol=1e-15)


def test_bicg_diagonal_with_exact_spai_converges_in_one_step():
    n = 50
    rng = np.random.default_rng(11)
    A = sp.diags(-rng.uniform(1, 5, n)).tocsr()
    e = rng.uniform(1, 2, n)
    s = 2.0
    P = spai.spai(A, e, s)  # diagonal pattern: the exact inverse
    M = (s * sp.diags(e) - A).tocsr()
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    res = bicg.solve(lambda v: M @ v, lambda v: M.T @ v, b, c, lambda v: P @ v,
                     lambda v: P.T @ v, tol=1e-12)
    assert res.iters == 1 and res.status == "ok"


def test_bicg_zero_right_hand_sides():
    A = laplacian_5pt(5)
    n = A.shape[0]
    M = (1.0 * sp.identity(n) - A).tocsr()
    b = np.random.default_rng(12).standard_normal(n)
    ops = (lambda v: M @ v, lambda v: M.T @ v)
    r0 = bicg.solve(*ops, np.zeros(n), np.zeros(n))
    assert r0.iters == 0 and not r0.x.any() and not r0.y.any()
    r1 = bicg.solve(*ops, b, np.zeros(n), tol=1e-12)
    assert not r1.y.any() and np.linalg.norm(M @ r1.x - b) <= 1e-12 * np.linalg.norm(b)
    r2 = bicg.solve(*ops, np.zeros(n), b, tol=1e-12)
    assert not r2.x.any() and np.linalg.norm(M.T @ r2.y - b) <= 1e-12 * np.linalg.norm(b)


def test_projection_hermite_interpolation():
    """Section II: H and H' of the reduced model match the full model at every shift
    (solutions from a sparse direct solver), and not elsewhere."""
    w = make_workload(0)
    n = w.n
    X = np.zeros((n, 6))
    Y = np.zeros((n, 6))
    for i, s in enumerate(w.rounds[0]):
        lu = spla.splu((s * sp.diags(w.e) - w.A).tocsc())
        X[:, i] = lu.solve(w.B[:, 0])
        Y[:, i] = lu.solve(w.C[:, 0].copy(), trans="T")
    Ar, Er, Br, Cr = projection.reduce(w.A, w.e, w.B, w.C, X, Y)
    for s in w.rounds[0]:
        H, dH = projection.full_transfer(w.A, w.e, w.B, w.C, s)
        Hr = projection.transfer(Ar, Er, Br, Cr, s)
        dHr = projection.transfer_derivative(Ar, Er, Br, Cr, s)
        assert abs(Hr - H).max() <= 1e-11 * abs(H).max()
        assert abs(dHr - dH).max() <= 1e-10 * abs(dH).max()
    H, _ = projection.full_transfer(w.A, w.e, w.B, w.C, 7.0)
    Hr = projection.transfer(Ar, Er, Br, Cr, 7.0)
    assert abs(Hr - H).max() > 1e-12 * abs(H).max()
    # basis invariance: any other basis of the same spaces gives the same H_r
    T = np.random.default_rng(13).standard_normal((6, 6)) + 6 * np.eye(6)
    Ar2, Er2, Br2, Cr2 = projection.reduce(w.A, w.e, w.B, w.C, X @ T, Y @ T.T)
    assert abs(projection.transfer(Ar2, Er2, Br2, Cr2, 7.0) - Hr).max() <= 1e-10 * abs(Hr).max()


def test_transfer_derivatives_against_central_differences():
    """H^(k) from the closed form against central differences of H^(k-1):
    a wrong sign, factorial or power of (sE - A)^{-1} E fails."""
    w = make_workload(0, N=8)
    Ar, Er = w.A.toarray(), np.diag(w.e)
    Br, Cr = w.B.reshape(-1, 1), w.C.reshape(-1, 1)
    s, h = 3.0, 1e-4
    for k in (1, 2, 3):
        d = projection.transfer_derivative_k(Ar, Er, Br, Cr, s, k)
        fd = (projection.transfer_derivative_k(Ar, Er, Br, Cr, s + h, k - 1)
              - projection.transfer_derivative_k(Ar, Er, Br, Cr, s - h, k - 1)) / (2 * h)
        assert abs(d - fd).max() <= 1e-6 * abs(d).max(), (k, d, fd)
        full = projection.full_transfer_derivative_k(w.A, w.e, w.B, w.C, s, k)
        assert abs(full - d).max() <= 1e-10 * abs(d).max()
    assert np.allclose(projection.transfer_derivative_k(Ar, Er, Br, Cr, s, 1),
                       projection.transfer_derivative(Ar, Er, Br, Cr, s), rtol=1e-12)


def test_moments_match_derivatives_to_order_2J_minus_1():
    """Two moments per shift on both sides: the reduced H and its first three
    derivatives equal the full ones at every shift (oracle moments by BiCG);
    away from the shifts the reduced model is only an approximation."""
    w = make_workload(1, N=6, nshift=3)
    sig = w.rounds[0]
    X, Y, stats = job.moments(w.A, w.e, w.B, w.C, sig, 2)
    assert all(st.status == "ok" for st in stats)
    # the first moments satisfy their defining systems
    E = sp.diags(w.e)
    for i, s in enumerate(sig):
        M = (s * E - w.A).tocsr()
        rhs = w.e * X[:, i]
        assert np.linalg.norm(M @ X[:, len(sig) + i] - rhs) <= 1e-9 * np.linalg.norm(rhs)
    Ar, Er, Br, Cr = projection.reduce(w.A, w.e, w.B, w.C, X, Y)
    for s in sig:
        for k in range(4):
            full = projection.full_transfer_derivative_k(w.A, w.e, w.B, w.C, s, k)
            red = projection.transfer_derivative_k(Ar, Er, Br, Cr, s, k)
            assert abs(red - full).max() <= 1e-7 * abs(full).max(), (s, k)
    full4 = projection.full_transfer_derivative_k(w.A, w.e, w.B, w.C, 7.0, 4)
    red4 = projection.transfer_derivative_k(Ar, Er, Br, Cr, 7.0, 4)
    assert abs(red4 - full4).max() > 1e-8 * abs(full4).max()


def test_gmres_matches_dense_lu_with_spai_chain():
    """GMRES(30) with the Algorithm-4 chain on the 45x45 workload (primal and
    transposed systems): true residuals <= 1e-10 and the LU error bound."""
    w = make_workload(0, N=30, nshift=3)
    specs, chains = chain.schedule(w.rounds)
    fs = job.build_factors(w.A, w.e, specs)
    Ad = w.A.toarray()
    for i, s in enumerate(w.rounds[0]):
        M = s * np.diag(w.e) - Ad
        ch = chains[0][i]
        rp, rd = gmres.solve_pair(lambda v: M @ v, lambda v: M.T @ v, w.B[:, 0], w.C[:, 0],
                                  lambda v: chain.apply(fs, ch, v),
                                  lambda v: chain.apply_transpose(fs, ch, v), tol=1e-10, m=30)
        assert rp.status == "ok" and rd.status == "ok"
        smin = np.linalg.eigvalsh(M)[0]
        for res, rhs, Mm in ((rp, w.B[:, 0], M), (rd, w.C[:, 0], M.T)):
            exact = np.linalg.solve(Mm, rhs)
            rel = np.linalg.norm(rhs - Mm @ res.x) / np.linalg.norm(rhs)
            assert rel <= 1e-10
            assert np.linalg.norm(res.x - exact) <= (rel + 1e-13) * np.linalg.norm(rhs) / smin


def test_gmres_iterate_minimises_the_residual():
    """After k steps the GMRES iterate has the least residual over
    P K_k(A P, b): brute-force least squares over an explicit Krylov basis."""
    n = 40
    A = _rand_sparse(n, 0.1, 31).toarray()
    rng = np.random.default_rng(32)
    Pm = np.eye(n) + 0.05 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    AP = A @ Pm
    for k in range(1, 7):
        x, steps, _ = gmres.cycle(lambda v: A @ v, lambda v: Pm @ v, np.zeros(n), b, 30, 0.0,
                                  steps=k)
        assert steps == k
        K = np.zeros((n, k))
        K[:, 0] = b
        for j in range(1, k):
            K[:, j] = AP @ K[:, j - 1]
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(AP @ Q, b, rcond=None)
        best = np.linalg.norm(b - AP @ Q @ y)
        got = np.linalg.norm(b - A @ x)
        assert abs(got - best) <= 1e-10 * np.linalg.norm(b), (k, got, best)


def test_gmres_converges_within_n_steps():
    n = 12
    A = _rand_sparse(n, 0.3, 33).toarray()
    b = np.random.default_rng(34).standard_normal(n)
    res = gmres.solve(lambda v: A @ v, b, tol=1e-10, m=n, max_restarts=0)
    assert res.status == "ok" and res.iters <= n and res.cycles == 1
    assert np.linalg.norm(res.x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(res.x)


def test_two_way_transfer_identity_from_oracle_solves():
    w = make_workload(0, nshift=3)
    out = job.run(w.A, w.e, w.B, w.C, w.rounds, tol=1e-12, project=False)
    X, Y = out["rounds"][0]["X"], out["rounds"][0]["Y"]
    for i, s in enumerate(w.rounds[0]):
        H, dH = projection.full_transfer(w.A, w.e, w.B, w.C, s)
        assert abs(w.C[:, 0] @ X[:, i] - H[0, 0]) <= 1e-9 * abs(H[0, 0])
        assert abs(Y[:, i] @ w.B[:, 0] - H[0, 0]) <= 1e-9 * abs(H[0, 0])
        assert abs(-(Y[:, i] * w.e) @ X[:, i] - dH[0, 0]) <= 1e-8 * abs(dH[0, 0])


def test_storage_rounding_bits():
    one = 1.0
    cases = {
        one: one,
        one + 2.0**-8: one,                      # tie -> even mantissa (0)
        one + 3 * 2.0**-8: one + 2.0**-6,        # tie -> even mantissa (2)
        one + 2.0**-8 + 2.0**-20: one + 2.0**-7,  # just above the tie
        -(one + 3 * 2.0**-8): -(one + 2.0**-6),
        2.0 - 2.0**-9: 2.0,                      # carry into the exponent
        3.4e38: math.inf,                        # above the largest BF16 -> inf
        0.0: 0.0,
    }
    for x, want in cases.items():
        got = round_storage(np.array([x]), "bf16")[0]
        assert got == want, (x, got, want)
    assert np.isnan(round_storage(np.array([np.nan]), "bf16")[0])
    v = np.array([1.0 + 2.0**-30, 1e-40, 123456.789])
    assert np.array_equal(round_storage(v, "f32"), v.astype(np.float32).astype(np.float64))
    assert np.array_equal(round_storage(v, "f64"), v)


def test_storage_rounding_agrees_with_torch_bf16():
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(14).standard_normal(20000) * 10.0 ** np.random.default_rng(15).uniform(-30, 30, 20000)
    f32 = torch.from_numpy(v.astype(np.float32))
    ref = f32.to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(round_storage(v, "bf16"), ref)


def test_generator_laplacian_spectrum_closed_form():
    """-A of the 5-point workload has eigenvalues (4/h^2)(sin^2(i pi h/2) + sin^2(j pi h/2))."""
    N = 9
    h = 1.0 / (N + 1)
    ev = np.sort(np.linalg.eigvalsh(-laplacian_5pt(N).toarray()))
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    want = np.sort((4 / h**2) * (s[:, None] + s[None, :]).ravel())
    assert np.allclose(ev, want, rtol=1e-12)


@pytest.mark.parametrize("idx,N,nnz", [(0, 45, 5 * 45**2 - 4 * 45), (1, 12, 7 * 12**3 - 6 * 12**2),
                                        (2, 11, 7 * 11**3 - 6 * 11**2), (4, 7, (3 * 7 - 2) ** 3)])
def test_generator_stencil_nnz(idx, N, nnz):
    w = make_workload(idx, N=N)
    assert w.nnz == nnz
    # sigma E - A is an M-matrix-like operator: weakly diagonally dominant rows
    M = (1.0 * sp.diags(w.e) - w.A).tocsr()
    d = M.diagonal()
    off = np.asarray(abs(M).sum(axis=1)).ravel() - abs(d)
    assert np.all(d > 0) and np.all(d >= off * (1 - 1e-12))


def test_irka_full_order_model_gives_the_mirror_poles_in_one_round():
    """With r = n the projection keeps the whole model, so the first round's
    mirror images are -eig(A, E) of the full pencil and the second round
    finds them unchanged."""
    import scipy.linalg as sla

    rng = np.random.default_rng(21)
    n = 5
    A = sp.diags([np.full(n - 1, 1.0), -4.0 - rng.uniform(0, 1, n), np.full(n - 1, 1.0)],
                 [-1, 0, 1]).tocsr()
    e = rng.uniform(1, 2, n)
    b = rng.standard_normal(n)
    full = np.sort(-sla.eigvals(A.toarray(), np.diag(e)).real)
    res = irka.run(A, e, b, b, [0.5, 1.0, 2.0, 3.0, 7.0], max_rounds=5, tol=1e-10)
    assert res.status == "converged" and res.rounds == 2
    assert np.allclose(res.sigmas, full, rtol=1e-10, atol=0)


def test_irka_fixed_point_satisfies_the_h2_interpolation_conditions():
    """At a converged shift set of a symmetric system with c = b the reduced
    poles are real, their mirror images are the shifts, and H and H' are
    interpolated there (the first-order H2-optimality conditions)."""
    w = make_workload(2, N=6)  # variable-coefficient 7-point, symmetric, n = 216
    b = w.B[:, 0]
    res = irka.run(w.A, w.e, b, b, [1.0, 10.0, 100.0, 1000.0], max_rounds=200, tol=1e-11)
    assert res.status == "converged", (res.status, res.rounds, res.change)
    assert np.abs(res.poles.imag).max() == 0.0
    assert np.allclose(np.sort(-res.poles.real), res.sigmas, rtol=1e-9, atol=0)
    for s in res.sigmas:
        H, dH = projection.full_transfer(w.A, w.e, b, b, s)
        Hr = projection.transfer(res.Ar, res.Er, res.Br, res.Cr, s)
        dHr = projection.transfer_derivative(res.Ar, res.Er, res.Br, res.Cr, s)
        assert abs(Hr - H).max() <= 1e-8 * abs(H).max()
        assert abs(dHr - dH).max() <= 1e-7 * abs(dH).max()


def test_irka_reports_complex_reduced_poles():
    """The nonsymmetric convection-diffusion operator gives a complex pole
    pair in its first round: the loop stops there with status "complex"."""
    w = make_workload(1, N=6)
    res = irka.run(w.A, w.e, w.B[:, 0], w.C[:, 0], w.rounds[0][:6], max_rounds=5)
    assert res.status == "complex" and res.rounds == 1
    assert np.abs(res.poles.imag).max() > 0.0
