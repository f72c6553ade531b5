"""Pins of the MIMO (tangential) IRKA-style loop of the oracle.

The conditions checked do not come from the loop itself: tangential Hermite
interpolation (right, left and bitangential derivative) holds for any model
projected on the tangential solves, the SISO loop is the m = q = 1 case, and
a converged loop reproduces its own shifts and directions.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import irka, projection
from paper_2003_12759_amd.workloads import make_workload


def _full(A, e, B, C, s):
    """H(s) = C^T (sE - A)^{-1} B and H'(s) by sparse LU."""
    M = (s * sp.diags(e) - A).tocsc()
    lu = spla.splu(M)
    X = lu.solve(B)
    H = C.T @ X
    dH = -C.T @ lu.solve(e[:, None] * X)
    return H, dH


def _reduced(Ar, Er, Br, Cr, s):
    M = s * Er - Ar
    X = np.linalg.solve(M, Br)
    return Cr.T @ X, -Cr.T @ np.linalg.solve(M, Er @ X)


def test_tangential_loop_is_the_siso_loop_for_one_input_and_output():
    w = make_workload(2, N=6)  # symmetric 7-point, n = 216
    b = w.B[:, :1]
    sig0 = [1.0, 10.0, 100.0, 1000.0]
    siso = irka.run(w.A, w.e, b[:, 0], b[:, 0], sig0, max_rounds=30, tol=1e-9)
    tang = irka.run_tangential(w.A, w.e, b, b, sig0, np.ones((1, 4)), np.ones((1, 4)),
                               max_rounds=30, tol=1e-9)
    assert siso.status == tang.status == "converged" and siso.rounds == tang.rounds
    assert np.allclose(tang.sigmas, siso.sigmas, rtol=1e-10, atol=0)
    assert np.all(tang.bdir == 1.0) and np.all(tang.cdir == 1.0)


def test_tangential_interpolation_holds_for_every_model():
    """With v_i = (s_i E - A)^{-1} B b_i in V and w_i = (s_i E - A)^{-T} C c_i in
    W: H(s_i) b_i = Hr(s_i) b_i, c_i^T H(s_i) = c_i^T Hr(s_i) and
    c_i^T H'(s_i) b_i = c_i^T Hr'(s_i) b_i, whatever the round."""
    w = make_workload(2, N=6)
    rng = np.random.default_rng(3)
    B, C = w.B, w.C  # 4 inputs, 4 outputs, C != B: a nonsymmetric transfer function
    r = 5
    sig0 = np.geomspace(2.0, 2000.0, r)
    bd0, cd0 = rng.standard_normal((4, r)), rng.standard_normal((4, r))
    for max_rounds in (1, 2):
        res = irka.run_tangential(w.A, w.e, B, C, sig0, bd0, cd0, max_rounds=max_rounds, tol=0.0)
        if res.status == "complex":
            continue
        for i, s in enumerate(res.sigmas):
            H, dH = _full(w.A, w.e, B, C, s)
            Hr, dHr = _reduced(res.Ar, res.Er, res.Br, res.Cr, s)
            b, c = res.bdir[:, i], res.cdir[:, i]
            assert np.allclose(Hr @ b, H @ b, rtol=1e-8, atol=1e-10 * abs(H).max())
            assert np.allclose(c @ Hr, c @ H, rtol=1e-8, atol=1e-10 * abs(H).max())
            assert abs(c @ dHr @ b - c @ dH @ b) <= 1e-7 * abs(dH).max()


def test_converged_loop_reproduces_its_shifts_and_directions():
    """Symmetric A, E and C = B give real poles; at convergence the next
    shifts and directions from the returned model equal the returned ones."""
    w = make_workload(2, N=6)
    rng = np.random.default_rng(5)
    r = 4
    d0 = rng.standard_normal((4, r))  # equal left and right directions keep W = V
    res = irka.run_tangential(w.A, w.e, w.B, w.B, np.geomspace(1.0, 5000.0, r), d0, d0,
                              max_rounds=100, tol=1e-9)
    assert res.status == "converged", (res.status, res.rounds, res.change)
    _, sig, bd, cd = irka.tangent_directions(res.Ar, res.Er, res.Br, res.Cr)
    assert np.allclose(sig, res.sigmas, rtol=1e-9, atol=0)
    assert np.allclose(bd, res.bdir, atol=1e-7) and np.allclose(cd, res.cdir, atol=1e-7)
    # and the bitangential H2 conditions hold there
    for i, s in enumerate(res.sigmas):
        H, dH = _full(w.A, w.e, w.B, w.B, s)
        Hr, dHr = _reduced(res.Ar, res.Er, res.Br, res.Cr, s)
        b, c = res.bdir[:, i], res.cdir[:, i]
        assert np.allclose(Hr @ b, H @ b, rtol=1e-8, atol=1e-10 * abs(H).max())
        assert abs(c @ dHr @ b - c @ dH @ b) <= 1e-7 * abs(dH).max()


def test_directions_are_the_residue_directions_of_the_reduced_model():
    """Hr(s) = sum_i c_i b_i^T / (s - lambda_i) with rank-one residues: the
    residue at lambda_i, taken as eps Hr(lambda_i + eps), has the right
    singular vector b_i and the left singular vector c_i (up to sign and
    scale), independently of any eigenvector routine."""
    rng = np.random.default_rng(9)
    r, m, q = 5, 3, 2
    lam = -np.array([0.5, 1.3, 2.0, 4.5, 9.0])
    S = rng.standard_normal((r, r)) + 3 * np.eye(r)
    Er = rng.standard_normal((r, r)) + 4 * np.eye(r)
    Ar = Er @ S @ np.diag(lam) @ np.linalg.inv(S)  # Er^{-1} Ar = S diag(lam) S^{-1}
    Br, Cr = rng.standard_normal((r, m)), rng.standard_normal((r, q))
    poles, sig, bd, cd = irka.tangent_directions(Ar, Er, Br, Cr)
    assert np.allclose(sig, -lam, rtol=1e-10)
    for i, s in enumerate(sig):
        l = -s
        eps = 1e-7 * abs(l)
        R = eps * (Cr.T @ np.linalg.solve((l + eps) * Er - Ar, Br))  # q x m
        U, sv, Vt = np.linalg.svd(R)
        assert sv[1] <= 1e-5 * sv[0]  # rank one
        assert np.allclose(irka._unit(Vt[0]), bd[:, i], atol=1e-5)
        assert np.allclose(irka._unit(U[:, 0]), cd[:, i], atol=1e-5)
