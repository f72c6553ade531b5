"""The algebra behind the normal-equations least-squares kernel, checked on
the CPU with dense matrices built from the definitions (no GPU, no library).

For column k with support J = J_k, shadow rows I = I_k and
M(s) = (s E - A)(I, J), the kernel never forms M.  It uses
* G0 = (A^T A)(J, J), which equals A(I, J)^T A(I, J) because I holds every
  row of the columns J of A;
* Ajj = A(J, J) and E_J, through
  M(s1)^T M(s2) = G0 - s2 Ajj^T E_J - s1 E_J Ajj + s1 s2 E_J^2,
  since E(I, J) has one entry E_j per column, in row J_j;
* the SPAI right-hand side M(s)^T e_k = s E_k e_a - Ajj(a, :)^T and the
  update right-hand side M(sn)^T (sp E - A)(I, k) = (M(sn)^T M(sp))(:, a),
  a being the position of k in J.
The normal-equations solution is then compared with the oracle's
least-squares columns (QR / lstsq).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pattern as opattern
from oracle import spai as ospai
from paper_2003_12759_amd.workloads import make_workload


def _cases():
    rng = np.random.default_rng(5)
    M = sp.random(60, 60, density=0.07, random_state=rng, format="csr")
    M.data = rng.standard_normal(M.nnz)
    A = (M + sp.diags(-6.0 - rng.uniform(0, 1, 60))).tolil()
    for i in range(0, 60, 7):
        A[i, i] = 0.0  # rows whose diagonal is only in the pattern
    A = A.tocsr()
    A.eliminate_zeros()
    yield "nonsym_random_n60", A, rng.uniform(1, 2, 60)
    w = make_workload(4, N=5)  # 27-point stencil, 125 rows
    yield "varcoef27_n125", w.A, w.e
    w = make_workload(1, N=5)  # 7-point upwind convection-diffusion
    yield "convdiff_n125", w.A, w.e


CASES = list(_cases())


def _dense_local(A, e, s, I, J):
    n = A.shape[0]
    Ms = (s * sp.diags(e) - A).toarray()
    return Ms[np.ix_(I, J)]


@pytest.mark.parametrize("name,A,e", CASES, ids=[c[0] for c in CASES])
def test_normal_equation_blocks_from_square_submatrices(name, A, e):
    S = opattern.pattern(A)
    Ad = A.toarray()
    AtA = Ad.T @ Ad
    s1, s2 = 2.5, 40.0
    for k in range(0, A.shape[0], 7):
        J = opattern.column_support(S, k)
        I = opattern.shadow_rows(S, J)
        # every row of the columns J of A lies in I
        rows = np.nonzero(np.abs(Ad[:, J]).sum(axis=1))[0]
        assert np.all(np.isin(rows, I))
        G0 = AtA[np.ix_(J, J)]
        Ajj = Ad[np.ix_(J, J)]
        EJ = np.diag(e[J])
        M1 = _dense_local(A, e, s1, I, J)
        M2 = _dense_local(A, e, s2, I, J)
        want = M1.T @ M2
        got = G0 - s2 * Ajj.T @ EJ - s1 * EJ @ Ajj + s1 * s2 * EJ @ EJ
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        a = int(np.nonzero(J == k)[0][0])
        ek = (I == k).astype(float)
        spai_rhs = s1 * e[k] * (np.arange(J.size) == a) - Ajj[a, :]
        assert np.abs(M1.T @ ek - spai_rhs).max() <= 1e-13 * max(1.0, np.abs(spai_rhs).max())
        col_prev = (s2 * sp.diags(e) - A).toarray()[I, k]
        assert np.abs(M1.T @ col_prev - want[:, a]).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("name,A,e", CASES, ids=[c[0] for c in CASES])
def test_normal_equation_solutions_match_oracle_columns(name, A, e):
    S = opattern.pattern(A)
    Ad = A.toarray()
    AtA = Ad.T @ Ad
    sp_, sn = 2.5, 40.0
    for k in range(0, A.shape[0], 5):
        J = opattern.column_support(S, k)
        G0 = AtA[np.ix_(J, J)]
        Ajj = Ad[np.ix_(J, J)]
        EJ = np.diag(e[J])
        a = int(np.nonzero(J == k)[0][0])

        def gram(s1, s2):
            return G0 - s2 * Ajj.T @ EJ - s1 * EJ @ Ajj + s1 * s2 * EJ @ EJ

        # SPAI column at sn
        L = np.linalg.cholesky(gram(sn, sn))
        b = sn * e[k] * (np.arange(J.size) == a) - Ajj[a, :]
        p = np.linalg.solve(L.T, np.linalg.solve(L, b))
        Jo, po = ospai.spai_column(A, e, sn, k)
        assert np.array_equal(J, Jo)
        assert np.linalg.norm(p - po) <= 1e-11 * np.linalg.norm(po)
        # update column from sp to sn
        q = np.linalg.solve(L.T, np.linalg.solve(L, gram(sn, sp_)[:, a]))
        Jo, qo = ospai.update_column(A, e, sp_, sn, k)
        assert np.linalg.norm(q - qo) <= 1e-11 * np.linalg.norm(qo)
