"""Elementwise parity of the solve's own product kernels, and bit-exact
parity of the factor schedules, through the C ABI.

The chain step (``k_chain_halo`` 8- and 32-slot, ``k_chain_narrow``,
``k_chain_step``) and the shifted pair (the halo chain kernel's shifted-pair
pass, ``k_spmv_pair``) are run by ``morx_chain_apply_batch`` /
``morx_shifted_apply_pair``, which launch them with the work lists, tile
widths and row blocks of a solve.  Factors are
imported from seeded random values on the pattern S (the same values, rounded
by the oracle's storage rounding, feed ``oracle.chain.apply``), so both sides
apply the same operator.

Bounds (elementwise, from the FP64 dot-product error of rows of at most 32
terms, gamma = 32 u, on each side):
* FP64 apply: pass k adds |F_k| B_{k-1} + 2 gamma |F_k| |t_{k-1}| to the bound
  B_{k-1} of its input (t the oracle's intermediates);
* FP32 apply: each pass result is rounded to FP32 on both sides, so values
  whose FP64 sums differ by d round to values that differ by at most
  d + 2^-23 |t_k|; the bound adds that one FP32 ulp per pass.
Halo and gather kernels sum every row's slots in the same order, so their
outputs are compared bit for bit.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import chain as ochain
from oracle import pattern as opattern
from oracle import spai as ospai
from oracle.precision import round_storage
from paper_2003_12759_amd.workloads import make_workload

pytestmark = pytest.mark.gpu

U = 2.0**-53
GAMMA = 32 * U * 1.01


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _rand_wide(n, seed):
    """Nonsymmetric pattern with rows of about 11 entries (no halo-narrow)."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=10.0 / n, random_state=rng, format="csr")
    M.data = rng.standard_normal(M.nnz)
    M = (M + sp.diags(-12.0 - rng.uniform(0, 1, n))).tocsr()
    M.sort_indices()
    return M


# 27-point grid of 1331 rows (21 slices: a last block of one partial slice),
# a 27-point grid of 32,768 rows, the 7-point convection-diffusion operator
# (rows <= 8: the narrow kernels), and a random pattern with rows of ~11
# entries
CASES = {
    "varcoef27_n1331": lambda: (make_workload(4, N=11).A, make_workload(4, N=11).e),
    # 32^3: 128 row blocks, a grid plane every 4: the halo kernels walk row
    # blocks a plane apart
    "varcoef27_n32768": lambda: (make_workload(4, N=32).A, make_workload(4, N=32).e),
    "convdiff_n1331": lambda: (make_workload(1, N=11).A, make_workload(1, N=11).e),
    "randwide_n1000": lambda: (_rand_wide(1000, 5), np.random.default_rng(6).uniform(1, 2, 1000)),
}


def _dev_block(X):
    return torch.as_tensor(np.ascontiguousarray(X.T), device="cuda").t()


def _colmajor(n, m):
    from paper_2003_12759_amd import morx

    return morx.colmajor(m, n)


def _random_factor_values(S, rng):
    """Random factor values on the CSR pattern of S, scaled so that chains of
    a dozen factors stay O(1)."""
    v = rng.standard_normal(S.nnz)
    rows = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    diag = S.indices == rows
    v[diag] += 3.0
    return v / 3.5


def _import(S_handle, vals, prec):
    from paper_2003_12759_amd import morx

    return morx.morx_factor_import(S_handle, torch.as_tensor(vals, device="cuda"), prec)


def _oracle_factor(Scsr, vals, prec):
    return sp.csr_matrix((round_storage(vals, prec), Scsr.indices, Scsr.indptr), shape=Scsr.shape)


class _OracleFactors:
    """The oracle's factors (rounded like the stored values), their
    transposes and elementwise absolute values."""

    def __init__(self, mats):
        self.F = mats
        self.FT = [m.T.tocsr() for m in mats]
        self.aF = [abs(m) for m in mats]
        self.aFT = [abs(m) for m in self.FT]


def _bound(of, chain, x, apply, trans):
    """The oracle's chain product of one column and an elementwise bound on
    |GPU - oracle| (see the module docstring)."""
    t = ochain._to_apply(np.asarray(x, dtype=np.float64), apply)
    B = np.zeros_like(t)
    order = list(reversed(chain)) if trans else list(chain)
    for f in order:
        F, aF = (of.FT[f], of.aFT[f]) if trans else (of.F[f], of.aF[f])
        s = F @ t
        B = aF @ B + 2.0 * GAMMA * (aF @ np.abs(t))
        t = ochain._to_apply(s, apply)
        if apply == "f32":
            B = B + 2.0**-23 * (1.01 * np.abs(t) + B)
    ref = (ochain.apply_transpose if trans else ochain.apply)(of.F, chain, x, apply)
    assert np.array_equal(ref, t)
    return ref, B


def _system(ctx, name):
    from paper_2003_12759_amd import api

    A, e = CASES[name]()
    S = api.System(ctx, A, e)
    Sref = opattern.pattern(A).tocsr()
    Sref.sort_indices()
    return A, e, S, Sref


def test_factor_import_rounds_like_the_oracle(ctx):
    """Imported values are stored exactly as the oracle rounds them, in both
    orders (the transposed order checked through a one-factor transposed
    apply of unit vectors)."""
    from paper_2003_12759_amd import morx

    A, e, S, Sref = _system(ctx, "varcoef27_n1331")
    rng = np.random.default_rng(11)
    vals = _random_factor_values(Sref, rng)
    vals[:5] = [1.0 + 2.0**-24, 1.0 + 3 * 2.0**-24, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -0.0]
    for prec in ("f64", "f32", "bf16"):
        _say(f"import {prec}")
        f = _import(S.handle, vals, prec)
        got = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
        morx.morx_factor_values(f, got)
        want = round_storage(vals, prec)
        assert np.array_equal(got.cpu().numpy().view(np.uint64), want.view(np.uint64))
        # transposed order: F^T e_j is row j of F
        n = A.shape[0]
        cols = [0, 7, n // 2, n - 1]
        X = np.zeros((n, len(cols)))
        for c, j in enumerate(cols):
            X[j, c] = 1.0
        Yt = _colmajor(n, len(cols))
        morx.morx_chain_apply_batch(S.handle, [[f]] * len(cols), None, None, _dev_block(X), Yt)
        F = _oracle_factor(Sref, vals, prec)
        for c, j in enumerate(cols):
            assert np.array_equal(Yt[:, c].cpu().numpy(), F.getrow(j).toarray().ravel())
        morx.morx_factor_destroy(f)
    S.close()


# (columns, cols_per_wave): chain tiles 1, 2, 3, 4, 6, 8, 10, 12, 16
TILES = [(16, 1), (16, 2), (16, 3), (16, 4), (16, 6), (16, 8), (10, 16), (12, 12), (16, 16)]


def _chain_case(ctx, name, prec, apply, kernel, ncol, ncmax, shared, seed=21):
    from paper_2003_12759_amd import morx

    A, e, S, Sref = _system(ctx, name)
    try:
        S.set_tune(cols_per_wave=ncmax, chain_kernel=kernel)
    except morx.MorxError:
        S.close()
        return None
    n = A.shape[0]
    rng = np.random.default_rng(seed)
    nf = 12
    vals = [_random_factor_values(Sref, rng) for _ in range(nf + ncol)]
    handles = [_import(S.handle, v, prec) for v in vals]
    oracle_f = _OracleFactors([_oracle_factor(Sref, v, prec) for v in vals])
    if shared:
        # Algorithm 4's batch: prefixes of one factor list, lengths 1..12
        chains = [list(range(1 + c % nf)) for c in range(ncol)]
    else:
        # every column its own chain (Table 2's first approach, serving)
        chains = [[0, nf + c] if c % 3 else [nf + c] for c in range(ncol)]
    X = rng.standard_normal((n, ncol))
    Xt = rng.standard_normal((n, ncol))
    Y, Yt = _colmajor(n, ncol), _colmajor(n, ncol)
    morx.morx_chain_apply_batch(S.handle, [[handles[k] for k in ch] for ch in chains],
                                _dev_block(X), Y, _dev_block(Xt), Yt, apply=apply)
    got, gott = Y.cpu().numpy(), Yt.cpu().numpy()
    for c, ch in enumerate(chains):
        ref, B = _bound(oracle_f, ch, X[:, c], apply, False)
        assert np.all(np.abs(got[:, c] - ref) <= B + 1e-300), \
            (c, len(ch), np.max(np.abs(got[:, c] - ref) / (B + 1e-300)))
        reft, Bt = _bound(oracle_f, ch, Xt[:, c], apply, True)
        assert np.all(np.abs(gott[:, c] - reft) <= Bt + 1e-300), \
            (c, len(ch), np.max(np.abs(gott[:, c] - reft) / (Bt + 1e-300)))
    for h in handles:
        morx.morx_factor_destroy(h)
    S.close()
    return got, gott


@pytest.mark.parametrize("ncol,ncmax", TILES)
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_chain_kernels_match_oracle_elementwise(ctx, name, kernel, ncol, ncmax):
    """Chains of 1..12 shared factors (forward and transposed at once), FP64
    storage and apply, every tile width, both chain kernels."""
    _say(f"chain {name} kernel={kernel} ncol={ncol} ncmax={ncmax}")
    if name == "varcoef27_n32768" and kernel == 1:
        from paper_2003_12759_amd import api

        A, e = CASES[name]()
        S = api.System(ctx, A, e)
        assert S.get_tune()["halo_stride"] == 4  # a 32 x 32 plane is 4 row blocks
        S.close()
    if _chain_case(ctx, name, "f64", "f64", kernel, ncol, ncmax, True) is None:
        pytest.skip(f"{name} has no halo layout")


@pytest.mark.parametrize("shared", [True, False])
@pytest.mark.parametrize("prec,apply", [("f32", "f64"), ("bf16", "f64"), ("f64", "f32"),
                                        ("f32", "f32"), ("bf16", "f32")])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_chain_kernels_storage_and_apply_precisions(ctx, name, kernel, prec, apply, shared):
    """FP32/BF16 storage widened on load, the FP32 apply, and chunks whose
    columns apply different factors."""
    _say(f"chain {name} kernel={kernel} prec={prec} apply={apply} shared={shared}")
    if _chain_case(ctx, name, prec, apply, kernel, 12, 6, shared) is None:
        pytest.skip(f"{name} has no halo layout")


@pytest.mark.parametrize("shared", [True, False])
@pytest.mark.parametrize("prec,apply", [("f64", "f64"), ("bf16", "f64"), ("f32", "f32")])
@pytest.mark.parametrize("ncol,ncmax", [(16, 2), (12, 12), (16, 16)])
@pytest.mark.parametrize("name", list(CASES))
def test_halo_equals_gather_bitwise(ctx, name, ncol, ncmax, prec, apply, shared):
    """The halo kernels sum each row's slots in the gather kernels' order."""
    _say(f"halo == gather {name} ncol={ncol} ncmax={ncmax} {prec}/{apply} shared={shared}")
    r0 = _chain_case(ctx, name, prec, apply, 0, ncol, ncmax, shared, seed=31)
    r1 = _chain_case(ctx, name, prec, apply, 1, ncol, ncmax, shared, seed=31)
    if r1 is None:
        pytest.skip(f"{name} has no halo layout")
    assert np.array_equal(r0[0], r1[0]) and np.array_equal(r0[1], r1[1])


def test_chain_apply_single_chain_entry(ctx):
    """morx_chain_apply (one chain for every column, one direction at a
    time) against the oracle, on imported factors."""
    from paper_2003_12759_amd import morx

    A, e, S, Sref = _system(ctx, "convdiff_n1331")
    n = A.shape[0]
    rng = np.random.default_rng(4)
    vals = [_random_factor_values(Sref, rng) for _ in range(3)]
    fs = [_import(S.handle, v, "f64") for v in vals]
    refs = _OracleFactors([_oracle_factor(Sref, v, "f64") for v in vals])
    X = rng.standard_normal((n, 3))
    for trans in (0, 1):
        _say(f"chain_apply trans={trans}")
        Yd = _colmajor(n, 3)
        morx.morx_chain_apply(S.handle, fs, trans, _dev_block(X), Yd)
        got = Yd.cpu().numpy()
        for j in range(3):
            ref, B = _bound(refs, [0, 1, 2], X[:, j], "f64", bool(trans))
            assert np.all(np.abs(got[:, j] - ref) <= B + 1e-300)
    for f in fs:
        morx.morx_factor_destroy(f)
    S.close()


SPMV_CASES = dict(CASES, laplace2d_n2025=lambda: (make_workload(0).A, make_workload(0).e))


@pytest.mark.parametrize("ncs", [1, 2, 4, 8])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", list(SPMV_CASES))
def test_shifted_pair_matches_oracle_elementwise(ctx, name, kernel, ncs):
    """q = (s E - A) p and q~ = (s E - A)^T p~ in one launch, per-column
    shifts, against the oracle's sparse products (|M| |x| bound); halo and
    gather kernels bit for bit."""
    from paper_2003_12759_amd import api, morx

    A, e = SPMV_CASES[name]()
    S = api.System(ctx, A, e)
    n = A.shape[0]
    ncol = 7
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, ncol))
    Xt = rng.standard_normal((n, ncol))
    sig = [0.0, 3.7, 1e3, 0.25, 12.0, 1.0, 77.0]
    outs = []
    for kern in (0, kernel):
        try:
            S.set_tune(spmv_cols_per_wave=ncs, chain_kernel=kern)
        except morx.MorxError:
            S.close()
            pytest.skip(f"{name} has no halo layout")
        _say(f"shifted pair {name} kernel={kern} ncs={ncs}")
        Y, Yt = _colmajor(n, ncol), _colmajor(n, ncol)
        morx.morx_shifted_apply_pair(S.handle, sig, _dev_block(X), Y, _dev_block(Xt), Yt)
        got, gott = Y.cpu().numpy(), Yt.cpu().numpy()
        for c, s in enumerate(sig):
            M = (s * sp.diags(e) - A).tocsr()
            for G, V, MM in ((got, X, M), (gott, Xt, M.T.tocsr())):
                ref = MM @ V[:, c]
                bound = 2.0 * GAMMA * (abs(MM) @ np.abs(V[:, c])) + 1e-300
                assert np.all(np.abs(G[:, c] - ref) <= bound), np.max(np.abs(G[:, c] - ref) / bound)
        outs.append((got, gott))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    S.close()


def _specs_of(specs, idx):
    return [specs[k] for k in idx]


@pytest.mark.parametrize("batched", [True, False])
def test_gpu_schedule_equals_algorithm4_over_three_rounds(ctx, batched):
    """The factor chains the solves ran with, spec by spec and bit for bit,
    against the oracle's Algorithm 4 schedule (RESET then NEXT_ROUND twice:
    horizontal chains, and the vertical link between first shifts)."""
    from paper_2003_12759_amd import api, morx

    w = make_workload(1, N=8, nshift=5, nrounds=3)
    S = api.System(ctx, w.A, w.e)
    specs, chains = ochain.schedule(w.rounds)
    for z, sig in enumerate(w.rounds):
        _say(f"schedule round {z} batched={batched}")
        S.solve_shifts(sig, w.B, w.C, prec="f32", next_round=z > 0, batched=batched)
        got = morx.morx_last_chains(S.handle)
        assert got == [_specs_of(specs, ch) for ch in chains[z]]
        for i, ch in enumerate(got):
            assert len(ch) == i + z + 1  # i + z - 1 with one-based i and z
    # a RESET call starts a new vertical chain
    S.solve_shifts(w.rounds[1], w.B, w.C, prec="f32", next_round=False, batched=batched)
    specs2, chains2 = ochain.schedule(w.rounds[1:2])
    assert morx.morx_last_chains(S.handle) == [_specs_of(specs2, ch) for ch in chains2[0]]
    S.close()


@pytest.mark.parametrize("policy", ["direct", "first"])
def test_gpu_schedule_equals_comparator_schedules(ctx, policy):
    from paper_2003_12759_amd import api, morx

    w = make_workload(1, N=8, nshift=5, nrounds=2)
    S = api.System(ctx, w.A, w.e)
    sched = ochain.schedule_direct if policy == "direct" else ochain.schedule_first
    for z, sig in enumerate(w.rounds):
        _say(f"schedule {policy} round {z}")
        S.solve_shifts(sig, w.B, w.C, prec="f32", policy=policy)
        specs, chains = sched([sig])
        assert morx.morx_last_chains(S.handle) == [_specs_of(specs, ch) for ch in chains[0]]
    # the GMRES comparator plans its chains the same way
    S.gmres_shifts(w.rounds[0], w.B, w.C, restart=20, prec="f32", policy=policy)
    specs, chains = sched(w.rounds[:1])
    assert morx.morx_last_chains(S.handle) == [_specs_of(specs, ch) for ch in chains[0]]
    S.close()


def test_factor_build_many_jobs_match_oracle(ctx):
    """Several shifts in one launch of the normal-equations kernel (so the
    two-wave blocks' second lane groups carry jobs 2 and 3), every column of
    every job against the oracle's least squares."""
    from paper_2003_12759_amd import api, morx

    w = make_workload(4, N=7)
    S = api.System(ctx, w.A, w.e)
    S.set_tune(factor_kernel=2)
    specs = [("spai", 2.5), ("update", 2.5, 40.0), ("update", 40.0, 0.3), ("update", 0.3, 7.0),
             ("spai", 900.0), ("update", 7.0, 7.5)]
    rp, ci = S.pattern()
    for prec in ("f64", "f32", "bf16"):
        _say(f"factor_build {len(specs)} jobs {prec}")
        fs = morx.morx_factor_build(S.handle, specs, prec)
        for f, spc in zip(fs, specs):
            ref = ospai.spai(w.A, w.e, spc[1]) if spc[0] == "spai" else \
                ospai.update(w.A, w.e, spc[1], spc[2])
            vals = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
            morx.morx_factor_values(f, vals)
            got = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=w.A.shape).tocsc()
            want = ref.tocsc()
            want.sort_indices()
            got.sort_indices()
            if prec == "f64":
                D = got - want
                colerr = np.sqrt(np.asarray(D.multiply(D).sum(axis=0))).ravel()
                colnorm = np.sqrt(np.asarray(want.multiply(want).sum(axis=0))).ravel()
                assert np.all(colerr <= 1e-11 * colnorm), (spc, np.max(colerr / colnorm))
            else:
                g = got.toarray()
                wd = want.toarray()
                wr = round_storage(wd, prec)
                # one storage step, plus the columns' FP64 difference (1e-11 of
                # the column norm), which can move a small entry's rounding
                ulp = np.abs(wr) * (2.0**-23 if prec == "f32" else 2.0**-7) + \
                    1e-11 * np.linalg.norm(wd, axis=0)[None, :]
                assert np.all(np.abs(g - wr) <= ulp), spc
            morx.morx_factor_destroy(f)
    S.close()


def test_normal_equations_fallback_on_a_late_job_of_a_wide_column(ctx):
    """A dense 20 x 20 system (|J_k| = 20: 32-lane groups; the groups of jobs
    2 and 3 lie on a block's second wave).
    With A = 2 I - B, the shifted matrix s I - A = (s - 2) I + B, where B is
    symmetric positive definite with eigenvalues 5e-4 and 1..5 and the
    eigenvector of 5e-4 is (e_0 - e_1)/sqrt(2): columns 0 and 1 of B nearly
    coincide.  Only at s = 2, the shift of jobs 2 and 3, is the local problem
    ill conditioned (condition number 1e4; the normal equations' second
    pivot falls to ~1e-7 of its diagonal).  Every column must be rebuilt by
    the Householder kernel, which matches the oracle to 1e-11; the normal
    equations alone would lose ~1e-8."""
    from paper_2003_12759_amd import api, morx

    rng = np.random.default_rng(9)
    n = 20
    G0 = rng.standard_normal((n, n))
    G0[:, 0] = 0.0
    G0[0, 0], G0[1, 0] = 1.0, -1.0
    Q, _ = np.linalg.qr(G0)
    Bm = (Q * np.concatenate([[5e-4], np.linspace(1.0, 5.0, n - 1)])) @ Q.T
    Ad = 2.0 * np.eye(n) - Bm
    A = sp.csr_matrix(Ad)
    e = np.ones(n)
    S = api.System(ctx, A, e)
    S.set_tune(factor_kernel=2)
    specs = [("spai", 3.0), ("update", 3.0, 5.0), ("spai", 2.0), ("update", 7.0, 2.0),
             ("update", 5.0, 7.0)]
    _say("normal equations fallback on jobs 2 and 3 of a 20-wide pattern")
    fs = morx.morx_factor_build(S.handle, specs, "f64")
    rp, ci = S.pattern()
    for f, spc in zip(fs, specs):
        ref = (ospai.spai(A, e, spc[1]) if spc[0] == "spai" else
               ospai.update(A, e, spc[1], spc[2])).toarray()
        vals = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
        morx.morx_factor_values(f, vals)
        got = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=A.shape).toarray()
        for k in range(n):
            assert np.linalg.norm(got[:, k] - ref[:, k]) <= 1e-11 * np.linalg.norm(ref[:, k]), \
                (spc, k, np.linalg.norm(got[:, k] - ref[:, k]) / np.linalg.norm(ref[:, k]))
        morx.morx_factor_destroy(f)
    # the full pattern makes the SPAI at the bad shift the exact inverse of B
    exact = np.linalg.inv(Bm)
    assert np.linalg.norm(ospai.spai(A, e, 2.0).toarray() - exact) <= 1e-9 * np.linalg.norm(exact)
    S.close()
