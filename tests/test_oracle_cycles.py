"""Pins of the oracle's cycle compositions against dense error operators.

Algorithm 1 (Section 3.1) with nu recursive calls, the "1 V-cycle / 2
V-cycles" preconditioners of Section 4.4 (reading R17: successive cycles,
the second from the first's result), the saddle point cycle with the sGS,
Braess-Sarazin and Vanka smoothers of Section 3.3, and the restart path of
flexible GMRES. Every expected operator is built here from dense matrices
(triangular solves, explicit inverses, Galerkin products P^T K P), not from
the oracle's own cycle code.
"""
import numpy as np
import pytest

from oracle import amg, krylov, workloads


def _dense_operator(apply, n):
    return np.stack([np.asarray(apply(e)).ravel() for e in np.eye(n)], axis=1)


def _block_id(n_nodes):
    return np.arange(3 * n_nodes) // 3


def _perm_triangular(A, order, lower):
    """Block lower (upper) triangle, diagonal blocks included, of A in the
    node order ``order``: returned in the original numbering."""
    n = A.shape[0] // 3
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    r = rank[_block_id(n)]
    keep = (r[:, None] >= r[None, :]) if lower else (r[:, None] <= r[None, :])
    return np.where(keep, A, 0.0)


def _smoother_error(lev, sm, A, pre):
    """Error operator of one SPD smoothing step: Gauss-Seidel sweeps are
    triangular solves in the colour order (forward: ascending, backward:
    descending), Jacobi is I - omega D^{-1} A with the 3x3 diagonal blocks."""
    n = A.shape[0]
    if sm.kind == "GS":
        forward = pre or sm.post_forward
        T = _perm_triangular(A, lev.order_fwd, lower=forward)
        return np.eye(n) - np.linalg.solve(T, A)
    blk = _block_id(n // 3)
    D = np.where(blk[:, None] == blk[None, :], A, 0.0)
    return np.eye(n) - sm.omega * np.linalg.solve(D, A)


def _spd_cycle_error(h, sm, l, nu):
    """E_l = S_post^m (I - P M_{l+1} P^T A_l) S_pre^m with M_{l+1} the
    approximate coarse inverse that nu successive cycles from zero give:
    (I - E_{l+1}^nu) A_{l+1}^{-1}, and the exact inverse on the coarsest level."""
    lev = h.levels[l]
    A = lev.A.dense()
    n = A.shape[0]
    Pk = np.kron(lev.P.toarray(), np.eye(3))
    Ac = Pk.T @ A @ Pk
    if l + 1 == h.L:
        Mc = np.linalg.inv(Ac)
    else:
        Ec = _spd_cycle_error(h, sm, l + 1, nu)
        Mc = (np.eye(Ac.shape[0]) - np.linalg.matrix_power(Ec, nu)) @ np.linalg.inv(Ac)
    Spre = np.linalg.matrix_power(_smoother_error(lev, sm, A, True), sm.pre)
    Spost = np.linalg.matrix_power(_smoother_error(lev, sm, A, False), sm.post)
    return Spost @ (np.eye(n) - Pk @ Mc @ Pk.T @ A) @ Spre


@pytest.fixture(scope="module")
def three_level():
    s = workloads.elasticity(3)
    h = amg.setup(s.A, s.nlin, s.nquad, coarse_max=30)
    assert h.L == 2
    return s, h


@pytest.mark.parametrize("name,nu", [("GS-1-1", 2), ("GS-1-1", 1), ("JA-2-2-0.5", 2), ("GS-2-2", 2)])
def test_cycle_error_operator_three_levels(three_level, name, nu):
    """Algorithm 1 from zero on three levels: the preconditioner's matrix M
    satisfies I - M A = E_0 for the recursively defined dense E_l, for the
    V-cycle (nu = 1) and the W-cycle (nu = 2)."""
    s, h = three_level
    sm = amg.Smoother.parse(name)
    A = s.A.dense()
    Mi = _dense_operator(amg.preconditioner(h, sm, nu=nu), A.shape[0])
    E = _spd_cycle_error(h, sm, 0, nu)
    assert np.abs(np.eye(A.shape[0]) - Mi @ A - E).max() < 1e-10
    if nu == 2:
        # the W-cycle is a different operator from the V-cycle
        E1 = _spd_cycle_error(h, sm, 0, 1)
        assert np.abs(E - E1).max() > 1e-3


def test_w_cycle_from_nonzero_guess(three_level):
    """One cycle from an arbitrary x: x_new - x* = E_0 (x - x*)."""
    s, h = three_level
    sm = amg.Smoother.parse("GS-1-1")
    A = s.A.dense()
    rng = np.random.default_rng(11)
    b = rng.standard_normal(A.shape[0])
    x = rng.standard_normal(A.shape[0])
    xs = np.linalg.solve(A, b)
    got = amg.cycle(h, 0, sm, b.reshape(-1, 3), x.reshape(-1, 3), nu=2).ravel()
    E = _spd_cycle_error(h, sm, 0, 2)
    assert np.abs(got - (xs + E @ (x - xs))).max() < 1e-10 * np.abs(xs).max()


@pytest.mark.parametrize("name", ["GS-1-1", "JA-1-1-0.5"])
def test_two_successive_cycles_square_the_error(three_level, name):
    """Reading R17: "2 V-cycles" per preconditioner application are two
    successive cycles, the second from the first's result, so the error
    operator is the square of one cycle's: I - M_2 A = (I - M_1 A)^2."""
    s, h = three_level
    sm = amg.Smoother.parse(name)
    A = s.A.dense()
    n = A.shape[0]
    E1 = np.eye(n) - _dense_operator(amg.preconditioner(h, sm, cycles=1), n) @ A
    E2 = np.eye(n) - _dense_operator(amg.preconditioner(h, sm, cycles=2), n) @ A
    assert np.abs(E2 - E1 @ E1).max() < 1e-10
    assert np.abs(E2 - _spd_cycle_error(h, sm, 0, 1) @ _spd_cycle_error(h, sm, 0, 1)).max() < 1e-10


# ---------------------------------------------------------------- saddle
def _saddle_dense(lev):
    A, B = lev.A.dense(), lev.B.dense()
    C = lev.C.dense() if lev.C is not None else np.zeros((B.shape[0], B.shape[0]))
    return A, B, C, np.block([[A, B.T], [B, -C]])


def _saddle_smoother_error(lev, sm, schur_inv=None):
    """I - K_hat^{-1} K of one step, K_hat written out from Section 3.3:
    sGS: [[M_A, 0], [B, -omega^{-1} S_d]] (M_A = D_b / damping, reading R14);
    Braess-Sarazin: [[A_hat, B^T], [B, B A_hat^{-1} B^T - S_hat]], A_hat = 2 diag(A);
    Vanka: the product over patches of (I - omega R_i^T K_i^{-1} R_i K)."""
    A, B, C, K = _saddle_dense(lev)
    nv, npr = A.shape[0], B.shape[0]
    nd = nv + npr
    if sm.kind == "SGS":
        blk = _block_id(nv // 3)
        D = np.where(blk[:, None] == blk[None, :], A, 0.0)
        MA_inv = sm.sgs_damping * np.linalg.inv(D)
        Sd = np.diag(np.diag(B @ MA_inv @ B.T + C)) if sm.sgs_scaled else np.eye(npr)
        Khat = np.block([[np.linalg.inv(MA_inv), np.zeros((nv, npr))], [B, -Sd / sm.sgs_omega]])
        return np.eye(nd) - np.linalg.solve(Khat, K)
    if sm.kind == "BS":
        Ahat = np.diag(2.0 * np.diag(A))
        Shat = np.linalg.inv(schur_inv)
        Khat = np.block([[Ahat, B.T], [B, B @ np.linalg.solve(Ahat, B.T) - Shat]])
        return np.eye(nd) - np.linalg.solve(Khat, K)
    assert sm.kind == "VANKA"
    V = amg.vanka_patches(lev)
    E = np.eye(nd)
    for i in V.order:
        idx = V.dofs[i]
        R = np.zeros((idx.size, nd))
        R[np.arange(idx.size), idx] = 1.0
        E = (np.eye(nd) - sm.omega * R.T @ np.linalg.solve(K[np.ix_(idx, idx)], R @ K)) @ E
    return E


def _saddle_prolongation(lev):
    """diag(P (x) I_3, H): velocity nodes by P, pressures by H (reading R6)."""
    Pk = np.kron(lev.P.toarray(), np.eye(3))
    H = lev.H.toarray()
    top = np.hstack([Pk, np.zeros((Pk.shape[0], H.shape[1]))])
    bot = np.hstack([np.zeros((H.shape[0], Pk.shape[1])), H])
    return np.vstack([top, bot])


def _saddle_cycle_error(h, sm, l, nu, schur_inv=None):
    lev = h.levels[l]
    _, _, _, K = _saddle_dense(lev)
    nd = K.shape[0]
    P = _saddle_prolongation(lev)
    Kc = P.T @ K @ P
    if l + 1 == h.L:
        Mc = np.linalg.inv(Kc)
    else:
        Ec = _saddle_cycle_error(h, sm, l + 1, nu, None if schur_inv is None else schur_inv[1:])
        Mc = (np.eye(Kc.shape[0]) - np.linalg.matrix_power(Ec, nu)) @ np.linalg.inv(Kc)
    S = _saddle_smoother_error(lev, sm, None if schur_inv is None else schur_inv[0])
    return (np.linalg.matrix_power(S, sm.post) @ (np.eye(nd) - P @ Mc @ P.T @ K)
            @ np.linalg.matrix_power(S, sm.pre))


@pytest.fixture(scope="module")
def saddle_two_level():
    s = workloads.mixed_elasticity(2, nu=0.3)
    h = amg.setup(s.A, s.nlin, s.nquad, B=s.B, C=s.C, singular=s.singular, coarse_max=100)
    assert h.L == 1
    return s, h


@pytest.mark.parametrize("name", ["sGS-1-1", "sGS-2-2", "sGS-1-1:literal", "BS-1-1", "Vanka-1-1"])
def test_saddle_two_level_error_operator(saddle_two_level, name):
    """The saddle V-cycle (Algorithm 1 on K = [[A, B^T], [B, -C]]) from zero
    on two levels: I - M K = S^m_post (I - P K_c^{-1} P^T K) S^m_pre with
    P = diag(P (x) I_3, H), K_c = P^T K P (dense) and S the dense error
    operator of the smoothing step."""
    s, h = saddle_two_level
    sm = amg.Smoother.parse(name.split(":")[0])
    sm.sgs_scaled = not name.endswith(":literal")
    schur_inv = None
    if sm.kind == "BS":
        amg.prepare_bs(h)
        npr = h.levels[0].npres
        schur_inv = [_dense_operator(lambda e: amg.scalar_vcycle(h.levels[0].schur, 0, e, np.zeros(npr)), npr)]
    _, _, _, K = _saddle_dense(h.levels[0])
    nd = K.shape[0]
    Mi = _dense_operator(amg.preconditioner(h, sm), nd)
    E = _saddle_cycle_error(h, sm, 0, 1, schur_inv)
    assert np.abs(np.eye(nd) - Mi @ K - E).max() < 1e-9 * max(1.0, np.abs(E).max())
    # and E is a contraction of the error in this setting
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0


def test_saddle_w_cycle_three_levels_and_two_cycles():
    """sGS saddle cycle on three levels with nu = 2, and "2 V-cycles" as the
    square of one cycle's error operator."""
    s = workloads.mixed_elasticity(3, nu=0.3)
    h = amg.setup(s.A, s.nlin, s.nquad, B=s.B, C=s.C, singular=s.singular, coarse_max=100)
    assert h.L == 2
    sm = amg.Smoother.parse("sGS-1-1")
    _, _, _, K = _saddle_dense(h.levels[0])
    nd = K.shape[0]
    Mw = _dense_operator(amg.preconditioner(h, sm, nu=2), nd)
    Ew = _saddle_cycle_error(h, sm, 0, 2)
    assert np.abs(np.eye(nd) - Mw @ K - Ew).max() < 1e-9 * max(1.0, np.abs(Ew).max())
    Ev = _saddle_cycle_error(h, sm, 0, 1)
    M2 = _dense_operator(amg.preconditioner(h, sm, cycles=2), nd)
    assert np.abs(np.eye(nd) - M2 @ K - Ev @ Ev).max() < 1e-9 * max(1.0, np.abs(Ev).max())


# ---------------------------------------------------------------- restarted GMRES
def _min_residual_step(A, r, k, Mp=None):
    """argmin over y in M K_k(A M, r) of ||r - A y||, by dense least squares."""
    Mp = np.eye(A.shape[0]) if Mp is None else Mp
    AM = A @ Mp
    K = np.stack([np.linalg.matrix_power(AM, j) @ r for j in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(AM @ Q, r, rcond=None)[0]
    return Mp @ Q @ c


@pytest.mark.parametrize("precond", [False, True])
def test_restarted_gmres_cycles_are_dense_minimisers(precond):
    """GMRES(m) restarts from x_m with the residual r_m: iterate m + k is
    x_m + argmin ||r_m - A y|| over M K_k(A M, r_m) (a fixed right
    preconditioner M; FGMRES with a fixed M is right-preconditioned GMRES).
    Checked at the end of the first cycle, inside the second and inside the
    third."""
    rng = np.random.default_rng(12)
    n, m = 40, 5
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    b = rng.standard_normal(n)
    Mp = np.linalg.inv(np.diag(np.diag(A)) + 0.3 * np.tril(rng.standard_normal((n, n)), -1)) if precond else None
    prec = (lambda v: Mp @ v) if precond else (lambda v: v)
    x = np.zeros(n)
    expect = {}
    for it in range(1, 3 * m):
        cyc_start = (it - 1) // m * m
        if it - 1 == cyc_start:
            x0 = x.copy()
        xk = x0 + _min_residual_step(A, b - A @ x0, it - cyc_start, Mp)
        expect[it] = np.linalg.norm(b - A @ xk) / np.linalg.norm(b)
        if it - cyc_start == m:
            x = xk
    for it in (m, m + 2, 2 * m + 3):
        res = krylov.fgmres(lambda v: A @ v, prec, b, tol=0.0, maxit=it, restart=m)
        assert res.iters == it
        assert abs(res.relres - expect[it]) < 1e-10, (it, res.relres, expect[it])
    # restarting loses optimality: GMRES(m) at 2m is no better than GMRES(2m)
    full = krylov.fgmres(lambda v: A @ v, prec, b, tol=0.0, maxit=2 * m, restart=50)
    assert full.relres <= expect[2 * m] + 1e-12
