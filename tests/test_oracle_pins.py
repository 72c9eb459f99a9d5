"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check uses a closed form,
an invariant, an independent numpy computation of the definition, or a number
printed in the paper (Table 1). These run on the CPU only.
"""

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# --------------------------------------------------------------------------
# counter-based generator
# --------------------------------------------------------------------------
def test_uniform_generator_range_and_moments():
    X = oracle.fill_uniform(300, 40, seed=7, stream=5)
    assert X.min() >= -1.0 and X.max() < 1.0
    assert abs(X.mean()) < 0.02 and abs(X.var() - 1.0 / 3.0) < 0.01
    # counter-based: entry (i, j) depends only on (seed, stream, i, j)
    Y = oracle.fill_uniform(10, 40, seed=7, stream=5)
    assert np.array_equal(X[:10], Y)
    assert oracle.uniform(7, (5 << 40) + 3 * 4096 + 2) == X[3, 2]
    assert not np.array_equal(X[:10], oracle.fill_uniform(10, 40, seed=7, stream=6))
    # values are multiples of 2^-52 (53-bit mantissa draws mapped to [-1, 1))
    assert np.all(np.mod(X * 2.0**52, 1.0) == 0.0)


def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea & Flood 2014) reference outputs: the first three
    64-bit values of the generators seeded with 0 and with 1234567."""
    assert [oracle.splitmix64(0, k) for k in range(3)] == [
        16294208416658607535, 7960286522194355700, 487617019471545679]
    assert [oracle.splitmix64(1234567, k) for k in range(3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_uniform_is_the_top_53_bits_mapped_to_pm1():
    for seed, k in [(0, 0), (0, 2), (1234567, 1)]:
        z = oracle.splitmix64(seed, k)
        assert oracle.uniform(seed, k) == (z >> 11) * 2.0**-52 - 1.0


# --------------------------------------------------------------------------
# one-sided Jacobi SVD
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(40, 30), (30, 40), (64, 64), (17, 5)])
def test_jacobi_prescribed_spectrum(m, n):
    p = min(m, n)
    sigma = np.geomspace(1e3, 1e-6, p)
    W, q1, q2 = synth.prescribed_spectrum(m, n, sigma, seed=11 + m + n)
    U, S, V = oracle.jacobi_svd(W)
    assert np.all(np.diff(S) <= 0)
    err = np.abs(S - sigma)
    assert np.all(err <= 1e-13 * sigma[0] + 1e-12 * sigma), err.max()
    assert np.abs(U.T @ U - np.eye(p)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(p)).max() < 1e-13
    assert np.linalg.norm(U * S @ V.T - W) <= 1e-13 * np.linalg.norm(W)


def test_jacobi_2x2_closed_form():
    a, b, d = 3.0, -7.5, 0.25
    U, S, V = oracle.jacobi_svd(np.array([[a, b], [0.0, d]]))
    # sigma1 * sigma2 = |det|, sigma1^2 + sigma2^2 = ||W||_F^2
    assert S[0] * S[1] == pytest.approx(abs(a * d), rel=1e-14)
    assert S[0] ** 2 + S[1] ** 2 == pytest.approx(a * a + b * b + d * d, rel=1e-14)


def test_jacobi_brute_force_tiny():
    g = np.random.default_rng(3)
    for shape in [(3, 3), (4, 2), (2, 5), (6, 6), (1, 4), (5, 1)]:
        W = g.standard_normal(shape)
        _, S, _ = oracle.jacobi_svd(W)
        ref = np.linalg.svd(W, compute_uv=False)
        assert np.allclose(S, ref, rtol=0, atol=1e-14 * ref[0])


def test_jacobi_rank_deficient_and_zero():
    g = np.random.default_rng(5)
    W = g.standard_normal((9, 3)) @ g.standard_normal((3, 7))
    U, S, V = oracle.jacobi_svd(W)
    assert np.all(S[3:] <= 1e-13 * S[0])
    assert np.abs(U.T @ U - np.eye(7)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(7)).max() < 1e-12
    U, S, V = oracle.jacobi_svd(np.zeros((5, 4)))
    assert np.all(S == 0)
    assert np.abs(U.T @ U - np.eye(4)).max() < 1e-15
    assert np.abs(V.T @ V - np.eye(4)).max() < 1e-15


def test_jacobi_sign_convention():
    W = synth.gaussian((12, 8), seed=9)
    U, S, V = oracle.jacobi_svd(W)
    for k in range(8):
        assert U[np.argmax(np.abs(U[:, k])), k] > 0


# --------------------------------------------------------------------------
# singular value thresholding, Eq. (4)
# --------------------------------------------------------------------------
def test_svt_closed_form_prescribed_spectrum():
    sigma = np.array([50.0, 20.0, 9.0, 4.0, 1.5, 0.5, 0.1])
    W, q1, q2 = synth.prescribed_spectrum(30, 20, sigma, seed=2)
    eps = 3.0
    A, S, r = oracle.svt_exact(W, eps)
    ref = (q1 * np.maximum(sigma - eps, 0.0)) @ q2.T
    assert r == 4
    assert np.linalg.norm(A - ref) <= 1e-13 * np.linalg.norm(ref)


def test_svt_is_the_prox_of_the_nuclear_norm():
    """Eq. (3): A minimises eps ||A||_* + 0.5 ||A - W||_F^2 (checked with numpy)."""
    g = np.random.default_rng(8)
    W = g.standard_normal((15, 12)) * 3.0
    eps = 2.0
    A, _, r = oracle.svt_exact(W, eps)

    def f(X):
        return eps * np.linalg.svd(X, compute_uv=False).sum() + 0.5 * np.sum((X - W) ** 2)

    f0 = f(A)
    for _ in range(50):
        H = g.standard_normal(W.shape)
        for t in (1e-2, 1e-4):
            assert f(A + t * H) >= f0 - 1e-12
    # KKT: W - A = eps (U_r V_r^T + Z), U_r^T Z = 0, Z V_r = 0, ||Z||_2 <= 1
    Ua, Sa, Vat = np.linalg.svd(A)
    Ur, Vr = Ua[:, :r], Vat[:r].T
    Z = (W - A) / eps - Ur @ Vr.T
    assert np.abs(Ur.T @ Z).max() < 1e-12 and np.abs(Z @ Vr).max() < 1e-12
    assert np.linalg.norm(Z, 2) <= 1.0 + 1e-12


def test_svt_threshold_above_spectrum_gives_zero():
    W = synth.gaussian((10, 10), seed=1)
    A, S, r = oracle.svt_exact(W, S_max := np.linalg.norm(W, 2) * 1.01)
    assert r == 0 and np.all(A == 0)


# --------------------------------------------------------------------------
# BLWS step (Algorithms 2-3 with k = 2, warm start)
# --------------------------------------------------------------------------
def _warm(W, b, delta, seed):
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(seed)
    m, n = W.shape
    Ui = np.linalg.qr(U0[:, :b] + delta * g.standard_normal((m, b)))[0]
    Vi = np.linalg.qr(V0t[:b].T + delta * g.standard_normal((n, b)))[0]
    return Ui, Vi


def _spectrum_case():
    sigma = np.r_[np.linspace(100, 50, 5), np.geomspace(5, 0.01, 45)]
    W, _, _ = synth.prescribed_spectrum(60, 50, sigma, seed=3)
    return W, sigma


def test_blws_matches_rayleigh_ritz_definition():
    """Ritz values = singular values of the projection of W on the block
    Krylov spaces span[U, W V] x span[V, W^T U], computed with numpy."""
    g = np.random.default_rng(12)
    W = g.standard_normal((45, 38))
    b = 6
    U = np.linalg.qr(g.standard_normal((45, b)))[0]
    V = np.linalg.qr(g.standard_normal((38, b)))[0]
    Un, Vn, S, A, r = oracle.blws_step(W, 1.5, U, V)
    Qu = np.linalg.qr(np.hstack([U, W @ V]))[0]
    Qv = np.linalg.qr(np.hstack([V, W.T @ U]))[0]
    Ub, sb, Vbt = np.linalg.svd(Qu.T @ W @ Qv)
    assert np.allclose(S, sb[:b], rtol=1e-12, atol=1e-13 * sb[0])
    rr = int(np.sum(sb[:b] > 1.5))
    Aref = (Qu @ Ub[:, :rr] * (sb[:rr] - 1.5)) @ (Qv @ Vbt[:rr].T).T
    assert r == rr
    assert np.linalg.norm(A - Aref) <= 1e-12 * np.linalg.norm(Aref)
    assert np.abs(Un.T @ Un - np.eye(b)).max() < 1e-13
    assert np.abs(Vn.T @ Vn - np.eye(b)).max() < 1e-13


def test_blws_equals_literal_block_lanczos_on_augmented_matrix():
    """Algorithm 2 with k = 2 on W~ = [[0, W], [W^T, 0]] from the start block
    blockdiag(U, V), then Algorithm 3: the positive Ritz values are the BLWS
    Ritz values (Theorem 1 applied to the projected matrix)."""
    g = np.random.default_rng(21)
    m, n, b = 20, 16, 3
    W = g.standard_normal((m, n))
    U = np.linalg.qr(g.standard_normal((m, b)))[0]
    V = np.linalg.qr(g.standard_normal((n, b)))[0]
    Wt = np.block([[np.zeros((m, m)), W], [W.T, np.zeros((n, n))]])
    X1 = np.zeros((m + n, 2 * b))
    X1[:m, :b] = U
    X1[m:, b:] = V
    M1 = X1.T @ Wt @ X1
    R1 = Wt @ X1 - X1 @ M1
    X2, B1 = np.linalg.qr(R1)
    M2 = X2.T @ Wt @ X2
    T2 = np.block([[M1, B1.T], [B1, M2]])
    lam = np.sort(np.linalg.eigvalsh(T2))[::-1]
    _, _, S, _, _ = oracle.blws_step(W, 0.0, U, V, want_A=False)
    assert np.allclose(S, lam[:b], rtol=1e-12)
    # Theorem 1 on the explicit augmented matrix
    ev = np.sort(np.linalg.eigvalsh(Wt))
    sv = np.linalg.svd(W, compute_uv=False)
    expect = np.sort(np.r_[sv, -sv, np.zeros(m - n)])
    assert np.allclose(ev, expect, atol=1e-12)


def test_blws_exact_warm_start_is_exact():
    """With the exact top-b subspaces the new Krylov directions vanish (R_1 = 0);
    the Householder completion keeps the block orthonormal and the step returns
    the exact top-b singular values and T_eps(W)."""
    W, sigma = _spectrum_case()
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    b = 8
    Un, Vn, S, A, r = oracle.blws_step(W, 3.5, U0[:, :b], V0t[:b].T)
    assert np.allclose(S, sigma[:b], rtol=1e-12)
    Aex, _, rex = oracle.svt_exact(W, 3.5)
    assert r == rex == 8
    assert np.linalg.norm(A - Aex) <= 1e-12 * np.linalg.norm(Aex)
    assert np.abs(Un.T @ Un - np.eye(b)).max() < 1e-13


def test_blws_warm_start_convergence_is_quadratic_in_sigma():
    W, sigma = _spectrum_case()
    b = 8
    errs = []
    for d in (1e-3, 1e-4, 1e-5):
        U, V = _warm(W, b, d, seed=0)
        _, _, S, _, _ = oracle.blws_step(W, 3.5, U, V, want_A=False)
        errs.append(np.abs(S - sigma[:b]).max() / sigma[0])
        # Ritz values interlace from below
        assert np.all(S <= sigma[:b] * (1 + 1e-13))
    assert errs[0] / errs[1] > 30 and errs[1] / errs[2] > 30, errs


def test_blws_rank_deficient_w():
    g = np.random.default_rng(4)
    W = g.standard_normal((30, 4)) @ g.standard_normal((4, 26))
    U = np.linalg.qr(g.standard_normal((30, 6)))[0]
    V = np.linalg.qr(g.standard_normal((26, 6)))[0]
    Un, Vn, S, A, r = oracle.blws_step(W, 0.0, U, V)
    sv = np.linalg.svd(W, compute_uv=False)
    assert np.allclose(S[:4], sv[:4], rtol=1e-11)
    assert np.all(S[4:] <= 1e-12 * sv[0])
    assert np.abs(Un.T @ Un - np.eye(6)).max() < 1e-12
    assert np.abs(Vn.T @ Vn - np.eye(6)).max() < 1e-12


@pytest.mark.parametrize("side", ["V", "U"])
@pytest.mark.parametrize("kappa", [1e8, 1e12])
def test_blws_ill_conditioned_krylov_block(side, kappa):
    """A new block with condition number kappa (not singular): every singular
    pair above the threshold lies in both halves of the block, so the step's
    values are the prescribed ones and A is T_eps(W) formed from the
    prescribed factors, whatever the QR step does with the near-dependent pair."""
    c = synth.ill_conditioned_block(200, 180, 12, kappa, side, seed=11)
    W, sig = c["W"], c["sigma"]
    Un, Vn, S, A, r = oracle.blws_step(W, 30.0, c["U"], c["V"])
    assert r == 11
    assert np.abs(S[:r] - sig[:r]).max() <= 1e-13 * sig[0]
    _, X, Y = synth.prescribed_spectrum(200, 180, sig, seed=11)
    A_def = (X[:, :r] * (sig[:r] - 30.0)) @ Y[:, :r].T
    assert np.linalg.norm(A - A_def) <= 1e-12 * np.linalg.norm(A_def)
    assert np.abs(Un.T @ Un - np.eye(12)).max() < 1e-13
    assert np.abs(Vn.T @ Vn - np.eye(12)).max() < 1e-13


def test_spectral_norm_by_blws():
    # a clear top gap: converged to rounding
    sigma = np.r_[10.0, np.linspace(8.0, 0.1, 59)]
    W, _, _ = synth.prescribed_spectrum(120, 90, sigma, seed=6)
    s, steps = oracle.spectral_norm_blws(W, bs=8)
    assert s == pytest.approx(10.0, rel=1e-13)
    # a Gaussian matrix (clustered top of the spectrum): converges from below
    g = np.random.default_rng(6)
    W = g.standard_normal((120, 90))
    s, steps = oracle.spectral_norm_blws(W, bs=8)
    ref = np.linalg.norm(W, 2)
    assert ref * (1 - 1e-9) <= s <= ref * (1 + 1e-14)
    U, V = oracle.cold_block(W, 8, 2, seed=1)
    assert np.abs(U.T @ U - np.eye(8)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(8)).max() < 1e-13


def _projector(X):
    Q = np.linalg.qr(X)[0]
    return Q @ Q.T


def test_cold_block_without_power_steps_spans_the_drawn_blocks():
    """pow_steps = 0: V spans the generator's block of stream s, U that of
    stream s + 1 (both orthonormal)."""
    W = synth.gaussian((70, 50), seed=4)
    U, V = oracle.cold_block(W, 6, 0, seed=99, stream_v=5)
    Rv = oracle.fill_uniform(50, 6, seed=99, stream=5)
    Ru = oracle.fill_uniform(70, 6, seed=99, stream=6)
    assert np.abs(V.T @ V - np.eye(6)).max() < 1e-14
    assert np.abs(U.T @ U - np.eye(6)).max() < 1e-14
    assert np.abs(_projector(V) - _projector(Rv)).max() < 1e-13
    assert np.abs(_projector(U) - _projector(Ru)).max() < 1e-13


def test_cold_block_power_steps_contract_like_subspace_iteration():
    """Each power half-step pair V <- orth(W^T orth(W V)) is one step of subspace
    iteration on W^T W: with the top b singular values equal (8) and one value
    (4) below them, the tangent of the largest principal angle between span(V)
    and the top right singular subspace shrinks by exactly (4/8)^2 per step once
    the much smaller rest of the spectrum has died out. U stays the independent
    draw of stream s + 1 whatever the number of steps."""
    b, m, n = 6, 150, 120
    sigma = np.r_[np.full(b, 8.0), 4.0, np.geomspace(0.05, 0.01, n - b - 1)]
    W, q1, q2 = synth.prescribed_spectrum(m, n, sigma, seed=17)
    top = q2[:, :b]
    tans = []
    for t in range(4):
        U, V = oracle.cold_block(W, b, t, seed=3, stream_v=1)
        cos = np.linalg.svd(top.T @ V, compute_uv=False).min()
        tans.append(np.sqrt(1.0 - cos * cos) / cos)
        assert np.abs(_projector(U) - _projector(oracle.fill_uniform(m, b, 3, 2))).max() < 1e-13
    ratios = [tans[t] / tans[t - 1] for t in range(1, 4)]
    assert ratios[0] < 0.2501, ratios
    assert all(abs(r - 0.25) < 1e-3 for r in ratios[1:]), ratios


def test_predict_rank_hand_worked():
    """Rank rule of the host solver: one more than the count above the threshold
    when it fell short of the prediction, else that count plus 5% of min(m, n),
    never beyond min(m, n)."""
    assert oracle.predict_rank(50, 60, 0.05, 2000) == 51
    assert oracle.predict_rank(0, 10, 0.05, 2000) == 1
    assert oracle.predict_rank(101, 101, 0.05, 2000) == 201
    assert oracle.predict_rank(10, 10, 0.05, 200) == 20
    assert oracle.predict_rank(1990, 1000, 0.05, 2000) == 2000
    assert oracle.predict_rank(1999, 2000, 0.05, 2000) == 2000


def test_block_width_hand_worked():
    """b = the predicted rank rounded up to a multiple of 16, at most p / 2."""
    assert oracle.block_width(101, 16, 2000) == 112
    assert oracle.block_width(112, 16, 2000) == 112
    assert oracle.block_width(113, 16, 2000) == 128
    assert oracle.block_width(1, 16, 2000) == 16
    assert oracle.block_width(201, 16, 2000) == 208
    assert oracle.block_width(1500, 16, 2000) == 1000
    assert oracle.block_width(5, 16, 20) == 10
    assert oracle.block_width(5, 4, 20) == 8


def test_resize_block_truncates_or_extends_the_span():
    g = np.random.default_rng(2)
    X = np.linalg.qr(g.standard_normal((40, 7)))[0]
    Y = oracle.resize_block(X, 4, seed=5, stream=11)
    assert np.array_equal(Y, X[:, :4])
    Y = oracle.resize_block(X, 12, seed=5, stream=11)
    R = oracle.fill_uniform(40, 5, seed=5, stream=11)
    assert np.array_equal(Y[:, :7], X)
    assert np.abs(Y.T @ Y - np.eye(12)).max() < 1e-14
    assert np.abs(_projector(Y) - _projector(np.hstack([X, R]))).max() < 1e-13


def test_rpca_snapshot_first_iteration_closed_form():
    """Iteration 1 of the RPCA loop: W = D + Y0/mu0 with Y0 = D / max(||D||_2,
    ||D||_inf / lambda), mu0 = 1.25 / ||D||_2 and eps = 1/mu0, ||D||_2 exact;
    the first block is 16 wide (predicted rank 10) and orthonormal."""
    inst = synth.rpca_instance(120, 90, 6, 0.05, 50.0, 1)
    D = inst["D"]
    W, U, V, eps = oracle.rpca_snapshot(D, 1)
    s1 = np.linalg.norm(D, 2)
    lam = 1.0 / np.sqrt(120)
    J = max(s1, np.abs(D).max() / lam)
    mu0 = 1.25 / s1
    assert eps == pytest.approx(1.0 / mu0, rel=1e-12)
    assert np.abs(W - (D + D / J / mu0)).max() <= 1e-12 * np.abs(D).max()
    assert U.shape == (120, 16) and V.shape == (90, 16)
    assert np.abs(U.T @ U - np.eye(16)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(16)).max() < 1e-13


# --------------------------------------------------------------------------
# inexact ALM for RPCA
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rpca_exact_recovery_small(seed):
    inst = synth.rpca_instance(200, 200, 10, 0.05, 50.0, seed)
    ex = oracle.rpca(inst["D"], mode="exact", want_Y=True)
    bl = oracle.rpca(inst["D"], mode="blws", want_Y=True)
    nA0 = np.linalg.norm(inst["A0"])
    for out in (ex, bl):
        info = out["info"]
        assert info["status"] == 0 and info["rel_residual"] < 1e-7
        assert info["rank"] == 10
        # ||D||_2 (it sets Y0 and mu0) to rounding in both modes
        assert info["norm2_D"] == pytest.approx(np.linalg.norm(inst["D"], 2), rel=1e-11)
        assert np.linalg.norm(out["A"] - inst["A0"]) / nA0 < 2e-6
        assert abs(info["nnz_E"] - inst["nnz"]) <= 10
        lam = 1.0 / np.sqrt(200)
        Y, E = out["Y"], out["E"]
        # E-step optimality: |Y| <= lambda with equality (and sign) on supp(E)
        # (the dual update Y + mu Z cancels in floating point: mu reaches 1e7 mu_0)
        assert np.abs(Y).max() <= lam * (1 + 1e-9)
        on = E != 0
        assert np.allclose(Y[on], lam * np.sign(E[on]), rtol=0, atol=1e-9 * lam)
        # dual feasibility for the nuclear norm at the optimum
        assert np.linalg.norm(Y, 2) <= 1.0 + 1e-3
    assert np.linalg.norm(ex["A"] - bl["A"]) / np.linalg.norm(ex["A"]) < 1e-6


def test_rpca_table1_m500_row():
    """Table 1, m = 500: rank(A^) = 50, ||E^||_0 within a few dozen of the
    25000 corruptions, relative error of order 1e-5, about 30 iterations."""
    inst = synth.rpca_instance(500, 500, 50, 0.10, 500.0, 0)
    out = oracle.rpca(inst["D"], mode="blws")
    info = out["info"]
    assert info["rank"] == 50
    assert 25000 <= info["nnz_E"] <= 25100
    err = np.linalg.norm(out["A"] - inst["A0"]) / np.linalg.norm(inst["A0"])
    assert err < 5e-5
    assert 15 <= info["iters"] <= 40


# --------------------------------------------------------------------------
# ALM matrix completion
# --------------------------------------------------------------------------
def test_mc_recovers_planted_low_rank():
    inst = synth.mc_instance(120, 100, 4, 0.45, seed=3)
    M = inst["L"] @ inst["R"].T
    res = {}
    for mode in ("exact", "blws"):
        out = oracle.mc(120, 100, inst["row_ptr"], inst["col_idx"], inst["values"], mode=mode,
                        r_cap=40, rho=1.1, tol=1e-8)
        A = out["U"] * out["S"] @ out["V"].T
        assert out["info"]["status"] == 0
        assert out["rank"] == 4
        assert np.linalg.norm(A - M) / np.linalg.norm(M) < 1e-6
        res[mode] = A
    assert np.linalg.norm(res["exact"] - res["blws"]) / np.linalg.norm(M) < 1e-6


# --------------------------------------------------------------------------
# the SVT algorithm for matrix completion (Table 2's host)
# --------------------------------------------------------------------------
def _planted_error(out, inst):
    """||U S V^T - L R^T||_F / ||L R^T||_F from the factors (no dense product)."""
    U, S, V, L, R = out["U"], out["S"], out["V"], inst["L"], inst["R"]
    nA2 = float(np.sum(S ** 2))
    nM2 = float(np.sum((L.T @ L) * (R.T @ R)))
    ip = float(np.sum(((U * S).T @ L) * (V.T @ R)))
    return np.sqrt(max(nA2 + nM2 - 2.0 * ip, 0.0)) / np.sqrt(nM2)


def _table2_instance(m, r, ratio, seed=0):
    s = ratio * r * (2 * m - r)  # s / d_r with d_r = r (2 m - r)
    return synth.mc_instance(m, m, r, s / float(m * m), seed)


def test_mc_svt_exact_and_blws_thresholding_agree():
    """Same host, exact (Jacobi) or BLWS thresholding: the same iterations and
    rank and the same completed matrix; recovery at the tolerance's scale."""
    inst = _table2_instance(200, 5, 6)
    ex = oracle.mc_svt(200, 200, inst["row_ptr"], inst["col_idx"], inst["values"], mode="exact",
                       r_cap=32)
    bl = oracle.mc_svt(200, 200, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                       r_cap=32)
    assert ex["info"]["status"] == bl["info"]["status"] == 0
    assert ex["info"]["iters"] == bl["info"]["iters"]
    assert ex["rank"] == bl["rank"] == 5
    Ae = ex["U"] * ex["S"] @ ex["V"].T
    Ab = bl["U"] * bl["S"] @ bl["V"].T
    assert np.linalg.norm(Ae - Ab) <= 1e-6 * np.linalg.norm(Ae)
    assert _planted_error(bl, inst) < 5e-4


@pytest.mark.parametrize("m,r,ratio,iters,err", [
    (5000, 10, 6, 123, 1.74e-4),
    (10000, 10, 6, 123, 1.70e-4),
    (5000, 50, 5, 108, 1.55e-4),
])
def test_mc_svt_table2_rows(m, r, ratio, iters, err):
    """Table 2, BLWS-SVT rows: m x m, rank r, s/d_r samples; the paper prints the
    iteration count and the relative error of the recovered matrix. The host's
    constants (tau = 5 m, delta = 1.2 m^2 / s, tol 1e-4, rank step 5) are those
    of the SVT algorithm's source; the draws are ours, so the counts match to a
    few iterations and the errors to a few percent."""
    inst = _table2_instance(m, r, ratio)
    out = oracle.mc_svt(m, m, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                        r_cap=128)
    info = out["info"]
    assert info["status"] == 0 and out["rank"] == r
    assert abs(info["iters"] - iters) <= 6, info["iters"]
    e = _planted_error(out, inst)
    assert err / 1.25 <= e <= err * 1.25, e


# ---------------------------------------------------------------------------
# Sec. 4.1 ablations: Algorithms 2-3 taken literally on [[0, W], [W^T, 0]]
# from the split, aug, and half-information start blocks, with k blocks.
# ---------------------------------------------------------------------------


def _warm_signed(W, b, delta, seed):
    """Noisy top-b singular subspaces with the signs of the exact vectors kept
    (column j of U and of V perturb u_j and v_j): the pairing that makes
    (U; V) / sqrt(2) close to eigenvectors of the augmented matrix."""
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(seed)
    m, n = W.shape

    def orth_signed(X):
        Q, R = np.linalg.qr(X)
        return Q * np.sign(np.diag(R))

    return (orth_signed(U0[:, :b] + delta * g.standard_normal((m, b))),
            orth_signed(V0t[:b].T + delta * g.standard_normal((n, b))))


def test_lanczos_split_k2_equals_blws_step():
    """The literal procedure on the explicit augmented matrix from
    blockdiag(U, V) gives the same Ritz values and SVT as the default step,
    which works on W only (two separate implementations)."""
    W, sigma = _spectrum_case()
    U, V = _warm(W, 8, 1e-3, seed=4)
    _, _, S1, A1, r1 = oracle.blws_step(W, 3.5, U, V)
    Ul, Vl, S2, A2, r2 = oracle.lanczos_svt(W, 3.5, U, V, "split", 2)
    assert r1 == r2
    assert np.abs(S1 - S2).max() <= 1e-13 * sigma[0]
    assert np.linalg.norm(A1 - A2) <= 1e-12 * np.linalg.norm(A1)
    assert np.abs(Ul.T @ Ul - np.eye(8)).max() < 1e-13
    assert np.abs(Vl.T @ Vl - np.eye(8)).max() < 1e-13


@pytest.mark.parametrize("start,k", [("split", 5), ("aug", 10), ("left", 10), ("right", 10)])
def test_lanczos_full_krylov_space_is_exact(start, k):
    """k blocks spanning all of R^(m+n): T_k is orthogonally similar to the
    augmented matrix, whose top eigenvalues are the singular values of W
    (Theorem 1), so the Ritz values and the SVT are exact."""
    g = np.random.default_rng(31)
    m, n, b = 6, 4, 1
    W = g.standard_normal((m, n))
    U = np.linalg.qr(g.standard_normal((m, b)))[0]
    V = np.linalg.qr(g.standard_normal((n, b)))[0]
    sv = np.linalg.svd(W, compute_uv=False)
    eps = 0.5 * (sv[0] + sv[1])  # only sigma_1 above the threshold
    Un, Vn, S, A, r = oracle.lanczos_svt(W, eps, U, V, start, k)
    assert abs(S[0] - sv[0]) <= 1e-13 * sv[0]
    Aex, _, rex = oracle.svt_exact(W, eps)
    assert r == rex == 1
    assert np.linalg.norm(A - Aex) <= 1e-12 * np.linalg.norm(Aex)


@pytest.mark.parametrize("start", ["left", "right"])
def test_lanczos_half_start_k2_closed_form(start):
    """From (U; 0) the second block is (0; orth(W^T U)) and both diagonal
    blocks of T_2 vanish, so T_2 = [[0, R^T], [R, 0]] with W^T U = G R: the Ritz
    values are the singular values of W^T U (of W V from (0; V))."""
    g = np.random.default_rng(32)
    m, n, b = 25, 19, 4
    W = g.standard_normal((m, n))
    U = np.linalg.qr(g.standard_normal((m, b)))[0]
    V = np.linalg.qr(g.standard_normal((n, b)))[0]
    _, _, S, _, _ = oracle.lanczos_svt(W, 0.0, U, V, start, 2, want_A=False)
    expect = np.linalg.svd(W.T @ U if start == "left" else W @ V, compute_uv=False)
    assert np.allclose(S, expect, rtol=1e-13, atol=0)


def test_lanczos_aug_start_on_exact_subspaces_is_exact():
    """With the exact top-b singular pairs, (U; V) / sqrt(2) spans an
    invariant subspace of the augmented matrix (W V = U S, W^T U = V S): the
    Ritz values are sigma_1..sigma_b and the SVT is exact."""
    W, sigma = _spectrum_case()
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    b = 8  # all eight values above eps = 3.5
    Un, Vn, S, A, r = oracle.lanczos_svt(W, 3.5, U0[:, :b], V0t[:b].T, "aug", 2)
    assert np.allclose(S, sigma[:b], rtol=1e-12)
    Aex, _, rex = oracle.svt_exact(W, 3.5)
    assert r == rex
    assert np.linalg.norm(A - Aex) <= 1e-11 * np.linalg.norm(Aex)


@pytest.mark.parametrize("start", ["split", "aug", "left", "right"])
def test_lanczos_ritz_values_rise_with_k(start):
    """The Krylov spaces are nested in k, so each Ritz value is
    nondecreasing in k (Cauchy interlacing) and never above sigma_i."""
    W, sigma = _spectrum_case()
    U, V = _warm_signed(W, 5, 1e-2, seed=6)
    prev = None
    for k in (2, 3, 4):
        _, _, S, _, _ = oracle.lanczos_svt(W, 0.0, U, V, start, k, want_A=False)
        assert np.all(S <= sigma[:5] * (1 + 1e-13))
        if prev is not None:
            assert np.all(S >= prev - 1e-12 * sigma[0])
        prev = S


def test_lanczos_aug_start_beats_half_starts():
    """Sec. 4.1: starting from both previous subspaces gives more precise
    Ritz values than either half-information start at the same k."""
    W, sigma = _spectrum_case()
    U, V = _warm_signed(W, 5, 1e-2, seed=7)
    err = {}
    for start in ("aug", "left", "right"):
        _, _, S, _, _ = oracle.lanczos_svt(W, 0.0, U, V, start, 2, want_A=False)
        err[start] = np.abs(S - sigma[:5]).max()
    assert err["aug"] < err["left"] and err["aug"] < err["right"], err
