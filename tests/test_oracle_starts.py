"""Pins for the level starts of the V-cycle (Sec. 4.1, Alg. 4): the Approach X
auxiliaries rebuilt from the interpolated solution, the Approach D start from
the transferred auxiliaries, and the auxiliary a finished coarse level hands
on (``final_aux``).

Closed forms use ramp images X[i, j] = s1 i + s2 j, whose gradient is s1 on
every entry of the row-difference block vec(D X) and s2 on every entry of the
column-difference block vec(X D^T) (Sec. 4.2 block order), so each expected
value below is a number worked out by hand, block by block.
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import solvers as S
from oracle import vcycle
from oracle.hierarchy import Hierarchy
import synth

EPS, TAU = 0.03, 0.005


def ramp(m, s1, s2):
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    return s1 * i + s2 * j


def blocks(q, m):
    nx = (m - 1) * m
    return q[:nx], q[nx:]


def test_irls_x_start_weights_closed_form():
    """Alg. 1 weights from the interpolated x: max(|Lx|, eps)^(-1/2).
    Slope 1/16 gives 4 exactly, slope 1/4 gives 2; a flat direction gives
    eps^(-1/2)."""
    m = 6
    st = S.init_state("irls", "X", m, x0=ramp(m, 1 / 16, 1 / 4), eps=EPS, tau=TAU)
    wx, wy = blocks(st["w"], m)
    assert np.all(wx == 4.0) and np.all(wy == 2.0)
    st = S.init_state("irls", "X", m, x0=ramp(m, 0.0, -1 / 16), eps=EPS, tau=TAU)
    wx, wy = blocks(st["w"], m)
    assert np.allclose(wx, 5.773502691896258, rtol=0, atol=1e-15)  # 0.03^(-1/2)
    assert np.all(wy == 4.0)


def test_mm_x_start_shift_closed_form():
    """Alg. 2 shift u (1 - (eps^2 / (u^2 + eps^2))^(1/2)): at u = eps sqrt(3)
    the root is 1/2, so the shift is u / 2; at u = 0 it is 0."""
    m = 5
    u = EPS * np.sqrt(3.0)
    st = S.init_state("mm", "X", m, x0=ramp(m, u, 0.0), eps=EPS, tau=TAU)
    wx, wy = blocks(st["w"], m)
    assert np.allclose(wx, 0.025980762113533160, rtol=0, atol=1e-16)  # eps sqrt(3) / 2
    assert np.all(wy == 0.0)
    st = S.init_state("mm", "X", m, x0=ramp(m, 0.0, -u), eps=EPS, tau=TAU)
    wx, wy = blocks(st["w"], m)
    assert np.all(wx == 0.0)
    assert np.allclose(wy, -0.025980762113533160, rtol=0, atol=1e-16)


def test_sb_x_start_is_one_shrink_step():
    """Split Bregman under Approach X: one shrinkage step on the interpolated
    x, d = shrink(Lx, tau), and the multiplier g = Lx - d (the Bregman
    update of Alg. 3 taken from g = 0).  Slope 1/16: d = 0.0575, g = 0.005;
    slope -1/4: d = -0.245, g = -0.005; slope 0.003 < tau: d = 0, g = 0.003."""
    m = 6
    st = S.init_state("sb", "X", m, x0=ramp(m, 1 / 16, -1 / 4), eps=EPS, tau=TAU)
    dx, dy = blocks(st["d"], m)
    gx, gy = blocks(st["g"], m)
    assert np.allclose(dx, 0.0575, rtol=0, atol=1e-15)
    assert np.allclose(gx, 0.005, rtol=0, atol=1e-15)
    assert np.allclose(dy, -0.245, rtol=0, atol=1e-15)
    assert np.allclose(gy, -0.005, rtol=0, atol=1e-15)
    st = S.init_state("sb", "X", m, x0=ramp(m, 0.003, 0.0), eps=EPS, tau=TAU)
    dx, _ = blocks(st["d"], m)
    gx, _ = blocks(st["g"], m)
    assert np.all(dx == 0.0)
    assert np.allclose(gx, 0.003, rtol=0, atol=1e-16)


def small_problem(m=16, seed=11):
    rng = np.random.default_rng(seed)
    X = synth.piecewise_constant_image(m, 6, rng)
    P = synth.gaussian_psf(1.3, 3)
    B = ops.blur(X, P)
    B = B + 0.02 * np.linalg.norm(B) * rng.standard_normal((m, m)) / m
    return X, P, B


def test_sb_running_sum_includes_the_x_start():
    """From an Approach X start the multiplier after K Bregman updates is
    g^(K) = sum_{j=0..K} (L x^(j) - d^(j)), where j = 0 is the shrink step of
    the start (Alg. 3 with g^(0) = L x^(0) - d^(0)).  A start with g^(0) = 0
    misses the j = 0 term."""
    m = 16
    _, P, B = small_problem(m)
    H = Hierarchy(P, m, 1, "haar")
    op = S.LevelOperator(H, 0)
    rng = np.random.default_rng(3)
    x0 = ops.prolong(rng.standard_normal((m // 2, m // 2)), ops.lowpass("haar"))
    st = S.init_state("sb", "X", m, x0=x0, eps=EPS, tau=TAU)
    acc = ops.grad(x0) - st["d"]
    assert np.max(np.abs(acc)) > 1e-3  # the j = 0 term is not negligible here
    for _ in range(4):
        st, _ = S.solve_level(op, B, "sb", st, k_out=1, k_in=25, mu=[0.05], tau=TAU)
        acc = acc + ops.grad(st["x"]) - st["d"]
        assert np.max(np.abs(st["g"] - acc)) < 1e-14


def spy_inner(log, k_in=20):
    def inner(sub):
        log.append({"w": None if sub.w is None else sub.w.copy(),
                    "c": None if sub.c is None else sub.c.copy()})
        return sub.solve_cgls(k_in)[0]
    return inner


@pytest.mark.parametrize("solver", ["irls", "mm", "sb"])
def test_final_aux_is_what_the_next_iteration_uses(solver):
    """The auxiliary a coarse level hands to Approach D is the one its solver
    would use in its next outer iteration (Sec. 4.1): IRLS weights and the MM
    shift from the last x, SB's c = d - g after the last Bregman update.
    Checked against the subproblem the level actually forms at iteration K
    of a longer run (a stale value, from the start of iteration K - 1, fails)."""
    m = 16
    _, P, B = small_problem(m)
    H = Hierarchy(P, m, 1, "haar")
    op = S.LevelOperator(H, 0)
    K = 3
    st0 = S.init_state(solver, "I", m)
    log = []
    S.solve_level(op, B, solver, st0, K + 1, 0, mu=[0.02] * (K + 1), inner=spy_inner(log))
    stK, _ = S.solve_level(op, B, solver, st0, K, 0, mu=[0.02] * K, inner=spy_inner([]))
    aux = S.final_aux(solver, stK, EPS)
    used = log[K]
    if solver == "irls":
        assert np.array_equal(aux["w"], used["w"])
        assert not np.array_equal(log[K - 1]["w"], used["w"])
    elif solver == "mm":
        assert np.array_equal(aux["w"], used["c"])
        assert not np.array_equal(log[K - 1]["c"], used["c"])
    else:
        assert np.array_equal(aux["d"] - aux["g"], used["c"])
        assert not np.array_equal(log[K - 1]["c"], used["c"])


def test_d_start_is_the_transferred_block_closed_form():
    """Approach D under Haar (Sec. 4.2): a flat coarse solution has L x = 0,
    so the IRLS weights it hands on are eps^(-1/2) everywhere.  The block
    transfer W~1 Q_x W1^T, W1 Q_y W~1^T of a constant c gives c/2 on every
    difference row (column) of the fine grid except row (column) m_f - 2,
    where W~1 has no entry, which gets 0.  The level starts from x = 0 with
    exactly those weights."""
    mc, mf = 4, 8
    coarse = {"x": np.full((mc, mc), 0.7)}
    aux = S.final_aux("irls", coarse, EPS)
    c = 5.773502691896258  # 0.03^(-1/2)
    assert np.allclose(aux["w"], c, rtol=0, atol=1e-15)
    h = ops.lowpass("haar")
    wf = ops.dtransfer_vec(aux["w"], mc, h)
    st = S.init_state("irls", "D", mf, aux={"w": wf})
    assert np.all(st["x"] == 0.0) and st["x"].shape == (mf, mf)
    Wx = ops.unvec(st["w"][: (mf - 1) * mf], mf - 1, mf)
    Wy = ops.unvec(st["w"][(mf - 1) * mf:], mf, mf - 1)
    expect_x = np.full((mf - 1, mf), c / 2)
    expect_x[mf - 2, :] = 0.0
    expect_y = np.full((mf, mf - 1), c / 2)
    expect_y[:, mf - 2] = 0.0
    assert np.allclose(Wx, expect_x, rtol=0, atol=1e-15)
    assert np.allclose(Wy, expect_y, rtol=0, atol=1e-15)


@pytest.mark.parametrize("solver", ["irls", "mm", "sb"])
@pytest.mark.parametrize("transfer", ["X", "D"])
def test_vcycle_hands_each_level_its_start(monkeypatch, solver, transfer):
    """Alg. 4 wiring: the coarsest grid starts as Approach I; every finer grid
    starts from the prolonged coarse x (X) or from x = 0 and the block
    transfer of the coarse level's final auxiliaries (D)."""
    m, levels = 16, 3
    _, P, B = small_problem(m)
    calls = []
    real = vcycle.solve_level

    def spy(op, Bi, solver_, state, *a, **kw):
        out = real(op, Bi, solver_, state, *a, **kw)
        calls.append((op.m, {k: np.array(v, copy=True) for k, v in state.items()}, out[0]))
        return out

    monkeypatch.setattr(vcycle, "solve_level", spy)
    vcycle.deblur(B, P, solver, "haar", levels, transfer, k_out=2, k_in=8,
                  mu=[[0.01] * 2] * levels)
    assert [c[0] for c in calls] == [4, 8, 16]
    first = calls[0][1]
    assert np.all(first["x"] == 0.0)
    if solver == "irls":
        assert np.all(first["w"] == 1.0)
    elif solver == "mm":
        assert np.all(first["w"] == 0.0)
    else:
        assert np.all(first["d"] == 0.0) and np.all(first["g"] == 0.0)
    h = ops.lowpass("haar")
    for (mc, _, out_c), (mf, start, _) in zip(calls, calls[1:]):
        if transfer == "X":
            assert np.array_equal(start["x"], ops.prolong(out_c["x"], h))
        else:
            assert np.all(start["x"] == 0.0)
            for key, v in S.final_aux(solver, out_c, EPS).items():
                assert np.array_equal(start[key], ops.dtransfer_vec(v, mc, h))
