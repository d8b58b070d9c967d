"""Pins of the oracle's fixed-budget lightweight mode (Alg. 1 with the inertia-only metric of Eq. 10).

* contact_blocks: Phi equals the pinned NCP function, and K, E are the derivatives of Phi with
  respect to the contact displacement and the multipliers (central differences away from kinks);
* inertia_metric: h^2 H M^-1 H^T written with the scene's masses and frames;
* step_lightweight: without contacts it is the exact step; with a large budget it converges to the
  exact step (the same fixed point, Sec. IV-B); frictionless contacts that stay active contract as
  e_{i+1} = (I - S^-1 W_nn) e_i, S = diag(h^2 / m_v), the closed form of the update with W~ = S on
  single-contact vertices; momentum balance holds whatever the budget.
"""
import math

import numpy as np
import pytest

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes


def _random_state(seed, c=5):
    rng = np.random.default_rng(seed)
    Y = rng.normal(scale=1e-3, size=(c, 3))
    lam = rng.normal(scale=0.5, size=(c, 3))
    lam[:, 0] = np.abs(lam[:, 0]) + 0.1
    d0 = rng.normal(scale=1e-3, size=c)
    dob = rng.normal(scale=1e-4, size=(c, 2))
    s = rng.uniform(1e-3, 1e-2, size=c)
    return Y, lam, d0, dob, s, 0.6


@pytest.mark.parametrize("seed", range(6))
def test_contact_blocks_match_ncp_function_and_its_derivatives(seed):
    Y, lam, d0, dob, s, mu = _random_state(seed)
    phi, Kb, Eb = O.contact_blocks(Y, lam, d0, dob, s, mu)
    # Phi equals the NCP function with W = 0 and y0 = Y (the pinned formula)
    csp = O.CSP(Y.reshape(-1), np.zeros((Y.size, Y.size)), d0, dob, s, mu, 1e10)
    ref, *_ = O.ncp_function(csp, lam)
    np.testing.assert_allclose(phi, ref, rtol=1e-13, atol=1e-16)
    # K = dPhi/dY and E = dPhi/dlambda by central differences (each contact independent)
    for j in range(Y.shape[0]):
        for a in range(3):
            for wrt, blk in (("Y", Kb), ("lam", Eb)):
                hstep = 1e-9 if wrt == "Y" else 1e-7
                Yp, Ym, lp, lm = Y.copy(), Y.copy(), lam.copy(), lam.copy()
                if wrt == "Y":
                    Yp[j, a] += hstep; Ym[j, a] -= hstep
                else:
                    lp[j, a] += hstep; lm[j, a] -= hstep
                pp, *_ = O.contact_blocks(Yp, lp, d0, dob, s, mu)
                pm, *_ = O.contact_blocks(Ym, lm, d0, dob, s, mu)
                num = (pp[j] - pm[j]) / (2 * hstep)
                scale = max(1.0, float(np.abs(blk[j][:, a]).max()))
                assert np.max(np.abs(num - blk[j][:, a])) <= 1e-5 * scale, (j, a, wrt)


def test_inertia_metric_blocks():
    sc = scenes.drop_cube(seed=1, hexes=2, drop_height=0.0005, jitter=0.0)
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    box = scenes.box((0.05 + 0.0015 + 0.02, 0.01, 0.0), (0.02, 0.05, 0.05))
    con = O.detect(sc.x0[0], sc.v0[0], [scenes.ground(), box], p)
    Wt = O.inertia_metric(oe, con, p.h).toarray()
    assert np.allclose(Wt, Wt.T)
    multi = 0
    for j in range(con.count):
        for k in range(con.count):
            blk = Wt[3 * j:3 * j + 3, 3 * k:3 * k + 3]
            if con.vertex[j] != con.vertex[k]:
                assert not blk.any()
            elif j == k:
                # orthonormal frame: (h^2 / m_v) I
                np.testing.assert_allclose(blk, p.h ** 2 / oe.mass[con.vertex[j]] * np.eye(3), rtol=1e-14)
            else:
                multi += 1
                # two obstacles' frames on one vertex: normal-normal coupling n_j . n_k
                nn = con.frame[j][:, 0] @ con.frame[k][:, 0]
                assert math.isclose(blk[0, 0], p.h ** 2 / oe.mass[con.vertex[j]] * nn, rel_tol=1e-13)
    assert multi > 0


def test_lightweight_step_without_contacts_is_the_exact_step():
    sc = scenes.drop_cube(seed=2, drop_height=1.0)
    oe = O.precompute(sc.envs[0], sc.params.h)
    a = O.step(oe, sc.x0[0], sc.v0[0], sc.obstacles[0], sc.params)
    b = O.step_lightweight(oe, sc.x0[0], sc.v0[0], sc.obstacles[0], sc.params, newton_iterations=3)
    assert a.contacts.count == 0 and b.contacts.count == 0
    np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-15)


def test_lightweight_step_converges_to_the_exact_step():
    """A soft block landing with friction: with enough lightweight updates per local-global
    iteration the step reaches the exact-metric step (the same fixed point)."""
    sc = scenes.drop_cube(seed=4, hexes=3, young=2e4, drop_height=0.0005, jitter=0.0)
    p = sc.params
    p.lg_iterations = 3
    oe = O.precompute(sc.envs[0], p.h)
    x = sc.x0[0]
    v = np.zeros_like(x)
    v[:, 0] = 0.02
    v[:, 1] = -0.05
    ex = O.step(oe, x, v, sc.obstacles[0], p, tol=1e-13)
    li = O.step_lightweight(oe, x, v, sc.obstacles[0], p, newton_iterations=4000, tol=1e-13)
    assert ex.contacts.count > 0
    assert li.residual <= 1e-12
    np.testing.assert_allclose(li.x, ex.x, rtol=0, atol=1e-10)
    assert li.info["newton"] > 3 * 5      # the inertia-only metric needs many more updates
    # a small budget does not reach it
    few = O.step_lightweight(oe, x, v, sc.obstacles[0], p, newton_iterations=2)
    assert few.residual > 1e-9


def test_frictionless_active_contacts_contract_at_the_closed_form_rate():
    """mu = 0, one local-global iteration (b fixed), every bottom vertex pressed into the ground:
    after the first update (which zeroes the tangential multipliers) the normal error contracts
    exactly as e_{i+1} = (I - S^-1 W_nn) e_i with W_nn the exact Delassus operator on the normal
    rows and S = diag(h^2 / m_v)."""
    sc = scenes.drop_cube(seed=6, hexes=2, drop_height=-0.0008, jitter=0.0, mu=0.0, young=3e5)
    p = sc.params
    p.lg_iterations = 1
    oe = O.precompute(sc.envs[0], p.h)
    x, v = sc.x0[0], sc.v0[0]
    li = O.step_lightweight(oe, x, v, sc.obstacles[0], p, newton_iterations=12)
    c = li.contacts.count
    assert c == 9 and len(set(li.contacts.vertex.tolist())) == 9
    # the exact solution of the same subproblem (b at q~, the only projection point)
    qt = O.predicted_state(x, v, p.h, p.gravity)
    qb = oe.solve(O.assemble_rhs(oe, qt, O.project(oe, qt), p.h))
    csp, _, _ = O.build_csp(oe, x, qb, li.contacts, p.h, p.max_force)
    lam_star, r, _ = O.solve_csp(csp, tol=1e-14)
    assert np.all(lam_star[:, 0] > 0) and np.allclose(lam_star[:, 1:], 0.0, atol=1e-12)
    Wnn = csp.W[0::3, 0::3]
    S = p.h ** 2 / oe.mass[li.contacts.vertex]
    M = np.eye(c) - Wnn / S[:, None]
    hist = li.info["lam_history"]
    e1 = hist[0][:, 0] - lam_star[:, 0]
    np.testing.assert_allclose(hist[0][:, 1:], 0.0, atol=1e-12)
    for i in range(1, len(hist)):
        assert np.all(hist[i][:, 0] > 0)
        pred = np.linalg.matrix_power(M, i) @ e1
        np.testing.assert_allclose(hist[i][:, 0] - lam_star[:, 0], pred, rtol=1e-7,
                                   atol=1e-9 * np.abs(lam_star[:, 0]).max())
    # the contraction is real but slow for a stiff block: the spectral radius is close to 1
    rho = max(abs(np.linalg.eigvals(M)))
    assert 0.5 < rho < 1.0


@pytest.mark.parametrize("budget", [1, 3])
def test_lightweight_momentum_balance_at_any_budget(budget):
    """sum_v m_v (v' - v) = h M g + sum_j P_j for whatever multipliers the budget reaches."""
    sc = scenes.squeeze_blocks(1, seed=3, hexes=3)
    p = sc.params
    p.lg_iterations = 4
    oe = O.precompute(sc.envs[0], p.h)
    x, v, obs = sc.x0[0], sc.v0[0], sc.obstacles[0]
    for _ in range(3):
        r = O.step_lightweight(oe, x, v, obs, p, newton_iterations=budget)
        lhs = (oe.mass[:, None] * (r.v - v)).sum(0)
        rhs = p.h * oe.mass.sum() * np.asarray(p.gravity) + r.impulse.sum(0)
        assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-13)
        x, v, obs = r.x, r.v, r.obstacles
    assert r.contacts.count > 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lightweight_update_is_newton_when_the_body_is_all_inertia(seed):
    """With negligible elasticity A = M, so W = W~: one lightweight update is then an undamped
    semismooth Newton step of the exact problem with proximal scale h^2 / m_v, computed here with
    the exact path's generalized Jacobian.  A single tet sliding onto the ground (stick, slip and
    separation rows all appear over the seeds)."""
    sc = scenes.single_tet_scene("ground", seed=seed, tang_speed=0.3)
    p = sc.params
    p.lg_iterations = 1
    env = sc.envs[0]
    env.young = 1e-9
    oe = O.precompute(env, p.h)
    x, v = sc.x0[0], sc.v0[0]
    rng = np.random.default_rng(seed)
    con = O.detect(x, v, sc.obstacles[0], p)
    lam0 = np.abs(rng.normal(scale=0.05, size=(con.count, 3)))
    li = O.step_lightweight(oe, x, v, sc.obstacles[0], p, newton_iterations=1, lam_warm=lam0)
    qt = O.predicted_state(x, v, p.h, p.gravity)
    qb = oe.solve(O.assemble_rhs(oe, qt, O.project(oe, qt), p.h))
    csp, _, _ = O.build_csp(oe, x, qb, li.contacts, p.h, p.max_force)
    s = p.h ** 2 / oe.mass[li.contacts.vertex]
    Jm, phi = O.generalized_jacobian(csp, lam0, s)
    d = np.linalg.solve(Jm, -phi.reshape(-1)).reshape(-1, 3)
    np.testing.assert_allclose(li.info["lam_history"][0], lam0 + d, rtol=1e-6, atol=1e-9)
