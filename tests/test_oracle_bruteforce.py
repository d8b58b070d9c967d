"""Brute-force enumeration of stick / slip / separate modes on 1-3 contacts.

For every assignment of modes the contact subproblem (Eq. 2b with the exact
Delassus operator) reduces to a small system: separate -> lambda = 0;
stick -> C_n = 0 and u_t = 0; slip -> C_n = 0, lambda_t = mu lambda_n d(theta)
and u_t = -gamma d(theta), gamma > 0.  Every feasible solution is collected;
the oracle's Newton solution must be one of them, and equal to it when the
feasible set is a single point.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import root

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes


def _csp_for(seed, lift, speed=0.2):
    sc = scenes.single_tet_scene(seed=seed, tang_speed=speed)
    x = sc.x0[0].copy()
    for i, dy in enumerate(lift):
        x[i, 1] += dy
    v = sc.v0[0]
    h = sc.params.h
    oe = O.precompute(sc.envs[0], h)
    c = O.detect(x, v, sc.obstacles[0], sc.params)
    qt = O.predicted_state(x, v, h, sc.params.gravity)
    qb = oe.solve(O.assemble_rhs(oe, qt, O.project(oe, qt), h))
    csp, _, _ = O.build_csp(oe, x, qb, c, h, 1e10)
    return csp, c


def _enumerate(csp):
    c = csp.d0.shape[0]
    mu = csp.mu
    sols = []
    for modes in itertools.product("0SL", repeat=c):
        slip = [j for j in range(c) if modes[j] == "L"]
        stick = [j for j in range(c) if modes[j] == "S"]

        def unpack(z):
            lam = np.zeros((c, 3))
            extra = {}
            k = 0
            for j in range(c):
                if modes[j] == "S":
                    lam[j] = z[k:k + 3]
                    k += 3
                elif modes[j] == "L":
                    ln, th, gam = z[k:k + 3]
                    k += 3
                    lam[j] = [ln, mu * ln * math.cos(th), mu * ln * math.sin(th)]
                    extra[j] = (th, gam)
            return lam, extra

        def fun(z):
            lam, extra = unpack(z)
            Y = (csp.y0 + csp.W @ lam.reshape(-1)).reshape(c, 3)
            res = []
            for j in range(c):
                if modes[j] == "S":
                    res += [csp.d0[j] + Y[j, 0], *(Y[j, 1:] - csp.dob[j])]
                elif modes[j] == "L":
                    th, gam = extra[j]
                    ut = Y[j, 1:] - csp.dob[j]
                    res += [csp.d0[j] + Y[j, 0], ut[0] + gam * math.cos(th), ut[1] + gam * math.sin(th)]
            return np.array(res) * 1e3

        nunk = 3 * (len(stick) + len(slip))
        starts = []
        if nunk == 0:
            starts = [np.zeros(0)]
        else:
            for a in range(8):
                z = []
                for j in range(c):
                    if modes[j] == "S":
                        z += [1.0, 0.0, 0.0]
                    elif modes[j] == "L":
                        z += [1.0, 2 * math.pi * a / 8 + 0.1 * j, 1e-3]
                starts.append(np.array(z))
        for z0 in starts:
            if nunk:
                sol = root(fun, z0, method="hybr", options={"xtol": 1e-14, "maxfev": 4000})
                if not np.all(np.isfinite(sol.x)) or np.max(np.abs(fun(sol.x))) > 1e-9:
                    continue
                z = sol.x
            else:
                z = z0
            lam, extra = unpack(z)
            Y = (csp.y0 + csp.W @ lam.reshape(-1)).reshape(c, 3)
            Cn = csp.d0 + Y[:, 0]
            ok = True
            for j in range(c):
                if modes[j] == "0":
                    ok &= Cn[j] >= -1e-13
                else:
                    ok &= lam[j, 0] >= -1e-12
                if modes[j] == "S":
                    ok &= np.linalg.norm(lam[j, 1:]) <= mu * lam[j, 0] * (1 + 1e-9) + 1e-13
                if modes[j] == "L":
                    ok &= extra[j][1] > 0
            if ok and not any(np.allclose(lam, s, rtol=1e-7, atol=1e-10) for s in sols):
                sols.append(lam)
    return sols


CASES = [
    (0, (0.0, 0.0, 0.0), 0.2),          # three sliding contacts
    (1, (0.0, 0.0, 0.0), 0.2),
    (2, (0.0, 0.003, 0.0), 0.2),        # one vertex lifts off
    (3, (0.003, 0.003, 0.0), 0.2),      # single active contact
    (4, (0.0, 0.0, 0.0006), 0.2),       # third vertex hovers in the margin
    (5, (0.0, 0.0, 0.0), 0.002),        # slow: friction sticks
    (6, (0.0, 0.0, 0.0), 0.002),
    (7, (0.0, 0.0012, 0.0), 0.0005),
    (8, (0.0, 0.0, 0.0), 0.02),         # near the stick/slip threshold
    (9, (0.0, 0.0, 0.0), 0.03),
]


@pytest.mark.parametrize("seed,lift,speed", CASES)
def test_newton_solution_is_an_enumerated_mode_solution(seed, lift, speed):
    csp, c = _csp_for(seed, lift, speed)
    assert 1 <= c.count <= 3
    sols = _enumerate(csp)
    assert len(sols) >= 1
    lam, r, info = O.solve_csp(csp, tol=1e-13)
    assert r <= 1e-13
    match = [np.allclose(lam, s, rtol=1e-6, atol=1e-9) for s in sols]
    assert any(match)
    if len(sols) == 1:
        assert match[0]


def test_frictionless_lcp_matches_active_set_enumeration():
    """mu = 0: the subproblem is an LCP; enumerate 2^c active sets of normal rows."""
    csp, c = _csp_for(0, (0.0, 0.0, 0.0))
    csp = O.CSP(csp.y0, csp.W, csp.d0, csp.dob, csp.s, 0.0, csp.max_force)
    n = csp.d0.shape[0]
    Wn = csp.W[0::3, 0::3]
    y0n = csp.y0[0::3]
    found = []
    for act in itertools.product([0, 1], repeat=n):
        A = [j for j in range(n) if act[j]]
        ln = np.zeros(n)
        if A:
            ln[A] = np.linalg.solve(Wn[np.ix_(A, A)], -(csp.d0[A] + y0n[A]))
        Cn = csp.d0 + y0n + Wn @ ln
        if np.all(ln >= -1e-14) and np.all(Cn >= -1e-14):
            found.append(ln)
    assert len(found) == 1
    lam, r, _ = O.solve_csp(csp, tol=1e-14)
    assert np.allclose(lam[:, 0], found[0], rtol=1e-9, atol=1e-12)
    assert np.allclose(lam[:, 1:], 0.0, atol=1e-12)
