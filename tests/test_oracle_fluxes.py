"""Pins of the oracle's limiters and Riemann fluxes against hand values,
textbook identities and symmetry properties.

Paper passages: Sec. "Limited Lax-Wendroff scheme" (limiters of van Leer and
Sweby), Sec. "The HLLC solver" (rotated Riemann problem, eq.
hllc_formulation_mutlicomponent).  The Roe flux is not in the paper (textbook).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import MINMOD, SWEBY, VANLEER, prim_to_W

LIMS = [(MINMOD, 1.0), (VANLEER, 1.0), (SWEBY, 1.0), (SWEBY, 1.5), (SWEBY, 2.0)]


@pytest.mark.parametrize("kind,beta", LIMS)
def test_slope_limiter_identities(kind, beta):
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = rng.normal(size=2) * 10 ** rng.uniform(-3, 3)
        L = oracle.slope_limiter(kind, beta, a, b)
        assert L == oracle.slope_limiter(kind, beta, b, a)            # symmetric
        if a * b <= 0:
            assert L == 0.0
        else:
            assert math.copysign(1, L) == math.copysign(1, a)
            assert abs(L) <= 2 * min(abs(a), abs(b)) * (1 + 1e-15)   # TVD bound
            assert abs(L) >= min(abs(a), abs(b)) * (1 - 1e-15) or kind == VANLEER
        assert oracle.slope_limiter(kind, beta, a, a) == pytest.approx(a, rel=1e-15)


def test_slope_limiter_hand_values():
    assert oracle.slope_limiter(MINMOD, 1, 1.0, 3.0) == 1.0
    assert oracle.slope_limiter(VANLEER, 1, 1.0, 3.0) == 1.5
    assert oracle.slope_limiter(SWEBY, 2.0, 1.0, 3.0) == 2.0           # superbee
    assert oracle.slope_limiter(SWEBY, 1.5, 1.0, 3.0) == 1.5
    assert oracle.slope_limiter(SWEBY, 1.0, -1.0, -3.0) == -1.0        # = minmod
    assert oracle.slope_limiter(oracle.FIRST_ORDER, 1, 1.0, 3.0) == 0.0
    assert oracle.slope_limiter(oracle.UNLIMITED, 1, 1.0, 3.0) == 2.0


@pytest.mark.parametrize("kind,beta", LIMS)
def test_psi_limiter_in_sweby_tvd_region(kind, beta):
    for R in np.linspace(-3, 6, 181):
        psi = oracle.psi_limiter(kind, beta, R, 1.0)
        if R <= 0:
            assert psi == 0.0
        else:
            assert 0.0 <= psi <= min(2 * R, 2.0) + 1e-15
    assert oracle.psi_limiter(kind, beta, 1.0, 1.0) == pytest.approx(1.0)  # second order at R = 1
    assert oracle.psi_limiter(kind, beta, 1.0, 0.0) == 0.0                 # b = 0 -> first order


def test_psi_limiter_hand_values():
    assert oracle.psi_limiter(VANLEER, 1, 3.0, 1.0) == pytest.approx(1.5)   # 2R/(1+R)
    assert oracle.psi_limiter(MINMOD, 1, 0.4, 1.0) == pytest.approx(0.4)
    assert oracle.psi_limiter(SWEBY, 2.0, 0.4, 1.0) == pytest.approx(0.8)   # superbee
    assert oracle.psi_limiter(SWEBY, 2.0, 3.0, 1.0) == pytest.approx(2.0)
    assert oracle.psi_limiter(oracle.UNLIMITED, 1, -5.0, 1.0) == 1.0


def test_euler_flux_hand_value():
    # rho = 1, u = (2, 0), p = 1, gamma = 1.4: rhoE = 2.5 + 2 = 4.5
    W = prim_to_W(1.0, [2.0, 0.0], 1.0)
    F = oracle.euler_flux(2, 0, W, np.array([1.0, 0.0]))
    np.testing.assert_allclose(F, [2.0, 5.0, 0.0, 11.0])
    F = oracle.euler_flux(2, 0, W, np.array([0.0, 2.0]))   # flux through a y-face of length 2
    np.testing.assert_allclose(F, [0.0, 0.0, 2.0, 0.0])


def _rand_state(rng, nd, nsp, mach=0.5):
    rho = rng.uniform(0.3, 2.0)
    p = rng.uniform(0.2, 3.0)
    a = math.sqrt(1.4 * p / rho)
    vel = rng.normal(size=nd) * mach * a
    Y = rng.dirichlet(np.ones(nsp)) if nsp else []
    return prim_to_W(rho, vel, p, 1.4, Y)


def _rot3(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q


def _rotate_W(W, R, nd):
    W = W.copy()
    W[1:1 + nd] = R @ W[1:1 + nd]
    return W


FLUXES = [("hllc", lambda nd, nsp, L, R, S: oracle.hllc(nd, nsp, L, R, S)),
          ("roe", lambda nd, nsp, L, R, S: oracle.roe(nd, nsp, L, R, S, fix=0.1))]


@pytest.mark.parametrize("name,flux", FLUXES)
@pytest.mark.parametrize("nd,nsp", [(2, 0), (3, 0), (3, 3)])
def test_consistency(name, flux, nd, nsp):
    rng = np.random.default_rng(2)
    for _ in range(50):
        W = _rand_state(rng, nd, nsp)
        S = rng.normal(size=nd)
        np.testing.assert_allclose(flux(nd, nsp, W, W, S), oracle.euler_flux(nd, nsp, W, S),
                                   rtol=1e-13, atol=1e-13 * np.abs(W).max() * np.abs(S).max())


@pytest.mark.parametrize("name,flux", FLUXES)
@pytest.mark.parametrize("nd,nsp", [(2, 0), (3, 2)])
def test_supersonic_upwinding(name, flux, nd, nsp):
    """All waves to the right: the flux is F(W_L) (for Roe this is the Roe
    property sum lambda alpha K = F_R - F_L)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = rng.normal(size=nd)
        n /= np.linalg.norm(n)
        WL = _rand_state(rng, nd, nsp, mach=0.1)
        WR = _rand_state(rng, nd, nsp, mach=0.1)
        for W in (WL, WR):  # add a normal velocity of Mach 3 to both sides
            rho = W[0]
            a = math.sqrt(1.4 * W[-1] / rho)
            u_old = W[1:1 + nd] / rho
            u_new = u_old + 3.0 * 3.3 * n
            W[1 + nd] += 0.5 * rho * (u_new @ u_new - u_old @ u_old)
            W[1:1 + nd] = rho * u_new
        S = 0.7 * n
        F = flux(nd, nsp, WL, WR, S)
        np.testing.assert_allclose(F, oracle.euler_flux(nd, nsp, WL, S), rtol=1e-12, atol=1e-12)
        F = flux(nd, nsp, WR, WL, -S)
        np.testing.assert_allclose(F, oracle.euler_flux(nd, nsp, WL, -S), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name,flux", FLUXES)
def test_stationary_contact_is_exact(name, flux):
    WL = prim_to_W(1.0, [0.0, 0.3], 0.7)
    WR = prim_to_W(0.2, [0.0, -0.4], 0.7)
    S = np.array([0.5, 0.0])
    F = flux(2, 0, WL, WR, S)
    np.testing.assert_allclose(F, [0.0, 0.35, 0.0, 0.0], atol=1e-15)


@pytest.mark.parametrize("name,flux", FLUXES)
@pytest.mark.parametrize("nd,nsp", [(2, 0), (3, 2)])
def test_rotation_invariance_and_antisymmetry(name, flux, nd, nsp):
    rng = np.random.default_rng(4)
    for _ in range(30):
        WL, WR = _rand_state(rng, nd, nsp, 1.2), _rand_state(rng, nd, nsp, 1.2)
        S = rng.normal(size=nd)
        F = flux(nd, nsp, WL, WR, S)
        R = _rot3(rng)[:nd, :nd] if nd == 3 else np.array([[0.6, -0.8], [0.8, 0.6]])
        Fr = flux(nd, nsp, _rotate_W(WL, R, nd), _rotate_W(WR, R, nd), R @ S)
        Fexp = F.copy()
        Fexp[1:1 + nd] = R @ F[1:1 + nd]
        np.testing.assert_allclose(Fr, Fexp, rtol=1e-12, atol=1e-12 * np.abs(F).max())
        Fa = flux(nd, nsp, WR, WL, -S)
        np.testing.assert_allclose(Fa, -F, rtol=1e-12, atol=1e-12 * np.abs(F).max())


def _normal_shock(M1=2.0, g=1.4):
    """Stationary normal shock from the Rankine-Hugoniot relations."""
    r1, p1 = 1.0, 1.0
    a1 = math.sqrt(g * p1 / r1)
    u1 = M1 * a1
    r2 = r1 * (g + 1) * M1 ** 2 / ((g - 1) * M1 ** 2 + 2)
    p2 = p1 * (1 + 2 * g / (g + 1) * (M1 ** 2 - 1))
    u2 = u1 * r1 / r2
    return prim_to_W(r1, [u1, 0.0], p1), prim_to_W(r2, [u2, 0.0], p2)


def test_roe_captures_stationary_shock_exactly():
    WL, WR = _normal_shock()
    S = np.array([1.0, 0.0])
    FL = oracle.euler_flux(2, 0, WL, S)
    np.testing.assert_allclose(oracle.euler_flux(2, 0, WR, S), FL, rtol=1e-13)
    np.testing.assert_allclose(oracle.roe(2, 0, WL, WR, S, fix=0.0), FL, rtol=1e-13, atol=1e-13)


def test_hllc_star_states_satisfy_rankine_hugoniot():
    """Recover the HLLC star state from the flux, U*_K = U_K + (F - F_K)/S_K,
    and check it against the Rankine-Hugoniot form of the star state (Toro,
    Ch. 10): density rho_K (S_K - q_K)/(S_K - S*), normal velocity S*,
    unchanged tangential velocity and species fractions, and energy
    (S_K - S*) (rho E)*_K = (S_K - q_K)(rho E)_K - p_K q_K + p* S* with
    p* = p_K + rho_K (S_K - q_K)(S* - q_K).  This exercises the energy
    entry of eq. (hllc_formulation_mutlicomponent)."""
    rng = np.random.default_rng(9)
    nd, nsp = 3, 2
    hits = {"L": 0, "R": 0}
    for _ in range(400):
        WL, WR = _rand_state(rng, nd, nsp, 0.8), _rand_state(rng, nd, nsp, 0.8)
        n = rng.normal(size=nd)
        n /= np.linalg.norm(n)
        F = oracle.hllc(nd, nsp, WL, WR, n)
        st = {}
        for k, W in (("L", WL), ("R", WR)):
            rho, p = W[0], W[-1]
            u = W[1:1 + nd] / rho
            st[k] = (rho, u, u @ n, p, math.sqrt(1.4 * p / rho), W[1 + nd])
        rL, _, qL, pL, aL, _ = st["L"]
        rR, _, qR, pR, aR, _ = st["R"]
        SL, SR = min(qL - aL, qR - aR), max(qL + aL, qR + aR)
        Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) / (rL * (SL - qL) - rR * (SR - qR))
        if not (SL < 0 < SR):
            continue
        k, SK, W = ("L", SL, WL) if Ss >= 0 else ("R", SR, WR)
        hits[k] += 1
        rho, u, q, p, a, rE = st[k]
        Us = W[:-1] + (F - oracle.euler_flux(nd, nsp, W, n)) / SK
        rs = rho * (SK - q) / (SK - Ss)
        ps = p + rho * (SK - q) * (Ss - q)
        assert Us[0] == pytest.approx(rs, rel=1e-11)
        us = Us[1:1 + nd] / Us[0]
        assert us @ n == pytest.approx(Ss, abs=1e-11)
        np.testing.assert_allclose(us - (us @ n) * n, u - q * n, atol=1e-11)
        np.testing.assert_allclose(Us[2 + nd:] / Us[0], W[2 + nd:-1] / rho, rtol=1e-11)
        assert Us[1 + nd] * (SK - Ss) == pytest.approx((SK - q) * rE - p * q + ps * Ss, rel=1e-11)
    assert hits["L"] > 20 and hits["R"] > 20
