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


# ---------------------------------------------------------------------------
# Roe's entropy fix and the HLLC wave speeds, pinned by properties that any
# correct form satisfies (Toro, Ch. 8 for Harten's fix, Ch. 10 for the Davis
# estimates), measured from the flux the oracle returns.
# ---------------------------------------------------------------------------

def _prim(W, nd=2, g=1.4):
    rho = W[0]
    u = W[1:1 + nd] / rho
    p = W[-1]
    return rho, u, p


def _roe_average(WL, WR, n, g=1.4):
    """Textbook Roe average (Toro, Ch. 11): normal velocity q, sound speed a,
    and the strengths of the two acoustic waves alpha_1, alpha_5."""
    rL, uL, pL = _prim(WL)
    rR, uR, pR = _prim(WR)
    HL = (WL[3] + pL) / rL
    HR = (WR[3] + pR) / rR
    wL, wR = math.sqrt(rL), math.sqrt(rR)
    u = (wL * uL + wR * uR) / (wL + wR)
    H = (wL * HL + wR * HR) / (wL + wR)
    a = math.sqrt((g - 1.0) * (H - 0.5 * u @ u))
    rho = wL * wR
    dq = (uR - uL) @ n
    dp = pR - pL
    al1 = (dp - rho * a * dq) / (2 * a * a)
    al5 = (dp + rho * a * dq) / (2 * a * a)
    return u @ n, a, u, H, al1, al5


def _shift_normal(W, c, n):
    """Add the velocity c n to a 2D state (a Galilean shift: the Roe sound
    speed is unchanged, every Roe eigenvalue moves by c)."""
    rho, u, p = _prim(W)
    return prim_to_W(rho, u + c * n, p)


def _fixed_eigenvalue(WL, WR, n, A, wave):
    """|lambda| after the entropy fix, read off the flux: only the fixed
    acoustic wave changes between fix on and off, by -A/2 (l_fix - |l|)
    alpha K with a unit mass entry in K."""
    q, a, u, H, al1, al5 = _roe_average(WL, WR, n)
    lam, al = (q - a, al1) if wave == 1 else (q + a, al5)
    S = A * n
    Fon = oracle.roe(2, 0, WL, WR, S, fix=0.1)
    Foff = oracle.roe(2, 0, WL, WR, S, fix=0.0)
    d = Fon - Foff
    lfix = abs(lam) - 2.0 * d[0] / (A * al)
    sgn = -1.0 if wave == 1 else 1.0
    K = np.array([1.0, *(u + sgn * a * n), H + sgn * (u @ n) * a])
    return lam, 0.1 * a, lfix, d, -0.5 * A * (lfix - abs(lam)) * al * K


@pytest.mark.parametrize("wave", [1, 5])
def test_roe_entropy_fix_properties(wave):
    """Harten's fix replaces |lambda| of an acoustic wave near a sonic point
    by a smooth positive function.  Whatever its exact form, it must (i)
    leave |lambda| >= delta unchanged, (ii) be continuous where it starts to
    act, at |lambda| = delta, (iii) never lower the dissipation, (iv) be
    even and grow with |lambda|, and (v) for the parabola of Harten and
    Hyman, give delta / 2 at the sonic point.  Only the fixed wave's
    dissipation may change: the flux difference is along its eigenvector."""
    n = np.array([0.8, 0.6])
    A = 0.37
    WL0 = prim_to_W(1.0, np.array([0.2, -0.1]), 1.0)
    WR0 = prim_to_W(0.7, np.array([0.05, 0.15]), 0.6)
    q0, a0, *_ = _roe_average(WL0, WR0, n)
    delta = 0.1 * a0
    target0 = (q0 - a0) if wave == 1 else (q0 + a0)
    lams, fixed = [], []
    for x in np.concatenate([np.linspace(-2.0, 2.0, 81), [-1 + 1e-9, 1 - 1e-9, 1 + 1e-9, 0.0]]):
        c = x * delta - target0
        WL, WR = _shift_normal(WL0, c, n), _shift_normal(WR0, c, n)
        lam, dl, lfix, d, dexp = _fixed_eigenvalue(WL, WR, n, A, wave)
        assert dl == pytest.approx(delta, rel=1e-12)
        assert lam == pytest.approx(x * delta, abs=1e-12)
        scale = np.abs(oracle.roe(2, 0, WL, WR, A * n, fix=0.0)).max()
        np.testing.assert_allclose(d, dexp, atol=1e-12 * scale)       # only this wave changes
        if abs(lam) >= delta * (1 + 1e-9):
            assert lfix == pytest.approx(abs(lam), abs=1e-11)         # (i)
        assert lfix >= abs(lam) - 1e-11                              # (iii)
        lams.append(lam)
        fixed.append(lfix)
    lams, fixed = np.array(lams), np.array(fixed)
    at = lambda v: fixed[np.argmin(np.abs(lams - v))]
    assert at(0.0) == pytest.approx(0.5 * delta, rel=1e-9)            # (v)
    for s in (-1, 1):                                                # (ii)
        assert at(s * (1 - 1e-9) * delta) == pytest.approx(delta, rel=1e-7)
    order = np.argsort(lams)
    L, Fx = lams[order], fixed[order]
    inside = np.abs(L) < delta
    assert np.allclose(np.interp(-L[inside], L, Fx), Fx[inside], rtol=1e-9)   # (iv) even
    neg, pos = inside & (L < 0), inside & (L > 0)
    assert np.all(np.diff(Fx[neg]) <= 1e-14) and np.all(np.diff(Fx[pos]) >= -1e-14)


def _with_normal_speed(rho, p, vt, target, n, t, kind):
    """State whose normal velocity puts q - a (kind -1) or q + a (kind +1)
    at target; vt is its tangential velocity."""
    a = math.sqrt(1.4 * p / rho)
    q = target - kind * a
    return prim_to_W(rho, q * n + vt * t, p)


def test_hllc_fully_upwind_exactly_when_every_wave_moves_one_way():
    """The Davis estimates bound the fan by the extreme characteristic speeds
    of the two states, S_L = min(q_L - a_L, q_R - a_R), S_R = max(q_L + a_L,
    q_R + a_R).  So the flux is the left physical flux exactly when the
    slowest speed of both states is >= 0, and differs from it as soon as one
    of them is negative (and mirrored for right-moving states); across the
    switch the flux is continuous."""
    n = np.array([0.6, -0.8])
    t = np.array([0.8, 0.6])
    S = 0.45 * n
    for kind in (-1, 1):
        fixed = _with_normal_speed(1.0, 1.0, 0.3, kind * -0.25, n, t, kind)
        for s in [-0.3, -0.1, -0.01, -1e-7, 0.0, 1e-7, 0.01, 0.3]:
            other = _with_normal_speed(0.4, 0.5, -0.2, -kind * s, n, t, kind)
            # kind -1: the left state is supersonic to the right (q_L - a_L =
            # 0.25) and the right state's slowest speed is s; kind +1 mirrors it
            WL, WR = (fixed, other) if kind == -1 else (other, fixed)
            F = oracle.hllc(2, 0, WL, WR, S)
            Fup = oracle.euler_flux(2, 0, WL if kind == -1 else WR, S)
            gap = np.abs(F - Fup).max() / np.abs(Fup).max()
            if s >= 0:
                assert gap <= 1e-15
            elif s <= -0.01:
                assert gap >= 1e-4
            else:
                assert gap <= 1e-5        # continuous through the switch


def _godunov_flux(WL, WR, n, g=1.4):
    """Exact Godunov flux through the unit normal n: the exact Riemann
    solution of the normal problem sampled at x/t = 0 (tests.exact_riemann,
    independent of the oracle), tangential velocity taken from the upwind
    side of the contact."""
    import exact_riemann as er
    t = np.array([-n[1], n[0]])
    rL, uL, pL = _prim(WL)
    rR, uR, pR = _prim(WR)
    L = (rL, uL @ n, pL)
    R = (rR, uR @ n, pR)
    rho, q, p = (v[0] for v in er.sample(L, R, [0.5], 1.0, x0=0.5, g=g))
    _, us = er.star_state(L, R, g)
    vt = (uL @ t) if us >= 0 else (uR @ t)
    W = prim_to_W(rho, q * n + vt * t, p, g)
    return oracle.euler_flux(2, 0, W, n)


@pytest.mark.parametrize("name,flux", FLUXES)
def test_weak_waves_match_the_exact_godunov_flux_to_second_order(name, flux):
    """For a jump of size eps whose three waves are not sonic, a flux whose
    wave speeds are the characteristic speeds to first order matches the
    exact Godunov flux up to O(eps^2) (HLLC: its star states satisfy the
    jump conditions at S_L, S* and S_R, which tend to q - a, q, q + a; Roe:
    exact linearisation).  A wrong speed estimate leaves an O(eps) error."""
    n = np.array([0.28, 0.96])
    t = np.array([-0.96, 0.28])
    base = np.array([1.0, 0.35, 0.2, 1.0])        # rho, q, vt, p: subsonic, 0 < q < a
    dirs = np.array([0.7, -0.4, 0.5, 0.9])
    errs = []
    epss = [4e-2, 2e-2, 1e-2, 5e-3]
    for eps in epss:
        a, b = base - 0.5 * eps * dirs, base + 0.5 * eps * dirs
        WL = prim_to_W(a[0], a[1] * n + a[2] * t, a[3])
        WR = prim_to_W(b[0], b[1] * n + b[2] * t, b[3])
        errs.append(np.abs(flux(2, 0, WL, WR, n) - _godunov_flux(WL, WR, n)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= 1.8, (errs, rates)
    assert errs[-1] <= 1e-4
