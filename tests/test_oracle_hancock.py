"""Pins of the oracle's MUSCL-Hancock predictor (the half-step evolution of
the face states the paper names after Toro, Chap. 14).

The half-step rate of a node is checked against time derivatives that two
exact smooth solutions of the Euler equations fix by other means:

* an isentropic vortex carried by a uniform stream is a steady solution in
  the moving frame, so every variable (and a passive mass fraction that
  depends on the radius only) obeys d/dt = -U0 . grad;
* a simple wave keeps every quantity constant along its C+ characteristics,
  so d/dt = -(u_n + c) d/dxi with xi the distance along the wave normal.

The vortex exercises the pressure gradient, the convective terms and the
cross terms between directions (it is divergence-free); the simple wave
exercises every div u term.  Gradients come from the complex-step
derivative of the closed-form fields, exact to rounding.

The scheme-level pin: with the unlimited reconstruction, one forward-Euler
stage with the predictor converges at second order on a smooth entropy wave
(the exact solution is its translation), where the same stage without it is
first order in time.
"""
import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import workloads as wl

GAMMA = 1.4


def _rows(nd, rho, vel, p, Y, gamma=GAMMA):
    """(rho, rho u, rho E, rho Y, p) from primitives (complex-safe)."""
    ke = 0.5 * rho * sum(v * v for v in vel)
    return [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke] + [rho * y for y in Y] + [p]


def _grad_complex_step(field, x, h=1e-30):
    """d field / dx_d at x for each d by the complex-step derivative."""
    x = np.asarray(x, dtype=np.complex128)
    cols = []
    for d in range(len(x)):
        xp = x.copy()
        xp[d] += 1j * h
        cols.append(np.imag(np.asarray(field(xp))) / h)
    return np.stack(cols, axis=1)   # [nr][nd]


def _vortex(nd, nsp, U0, eps=5.0, gamma=GAMMA):
    def field(x):
        xb, yb = x[0] - 0.3, x[1] + 0.2
        r2 = xb * xb + yb * yb
        f = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
        T = 1.0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        vel = [U0[0] - f * yb, U0[1] + f * xb] + ([U0[2]] if nd == 3 else [])
        Y = [0.3 + 0.2 * (k + 1) * np.exp(-0.7 * r2) for k in range(nsp)]
        return _rows(nd, rho, vel, p, Y, gamma)
    return field


def _simple_wave(nd, nsp, n, ut, gamma=GAMMA):
    """Right-running simple wave along the unit normal n with a uniform
    tangential velocity ut (orthogonal to n) and uniform mass fractions.
    u_n(xi) is smooth; the Riemann invariant u_n - 2c/(gamma-1) is uniform."""
    rho0, p0, u0 = 1.2, 0.9, 0.4
    c0 = np.sqrt(gamma * p0 / rho0)

    def state(x):
        xi = sum(n[d] * x[d] for d in range(nd))
        un = u0 + 0.3 * np.sin(2.0 * xi) + 0.1 * np.cos(3.0 * xi)
        c = c0 + 0.5 * (gamma - 1.0) * (un - u0)
        rho = rho0 * (c / c0) ** (2.0 / (gamma - 1.0))
        p = p0 * (rho / rho0) ** gamma
        vel = [un * n[d] + ut[d] for d in range(nd)]
        Y = [0.1 * (k + 1) for k in range(nsp)]
        return _rows(nd, rho, vel, p, Y, gamma), un, c
    return state


@pytest.mark.parametrize("nd,nsp", [(2, 0), (2, 2), (3, 0), (3, 9)])
def test_rate_of_an_advected_isentropic_vortex_is_its_translation(nd, nsp):
    U0 = [0.7, -0.4, 0.25][:nd]
    field = _vortex(nd, nsp, U0)
    rng = np.random.default_rng(nd * 10 + nsp)
    for _ in range(6):
        x = rng.uniform(-1.5, 1.5, size=nd)
        w = np.real(np.asarray(field(x.astype(np.complex128))))
        g = _grad_complex_step(field, x)
        rate = oracle.hancock_rate(nd, nsp, w, g, GAMMA)
        want = -g @ np.asarray(U0)
        scale = np.abs(g).sum(axis=1) * np.abs(U0).max() + np.abs(want)
        assert np.all(np.abs(rate - want) <= 1e-13 * scale + 1e-15), (rate, want)


@pytest.mark.parametrize("nd,nsp", [(2, 0), (2, 2), (3, 0), (3, 2)])
def test_rate_of_a_simple_wave_follows_its_characteristics(nd, nsp):
    rng = np.random.default_rng(100 + nd * 10 + nsp)
    for _ in range(6):
        n = rng.normal(size=nd)
        n /= np.linalg.norm(n)
        t = rng.normal(size=nd)
        t -= (t @ n) * n
        ut = 0.5 * t
        st = _simple_wave(nd, nsp, n, ut)
        x = rng.uniform(-1.0, 1.0, size=nd)
        rows, un, c = st(x.astype(np.complex128))
        w = np.real(np.asarray(rows))
        g = _grad_complex_step(lambda y: st(y)[0], x)
        rate = oracle.hancock_rate(nd, nsp, w, g, GAMMA)
        # every quantity is a function of xi - (u_n + c) t along C+
        want = -np.real(un + c) * (g @ n)
        scale = np.abs(g).sum(axis=1) * 3.0 + np.abs(want)
        assert np.all(np.abs(rate - want) <= 1e-13 * scale + 1e-15), (rate, want)


def test_rate_of_a_uniform_state_is_zero():
    w = np.array([1.3, 0.4, -0.2, 2.9, 0.26, 1.1])
    rate = oracle.hancock_rate(2, 1, w, np.zeros((6, 2)), GAMMA)
    assert np.array_equal(rate, np.zeros(6))


def _entropy_wave_error(nx, predictor, t_end=0.5):
    """L1 density error of a sine entropy wave carried at u = 1 through a
    periodic strip of nx x 3 quads (split in triangles), one forward-Euler
    stage per step, unlimited reconstruction, HLLC."""
    m = wl.tri_rect_mesh(nx, 3, 1.0, 3.0 / nx, periodic=True)
    x = m.xyz[0]
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * x)
    P = np.stack([rho, np.ones_like(x), np.zeros_like(x), np.ones_like(x)])
    ph = oracle.Phys(limiter=4, rk=1, closure=0, cfl=0.4, predictor=predictor)  # 4: unlimited
    U = oracle.conserved_from_primitive(2, ph, P)
    Ue, t, *_ = oracle.OracleMesh(m).step(ph, U, nsteps=100000, t_end=t_end)
    assert t == pytest.approx(t_end, abs=1e-14)
    exact = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x - t_end))
    return np.mean(np.abs(Ue[0] - exact))


def test_predictor_makes_the_single_stage_second_order():
    ns = (16, 32, 64)
    with_p = [_entropy_wave_error(n, 1) for n in ns]
    without = [_entropy_wave_error(n, 0) for n in ns]
    rate_p = np.log2(with_p[1] / with_p[2])
    rate_0 = np.log2(without[1] / without[2])
    print(f"errors with predictor {with_p} (rate {rate_p:.2f}), without {without} (rate {rate_0:.2f})")
    assert rate_p >= 1.8
    assert rate_0 <= 1.3
    assert with_p[2] < 0.2 * without[2]


def test_predictor_keeps_uniform_flow_exact():
    """A uniform stream through a jittered periodic mesh stays uniform: the
    rate of a uniform state is zero and the fluxes cancel."""
    m = wl.tri_rect_mesh(9, 7, 1.0, 0.8, jitter=0.25, seed=3, periodic=True)
    nn = m.nnodes
    ph = oracle.Phys(limiter=2, rk=1, closure=0, predictor=1)
    P = np.stack([np.full(nn, 1.1), np.full(nn, 0.3), np.full(nn, -0.2), np.full(nn, 0.9)])
    U = oracle.conserved_from_primitive(2, ph, P)
    Ue, *_ = oracle.OracleMesh(m).step(ph, U, nsteps=5)
    assert np.allclose(Ue, U, rtol=0, atol=1e-13)


@pytest.mark.parametrize("bad", [dict(rk=2), dict(model=oracle.DRIFT_DIFFUSION, nspecies=1)])
def test_predictor_combinations_outside_its_definition_are_rejected(bad):
    m = wl.tri_rect_mesh(4, 3, periodic=True)
    ph = oracle.Phys(rk=1, predictor=1, closure=0)
    for k, v in bad.items():
        setattr(ph, k, v)
    nvar = ph.nvar(2)
    U = np.ones((nvar, m.nnodes))
    with pytest.raises(oracle.OracleError):
        oracle.OracleMesh(m).residual(ph, U, E=np.zeros((2, m.nnodes)), dt=1e-3)


@pytest.mark.parametrize("nd", [2, 3])
def test_predicted_residual_does_not_depend_on_the_vertex_order(nd):
    """The face states of an edge take each end's own half-step rate: the
    residual is the same whichever end a cell lists first."""
    if nd == 2:
        m = wl.tri_rect_mesh(8, 6, 1.0, 0.7, jitter=0.2, seed=5, periodic=True)
    else:
        m = wl.kuhn_tet_mesh(4, 3, 3, jitter=0.15, seed=5, periodic=True)
    rng = np.random.default_rng(7)
    nn, x = m.nnodes, m.xyz
    ph = oracle.Phys(limiter=2, rk=1, closure=0, predictor=1, nspecies=1)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])
    vel = [0.4 + 0.2 * np.cos(2 * np.pi * x[1])] + [0.1 * np.sin(2 * np.pi * x[0])] * (nd - 1)
    p = 1.0 + 0.2 * np.cos(2 * np.pi * (x[0] + x[1])) + 0.01 * rng.random(nn)
    P = np.stack([rho, *vel, p, 0.5 + 0.3 * np.sin(2 * np.pi * x[0])])
    U = oracle.conserved_from_primitive(nd, ph, P)
    r0 = oracle.OracleMesh(m).residual(ph, U, dt=0.02)
    rev = wl.Mesh(m.xyz, m.cells[::-1].copy(), m.period, m.name + "-rev", dict(m.meta))
    for mm in (rev, wl.fix_orientation_free(m)):
        r1 = oracle.OracleMesh(mm).residual(ph, U, dt=0.02)
        assert np.allclose(r1, r0, rtol=0, atol=1e-12 * np.abs(r0).max())
    # and the predictor changes the residual (dt enters)
    r2 = oracle.OracleMesh(m).residual(ph, U, dt=0.0)
    assert np.abs(r2 - r0).max() > 1e-4 * np.abs(r0).max()
