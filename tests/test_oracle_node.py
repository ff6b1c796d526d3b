"""Pins of the oracle's per-node arithmetic against what the paper and the mathematics fix.

Each test would fail for a plausible mistake in one oracle function: a wrong sign or
factor in the guided equilibrium, a wrong index in the OReg double sum, a swapped link
set in the corrections, a typo in the stress-error cases.
"""
import numpy as np
import pytest

import oracle
from tests.lbm_diag import CX, CY, node_moments

THETAS = [0.25, 0.3, 1.0 / 3.0, 0.4, 0.5, 0.55]
MODELS = ["bgk", "uc", "partial", "complete"]


def _states(seed, n=24, u_max=0.3, amp=2e-3):
    """Random near-equilibrium states: f = f^eq(rho, u) + perturbation."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        th = float(rng.choice(THETAS))
        rho = float(rng.uniform(0.7, 1.4))
        ux, uy = rng.uniform(-u_max, u_max, size=2)
        f = oracle.guided_equilibrium(rho, ux, uy, th) + amp * rng.uniform(-1, 1, size=9)
        out.append((th, f))
    return out


# --- guided equilibrium (eq:guidedEq) ---------------------------------------------------

def test_geq_six_moments():
    """Sec. 2: the equilibrium carries rho, rho u and the Maxwell-Boltzmann pressure tensor
    rho (u u + theta delta) (eq:density-momentum, eq:ideal-gas-eos-eq-pressure-tensor)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        th = rng.uniform(0.2, 0.6)
        rho = rng.uniform(0.5, 2.0)
        ux, uy = rng.uniform(-0.45, 0.45, size=2)
        r, jx, jy, pxx, pyy, pxy = node_moments(oracle.guided_equilibrium(rho, ux, uy, th))
        np.testing.assert_allclose([r, jx, jy, pxx, pyy, pxy],
                                   [rho, rho * ux, rho * uy, rho * (ux * ux + th), rho * (uy * uy + th),
                                    rho * ux * uy], rtol=0, atol=1e-14 * rho)


def test_geq_rest_state_is_textbook_d2q9_weights():
    """At theta = 1/3 and u = 0 the equilibrium is rho times the D2Q9 weights 4/9, 1/9, 1/36."""
    feq = oracle.guided_equilibrium(1.0, 0.0, 0.0, 1.0 / 3.0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    np.testing.assert_allclose(feq, w, rtol=4e-16, atol=0)


def test_geq_agrees_with_second_order_hermite_equilibrium_to_third_order():
    """At theta = 1/3 the product-form equilibrium equals the textbook quadratic equilibrium
    w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2] up to O(u^3)."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    errs = []
    for eps in (1e-2, 1e-3):
        ux, uy = 0.6 * eps, -0.8 * eps
        cu = CX * ux + CY * uy
        fh = w * 1.1 * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
        errs.append(np.max(np.abs(oracle.guided_equilibrium(1.1, ux, uy, 1 / 3) - fh)))
    assert errs[0] < 1e-6
    assert 500 < errs[0] / errs[1] < 2000  # cubic scaling


# --- OReg population (eq:oreg) ----------------------------------------------------------

def _N(f, feq):
    """Traceless non-equilibrium stress: N_xx = (P_xx - P_yy)/2, N_xy = P_xy of f - f^eq."""
    _, _, _, pxx, pyy, pxy = node_moments(f - feq)
    return 0.5 * (pxx - pyy), pxy


def test_oreg_carries_no_mass():
    for th, f in _states(2):
        p = oracle.collide_node(f, "uc", th, 0.8)
        assert abs(np.sum(p["fo"])) < 1e-17


def test_oreg_reduces_to_projective_regularization_at_rest():
    """At u = 0 and theta = 1/3, f^OReg is the textbook regularized non-equilibrium
    population w_i/(2 c_s^4) (c_i c_i - c_s^2 delta) : dev(Pi^neq), c_s^2 = 1/3."""
    rng = np.random.default_rng(3)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    A = np.stack([np.ones(9), CX, CY], axis=1)
    for _ in range(20):
        d = 1e-3 * rng.uniform(-1, 1, size=9)
        d -= A @ np.linalg.solve(A.T @ A, A.T @ d)  # no mass, no momentum
        f = 1.2 * w + d
        p = oracle.collide_node(f, "uc", 1 / 3, 0.8)
        assert np.max(np.abs(p["u"])) < 1e-15
        _, _, _, pxx, pyy, pxy = node_moments(f - p["feq"])
        tr = 0.5 * (pxx + pyy)
        dev = np.array([[pxx - tr, pxy], [pxy, pyy - tr]])
        cs2 = 1 / 3
        H = lambda a, b, i: (CX[i], CY[i])[a] * (CX[i], CY[i])[b] - cs2 * (a == b)
        ref = np.array([w[i] * p["rho"] / (2 * cs2 ** 2) / p["rho"] *
                        sum(H(a, b, i) * dev[a, b] for a in range(2) for b in range(2)) for i in range(9)])
        np.testing.assert_allclose(p["fo"], ref, rtol=0, atol=1e-15)


def test_oreg_first_moment_closed_form():
    """psi = sum_i c_i f^OReg. With the product form of f^eq its 1-D moments give
    psi_x = -N_xx u_x (u_x^2 + 3 theta - 1)/(2 theta^2),
    psi_y = +N_xx u_y (u_y^2 + 3 theta - 1)/(2 theta^2)   (derivation in the design doc)."""
    for th, f in _states(4):
        p = oracle.collide_node(f, "partial", th, 0.8)
        nxx, _ = _N(f, p["feq"])
        ux, uy = p["u"]
        _, jx, jy, *_ = node_moments(p["fo"])
        ref = [-nxx * ux * (ux * ux + 3 * th - 1) / (2 * th * th), nxx * uy * (uy * uy + 3 * th - 1) / (2 * th * th)]
        np.testing.assert_allclose([jx, jy], ref, rtol=0, atol=1e-16)
        np.testing.assert_allclose(p["psi"], ref, rtol=0, atol=1e-16)


def test_oreg_second_moment_is_paper_variable_viscosity():
    """eq:guidedEq-oreg-viscosity: Pi^OReg_aa = mu_aa N_aa with
    mu_aa = (theta - u_a^2)(1 - theta - u_a^2)/(2 theta^2); off-diagonal
    Pi^OReg_xy = N_xy + N_xx u_x u_y (u_y^2 - u_x^2)/(2 theta^2)."""
    for th, f in _states(5):
        p = oracle.collide_node(f, "uc", th, 0.8)
        nxx, nxy = _N(f, p["feq"])
        ux, uy = p["u"]
        mu = lambda u: (th - u * u) * (1 - th - u * u) / (2 * th * th)
        _, _, _, pxx, pyy, pxy = node_moments(p["fo"])
        np.testing.assert_allclose([pxx, pyy, pxy],
                                   [mu(ux) * nxx, -mu(uy) * nxx, nxy + nxx * ux * uy * (uy * uy - ux * ux) / (2 * th * th)],
                                   rtol=0, atol=2e-16)


# --- corrections (eq:correction, eq:partial-corrections, eq:complete-corrections) --------

def test_partial_corrections_remove_compatibility_error_only():
    """eq:correction with the deviation set relaxed to {psi, 0}: sum Psi = 0,
    sum c Psi = -psi, sum c c Psi = 0."""
    for th, f in _states(6):
        p = oracle.collide_node(f, "partial", th, 0.8)
        r, jx, jy, pxx, pyy, pxy = node_moments(p["Psi"])
        np.testing.assert_allclose([r, jx, jy, pxx, pyy, pxy], [0, -p["psi"][0], -p["psi"][1], 0, 0, 0],
                                   rtol=0, atol=1e-17)
        assert p["Psi"][0] == 0 and np.all(p["Psi"][5:] == 0)


def test_complete_corrections_satisfy_constraints():
    """eq:correction: sum {1, c, c c} Psi^C + {0, psi, Pi~} = 0."""
    for th, f in _states(7):
        p = oracle.collide_node(f, "complete", th, 0.8)
        r, jx, jy, pxx, pyy, pxy = node_moments(p["Psi"])
        Pi = p["Pi"]
        np.testing.assert_allclose([r, jx, jy, pxx, pyy, pxy],
                                   [0, -p["psi"][0], -p["psi"][1], -Pi[0, 0], -Pi[1, 1], -Pi[0, 1]],
                                   rtol=0, atol=1e-16)


def test_stress_error_is_oreg_stress_minus_ns_stress():
    """Pi~ is the deviation of the OReg stress from the Navier-Stokes stress
    (eq:oreg-pressure-tensor). With the exact discrete identities
    Pi^OReg = mu N (diagonal) and the NS stress equal to N, the paper's three cases
    (eq:guidedEq-oreg-stress-tensor-error) must equal (pref / X) (Pi^OReg - N), where
    X = -N_xx/(2 theta^2) is the prefactor's value at the Navier-Stokes level."""
    for th, f in _states(8):
        p = oracle.collide_node(f, "complete", th, 0.8)
        nxx, nxy = _N(f, p["feq"])
        _, _, _, pxx, pyy, pxy = node_moments(p["fo"])
        X = -nxx / (2 * th * th)
        dev = np.array([[pxx - nxx, pxy - nxy], [pxy - nxy, pyy + nxx]])
        np.testing.assert_allclose(p["Pi"] * X, p["pref"] * dev, rtol=0, atol=1e-19)


def test_prefactor_from_oreg_moment():
    """eq:geq-prefactor-evaluation with the paper's variable viscosity:
    pref = -(Pi^OReg_xx - Pi^OReg_yy)/(4 theta^2) = -N_xx (mu_xx + mu_yy)/(4 theta^2)."""
    for th, f in _states(9):
        p = oracle.collide_node(f, "complete", th, 0.8)
        nxx, _ = _N(f, p["feq"])
        ux, uy = p["u"]
        mu = lambda u: (th - u * u) * (1 - th - u * u) / (2 * th * th)
        np.testing.assert_allclose(p["pref"], -nxx * (mu(ux) + mu(uy)) / (4 * th * th), rtol=0, atol=1e-16)


# --- collision ---------------------------------------------------------------------------

@pytest.mark.parametrize("model", MODELS)
def test_collision_conservation(model):
    """Mass is conserved by every model; momentum by LBGK and the corrected models, not by
    the uncorrected OReg model, whose populations carry momentum psi (eq:CEcontinuity)."""
    tau = 0.7
    for th, f in _states(10, u_max=0.25, amp=5e-3):
        p = oracle.collide_node(f, model, th, tau)
        r0, jx0, jy0, *_ = node_moments(f)
        r1, jx1, jy1, *_ = node_moments(p["fstar"])
        assert abs(r1 - r0) < 1e-15
        dj = np.array([jx1 - jx0, jy1 - jy0])
        if model == "uc":
            psi = np.array(node_moments(p["fo"])[1:3])
            np.testing.assert_allclose(dj, (1 - 1 / tau) * psi, rtol=0, atol=4e-16)
            assert np.max(np.abs(psi)) > 1e-9
        else:
            assert np.max(np.abs(dj)) < 4e-16


def test_collision_relaxes_second_moment():
    """The non-equilibrium stress after collision is (1 - 1/tau) times that of
    f^GOReg = f^OReg + Psi (eq:lbe with f^neq replaced, Sec. 3); for the complete model it
    is (1 - 1/tau)(Pi^OReg - Pi~)."""
    tau = 0.9
    for th, f in _states(11):
        p = oracle.collide_node(f, "complete", th, tau)
        _, _, _, pxx, pyy, pxy = node_moments(p["fstar"] - p["feq"])
        _, _, _, oxx, oyy, oxy = node_moments(p["fo"])
        Pi = p["Pi"]
        np.testing.assert_allclose([pxx, pyy, pxy],
                                   (1 - 1 / tau) * np.array([oxx - Pi[0, 0], oyy - Pi[1, 1], oxy - Pi[0, 1]]),
                                   rtol=0, atol=1e-16)


def test_equilibrium_is_fixed_point():
    """f = f^eq has no non-equilibrium part: every model returns it unchanged."""
    for th, _ in _states(12):
        feq = oracle.guided_equilibrium(1.05, 0.1, -0.07, th)
        for m in MODELS:
            np.testing.assert_allclose(oracle.collide_node(feq, m, th, 0.6)["fstar"], feq, rtol=0, atol=4e-16)
