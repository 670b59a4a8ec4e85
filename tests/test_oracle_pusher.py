"""Pins for the oracle's pushers (CPU only).

The modified pusher is the paper's fix for the inexact electric/magnetic
cancellation of the Boris pusher (Sec. 2, first paragraph; Vay 2008).  Each
test pins it against a closed form that does not re-use its formula.
"""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

DT = 0.1
EPS = -0.5 * DT  # electron, q/m = -1


def _gamma(u):
    return math.sqrt(1.0 + float(np.dot(u, u)))


@pytest.mark.parametrize("gamma", [10.0, 1e2, 1e4, 1e6])
def test_vay_crossed_fields_straight_line(ora, gamma):
    """E = -v0 x B: the exact discrete solution is u = u0 for all steps."""
    u0 = math.sqrt(gamma * gamma - 1.0)
    v0 = u0 / math.sqrt(1.0 + u0 * u0)
    E = np.array([v0, 0.0, 0.0])  # -(v0 z) x (y) = v0 x
    B = np.array([0.0, 1.0, 0.0])
    u = np.array([0.0, 0.0, u0])
    for _ in range(200):
        u = ora.push(u, E, B, EPS, ora.VAY)
    assert np.linalg.norm(u - [0.0, 0.0, u0]) / u0 < 1e-13
    assert abs(u[0]) / u0 < 1e-13


@pytest.mark.parametrize("gamma", [1e2, 1e3, 1e4])
def test_beam_self_field_vay_exact_boris_error_grows(ora, gamma):
    """A particle co-moving with a beam of fixed rest-frame field E_rest sees
    lab fields E_r = gamma E_rest, B = beta E_r.  The physical net transverse
    force is q E_r / gamma^2.  The modified pusher reproduces the kick; the
    Boris pusher's relative error grows like gamma^2 (the paper's claim)."""
    b = math.sqrt(1.0 - 1.0 / gamma**2)
    Er = 1.0 * gamma
    E = np.array([Er, 0.0, 0.0])
    B = np.array([0.0, b * Er, 0.0])
    phys = -DT * Er / gamma**2
    u0 = np.array([0.0, 0.0, gamma * b])
    uv = ora.push(u0, E, B, EPS, ora.VAY)
    ub = ora.push(u0, E, B, EPS, ora.BORIS)
    err_v = abs(uv[0] - phys) / abs(phys)
    err_b = abs(ub[0] - phys) / abs(phys)
    assert err_v < 1e-6
    # Boris: relative error ~ (eps E_r)^2 / 2 ~ 1.25e-3 gamma^2
    assert err_b == pytest.approx(1.25e-3 * gamma**2, rel=0.05)


@pytest.mark.parametrize("pusher", ["vay", "boris"])
@pytest.mark.parametrize("gamma", [1.5, 1e2, 1e6])
@pytest.mark.parametrize("upar_frac", [0.0, 0.3])
def test_uniform_B_gamma_and_phase(ora, pusher, gamma, upar_frac):
    """E = 0, uniform B: gamma is conserved exactly; u_perp rotates by
    theta = 2 atan(|eps B| / gamma) per step; u_par is unchanged."""
    P = ora.VAY if pusher == "vay" else ora.BORIS
    Bmag = 1.0
    B = np.array([0.0, 0.0, Bmag])
    umag = math.sqrt(gamma * gamma - 1.0)
    upar = upar_frac * umag
    uperp = math.sqrt(umag * umag - upar * upar)
    phi0 = 0.7
    u = np.array([uperp * math.cos(phi0), uperp * math.sin(phi0), upar])
    E = np.zeros(3)
    n = 500
    for _ in range(n):
        u = ora.push(u, E, B, EPS, P)
    assert abs(_gamma(u) - gamma) / gamma < 1e-13
    assert abs(u[2] - upar) <= 1e-12 * umag
    theta = 2.0 * math.atan(abs(EPS) * Bmag / gamma)
    # electron (q<0) in B along +z rotates counter-clockwise seen from +z
    phi = math.atan2(u[1], u[0])
    expect = phi0 + n * theta
    dphi = (phi - expect + math.pi) % (2 * math.pi) - math.pi
    assert abs(dphi) < 1e-10 * max(1.0, n * theta)


@pytest.mark.parametrize("pusher", ["vay", "boris"])
def test_pure_electric_field_exact(ora, pusher):
    """B = 0: u_new = u + (q dt / m) E exactly."""
    P = ora.VAY if pusher == "vay" else ora.BORIS
    rng = np.random.default_rng(11)
    for _ in range(20):
        u = rng.normal(size=3) * 10
        E = rng.normal(size=3) * 3
        out = ora.push(u, E, np.zeros(3), EPS, P)
        np.testing.assert_allclose(out, u - DT * E, rtol=1e-14, atol=1e-14)


def test_vay_reduces_to_boris_rotation_when_nonrelativistic(ora):
    """At gamma -> 1 with weak fields both pushers agree to O((eps E)^2)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.normal(size=3) * 1e-3
        E = rng.normal(size=3) * 1e-3
        B = rng.normal(size=3)
        a = ora.push(u, E, B, EPS, ora.VAY)
        b = ora.push(u, E, B, EPS, ora.BORIS)
        assert np.linalg.norm(a - b) < 1e-7


def test_push_many_matches_single(ora):
    rng = np.random.default_rng(5)
    n = 16
    u = rng.normal(size=(n, 3)) * 100
    E = rng.normal(size=(n, 3))
    B = rng.normal(size=(n, 3))
    pos = rng.uniform(size=(n, 3))
    u2, p2 = ora.push_many(u, E, B, pos, DT, 7, ora.VAY)
    for i in range(n):
        ui = u[i].copy()
        pi = pos[i].copy()
        for _ in range(7):
            ui = ora.push(ui, E[i], B[i], EPS, ora.VAY)
            pi = pi + DT * ui / _gamma(ui)
        np.testing.assert_allclose(u2[i], ui, rtol=1e-15)
        np.testing.assert_allclose(p2[i], pi, rtol=1e-15)


def test_philox_known_answers(ora):
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
    n = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        c, k, o = [[int(w, 16) for w in part.split()] for part in line.split("|")]
        assert ora.philox4x64_10(c, k) == o
        n += 1
    assert n == 3


def test_philox_matches_numpy(ora):
    """numpy's Philox is Philox4x64-10; it increments the counter before the
    first block, so its first draw for counter c equals ours for c + 1."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(1, 2**63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        c = np.array([ctr[0] - 1] + ctr[1:], dtype=np.uint64)
        bg = np.random.Philox(counter=c, key=np.array(key, dtype=np.uint64))
        ref = [int(v) for v in bg.random_raw(4)]
        assert ora.philox4x64_10(ctr, key) == ref
