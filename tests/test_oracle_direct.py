"""Pins of the oracle's direct sum (O-D), generators and leapfrog against closed forms,
invariants and analytic profiles (not against the oracle's own formulas)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I


def _set(pos, m, eps, vel=None):
    pos = np.asarray(pos, float)
    n = pos.shape[0]
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, float)
    return I._pack(pos.copy(), vel.copy(), np.asarray(m, float).copy(), np.full(n, float(eps)))


def test_two_body_closed_form():
    # |a_1| = m_2 d / (d^2 + eps^2)^{3/2}, pointing at body 2; phi_1 = -m_2 / sqrt(d^2+eps^2)
    d, eps, m1, m2 = 0.7, 0.1, 0.3, 1.9
    ps = _set([[0, 0, 0], [d, 0, 0]], [m1, m2], eps)
    a = O.direct(ps)
    den = (d * d + eps * eps) ** 1.5
    assert a[0, 0] == pytest.approx(m2 * d / den, rel=1e-15)
    assert a[1, 0] == pytest.approx(-m1 * d / den, rel=1e-15)
    assert abs(a[0, 1]) == 0 and abs(a[0, 2]) == 0
    assert a[0, 3] == pytest.approx(-m2 / math.sqrt(d * d + eps * eps), rel=1e-15)
    assert a[1, 3] == pytest.approx(-m1 / math.sqrt(d * d + eps * eps), rel=1e-15)


def test_equilateral_triangle():
    # three equal masses on a triangle of side s: each acceleration points at the centroid
    # with magnitude 2 m s cos(30 deg) / (s^2 + eps^2)^{3/2}
    s, eps, m = 1.3, 0.05, 0.4
    h = s * math.sqrt(3) / 2
    pos = np.array([[0, 0, 0], [s, 0, 0], [s / 2, h, 0]])
    a = O.direct(_set(pos, [m] * 3, eps))
    mag = 2 * m * s * math.cos(math.pi / 6) / (s * s + eps * eps) ** 1.5
    cen = pos.mean(axis=0)
    for i in range(3):
        u = (cen - pos[i]) / np.linalg.norm(cen - pos[i])
        assert np.allclose(a[i, :3], mag * u, rtol=1e-14, atol=1e-14)
        assert a[i, 3] == pytest.approx(-2 * m / math.sqrt(s * s + eps * eps), rel=1e-15)


def test_newton_third_law():
    ps = I.plummer(2000, seed=11, eps=0.01)
    a = O.direct(ps)
    f = ps.m[:, None] * a[:, :3]
    assert np.linalg.norm(f.sum(axis=0)) <= 1e-13 * np.sum(np.linalg.norm(f, axis=1))


def test_self_term_excluded_and_system_isolation():
    # two identical systems laid end to end feel nothing from each other
    a_set = I.plummer(300, seed=5, eps=0.02)
    b_set = I.plummer(300, seed=5, eps=0.02)
    b_set.x += 100.0
    both = I.concat([a_set, b_set])
    a1 = O.direct(a_set)
    a2 = O.direct(both)
    assert np.array_equal(a2[:300], a1)
    # the shifted copy differs only by the rounding of coordinates near x = 100
    assert np.allclose(a2[300:], a1, rtol=1e-10, atol=1e-12)


def test_plummer_analytic_potential_and_virial():
    n = 16384
    ps = I.plummer(n, seed=7, eps=1e-3)
    a = O.direct(ps)
    r = np.sqrt(ps.x ** 2 + ps.y ** 2 + ps.z ** 2)
    # shell-averaged potential against -1/sqrt(r^2+1) (truncation at 20a shifts it by
    # O(1e-3) because 0.37 % of the mass beyond 20a is missing)
    for lo, hi in [(0.2, 0.4), (0.6, 0.9), (1.2, 1.6), (2.5, 3.5)]:
        sel = (r > lo) & (r < hi)
        rm = r[sel].mean()
        phi_model = -1.0 / math.sqrt(rm * rm + 1.0)
        assert a[sel, 3].mean() == pytest.approx(phi_model, rel=0.03)
    # radial acceleration against -r/(r^2+1)^{3/2}
    sel = (r > 0.8) & (r < 1.2)
    ar = (a[sel, 0] * ps.x[sel] + a[sel, 1] * ps.y[sel] + a[sel, 2] * ps.z[sel]) / r[sel]
    model = -r[sel] / (r[sel] ** 2 + 1.0) ** 1.5
    assert np.mean(ar / model) == pytest.approx(1.0, abs=0.03)
    # potential energy W -> -3 pi / 32 for a complete unit Plummer sphere
    K, W, E = O.energy(ps, a[:, 3])
    assert W == pytest.approx(-3 * math.pi / 32, rel=0.02)
    # virial ratio 2K/|W| ~ 1 for the equilibrium distribution function
    assert 2 * K / abs(W) == pytest.approx(1.0, abs=0.05)


def test_generator_radii_distribution():
    from scipy import stats
    ps = I.plummer(20000, seed=3, eps=0.01)
    # undo the COM shift's tiny offset by measuring around the COM (which is 0 after shift)
    r = np.sqrt(ps.x ** 2 + ps.y ** 2 + ps.z ** 2)
    mtrunc = 20.0 ** 3 / (20.0 ** 2 + 1) ** 1.5

    def cdf(x):
        x = np.asarray(x)
        return np.minimum(1.0, x ** 3 / (x * x + 1) ** 1.5 / mtrunc)

    ks = stats.kstest(r, cdf)
    assert ks.pvalue > 1e-3
    # half-mass radius of the (untruncated) Plummer sphere: (2^{2/3} - 1)^{-1/2} = 1.3048
    assert np.median(r) == pytest.approx(1.3048, rel=0.03)


def test_generator_frame_and_determinism():
    a = I.plummer(5000, seed=9, eps=0.01)
    b = I.plummer(5000, seed=9, eps=0.01)
    c = I.plummer(5000, seed=10, eps=0.01)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.vz, b.vz)
    assert not np.array_equal(a.x, c.x)
    for arr in (a.x, a.y, a.z, a.vx, a.vy, a.vz):
        assert abs(np.sum(a.m * arr)) < 1e-14
    assert np.sum(a.m) == pytest.approx(1.0, rel=1e-14)


def test_clustered_and_ensemble_structure():
    ps = I.clustered(n_background=4096, n_clusters=4, n_per_cluster=1024, seed=1)
    assert ps.n == 8192
    assert np.all(ps.m == 1.0 / 8192)
    ens = I.ensemble(n_sys=6, seed=4, nmin=64, nmax=512)
    off = ens.offsets()
    assert off[0] == 0 and off[-1] == ens.n and np.all(np.diff(off) >= 64)
    for s in range(6):
        sl = slice(off[s], off[s + 1])
        ns = off[s + 1] - off[s]
        assert np.allclose(ens.eps[sl], 4.0 / ns ** (1 / 3))
        assert np.sum(ens.m[sl]) == pytest.approx(1.0)


def _kdk(ps, dt, nsteps, acc):
    """Leapfrog of the sample program: predict (half kick + drift), force, correct."""
    x = np.stack([ps.x, ps.y, ps.z], 1)
    v = np.stack([ps.vx, ps.vy, ps.vz], 1)
    a = acc(x)
    for _ in range(nsteps):
        O.kick(v, a, dt)
        O.drift(x, v, dt)
        a = acc(x)
        O.kick(v, a, dt)
    return x, v


def _direct_acc(ps):
    def acc(x):
        q = I._pack(x.copy(), np.zeros_like(x), ps.m, ps.eps)
        return O.direct(q)[:, :3]
    return acc


def test_leapfrog_time_reversible():
    ps = I.plummer(64, seed=2, eps=0.05)
    x0 = np.stack([ps.x, ps.y, ps.z], 1).copy()
    v0 = np.stack([ps.vx, ps.vy, ps.vz], 1).copy()
    x1, v1 = _kdk(ps, 1 / 128, 40, _direct_acc(ps))
    back = I._pack(x1, -v1, ps.m, ps.eps)
    x2, v2 = _kdk(back, 1 / 128, 40, _direct_acc(ps))
    assert np.max(np.abs(x2 - x0)) < 1e-12
    assert np.max(np.abs(-v2 - v0)) < 1e-12


def test_leapfrog_circular_orbit():
    # equal masses m on a circle of separation d: speed of each v = sqrt(m / (2 d)) (eps -> 0)
    m, d = 0.5, 1.0
    v = math.sqrt(m / (2 * d))
    ps = _set([[-d / 2, 0, 0], [d / 2, 0, 0]], [m, m], 1e-8, vel=[[0, -v, 0], [0, v, 0]])
    period = 2 * math.pi * (d / 2) / v
    nsteps = 2000
    x, vv = _kdk(ps, period / nsteps, nsteps, _direct_acc(ps))
    # back to the start after one period; separation stays d
    assert np.linalg.norm(x[1] - x[0]) == pytest.approx(d, rel=1e-4)
    assert np.allclose(x, [[-d / 2, 0, 0], [d / 2, 0, 0]], atol=1e-3)


def test_leapfrog_energy_plummer():
    ps = I.plummer(512, seed=4, eps=0.05)
    acc = _direct_acc(ps)
    a0 = O.direct(ps)
    E0 = O.energy(ps, a0[:, 3])[2]
    x, v = _kdk(ps, 1 / 256, 64, acc)
    q = I._pack(x, v, ps.m, ps.eps)
    E1 = O.energy(q, O.direct(q)[:, 3])[2]
    assert abs(E1 - E0) / abs(E0) < 1e-4
