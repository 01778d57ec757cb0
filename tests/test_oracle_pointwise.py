"""Pins of the oracle's pointwise pieces against the paper's printed values,
closed forms, identities and brute force (no GPU)."""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ---------------- lattices (Table LBM_Schemes, lattice figure) -------------

def test_d2q9_matches_paper_table(oracle):
    c, w, opp = oracle.lattice(2)
    rows = _read_table("lattice_d2q9.txt")
    assert len(rows) == 9
    for k, cx, cy, wk in rows:
        k = int(k)
        assert (c[k, 0], c[k, 1]) == (int(cx), int(cy))
        assert w[k] == pytest.approx(float(Fraction(wk)), abs=1e-16)
    for k in range(9):
        assert np.all(c[opp[k]] == -c[k])


def test_d3q27_matches_paper_table(oracle):
    c, w, opp = oracle.lattice(3, 27)
    rows = _read_table("lattice_d3q27.txt")
    assert len(w) == 27
    for k0, k1, len2, wk in rows:
        for k in range(int(k0), int(k1) + 1):
            assert int((c[k] ** 2).sum()) == int(len2)
            assert w[k] == pytest.approx(float(Fraction(wk)), abs=1e-16)
    assert len({tuple(v) for v in c}) == 27


LATTICES = [(2, 9), (3, 19), (3, 27)]


@pytest.mark.parametrize("dim,Q", LATTICES)
def test_lattice_isotropy(oracle, dim, Q):
    """Unity sum, symmetry and isotropy of the weights (App. A requires
    them); 2nd moment c_s^2 I with c_s^2 = 1/3, 4th moment isotropic."""
    c, w, opp = oracle.lattice(dim, Q)
    assert len(w) == Q
    assert len({tuple(v) for v in c}) == Q
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-16
    m2 = np.einsum("k,ka,kb->ab", w, c, c)
    assert np.abs(m2 - np.eye(dim) / 3.0).max() < 1e-15
    m3 = np.einsum("k,ka,kb,kc->abc", w, c, c, c)
    assert np.abs(m3).max() < 1e-16
    m4 = np.einsum("k,ka,kb,kc,kd->abcd", w, c, c, c, c)
    I = np.eye(dim)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.abs(m4 - iso).max() < 1e-15
    for k in range(Q):
        assert np.all(c[opp[k]] == -c[k])
        assert w[opp[k]] == w[k]


# ---------------- equilibrium and forcing moments --------------------------

@pytest.mark.parametrize("dim,Q", LATTICES)
def test_feq_moments(oracle, dim, Q):
    c, w, _ = oracle.lattice(dim, Q)
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(dim)
        f = oracle.feq(dim, rho, np.pad(u, (0, 3 - dim)), Q)
        assert f.sum() == pytest.approx(rho, abs=1e-15)
        assert np.abs(c.T @ f - rho * u).max() < 1e-16
        P = np.einsum("k,ka,kb->ab", f, c, c)
        assert np.abs(P - rho * (np.eye(dim) / 3.0 + np.outer(u, u))).max() < 1e-15


@pytest.mark.parametrize("dim,Q", LATTICES)
def test_guo_source_moments(oracle, dim, Q):
    """Discrete force, read as Guo's scheme: zeroth moment 0, first
    (1 - 1/2tau) F, second (1 - 1/2tau)(uF + Fu)."""
    c, w, _ = oracle.lattice(dim, Q)
    rng = np.random.default_rng(4)
    for tau in (0.6, 0.8, 1.3):
        u = 0.05 * rng.standard_normal(dim)
        F = 1e-3 * rng.standard_normal(dim)
        S = oracle.guo(dim, tau, np.pad(u, (0, 3 - dim)), np.pad(F, (0, 3 - dim)), Q)
        pref = 1.0 - 0.5 / tau
        assert abs(S.sum()) < 1e-18
        assert np.abs(c.T @ S - pref * F).max() < 1e-18
        P = np.einsum("k,ka,kb->ab", S, c, c)
        assert np.abs(P - pref * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


# ---------------- anisotropy --------------------------------------------------

def test_aniso_2d_is_fourfold_cosine(oracle):
    """In 2D the cubic form equals 1 + delta cos(4 theta)."""
    for delta in (0.0, 0.02, 0.05):
        for th in np.linspace(0, 2 * np.pi, 37):
            for r in (1e-3, 1.0, 7.0):
                q = r * np.array([np.cos(th), np.sin(th)])
                assert oracle.aniso_ac(q, delta) == pytest.approx(
                    1 + delta * np.cos(4 * th), abs=1e-14)


def test_aniso_3d_special_directions(oracle):
    d = 0.03
    for q, expect in (([2.0, 0, 0], 1 + d), ([0, -1.0, 0], 1 + d), ([1.0, 1.0, 1.0], 1 - 5 * d / 3),
                      ([1.0, 1.0, 0], 1 - d), ([0, 3.0, -3.0], 1 - d)):
        assert oracle.aniso_ac(q, d) == pytest.approx(expect, abs=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_aniso_energy_symmetries(oracle, dim):
    """A(q) = gamma a_c^2 |q|^2 is even, degree-2 homogeneous and invariant
    under the cubic group (axis permutations and reflections)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        q = rng.standard_normal(dim)
        A = oracle.aniso_A(q, 1.3, 0.04)
        assert oracle.aniso_A(-q, 1.3, 0.04) == pytest.approx(A, rel=1e-15)
        assert oracle.aniso_A(2.5 * q, 1.3, 0.04) == pytest.approx(6.25 * A, rel=1e-14)
        for perm in itertools.permutations(range(dim)):
            assert oracle.aniso_A(q[list(perm)] * (-1) ** np.arange(dim), 1.3, 0.04) == \
                pytest.approx(A, rel=1e-14)
        assert oracle.aniso_A(q, 1.3, 0.0) == pytest.approx(1.3 * (q @ q), rel=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_aniso_gradient_vs_complex_step(oracle, dim):
    """The analytic dA/dq used by the step equals the complex-step
    derivative (Squire and Trapp 1998) of A itself."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        q = rng.standard_normal(dim) * 10 ** rng.uniform(-5, 1)
        for delta in (0.0, 0.02, 0.05):
            g = oracle.aniso_dAdq(q, 1.0, delta)
            gcs = oracle.aniso_dAdq_cs(q, 1.0, delta)
            assert np.abs(g - gcs).max() <= 1e-13 * np.abs(gcs).max() + 1e-300


def test_aniso_regularised_below_threshold(oracle):
    q = np.array([3e-13, -1e-13])
    assert oracle.aniso_ac(q, 0.05) == 1.0
    assert np.allclose(oracle.aniso_dAdq(q, 1.0, 0.05), 2 * q, rtol=0, atol=1e-300)


# ---------------- simplex projection ------------------------------------------

def _kkt_bruteforce(v):
    """Enumerate supports; the unique one satisfying the KKT conditions of
    min |x - v|^2 on the simplex gives the projection."""
    m = len(v)
    sols = []
    for r in range(1, m + 1):
        for S in itertools.combinations(range(m), r):
            theta = (sum(v[i] for i in S) - 1.0) / r
            x = np.zeros(m)
            ok = True
            for i in range(m):
                if i in S:
                    x[i] = v[i] - theta
                    ok &= x[i] >= -1e-15
                else:
                    ok &= v[i] - theta <= 1e-15
            if ok:
                sols.append(x)
    assert sols
    for s in sols[1:]:
        assert np.allclose(s, sols[0], atol=1e-14)
    return sols[0]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_projection_vs_bruteforce(oracle, m):
    rng = np.random.default_rng(10 + m)
    for _ in range(300):
        v = rng.uniform(-1.0, 2.0, m)
        x = oracle.project(v)
        assert np.abs(x - _kkt_bruteforce(v)).max() < 1e-14
        assert x.min() >= 0.0
        assert x.sum() == pytest.approx(1.0, abs=1e-14)


def test_projection_fixed_points(oracle):
    for v in ([1.0], [0.25, 0.75], [0.2, 0.3, 0.5], [1.0, 0.0, 0.0]):
        assert np.array_equal(oracle.project(v), np.array(v))
    assert np.allclose(oracle.project([2.0, 0.0]), [1.0, 0.0])
    assert np.allclose(oracle.project([0.6, 0.6]), [0.5, 0.5])


# ---------------- interpolation -------------------------------------------------

@pytest.mark.parametrize("N", [2, 3, 4])
def test_h_partition_of_unity_and_derivative(oracle, N):
    rng = np.random.default_rng(20 + N)
    for _ in range(100):
        phi = rng.dirichlet(np.ones(N))
        h, dh = oracle.interp_h(phi)
        assert h.sum() == pytest.approx(1.0, abs=1e-15)
        assert np.all(h >= -1e-15)
        # derivative by 4th-order central differences of h itself
        for a in range(N):
            e = np.zeros(N)
            e[a] = 1e-3
            num = (-oracle.interp_h(phi + 2 * e)[0] + 8 * oracle.interp_h(phi + e)[0]
                   - 8 * oracle.interp_h(phi - e)[0] + oracle.interp_h(phi - 2 * e)[0]) / 12e-3
            assert np.abs(num - dh[:, a]).max() < 1e-10
    # vertices of the simplex: h_a = 1 at its own vertex, flat there
    for a in range(N):
        phi = np.zeros(N)
        phi[a] = 1
        h, dh = oracle.interp_h(phi)
        assert np.array_equal(h, phi)
        assert np.abs(dh).max() == 0.0


@pytest.mark.parametrize("N", [3, 4])
def test_h_reduces_to_two_phases_on_every_edge(oracle, N):
    """On the edge phi_a + phi_b = 1 of the simplex the multiphase h is the
    two-phase phi^2 (3 - 2 phi) for a and b and 0 for every other phase; on a
    face (three phases present) it is the three-phase h."""
    s = np.linspace(0.0, 1.0, 11)
    for a in range(N):
        for b in range(N):
            if a == b:
                continue
            for t in s:
                phi = np.zeros(N)
                phi[a], phi[b] = t, 1 - t
                h, _ = oracle.interp_h(phi)
                assert h[a] == pytest.approx(t * t * (3 - 2 * t), abs=1e-15)
                assert h[b] == pytest.approx((1 - t) ** 2 * (1 + 2 * t), abs=1e-15)
                assert np.abs(np.delete(h, [a, b])).max(initial=0.0) == 0.0
    if N == 4:
        rng = np.random.default_rng(7)
        for _ in range(20):
            keep = rng.choice(4, 3, replace=False)
            phi = np.zeros(4)
            phi[keep] = rng.dirichlet(np.ones(3))
            h4, _ = oracle.interp_h(phi)
            h3, _ = oracle.interp_h(phi[keep])
            assert np.abs(h4[keep] - h3).max() < 1e-15


def test_normal_generator_statistics(oracle):
    """Counter-based SplitMix64 + Box-Muller: mean 0, variance 1."""
    z = np.array([oracle.normal(1, j) for j in range(20000)])
    assert abs(z.mean()) < 0.03
    assert abs(z.var() - 1.0) < 0.04
    assert oracle.normal(1, 5) == oracle.normal(1, 5)
    assert oracle.normal(1, 5) != oracle.normal(2, 5)


def test_splitmix64_published_vector(oracle):
    """First outputs of SplitMix64 seeded with 0 (reference values of the
    published generator) through the uniform of counter 0."""
    # splitmix64 from state 0: first output 0xE220A8397B1DCDAF
    first = 0xE220A8397B1DCDAF
    u1 = ((first >> 11) + 1) * 2.0 ** -53
    second = 0x6E789E6AA1B965F4
    u2 = (second >> 11) * 2.0 ** -53
    expect = math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
    assert oracle.normal(0, 0) == pytest.approx(expect, rel=1e-15)
