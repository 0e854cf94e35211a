"""Pins of the oracle's model pieces against facts that do not come from the
oracle itself: the moment-polynomial definitions behind the printed matrices,
orthogonality, lattice isotropy, the agreement of the two printed forms of each
equilibrium, the velocity-space forcing, and the implicit velocity equation."""
import itertools

import numpy as np
import pytest

import oracle

pytestmark = []

CS2 = 1.0 / 3.0


def _moment_polynomials_d3q19(e):
    """Row polynomials of the D3Q19 moment basis m = (rho, e, eps, jx, qx, jy,
    qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pzx, mx, my, mz) (Eq. 20),
    as defined by d'Humieres et al. (2002), the paper's Ref. [49]."""
    x, y, z = (e[a].astype(float) for a in range(3))
    r2 = x * x + y * y + z * z
    return np.array([
        np.ones_like(x),
        19 * r2 - 30,
        (21 * r2 * r2 - 53 * r2 + 24) / 2,
        x, (5 * r2 - 9) * x,
        y, (5 * r2 - 9) * y,
        z, (5 * r2 - 9) * z,
        3 * x * x - r2,
        (3 * r2 - 5) * (3 * x * x - r2),
        y * y - z * z,
        (3 * r2 - 5) * (y * y - z * z),
        x * y, y * z, z * x,
        (y * y - z * z) * x,
        (z * z - x * x) * y,
        (x * x - y * y) * z,
    ])


def _moment_polynomials_d3q15(e):
    """Row polynomials of the D3Q15 basis (Eq. 13), Ref. [49]."""
    x, y, z = (e[a].astype(float) for a in range(3))
    r2 = x * x + y * y + z * z
    return np.array([
        np.ones_like(x),
        r2 - 2,
        (15 * r2 * r2 - 55 * r2 + 32) / 2,
        x, (5 * r2 - 13) / 2 * x,
        y, (5 * r2 - 13) / 2 * y,
        z, (5 * r2 - 13) / 2 * z,
        3 * x * x - r2,
        y * y - z * z,
        x * y, y * z, z * x,
        x * y * z,
    ])


@pytest.mark.parametrize("q", [19, 15])
def test_velocity_set_structure(q):
    e = oracle.velocities(q)
    cols = {tuple(c) for c in e.T}
    assert len(cols) == q
    assert (0, 0, 0) in cols
    # closed under reversal
    for c in cols:
        assert tuple(-v for v in c) in cols
    r2 = (e * e).sum(0)
    if q == 19:
        assert sorted(np.bincount(r2)) == sorted([1, 6, 12])
    else:
        assert list(np.bincount(r2)) == [1, 6, 0, 8]
    # first seven columns are the D3Q7 set of Eq. 12
    assert np.array_equal(e[:, :7], oracle.velocities(7))


@pytest.mark.parametrize("q", [19, 15])
def test_weights_isotropy(q):
    """sum w = 1, sum w e_a e_b = cs^2 delta, fourth moment = cs^4 (ddd); odd
    moments vanish.  These fix the weights of Eqs. 18 and 24 to the lattice."""
    e = oracle.velocities(q).astype(float)
    w = oracle.weights(q)
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((w * e[a] * e[b]).sum() - CS2 * d[a, b]) < 1e-15
        assert abs((w * e[a]).sum()) < 1e-15
        for c in range(3):
            assert abs((w * e[a] * e[b] * e[c]).sum()) < 1e-15
            for dd in range(3):
                iso = CS2 * CS2 * (d[a, b] * d[c, dd] + d[a, c] * d[b, dd] + d[a, dd] * d[b, c])
                assert abs((w * e[a] * e[b] * e[c] * e[dd]).sum() - iso) < 1e-15


def test_d3q7_weights_second_moment():
    """omega_0 = 1 - varpi, omega_1..6 = varpi/6: sum = 1 and
    sum omega e_a e_b = csT^2 delta with csT^2 = varpi/3 (Eq. 40)."""
    for varpi in (0.2, 0.5, 0.9):
        e = oracle.velocities(7).astype(float)
        w = oracle.weights(7, varpi)
        assert abs(w.sum() - 1) < 1e-15
        for a, b in itertools.product(range(3), repeat=2):
            assert abs((w * e[a] * e[b]).sum() - varpi / 3 * (a == b)) < 1e-15


@pytest.mark.parametrize("q,poly", [(19, _moment_polynomials_d3q19), (15, _moment_polynomials_d3q15)])
def test_matrix_rows_are_moment_polynomials(q, poly):
    """The printed M (Eq. A2 / A1) equals the moment basis polynomials evaluated
    on the velocity set, entry by entry."""
    M = oracle.matrix(q)
    expect = poly(oracle.velocities(q))
    assert np.array_equal(M, expect)


@pytest.mark.parametrize("q", [19, 15])
def test_matrix_orthogonal_and_inverse(q):
    M = oracle.matrix(q)
    Minv = oracle.matrix_inverse(q)
    G = M @ M.T
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0  # rows mutually orthogonal
    # the Gauss-Jordan inverse equals M^T diag(1/|row|^2), which holds for orthogonal rows
    assert np.max(np.abs(Minv - M.T / np.diag(G))) < 1e-15
    assert np.max(np.abs(M @ Minv - np.eye(q))) < 1e-14
    assert np.max(np.abs(Minv @ M - np.eye(q))) < 1e-14


def test_row_norms_d3q19():
    M = oracle.matrix(19)
    assert list((M * M).sum(1)) == [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24,
                                    4, 4, 4, 8, 8, 8]


def test_N_and_printed_inverse():
    """Eq. 36 times Eq. 43 is the identity; N's rows are the basis vectors the
    paper names (1, e_x, e_y, e_z, |e|^2, e_x^2 - e_y^2, e_x^2 - e_z^2)."""
    N = oracle.matrix(7)
    Ninv = oracle.matrix_inverse(7)
    assert np.max(np.abs(N @ Ninv - np.eye(7))) < 1e-15
    assert np.max(np.abs(Ninv @ N - np.eye(7))) < 1e-15
    x, y, z = oracle.velocities(7)
    basis = np.array([np.ones(7), x, y, z, x * x + y * y + z * z, x * x - y * y, x * x - z * z])
    assert np.array_equal(N, basis)


@pytest.mark.parametrize("q", [19, 15])
def test_meq_equals_M_feq(q):
    """The moment-space equilibria (Eq. 21 / Eq. 15) and the velocity-space
    ones (Eq. 24 / Eq. 18) are two statements of one object: M f^eq = m^eq."""
    rng = np.random.default_rng(11)
    M = oracle.matrix(q)
    for _ in range(50):
        rho = 1 + 0.2 * rng.uniform(-1, 1)
        u = 0.1 * rng.uniform(-1, 1, 3)
        phi = rng.uniform(0.2, 1.0)
        d = M @ oracle.feq(q, rho, u, phi) - oracle.meq(q, rho, u, phi)
        assert np.max(np.abs(d)) < 2e-14


def test_neq_equals_N_geq():
    """N g^eq (Eq. 42) = n^eq (Eq. 37)."""
    rng = np.random.default_rng(12)
    N = oracle.matrix(7)
    for _ in range(50):
        T = rng.uniform(-1, 1)
        u = 0.1 * rng.uniform(-1, 1, 3)
        sigma = rng.uniform(0.5, 2.0)
        varpi = rng.uniform(0.1, 0.9)
        d = N @ oracle.geq(T, u, sigma, varpi) - oracle.neq(T, u, sigma, varpi)
        assert np.max(np.abs(d)) < 1e-15


@pytest.mark.parametrize("q", [19, 15])
def test_forcing_moments_equal_velocity_space_source(q):
    """S~ = M S (Eq. 11) with the velocity-space source of the generalized
    lattice Boltzmann model (Ref. [25]):
    S_i = w_i rho0 [e_i.F/cs^2 + ((e_i.u)(e_i.F) - cs^2 u.F)/(phi cs^4)]."""
    rng = np.random.default_rng(13)
    e = oracle.velocities(q).astype(float)
    w = oracle.weights(q)
    M = oracle.matrix(q)
    for _ in range(50):
        u = 0.1 * rng.uniform(-1, 1, 3)
        F = 1e-3 * rng.uniform(-1, 1, 3)
        phi = rng.uniform(0.2, 1.0)
        eu = e.T @ u
        eF = e.T @ F
        S = w * (eF / CS2 + (eu * eF - CS2 * (u @ F)) / (phi * CS2 * CS2))
        d = M @ S - oracle.forcing_moments(q, u, F, phi)
        assert np.max(np.abs(d)) < 1e-16


def test_total_force_special_cases():
    """Eq. 4: at rest F = phi G; with G = 0 and F_phi = 0 it is the Darcy drag."""
    G = np.array([1e-3, -2e-3, 5e-4])
    assert np.allclose(oracle.total_force([0, 0, 0], G, 0.4, 0.1, 2.0, 0.5), 0.4 * G, rtol=0, atol=1e-18)
    u = np.array([0.01, 0.02, -0.03])
    F = oracle.total_force(u, [0, 0, 0], 0.5, 0.1, 4.0, 0.0)
    assert np.allclose(F, -0.5 * 0.1 / 4.0 * u, rtol=1e-15, atol=0)
    # the Forchheimer term is quadratic and anti-parallel to u
    F1 = oracle.total_force(u, [0, 0, 0], 0.5, 0.0, 4.0, 0.3)
    F2 = oracle.total_force(2 * u, [0, 0, 0], 0.5, 0.0, 4.0, 0.3)
    assert np.allclose(F2, 4 * F1, rtol=1e-14, atol=0)
    assert (F1 @ u) < 0


@pytest.mark.parametrize("q", [19, 15])
def test_velocity_closure_solves_eq26(q):
    """Eqs. 27-28 solve the implicit Eq. 26: rho0 u = sum_i e_i f_i + rho0 F(u)/2
    with F of Eq. 4 evaluated at the returned u."""
    rng = np.random.default_rng(14)
    e = oracle.velocities(q).astype(float)
    for _ in range(100):
        f = rng.uniform(0.01, 0.1, q)
        G = 1e-2 * rng.uniform(-1, 1, 3)
        phi = rng.uniform(0.2, 1.0)
        nu = rng.uniform(0.01, 0.3)
        K = 10 ** rng.uniform(-1, 2)
        Fphi = rng.uniform(0, 1.5)
        u = oracle.velocity(q, f, G, phi, nu, K, Fphi)
        F = oracle.total_force(u, G, phi, nu, K, Fphi)
        res = u - (e @ f + 0.5 * F)
        assert np.max(np.abs(res)) < 1e-16 + 1e-14 * np.max(np.abs(u))


def test_splitmix64_matches_python_definition():
    """Counter-based noise: SplitMix64 (Steele, Lea & Flood 2014), written here
    again in Python from its published definition."""
    mask = (1 << 64) - 1

    def sm(s):
        z = (s + 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    for s in [0, 1, 2, 12345, mask, 0xDEADBEEF << 20]:
        assert oracle.splitmix64(s) == sm(s)
    vals = np.array([oracle.noise(5, n, 1e-3) for n in range(4096)])
    assert vals.min() >= -1e-3 and vals.max() <= 1e-3
    assert abs(vals.mean()) < 5e-5          # uniform on [-amp, amp]
    assert abs(vals.std() - 1e-3 / np.sqrt(3)) < 2e-5
    r = (sm(5 ^ 17) >> 11) * 2.0 ** -53
    assert oracle.noise(5, 17, 1e-3) == 1e-3 * (2 * r - 1)
