"""Pins of the oracle's node collision (Eqs. 9-11, 34) and parameter mapping
(Eqs. 6, 7, 28, 32, 41, 51, 56) through conservation laws and invariants."""
import numpy as np
import pytest

import lbm_inputs
import oracle


def _lattice(q=19, **kw):
    wl = lbm_inputs.cavity(8, lattice=q, **kw)
    return oracle.Oracle(wl)


@pytest.mark.parametrize("q", [19, 15])
@pytest.mark.parametrize("s_j", [1.0, 0.7, 1.6])
def test_collision_conserves_mass_heat_and_adds_force(q, s_j):
    """Sum f* = sum f; sum g* = sum g; sum e f* - sum e f = rho0 F for every s_j
    (the conserved-moment equilibria are those of M f^eq, reading R3)."""
    rng = np.random.default_rng(21)
    e = oracle.velocities(q).astype(float)
    with _lattice(q, porosity=0.45, darcy=1e-2, rayleigh=1e5, s_j=s_j) as o:
        for _ in range(20):
            f, g = lbm_inputs.random_state(q, (1, 1, 1), int(rng.integers(1 << 30)))
            f = f[:, 0, 0, 0]
            g = g[:, 0, 0, 0]
            fo, go, mac = o.collide_node(f, g)
            assert abs(fo.sum() - f.sum()) < 1e-15
            assert abs(go.sum() - g.sum()) < 1e-15
            dj = e @ fo - e @ f
            assert np.max(np.abs(dj - mac["F"])) < 5e-16  # rounding of O(0.1) sums
            assert abs(mac["rho"] - f.sum()) < 1e-15
            assert abs(mac["T"] - g.sum()) < 1e-15


@pytest.mark.parametrize("q", [19, 15])
def test_equilibrium_at_rest_is_a_fixed_point(q):
    """With G = 0 and u = 0 the force vanishes, so f^eq(rho, 0) and g^eq(T, 0)
    are left unchanged by the collision."""
    with _lattice(q, rayleigh=1e4) as o:
        d = o.derived()
        for rho, T in [(1.0, 0.0), (1.03, 0.0), (0.97, 0.0)]:
            # T = T_ref (= 0 for the cavity) so that G = 0
            f = oracle.feq(q, rho, [0, 0, 0], 0.6)
            g = oracle.geq(T, [0, 0, 0])
            fo, go, mac = o.collide_node(f, g)
            assert np.max(np.abs(fo - f)) < 1e-16
            assert np.max(np.abs(go - g)) < 1e-16
        assert d["K"] > 0


def test_thermal_collision_relaxes_each_moment_independently():
    """n* - n = -Q (n - n^eq) (Eq. 34): with the rates of Eq. 38, the change in
    each moment of g is proportional to its own departure."""
    rng = np.random.default_rng(22)
    N = oracle.matrix(7)
    with _lattice(19, rayleigh=1e4) as o:
        za = o.derived()["zeta_alpha"]
        Qd = np.array([1.0, za, za, za, 1.2, 1.2, 1.2])
        for _ in range(10):
            f, g = lbm_inputs.random_state(19, (1, 1, 1), int(rng.integers(1 << 30)))
            f, g = f[:, 0, 0, 0], g[:, 0, 0, 0]
            fo, go, mac = o.collide_node(f, g)
            n = N @ g
            ne = oracle.neq(mac["T"], mac["u"])
            assert np.max(np.abs((N @ go - n) + Qd * (n - ne))) < 1e-16


def test_cavity_mapping_closes_eq7():
    """The derived rates of Eq. 56 reproduce the dimensionless groups they came
    from: Ma = sqrt(gbeta dT L)/cs, Pr = nu/alpha, J = nu_e/nu, Gamma = alpha_e/alpha,
    Ra = gbeta dT L^3/(nu alpha), Da = K/L^2, and nu_e, alpha_e are Eqs. 32, 41."""
    for (n, phi, da, ra, pr) in [(32, 0.6, 1e-2, 1e4, 1.0), (48, 0.4, 1e-4, 1e6, 1.0),
                                (64, 0.8, 1e-3, 1e5, 0.71)]:
        # the box is (n, 2, 2): the mapping depends on the size only through L = nx
        with oracle.Oracle(lbm_inputs.cavity((n, 2, 2), porosity=phi, darcy=da,
                                             rayleigh=ra, prandtl=pr)) as o:
            d = o.derived()
        L = n
        cs = 1 / np.sqrt(3)
        assert abs(np.sqrt(d["gbeta"] * 1.0 * L) / cs - 0.1) < 1e-14
        assert abs(d["nu"] / d["alpha"] - pr) < 1e-13
        assert abs(d["gbeta"] * L ** 3 / (d["nu"] * d["alpha"]) - ra) < 1e-9 * ra
        assert abs(d["K"] - da * L * L) < 1e-12
        assert abs(d["nu_e"] - (1 / d["s_nu"] - 0.5) / 3) < 1e-16
        assert abs(d["alpha_e"] - (1 / d["zeta_alpha"] - 0.5) / 6) < 1e-16
        assert abs(d["F_phi"] - 1.75 / np.sqrt(150 * phi ** 3)) < 1e-15
        assert 0 < d["s_nu"] < 2 and 0 < d["zeta_alpha"] < 2


def test_cavity_32_derived_values():
    """Config values for the 32^3 cavity: phi 0.6, Da 1e-2, Ra 1e4, Pr 1."""
    with oracle.Oracle(lbm_inputs.config_cavity_fp64()) as o:
        d = o.derived()
    assert abs(d["s_nu"] - 1.800421) < 1e-6
    assert abs(d["zeta_alpha"] - 1.637060) < 1e-6
    assert abs(d["K"] - 10.24) < 1e-12


def test_channel_mapping_reads_eq51_as_inverse():
    """Eq. 51 read as 1/s_nu = 1/2 + J H u / (cs^2 Re) (reading R4): the derived
    viscosity satisfies Re = H u_c / nu."""
    wl = lbm_inputs.periodic_box((4, 32, 4), reynolds=5.0, u_char=0.01, length_axis=1)
    with oracle.Oracle(wl) as o:
        d = o.derived()
    assert abs(32 * 0.01 / d["nu"] - 5.0) < 1e-12
    assert abs(d["nu"] / d["alpha"] - 1.0) < 1e-12


def test_invalid_parameters_are_rejected():
    bad = [dict(porosity=0.0), dict(porosity=1.5), dict(darcy=0.0), dict(prandtl=-1.0)]
    for kw in bad:
        with pytest.raises(RuntimeError):
            oracle.Oracle(lbm_inputs.cavity(8, **kw))
    # rates outside (0, 2) are rejected too
    with pytest.raises(RuntimeError):
        oracle.Oracle(lbm_inputs.cavity(8, s_nu_set=2.5))
    with pytest.raises(RuntimeError):
        oracle.Oracle(lbm_inputs.cavity(8, zeta_alpha_set=2.0))
    # Eq. 56 needs Ra > 0 unless the rates are given
    with pytest.raises(RuntimeError):
        oracle.Oracle(lbm_inputs.cavity(8, rayleigh=0.0))
