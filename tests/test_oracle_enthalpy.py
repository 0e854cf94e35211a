"""Pins of the oracle's enthalpy-based D3Q7-MRT model (App. B, Eqs. B4-B13)
in the conduction setting of the paper's melting test (Sec. 4.3, u = 0)."""
import numpy as np
import pytest

import lbm_inputs
import oracle
from oracle import closed_forms as cf


def test_eta_reduces_to_the_classical_one_phase_stefan_root():
    """With the solid at the melting point Eq. 59 loses its second term and
    becomes Neumann's one-phase condition eta e^{eta^2} erf(eta) = St/sqrt(pi);
    for St = 1 the tabulated root is 0.6201."""
    from scipy.special import erf
    eta = cf.melting_eta(0.02, 0.02, 1.0, 1.0, 1.0, 0.0, 0.0, 1.0, 1.0)
    assert abs(eta - 0.6201) < 1e-4
    assert abs(eta * np.exp(eta * eta) * erf(eta) - 1.0 / np.sqrt(np.pi)) < 1e-12


def test_phase_map_is_continuous_and_monotone():
    """Eqs. B8-B9: T(En) is continuous at En_s and En_l and non-decreasing,
    f_l rises from 0 to 1 across the mushy range, and the two limits have
    slope 1/(sigma c_pl)."""
    wl = lbm_inputs.melting(4, 1, 1, mushy=0.3, porosity=0.6, matrix_heat=0.8, c_ps=0.7)
    with oracle.EnthalpyOracle(wl) as o:
        sig_l = 0.6 + 0.4 * 0.8
        sig_s = 0.6 * 0.7 + 0.4 * 0.8
        En_s = sig_s * 1.0 * 0.0
        En_l = sig_l * 1.0 * 0.3 + 0.6 * wl["latent"]
        E = np.linspace(-2.0, 3.0, 2001)
        T = np.array([o.phase(e)[0] for e in E])
        fl = np.array([o.phase(e)[1] for e in E])
        assert np.all(np.diff(T) >= -1e-15)
        assert np.all((fl >= 0) & (fl <= 1)) and fl[0] == 0.0 and fl[-1] == 1.0
        for e, Tb in ((En_s, 0.0), (En_l, 0.3)):
            lo, hi = o.phase(e - 1e-12)[0], o.phase(e + 1e-12)[0]
            assert abs(lo - Tb) < 1e-9 and abs(hi - Tb) < 1e-9
        assert abs(o.phase(-1.0)[0] - (-1.0 / sig_s)) < 1e-15
        assert abs(o.phase(En_l + 1.0)[0] - (0.3 + 1.0 / sig_l)) < 1e-14
        assert abs(o.phase(0.5 * (En_s + En_l))[1] - 0.5) < 1e-14


def test_without_latent_heat_it_is_the_temperature_model():
    """L_a = 0, sigma = c_pl = c_p,ref = 1 and one diffusivity: the enthalpy
    model is the temperature model of Sec. 3.2 at u = 0 (n_0 = En = T,
    n_4^eq = varpi T, same wall rules).  Both oracles must agree to rounding on
    a box with isothermal, adiabatic and periodic faces."""
    wl = lbm_inputs.melting(9, 5, 4, stefan=1e30, alpha_s=0.05, T_init=0.2)
    wl["latent"] = 0.0
    wl["faces"] = [lbm_inputs.face("wall", "isothermal", 1.0), lbm_inputs.face("wall", "isothermal", -0.5),
                   lbm_inputs.face("wall", "adiabatic"), lbm_inputs.face("wall", "adiabatic"),
                   lbm_inputs.face("periodic", "periodic"), lbm_inputs.face("periodic", "periodic")]
    zeta_alpha = 1.0 / (0.5 + 0.05 / (0.5 / 3.0))
    tw = lbm_inputs.cavity((9, 5, 4), rayleigh=0.0, reynolds=10.0, u_char=0.05, zeta_alpha_set=zeta_alpha,
                           noise_amp=0.0, init_axis=-1, T_ref=0.2, delta_T=1.0, porosity=1.0)
    tw["faces"] = wl["faces"]
    with oracle.EnthalpyOracle(wl) as e, oracle.Oracle(tw) as t:
        for n in (1, 7, 40):
            e.step(n)
            t.step(n)
            ge = e.get_state()
            f, gt = t.get_state()
            assert np.max(np.abs(ge - gt)) < 1e-14, (e.time, np.max(np.abs(ge - gt)))
            assert np.max(np.abs(t.fields()["ux"])) < 1e-15


def test_enthalpy_is_conserved_in_a_closed_box():
    """Adiabatic walls and periodic faces: sum En (Eq. B7) is constant, with a
    random state that straddles the solid, mushy and liquid ranges."""
    wl = lbm_inputs.melting(7, 6, 5, mushy=0.2, stefan=0.5, alpha_ratio=3.0)
    wl["faces"] = [lbm_inputs.face("wall", "adiabatic")] * 2 + [lbm_inputs.face("periodic", "periodic")] * 2 \
        + [lbm_inputs.face("wall", "adiabatic")] * 2
    rng = np.random.default_rng(17)
    with oracle.EnthalpyOracle(wl) as o:
        g = rng.uniform(-0.3, 0.7, size=(7,) + o.shape)
        o.set_state(g)
        total0 = o.fields()["En"].sum()
        fl0 = o.fields()["fl"]
        assert 0 < np.mean((fl0 > 0) & (fl0 < 1)) < 1 and np.any(fl0 == 0) and np.any(fl0 == 1)
        for _ in range(5):
            o.step(3)
            assert abs(o.fields()["En"].sum() - total0) < 1e-13 * abs(total0)


@pytest.mark.parametrize("ratio,e_bound,front_bound", [(1.0, 2e-3, 0.5), (4.0, 3e-3, 1.0), (12.0, 1.5e-2, 2.0)])
def test_two_region_melting_matches_the_closed_form(ratio, e_bound, front_bound):
    """Sec. 4.3 setting (T_h = 1, T_m = 0, T_i = -1, alpha_s = 0.02, St = 1,
    phi = sigma = c_pl = c_ps = 1) at Fo = t alpha_s / L^2 = 0.01 with L = 400:
    the temperature against Eqs. 57-58 (relative global error of Eq. 52) and
    the front (molten volume per unit area) against x_m = 2 eta sqrt(alpha_l t).
    The bounds are about twice the errors of the oracle as written; a wrong
    latent-heat factor, diffusivity interpolation or wall value fails them."""
    wl = lbm_inputs.melting(400, 1, 1, alpha_ratio=ratio)
    t = int(0.01 * 400 ** 2 / wl["alpha_s"])
    with oracle.EnthalpyOracle(wl) as o:
        o.step(t)
        f = o.fields()
    x = np.arange(400) + 0.5
    al, als = wl["alpha_l"], wl["alpha_s"]
    Ta, xm, _ = cf.two_region_melting(x, t, al, als, al, als, 1.0, 0.0, -1.0, wl["latent"], 1.0)
    T = f["T"][0, 0]
    assert cf.relative_global_error(T, Ta) < e_bound
    assert abs(f["fl"][0, 0].sum() - xm) < front_bound
