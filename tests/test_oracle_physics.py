"""Pins of the oracle's whole time step (collision + streaming + walls) against
closed forms, exact discrete balances and symmetry."""
import numpy as np
import pytest

import lbm_inputs
import oracle
from lbm_inputs import face
from oracle import closed_forms as cf


def _run_to_steady(o, key, chunk=500, tol=1e-14, max_steps=200000):
    prev = o.fields()[key]
    steps = 0
    while steps < max_steps:
        o.step(chunk)
        steps += chunk
        cur = o.fields()[key]
        if np.max(np.abs(cur - prev)) <= tol * max(1e-30, np.max(np.abs(cur))):
            return cur
        prev = cur
    raise AssertionError(f"no steady state after {steps} steps")


# --------------------------------------------------------------- conduction
def _conduction(n, zeta, side_walls, q=19):
    side = face("wall", "adiabatic") if side_walls else face("periodic", "periodic")
    wl = lbm_inputs.cavity((n, 3 if side_walls else 1, 3 if side_walls else 1), lattice=q,
                           rayleigh=0.0, s_nu_set=1.0, zeta_alpha_set=zeta, noise_amp=0.0)
    wl["faces"] = [face("wall", "isothermal", 0.5), face("wall", "isothermal", -0.5),
                   side, side, side, side]
    wl["init_axis"] = -1
    return oracle.Oracle(wl)


@pytest.mark.parametrize("n,zeta,side_walls,q", [(8, 1.0, False, 19), (12, 0.4, False, 19),
                                                (8, 1.7, True, 19), (10, 1.2, True, 15)])
def test_pure_conduction_is_exactly_linear(n, zeta, side_walls, q):
    """Ra = 0: u stays zero, T relaxes to the linear profile between the
    anti-bounce-back walls, and both face Nusselt numbers are exactly 1."""
    with _conduction(n, zeta, side_walls, q) as o:
        T = _run_to_steady(o, "T", chunk=2000, tol=1e-15)
        fl = o.fields()
        x = cf.node_coords(n)
        T_lin = 0.5 - x / n
        assert np.max(np.abs(T - T_lin[None, None, :])) < 1e-13
        for k in ("ux", "uy", "uz"):
            assert np.max(np.abs(fl[k])) < 1e-15  # zero up to the rounding of M^-1
        nu = o.nusselt()
        assert abs(nu[0] - 1.0) < 1e-12 and abs(nu[1] + 1.0) < 1e-12
        assert np.all(nu[2:] == 0.0)


# --------------------------------------------------------------- conservation
def _closed_box(q=19, isothermal=True, seed=3):
    wl = lbm_inputs.cavity((6, 5, 7), lattice=q, porosity=0.5, darcy=1e-2, rayleigh=1e5)
    if not isothermal:
        wl["faces"][0] = face("wall", "adiabatic")
        wl["faces"][1] = face("wall", "adiabatic")
    o = oracle.Oracle(wl)
    f, g = lbm_inputs.random_state(q, o.shape, seed, f_base=1.0 / q, amp=0.02, T_amp=0.3)
    o.set_state(f, g)
    return o


@pytest.mark.parametrize("q", [19, 15])
def test_closed_box_conserves_mass_and_adiabatic_heat(q):
    with _closed_box(q, isothermal=False) as o:
        f0, g0 = o.get_state()
        m0, h0 = f0.sum(), g0.sum()
        for _ in range(30):
            o.step(1)
            f, g = o.get_state()
            assert abs(f.sum() - m0) < 1e-13 * abs(m0)
            assert abs(g.sum() - h0) < 1e-13 * max(1.0, abs(h0))


@pytest.mark.parametrize("q", [19, 15])
def test_heat_balance_equals_wall_fluxes(q):
    """sum sigma T(t+1) - sum sigma T(t) equals the heat the anti-bounce-back
    walls put in during the streaming, which is what the face Nusselt numbers
    report (scaled by L / (alpha_e dT))."""
    with _closed_box(q, isothermal=True) as o:
        d = o.derived()
        shape = o.shape  # (nz, ny, nx)
        face_nodes = [shape[0] * shape[1]] * 2 + [shape[0] * shape[2]] * 2 + [shape[1] * shape[2]] * 2
        _, g = o.get_state()
        h_prev = g.sum()
        for _ in range(30):
            o.step(1)
            _, g = o.get_state()
            h = g.sum()
            nu = o.nusselt()
            flux = sum(nu[k] * face_nodes[k] for k in range(6)) * d["alpha_e"] * 1.0 / d["L"]
            assert abs((h - h_prev) - flux) < 1e-13
            h_prev = h


def test_periodic_box_momentum_changes_by_the_force():
    """In a periodic box streaming only permutes populations, so
    sum_x j(t+1) - sum_x j(t) = sum_x rho0 F(t), and by Eq. 26 F = 2 (u - j)."""
    wl = lbm_inputs.periodic_box((5, 4, 6), porosity=0.55, darcy=1e-3, rayleigh=1e5)
    with oracle.Oracle(wl) as o:
        f, g = lbm_inputs.random_state(19, o.shape, 9, amp=0.05, T_amp=0.4)
        o.set_state(f, g)
        e = oracle.velocities(19).astype(float)
        for _ in range(10):
            f, _ = o.get_state()
            j = np.einsum("aq,qzyx->azyx", e, f)
            fl = o.fields()
            u = np.stack([fl["ux"], fl["uy"], fl["uz"]])
            F = 2 * (u - j)
            o.step(1)
            f1, _ = o.get_state()
            j1 = np.einsum("aq,qzyx->azyx", e, f1)
            assert np.max(np.abs((j1 - j).sum((1, 2, 3)) - F.sum((1, 2, 3)))) < 1e-14


# --------------------------------------------------------------- symmetry
@pytest.mark.parametrize("q", [19, 15])
def test_noise_free_cavity_keeps_its_symmetries(q):
    """The cavity (hot -x, cold +x, buoyancy along z, T0 = 0) is invariant under
    the half-turn about the y axis combined with T -> -T, and under the mirror
    y -> -y.  A noise-free run must keep both to rounding."""
    wl = lbm_inputs.cavity((9, 6, 9), lattice=q, porosity=0.7, darcy=1e-2, rayleigh=1e5,
                           noise_amp=0.0)
    with oracle.Oracle(wl) as o:
        o.step(400)
        fl = o.fields()
    T, ux, uy, uz = fl["T"], fl["ux"], fl["uy"], fl["uz"]   # (z, y, x)
    rot = lambda a: a[::-1, :, ::-1]
    mir = lambda a: a[:, ::-1, :]
    assert np.max(np.abs(uz)) > 1e-4  # there is a flow to test
    su = np.max(np.abs(ux))
    assert np.max(np.abs(T + rot(T))) < 1e-12
    assert np.max(np.abs(ux + rot(ux))) < 1e-12 * su
    assert np.max(np.abs(uy - rot(uy))) < 1e-12 * su
    assert np.max(np.abs(uz + rot(uz))) < 1e-12 * su
    assert np.max(np.abs(T - mir(T))) < 1e-12
    assert np.max(np.abs(uy + mir(uy))) < 1e-12 * su
    assert np.max(np.abs(ux - mir(ux))) < 1e-12 * su


# --------------------------------------------------------------- channels
def _channel(n, q=19, forch=0.0, darcy=1e-2, phi=0.6, s_nu=1.0, a=None):
    side_p = face("periodic", "periodic")
    wall = face("wall", "adiabatic")
    a = 0.1 / (n * n) if a is None else a
    wl = {
        "nx": 1, "ny": n, "nz": 1, "q": q, "porosity": phi, "darcy": darcy,
        "rayleigh": 0.0, "prandtl": 1.0, "forchheimer": forch,
        "s_nu_set": s_nu, "zeta_alpha_set": 1.0, "length_axis": 1, "gravity_axis": 1,
        "T_ref": 0.0, "delta_T": 1.0, "accel": (a, 0.0, 0.0),
        "faces": [side_p, side_p, wall, wall, side_p, side_p],
        "init_axis": -1, "noise_amp": 0.0,
    }
    return oracle.Oracle(wl), a


def _brinkman_error(n, q=19):
    o, a = _channel(n, q)
    with o:
        u = _run_to_steady(o, "ux", chunk=2000, tol=1e-13)[0, :, 0]
        d = o.derived()
    ua = cf.brinkman_channel(n, a, d["K"], d["nu"], d["nu_e"], 0.6)
    return cf.relative_global_error(ua, u)


@pytest.mark.parametrize("q", [19, 15])
def test_brinkman_channel_profile(q):
    """Body-force-driven porous channel with F_phi = 0 against the closed form
    of Eqs. 2 + 4 (Sec. 4.1 uses the same model without the Forchheimer term)."""
    err = _brinkman_error(32, q)
    assert err < 2e-3


@pytest.mark.slow
def test_brinkman_channel_second_order():
    """Observed order of the relative global error (Eq. 52) over N_y = 16..64 is
    about two, the paper's stated accuracy (Sec. 4.1, Fig. 6)."""
    ns = np.array([16, 24, 32, 48, 64])
    errs = np.array([_brinkman_error(int(n)) for n in ns])
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2, (errs, slope)


def test_forchheimer_channel_profile():
    """With the Forchheimer drag the steady profile is compared with a
    Richardson-extrapolated Newton solution of the 1-D boundary value problem."""
    n = 32
    o, a = _channel(n, forch=1.0, darcy=1e-2, a=5e-4)  # u_max ~ 0.026
    with o:
        u = _run_to_steady(o, "ux", chunk=2000, tol=1e-13)[0, :, 0]
        d = o.derived()
    ua = cf.forchheimer_channel(n, a, d["K"], d["nu"], d["nu_e"], 0.6, d["F_phi"], refine=16)
    ub = cf.brinkman_channel(n, a, d["K"], d["nu"], d["nu_e"], 0.6)
    err = cf.relative_global_error(ua, u)
    assert err < 1e-3
    # the Forchheimer drag changes the profile by ~10% here
    assert cf.relative_global_error(ub, ua) > 10 * err


def test_mixed_convection_channel_eqs_48_49():
    """Mixed convection in a porous channel (Sec. 4.1, E1 setup): the paper's
    closed forms Eqs. 48-50 for u_x and T with the wall-normal acceleration of
    Eq. 47.  The walls carry a normal velocity, which bounce-back and
    anti-bounce-back treat only approximately, so the bound is loose."""
    n = 32
    phi, Re, Pr, Ra, da = 0.6, 5.0, 1.0, 100.0, 1e-2
    nu = (1 / 1.0 - 0.5) / 3  # s_nu = 1
    u1 = Re * nu / n
    u0 = u1
    wl = {
        "nx": 1, "ny": n, "nz": 1, "q": 19, "porosity": phi, "darcy": da,
        "rayleigh": Ra, "prandtl": Pr, "forchheimer": 0.0, "s_nu_set": 1.0,
        "length_axis": 1, "gravity_axis": 1, "T_ref": 0.0, "delta_T": 1.0,
        "faces": [face("periodic", "periodic")] * 2 +
                 [face("wall", "isothermal", -0.5, (0.0, u1, 0.0)),
                  face("wall", "isothermal", 0.5, (u0, u1, 0.0))] +
                 [face("periodic", "periodic")] * 2,
        "init_axis": -1, "noise_amp": 0.0,
    }
    with oracle.Oracle(wl) as o:
        d = o.derived()
        ay = cf.mixed_convection_accel(n, u1, d["nu"], d["K"], d["gbeta"], 1.0, d["alpha_e"])
        acc = np.zeros((3,) + o.shape)
        acc[1, 0, :, 0] = ay
        o.set_accel_field(acc)
        _run_to_steady(o, "ux", chunk=2000, tol=1e-12)
        fl = o.fields()
    ua, Ta = cf.mixed_convection_channel(n, u0, u1, d["nu"], d["nu_e"], d["alpha_e"], phi,
                                         1.0, da, -0.5, 0.5)
    eu = cf.relative_global_error(ua, fl["ux"][0, :, 0])
    eT = cf.relative_global_error(Ta, fl["T"][0, :, 0])
    uy = fl["uy"][0, :, 0]
    assert eu < 2e-2, eu
    assert eT < 2e-2, eT
    assert np.max(np.abs(uy - u1)) < 0.05 * u1


# --------------------------------------------------------------- open boundaries
@pytest.mark.parametrize("q,forch", [(19, 0.0), (19, 1.0), (15, 1.0)])
def test_plug_flow_through_porous_slab_obeys_darcy_forchheimer(q, forch):
    """Uniform inflow U through a moving-wall inlet, an open outlet at rho0:
    mass conservation makes u = U exactly, and the momentum balance of Eq. 2
    with Eq. 4 gives cs^2 d(rho)/dx = F = -(phi nu/K) U - (phi F_phi/sqrt K) U^2.
    The inlet temperature is carried through unchanged."""
    U, n, phi = 0.02, 48, 0.7
    per = face("periodic", "periodic")
    wl = {"nx": n, "ny": 1, "nz": 1, "q": q, "porosity": phi, "darcy": 1e-1, "rayleigh": 0.0,
          "prandtl": 1.0, "forchheimer": forch, "s_nu_set": 1.2, "zeta_alpha_set": 1.0,
          "length_axis": 0, "gravity_axis": 1, "T_ref": 0.0, "delta_T": 1.0,
          "faces": [face("wall", "isothermal", 0.3, (U, 0.0, 0.0)), face("outlet", "outflow"),
                    per, per, per, per],
          "init_axis": -1, "noise_amp": 0.0, "init_u": (U, 0.0, 0.0)}
    with oracle.Oracle(wl) as o:
        d = o.derived()
        _run_to_steady(o, "rho", chunk=2000, tol=1e-13)
        fl = o.fields()
    ux, rho, T = fl["ux"][0, 0], fl["rho"][0, 0], fl["T"][0, 0]
    F = -phi * d["nu"] / d["K"] * U - phi * d["F_phi"] / np.sqrt(d["K"]) * U * U
    slope = np.polyfit(np.arange(n), rho, 1)[0]
    assert np.max(np.abs(ux - U)) < 1e-13
    # (exact to 1e-12 for D3Q19; D3Q15 carries an O(U^2 drho) compressibility term)
    assert abs(slope / (F / (1.0 / 3.0)) - 1.0) < 1e-6
    # linear away from the last nodes (D3Q15 has a thin outlet layer in rho)
    assert np.max(np.abs(np.diff(rho)[:-4] - slope)) < 1e-5 * abs(slope)
    # the open boundary holds rho0 at the outlet face to O(U^2)
    assert abs(rho[-1] + 0.5 * slope - 1.0) < U * U
    assert np.max(np.abs(T - 0.3)) < 1e-13
