"""Oracle pins for the point-implicit BGK source and for jet inflow on any wall.  CPU only.

Point-implicit source (forward Euler transport, then the source alone by backward Euler;
Section 4.3 names point-implicit sources as the remedy for stiff collisions):
  * the result solves the backward-Euler equation U = U_t + dt C(U) with C the paper's BGK
    source formulas (Sections 2.3-2.4; pinned to quadrature elsewhere), to rounding;
  * a uniform state relaxes as U_M + (U_0 - U_M) (1 + dt/tau)^-n;
  * in the stiff limit dt/tau -> infinity one step lands on the local Maxwellian.
Jets on any wall: a jet on the bottom wall at 90 degrees is the x <-> y mirror image of a
jet on the left wall at 0 degrees (the left-wall path is pinned by the jet tests), for the
whole residual.
"""
import math

import numpy as np
import pytest

from oracle import moments as mo, scheme as sc
from paper_2401_15233_amd import inputs as I


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize('system', [5, 14])
@pytest.mark.parametrize('tau_mode', ['local', 'const'])
@pytest.mark.parametrize('h', [1e-3, 1.0, 1e3])
def test_backward_euler_equation_holds(system, tau_mode, h):
    if system == 14:
        W = I.random_states14(64, seed=5)
        s = sc.Setup(system=14, dim=1, nx=64, tau_mode=tau_mode, integrator='fe', source_implicit=True)
        Ut = mo.prim_to_cons14(W)
        T = mo.pressure14(W) / W[0]
    else:
        W = I.random_states5(64, seed=6)
        s = sc.Setup(system=5, dim=1, nx=64, tau_mode=tau_mode, integrator='fe', source_implicit=True)
        Ut = mo.prim_to_cons5(W)
        T = W[2] / W[0]
    tau_ref = 0.01
    tau = tau_ref * (1.0 / W[0]) * np.sqrt(1.0 / T) if tau_mode == 'local' else tau_ref + 0 * T
    dt = h * np.median(tau)
    U = sc.relax_backward_euler(Ut, dt, s, tau_ref)
    Wn = sc.cons_to_prim(U, s)
    resid = U - Ut - dt * sc.bgk_source(Wn, s, tau_ref)
    scale = np.maximum(np.abs(Ut), np.abs(U)).max(axis=1, keepdims=True)
    # dt C(U) is h times a difference of nearly equal moments: rounding grows like (1 + h)
    assert np.max(np.abs(resid) / scale) < 1e-11 * (1.0 + h)
    # rho, rho u and the energy are untouched
    keep = [0, 1, 2] if system == 5 else [0, 1, 2, 3]
    assert np.max(np.abs(U[keep] - Ut[keep]) / scale[keep]) < 1e-15
    if system == 14:
        assert rel(U[4] + U[7] + U[9], Ut[4] + Ut[7] + Ut[9]) < 1e-14


@pytest.mark.parametrize('system', [5, 14])
def test_homogeneous_implicit_relaxation_closed_form(system):
    nx = 8
    if system == 14:
        W0 = I.random_states14(1, seed=19)
        s = sc.Setup(system=14, dim=2, nx=nx, ny=4, bc=('periodic',) * 4, integrator='fe',
                     source_implicit=True)
        U0 = np.broadcast_to(mo.prim_to_cons14(W0)[:, :, None], (14, 4, nx)).copy()
        p = mo.pressure14(W0)[0]
        UM = mo.prim_to_cons14(mo.maxwellian_prim14(W0[0], W0[1:4].T, np.array([p])))[:, 0]
        T = p / W0[0, 0]
    else:
        W0 = I.random_states5(1, seed=20)
        s = sc.Setup(system=5, dim=1, nx=nx, bc=('periodic',) * 4, integrator='fe',
                     source_implicit=True)
        U0 = np.broadcast_to(mo.prim_to_cons5(W0), (5, nx)).copy()
        UM = mo.prim_to_cons5(mo.maxwellian_prim5(W0[0], W0[1], W0[2]))[:, 0]
        T = W0[2, 0] / W0[0, 0]
    tau_ref = 0.05
    tau = tau_ref * (1.0 / W0[0, 0]) * math.sqrt(1.0 / T)
    shape = (-1,) + (1,) * (U0.ndim - 1)
    for z in (0.3, 5.0, 1e4):      # far beyond the explicit limit z < 2
        U, t, n = sc.run(U0, s, tau_ref, nsteps=7, dt=z * tau, check=False)
        expect = UM.reshape(shape) + (1.0 + z) ** -7 * (U0 - UM.reshape(shape))
        assert rel(U, expect) < 1e-12, z


def test_stiff_limit_is_the_local_maxwellian():
    W = I.random_states14(32, seed=8)
    s = sc.Setup(system=14, dim=1, nx=32, integrator='fe', source_implicit=True)
    Ut = mo.prim_to_cons14(W)
    U = sc.relax_backward_euler(Ut, 1e14, s, 1e-3)
    p = mo.pressure14(W)
    UM = mo.prim_to_cons14(mo.maxwellian_prim14(W[0], W[1:4].T, p))
    assert rel(U, UM) < 1e-12


def test_implicit_source_needs_forward_euler():
    s = sc.Setup(system=5, dim=1, nx=8, integrator='ssprk2', source_implicit=True)
    with pytest.raises(ValueError):
        sc.step(mo.prim_to_cons5(I.sod_prims(5, 8)), 1e-3, s, 0.01)


def _swap_xy(W):
    """x <-> y mirror of a 14-moment primitive field [14][ny][nx] -> [14][nx][ny]."""
    perm = [0, 2, 1, 3, 7, 5, 8, 4, 6, 9, 11, 10, 12, 13]
    return np.swapaxes(W[perm], 1, 2)


@pytest.mark.parametrize('order', [1, 2])
def test_bottom_wall_jet_mirrors_left_wall_jet(order):
    nx, ny = 14, 11
    W = I.random_smooth_field14(nx, ny, seed=4)
    common = dict(system=14, dim=2, order=order, jet_mach=5.0, jet_rho=1.0, jet_T=1.0)
    left = sc.Setup(nx=nx, ny=ny, bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
                    jets=[(0.45, 0.3, 20.0, 0)], **common)
    bottom = sc.Setup(nx=ny, ny=nx, bc=('transmissive', 'transmissive', 'jet', 'transmissive'),
                      jets=[(0.45, 0.3, 70.0, 2)], **common)
    L1 = sc.residual(mo.prim_to_cons14(W), left, 0.02)
    Wm = _swap_xy(W)
    L2 = sc.residual(mo.prim_to_cons14(Wm), bottom, 0.02)
    # mirror the residual of the conserved field back
    perm = [0, 2, 1, 3, 7, 5, 8, 4, 6, 9, 11, 10, 12, 13]
    back = np.swapaxes(L2[perm], 1, 2)
    assert rel(back, L1) < 1e-13
    # and the jet really enters: residual differs from the all-transmissive one
    plain = sc.Setup(nx=nx, ny=ny, bc=('transmissive',) * 4, **common)
    assert rel(sc.residual(mo.prim_to_cons14(W), plain, 0.02), L1) > 1e-3


def test_right_and_top_wall_jets_mirror_left_wall_jet():
    nx, ny = 12, 12
    W = I.random_smooth_field14(nx, ny, seed=9)
    common = dict(system=14, dim=2, order=2, jet_mach=2.0, jet_rho=0.5, jet_T=1.5, nx=nx, ny=ny)
    left = sc.Setup(bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
                    jets=[(0.4, 0.25, 10.0, 0)], **common)
    right = sc.Setup(bc=('transmissive', 'jet', 'transmissive', 'transmissive'),
                     jets=[(0.4, 0.25, 170.0, 1)], **common)
    # mirror x -> -x: reverse the x axis and negate the x-odd components
    odd = [1, 5, 6, 10]
    def mirror(A):
        B = A[:, :, ::-1].copy()
        B[odd] = -B[odd]
        return B
    L1 = sc.residual(mo.prim_to_cons14(W), left, 0.02)
    L2 = sc.residual(mo.prim_to_cons14(mirror(W)), right, 0.02)
    assert rel(mirror(L2), L1) < 1e-13
    top = sc.Setup(bc=('transmissive', 'transmissive', 'transmissive', 'jet'),
                   jets=[(0.4, 0.25, -80.0, 3)], **common)
    bottom = sc.Setup(bc=('transmissive', 'transmissive', 'jet', 'transmissive'),
                      jets=[(0.4, 0.25, 80.0, 2)], **common)
    oddy = [2, 5, 8, 11]
    def mirror_y(A):
        B = A[:, ::-1, :].copy()
        B[oddy] = -B[oddy]
        return B
    L3 = sc.residual(mo.prim_to_cons14(W), bottom, 0.02)
    L4 = sc.residual(mo.prim_to_cons14(mirror_y(W)), top, 0.02)
    assert rel(mirror_y(L4), L3) < 1e-13
