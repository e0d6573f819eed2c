"""Flux-Jacobian eigenvalues of the closed systems (oracle/eigen.py) and what they say about
the approximate wave speeds (Section 5.1, Appendix B).  CPU only.

Pins of the eigenvalue tool itself:
  * 5-moment equilibrium: as sigma_lim -> 0 the closure's linearisation tends to the
    Gaussian one, whose characteristic speeds are the roots of the Hermite polynomial He_5,
    0, +-sqrt(5 - sqrt 10), +-sqrt(5 + sqrt 10) (in units of sqrt(P/rho)).  The limited
    closure deviates in proportion to sqrt(sigma_lim) (its (10 - 8 sqrt(sigma_bar)) q* term),
    so a Richardson extrapolation in sqrt(sigma_lim) must land on the closed form.
  * 14 -> 5 collapse: when the transverse temperatures vanish the 14-moment system along x
    reduces to the 1D1V 5-moment system (Appendix B); the extreme eigenvalues of the two
    Jacobians must then agree.
  * Galilean shift and the x <-> y rotation covariance.
Then the diagnostics: Baradaran's 5-moment fit and the paper's 14-moment fit against the
numerical extreme eigenvalues.
"""
import numpy as np
import pytest

from oracle import closure, eigen, moments, wavespeeds
from paper_2401_15233_amd import inputs


def test_5moment_equilibrium_tends_to_hermite_roots():
    """In units rho = P = 1 at rest (Galilean shift and scaling are checked separately).  The
    difference step must stay below sigma_lim, so that the perturbed states keep
    sigma_bar = sigma_lim: h = 1e-3 sigma_lim."""
    W = moments.maxwellian_prim5(np.array([1.0]), np.array([0.0]), np.array([1.0]))
    lam = {}
    for sl in (1e-6, 1e-8):
        lam[sl] = np.sort(eigen.eigen_speeds5(W, sl, h=1e-3 * sl)[3].real[0])
    # deviation ~ sqrt(sigma_lim): extrapolate from sqrt = 1e-3 and 1e-4 to 0
    lim = lam[1e-8] + (lam[1e-8] - lam[1e-6]) / 9.0
    s10 = np.sqrt(10.0)
    exact = np.array([-np.sqrt(5 + s10), -np.sqrt(5 - s10), 0.0, np.sqrt(5 - s10), np.sqrt(5 + s10)])
    assert np.max(np.abs(lim - exact)) < 5e-6, lim - exact
    # and the unextrapolated deviation really scales with sqrt(sigma_lim)
    d6, d8 = lam[1e-6][-1] - exact[-1], lam[1e-8][-1] - exact[-1]
    assert d6 < 0 and 9.0 < d6 / d8 < 11.0


@pytest.mark.parametrize('qs,sig', [(0.0, 0.3), (0.5, 0.4), (-1.0, 0.6), (1.5, 0.8)])
def test_14moment_collapses_to_5moment(qs, sig):
    W5 = eigen.state5_from_star(np.array([qs]), np.array([sig]))
    l5 = eigen.eigen_speeds5(W5, 1e-4)
    rho, u, P, q, r = W5[:, 0]
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        # transverse temperatures eps with Gaussian transverse moments: R = r + 4 P eps + 8 eps^2
        W = np.array([rho, u, 0, 0, P, 0, 0, eps, 0, eps, q, 0, 0,
                      r + 4.0 * P * eps / rho + 8.0 * eps * eps / rho])[:, None]
        s14 = closure.sigma14_star(*closure.nondim14(W)[4:])
        assert abs(s14[0] - sig) < 1e-3
        l14 = eigen.eigen_speeds14(W, 0, 1e-4)
        errs.append(max(abs(l14[0][0] - l5[0][0]), abs(l14[1][0] - l5[1][0])))
    assert errs[-1] < 1e-5 and errs[0] > errs[1] > errs[2], errs


def test_galilean_shift_and_rotation():
    W = eigen.state14_from_star(1.3, 0.4, 0.3, 0.5)
    a = eigen.eigen_speeds14(W, 0, 1e-4)
    Wu = W.copy()
    Wu[1] += 0.7
    Wu[2] -= 0.2
    b = eigen.eigen_speeds14(Wu, 0, 1e-4)
    assert abs(b[0][0] - 0.7 - a[0][0]) < 1e-8 and abs(b[1][0] - 0.7 - a[1][0]) < 1e-8
    perm = [0, 2, 1, 3, 7, 5, 8, 4, 6, 9, 11, 10, 12, 13]   # x <-> y
    c = eigen.eigen_speeds14(W[perm], 1, 1e-4)
    assert abs(c[0][0] - a[0][0]) < 1e-9 and abs(c[1][0] - a[1][0]) < 1e-9


def test_difference_step_does_not_matter():
    W = eigen.state14_from_star(np.array([0.7, 1.0, 1.6]), np.array([-0.5, 0.8, 0.2]),
                                np.array([0.2, 0.0, 0.6]), np.array([0.3, 0.6, 0.9]))
    a = eigen.eigen_speeds14(W, 0, 1e-4, h=1e-5)
    b = eigen.eigen_speeds14(W, 0, 1e-4, h=1e-4)
    assert np.max(np.abs(a[1] - b[1])) < 1e-6 and np.max(np.abs(a[0] - b[0])) < 1e-6


def test_5moment_fit_within_twenty_percent():
    """Baradaran's approximation against the 5-moment Jacobian over q* in [-3, 3], sigma in
    [0.02, 0.98]: every state within 20 % (measured: -11 % .. +4 %, mostly below)."""
    Q, S = np.meshgrid(np.linspace(-3, 3, 61), np.linspace(0.02, 0.98, 25))
    W = eigen.state5_from_star(Q.ravel(), S.ravel())
    assert np.max(np.abs(closure.sigma5_star(W[3], W[4]) - S.ravel())) < 1e-13
    lmin, lmax, im, _ = eigen.eigen_speeds5(W, 1e-4)
    fmin, fmax = wavespeeds.wavespeeds5(W, 1e-4)
    assert im.max() < 1e-8
    r = fmax / lmax - 1.0
    rm = fmin / lmin - 1.0
    print('5-moment fit / eigenvalue - 1: quantiles 0, 50, 100 %:', np.quantile(r, [0, .5, 1]).round(3))
    assert np.all(np.abs(r) < 0.2) and np.all(np.abs(rm) < 0.2)


def test_14moment_fit_near_isotropic_pressure():
    """The paper reports the fit's error below 20 % over most of the domain (Appendix B.2).
    On the axisymmetric states with P*_xx = 1 (q*_x in [-2, 2], sigma in [0.05, 0.95]) the
    measured error lies in [-19.9 %, +2.1 %]; away from P*_xx = 1 the fit errs more, mostly by
    underestimating (up to -62 % at P*_xx = 2.5 without transverse heat flux)."""
    QX, SG = np.meshgrid(np.linspace(-2, 2, 21), np.linspace(0.05, 0.95, 10))
    W = eigen.state14_from_star(1.0, QX.ravel(), 0.0, SG.ravel())
    lmin, lmax, im, _ = eigen.eigen_speeds14(W, 0, 1e-4)
    fmin, fmax = wavespeeds.wavespeeds14(W, 1e-4, 0)
    r = fmax / lmax - 1.0
    print('14-moment fit / eigenvalue - 1 at P*_xx = 1: quantiles 0, 50, 100 %:',
          np.quantile(r, [0, .5, 1]).round(3))
    assert np.mean(np.abs(r) < 0.2) >= 0.95
    # lambda_min follows from lambda_max by the mirror relation in both the fit and the system
    rm = fmin / lmin - 1.0
    assert np.max(np.abs(rm.reshape(QX.shape) - r.reshape(QX.shape)[:, ::-1])) < 1e-6


def test_inflation_bounds_most_jet_states():
    """On the synthetic developed crossed-jets field the fit (k = 1) falls short of the true
    extreme eigenvalue (measured from the bulk velocity) in about a third of the cells along x,
    by up to a third; the inflation k = 1.2 used for the jets covers about 95 % of them."""
    W = inputs.crossed_jets_developed(48, 48, seed=2).reshape(14, -1)
    lmin, lmax, im, _ = eigen.eigen_speeds14(W, 0, 1e-4)
    fmin, fmax = wavespeeds.wavespeeds14(W, 1e-4, 0)
    u = W[1]
    ratio = (fmax - u) / (lmax - u)
    short = np.mean(ratio < 1.0)
    covered = np.mean(1.2 * ratio >= 1.0)
    print(f'fit short of the eigenvalue in {short:.3f} of the cells; k = 1.2 covers {covered:.3f}; '
          f'worst ratio {ratio.min():.3f}')
    assert 0.1 < short < 0.6 and covered > 0.9 and ratio.min() > 0.5
