"""Independent references for pinning the oracle (test code, not part of the oracle).

* Weighted particle sets: moments and exact fluxes by direct summation over particles
  (the definition of a moment, <psi f> = sum_k w_k psi(v_k)).
* Gauss-Hermite quadrature of a Maxwellian (exact for the polynomial moments used here).
* The exact Riemann solver of the Euler equations for a polytropic gas (textbook
  two-rarefaction / two-shock Newton iteration on the star pressure).
"""
import math

import numpy as np

SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


# ---------------------------------------------------------------- particles, 3V
def particle_psi14(v):
    """The 14 generating functions psi(v) for velocities v (..., 3):
    1, v_i, v_i v_j (6 stored), v_i |v|^2, |v|^4."""
    vv = (v * v).sum(-1)
    comps = [np.ones_like(vv), v[..., 0], v[..., 1], v[..., 2]]
    comps += [v[..., i] * v[..., j] for (i, j) in SYM]
    comps += [v[..., i] * vv for i in range(3)]
    comps += [vv * vv]
    return np.stack(comps, -1)


def particle_state14(w, v):
    """Primitive state and full central moment tensors of a weighted particle set.
    w (M,), v (M, 3).  Returns W (14,), Q (3,3,3), R_ijkk (3,3), S_ijjkk (3,)."""
    rho = w.sum()
    u = (w[:, None] * v).sum(0) / rho
    c = v - u
    P = np.einsum('k,ki,kj->ij', w, c, c)
    Q = np.einsum('k,ki,kj,kl->ijl', w, c, c, c)
    cc = (c * c).sum(1)
    Rt = np.einsum('k,ki,kj,k->ij', w, c, c, cc)
    S = np.einsum('k,ki,k->i', w, c, cc * cc)
    q = np.einsum('k,ki,k->i', w, c, cc)
    R = (w * cc * cc).sum()
    W = np.array([rho, *u, P[0, 0], P[0, 1], P[0, 2], P[1, 1], P[1, 2], P[2, 2], *q, R])
    return W, Q, Rt, S


def particle_cons_flux14(w, v, k):
    """<psi> and <v_k psi> by direct summation."""
    psi = particle_psi14(v)
    return (w[:, None] * psi).sum(0), (w[:, None] * v[:, k:k + 1] * psi).sum(0)


# ---------------------------------------------------------------- particles, 1V
def particle_state5(w, v):
    rho = w.sum()
    u = (w * v).sum() / rho
    c = v - u
    return np.array([rho, u, (w * c**2).sum(), (w * c**3).sum(), (w * c**4).sum()]), (w * c**5).sum()


def particle_cons_flux5(w, v):
    psi = np.stack([v**0, v, v**2, v**3, v**4], -1)
    return (w[:, None] * psi).sum(0), (w[:, None] * v[:, None] * psi).sum(0)


# ---------------------------------------------------------------- Maxwellian quadrature
def maxwellian_moments14(rho, u, T, npts=6):
    """<psi M> for a 3V Maxwellian by tensor Gauss-Hermite quadrature (exact to degree
    2 npts - 1 per axis)."""
    x, wq = np.polynomial.hermite_e.hermegauss(npts)   # weight exp(-x^2/2)
    wq = wq / math.sqrt(2 * math.pi)
    X, Y, Z = np.meshgrid(x, x, x, indexing='ij')
    Wt = (wq[:, None, None] * wq[None, :, None] * wq[None, None, :]).ravel()
    s = math.sqrt(T)
    v = np.stack([u[0] + s * X.ravel(), u[1] + s * Y.ravel(), u[2] + s * Z.ravel()], -1)
    return rho * (Wt[:, None] * particle_psi14(v)).sum(0)


def maxwellian_moments5(rho, u, T, npts=6):
    x, wq = np.polynomial.hermite_e.hermegauss(npts)
    wq = wq / math.sqrt(2 * math.pi)
    v = u + math.sqrt(T) * x
    psi = np.stack([v**0, v, v**2, v**3, v**4], -1)
    return rho * (wq[:, None] * psi).sum(0)


# ---------------------------------------------------------------- exact Euler Riemann
def exact_riemann(left, right, gamma, xi):
    """Exact solution of the Euler Riemann problem at similarity coordinates xi = x/t.
    left/right = (rho, u, p).  Returns rho, u, p arrays."""
    rl, ul, pl = left
    rr, ur, pr = right
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1) / (2 * gamma)
    g2 = (gamma + 1) / (2 * gamma)

    def f(p, r, pk, ak):
        if p > pk:
            A = 2 / ((gamma + 1) * r)
            B = (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ak / (gamma - 1) * ((p / pk)**g1 - 1)

    # bisection on the star pressure (monotone function)
    lo, hi = 1e-12, 10 * max(pl, pr) + 10
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid, rl, pl, al) + f(mid, rr, pr, ar) + (ur - ul) > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (f(ps, rr, pr, ar) - f(ps, rl, pl, al))
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (gamma - 1) / (gamma + 1)
    for n, s in enumerate(xi):
        if s <= us:   # left of contact
            if ps > pl:
                rs = rl * ((ps / pl + gm) / (gm * ps / pl + 1))
                S = ul - al * math.sqrt(g2 * ps / pl + g1)
                rho[n], u[n], p[n] = (rl, ul, pl) if s <= S else (rs, us, ps)
            else:
                rs = rl * (ps / pl)**(1 / gamma)
                ast = al * (ps / pl)**g1
                if s <= ul - al:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= us - ast:
                    rho[n], u[n], p[n] = rs, us, ps
                else:
                    uu = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s)
                    c = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * (ul - s))
                    rho[n] = rl * (c / al)**(2 / (gamma - 1))
                    u[n] = uu
                    p[n] = pl * (c / al)**(2 * gamma / (gamma - 1))
        else:
            if ps > pr:
                rs = rr * ((ps / pr + gm) / (gm * ps / pr + 1))
                S = ur + ar * math.sqrt(g2 * ps / pr + g1)
                rho[n], u[n], p[n] = (rr, ur, pr) if s >= S else (rs, us, ps)
            else:
                rs = rr * (ps / pr)**(1 / gamma)
                ast = ar * (ps / pr)**g1
                if s >= ur + ar:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= us + ast:
                    rho[n], u[n], p[n] = rs, us, ps
                else:
                    uu = 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s)
                    c = 2 / (gamma + 1) * (ar - (gamma - 1) / 2 * (ur - s))
                    rho[n] = rr * (c / ar)**(2 / (gamma - 1))
                    u[n] = uu
                    p[n] = pr * (c / ar)**(2 * gamma / (gamma - 1))
    return rho, u, p
