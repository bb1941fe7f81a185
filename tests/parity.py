"""Shared helpers of the GPU parity tests (test infrastructure)."""

import numpy as np

from oracle.dg import DG
from oracle.euler import flux
from oracle.quadrature import gauss_legendre, lagrange_deriv

TOL = 1e-12   # FP64 parity bar of the hot path


def summand_scale(dg, Q):
    """Per field: max over nodes of sum_d (2/h_d) |F^d_f| times
    max_i sum_a |w_a D_ai / w_i| -- the size of the terms whose differences
    make up the right-hand side (cancellation scale)."""
    q = np.asarray(Q).reshape(5, -1)
    xi, w = gauss_legendre(dg.N)
    dh = 1.0
    if dg.N > 1:
        D = lagrange_deriv(xi, xi)
        dh = max(1.0, float(np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0))))
    s = np.zeros_like(q)
    for d in range(3):
        s = s + (2.0 / dg.h[d]) * np.abs(flux(q, d, dg.gamma))
    return np.max(s, axis=1) * dh


def rhs_errors(dg, Q, R_gpu, R_ora):
    """(plain relative, summand-scaled) error per field:
    plain_f = |dR_f|_inf / |R_ora_f|_inf,
    scaled_f = |dR_f|_inf / (|R_ora_f|_inf + S_f)."""
    d = np.abs(np.asarray(R_gpu) - np.asarray(R_ora)).reshape(5, -1).max(axis=1)
    ref = np.abs(np.asarray(R_ora)).reshape(5, -1).max(axis=1)
    S = summand_scale(dg, Q)
    plain = d / np.maximum(ref, 1e-300)
    scaled = d / (ref + S)
    return plain, scaled


def patch_rhs(n, p, L, Q, elems, gamma=1.4, make=DG):
    """Oracle right-hand side at selected elements of a large periodic mesh.
    The RHS of an element depends only on it and its six face neighbours, so
    it equals the RHS of the centre element of the 3x3x3 periodic patch
    around it (same element size).  Returns {(ex,ey,ez): R[5,N,N,N]}."""
    nx, ny, nz = n
    h = np.array(L, dtype=np.float64) / np.array(n)
    small = make((3, 3, 3), p, L=tuple(3 * h), gamma=gamma)
    out = {}
    for (ex, ey, ez) in elems:
        xs = [(ex + o) % nx for o in (-1, 0, 1)]
        ys = [(ey + o) % ny for o in (-1, 0, 1)]
        zs = [(ez + o) % nz for o in (-1, 0, 1)]
        patch = Q[:, zs][:, :, ys][:, :, :, xs]
        R = small.rhs(np.ascontiguousarray(patch))
        out[(ex, ey, ez)] = R[:, 1, 1, 1]
    return out


def visc_summand_scale(ns, Q):
    """Per field: the summand scale of the viscous rate, max over nodes of
    sum_d (2/h_d) |F_v^d_f| times max_i sum_a |w_a D_ai / w_i| (F_v the
    oracle's nodal viscous flux), plus the same for the gradients that
    F_v is built from, scaled by the viscosity."""
    xi, w = gauss_legendre(ns.N)
    dh = 1.0
    if ns.N > 1:
        D = lagrange_deriv(xi, xi)
        dh = max(1.0, float(np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0))))
    th = ns.gradients(Q)
    Fv = ns.viscous_flux(Q, th)
    s = np.zeros(Fv.shape[1:])
    for d in range(3):
        s = s + (2.0 / ns.h[d]) * np.abs(Fv[d])
    out = np.max(s.reshape(5, -1), axis=1) * dh
    # the gradients' own summands enter every stress through mu (and the
    # energy through kappa): (2/h)^2 times the largest primitive magnitude
    P = np.abs(ns.primitives(Q)).reshape(4, -1).max(axis=1)
    g = (2.0 / ns.h.min()) ** 2 * dh * dh
    out[1:4] += ns.mu * g * P[:3].max()
    out[4] += (ns.kappa * P[3] + ns.mu * P[:3].max() ** 2) * g
    return out


def patch_rhs_viscous(n, p, L, Q, elems, mu, prandtl, gamma=1.4):
    """Oracle Navier-Stokes right-hand side at selected elements of a large
    periodic mesh: the viscous rate of an element depends on the elements
    within two face steps of it (the gradients of its face neighbours use
    their neighbours), so it equals the rate of the centre element of the
    5x5x5 periodic patch around it.  Returns {(ex,ey,ez): R[5,N,N,N]}."""
    from oracle.viscous import NavierStokesDG
    nx, ny, nz = n
    h = np.array(L, dtype=np.float64) / np.array(n)
    small = NavierStokesDG((5, 5, 5), p, L=tuple(5 * h), gamma=gamma, mu=mu, prandtl=prandtl)
    out = {}
    for (ex, ey, ez) in elems:
        xs = [(ex + o) % nx for o in range(-2, 3)]
        ys = [(ey + o) % ny for o in range(-2, 3)]
        zs = [(ez + o) % nz for o in range(-2, 3)]
        patch = Q[:, zs][:, :, ys][:, :, :, xs]
        R = small.rhs(np.ascontiguousarray(patch))
        out[(ex, ey, ez)] = R[:, 2, 2, 2]
    return out


def split_summand_scale(dg, Q):
    """Per field: the summand scale of the split-form rate, the inviscid one
    with the larger of max_i sum_a |D_ia| and max_i sum_a |w_a D_ai / w_i|
    (both line operators appear) and a factor 2 for the two-point sums."""
    q = np.asarray(Q).reshape(5, -1)
    xi, w = gauss_legendre(dg.N)
    dh = 1.0
    if dg.N > 1:
        D = lagrange_deriv(xi, xi)
        dh = max(1.0, float(np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0))),
                 float(np.max(np.sum(np.abs(D), axis=1))))
    s = np.zeros_like(q)
    for d in range(3):
        s = s + (2.0 / dg.h[d]) * np.abs(flux(q, d, dg.gamma))
    return 2.0 * np.max(s, axis=1) * dh
