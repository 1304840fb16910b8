"""Condition-aware tolerances shared by the GPU parity tests.

A floating-point output y of the HIP path passes against the oracle's y*
when |y - y*| <= 1e-12 max(|y*|, s), where s is the oracle's scale of y*:
the sum of the magnitudes of the terms that make y* up, propagated through
every step (fill, surface evaluation, force sum, adjoint sweeps).  The
oracle's scale functions are pinned in tests/test_oracle_scales.py."""
import numpy as np

TOL = 1e-12


def check(got, want, scale, what, tol=TOL):
    got, want, scale = np.asarray(got), np.asarray(want), np.asarray(scale)
    err = np.abs(got - want)
    bound = tol * np.maximum(np.abs(want), scale)
    bad = ~(err <= bound)
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside {tol:g} rel; worst err "
                           f"{err[bad].max()}, its bound {bound[bad][np.argmax(err[bad])]}")


def force_scale(op, q, want, cs, p_idx, u_idx, mu):
    """Scale of each component of F = sum_q w_q (-p n + mu (grad u + grad
    u^T) n): sum_q |w_q| (s_p |n_i| + mu sum_j (s(du_i/dx_j) + s(du_j/dx_i))
    |n_j|), with s the oracle's surface scales from the cell scales cs."""
    d = op.dim
    _, _, _, ps = op.surface_query(q.x, want[p_idx:p_idx + 1], field_scale=cs[p_idx:p_idx + 1])
    _, _, _, us = op.surface_query(q.x, np.stack([want[i] for i in u_idx]),
                                   field_scale=np.stack([cs[i] for i in u_idx]))
    an = np.abs(q.n)
    out = np.zeros(d)
    for i in range(d):
        t = ps[0, 0] * an[i]
        for j in range(d):
            t = t + mu * (us[i, 1 + j] + us[j, 1 + i]) * an[j]
        out[i] = np.sum(np.abs(q.w) * t)
    return out


def force_seeds(q, d, mu, gF, nf, p_idx, u_idx, absval=False):
    """d(gF . F)/d(surface values, gradients) per field: the inputs of the
    oracle's surface adjoint for the force functional (absval: the sums of
    the magnitudes of their terms instead)."""
    nq = q.x.shape[1]
    gF = np.asarray(gF, dtype=np.float64)
    a = np.abs if absval else (lambda x: x)
    gval = np.zeros((nf, nq))
    ggrad = np.zeros((nf, d, nq))
    gval[p_idx] = a(-q.w[None, :] * gF[:, None] * q.n).sum(0)
    for i in range(d):
        for j in range(d):
            ggrad[u_idx[i], j] += a(mu * q.w * gF[i] * q.n[j]) + a(mu * q.w * gF[j] * q.n[i])
    return gval, ggrad


def force_gradient(op, q, mu, gF, kinds, p_idx, u_idx):
    """Oracle gradient of gF . F with respect to the interior field values
    and the boundary data, and the scales of both."""
    d = op.dim
    nf = len(kinds)
    gval, ggrad = force_seeds(q, d, mu, gF, nf, p_idx, u_idx)
    L0 = op.surface_query_adjoint(q.x, gval, ggrad, np.zeros((nf, op.n_cells)))
    G, Gb = op.fill_adjoint(L0, kinds)
    sval, sgrad = force_seeds(q, d, mu, gF, nf, p_idx, u_idx, absval=True)
    S0 = op.surface_query_adjoint_scale(q.x, sval, sgrad, np.zeros((nf, op.n_cells)))
    S, Sb = op.fill_adjoint_scale(S0, kinds)
    return G, Gb, S, Sb
