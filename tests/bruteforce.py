"""Independent brute-force evaluators used to pin the oracle.

Nothing here follows the paper's update formulas: the reconstruction is the
dense Tucker model built by successive n-mode products (Sec. 2.1), derivatives
come from linearity (replacing one factor row by a unit vector), and minimisers
come from fitting the loss along one coordinate.  Only tiny tensors.
"""
import numpy as np


def full_tensor(core, factors):
    """G x_1 A1 x_2 A2 ... x_N AN as a dense array (n-mode products, Sec. 2.1)."""
    t = np.asarray(core, dtype=np.float64)
    for n, A in enumerate(factors):
        t = np.moveaxis(np.tensordot(A, t, axes=([1], [n])), 0, n)
    return t


def recon_at(idx, core, factors):
    return full_tensor(core, factors)[tuple(idx.T)]


def sse(idx, val, core, factors):
    r = val - recon_at(idx, core, factors)
    return float(np.sum(r * r))


def loss(idx, val, core, factors, reg, lam):
    s = sse(idx, val, core, factors)
    if reg == 0:
        p = np.sum(core ** 2) + sum(np.sum(A ** 2) for A in factors)
    else:
        p = np.sum(np.abs(core)) + sum(np.sum(np.abs(A)) for A in factors)
    return s + lam * p


def delta_by_linearity(idx, core, factors, n):
    """[nnz, J_n]: derivative of B(alpha) w.r.t. a^(n)_{i_n j}.

    B(alpha) is linear in row i_n of A^(n); replacing that row by the unit
    vector e_j gives the coefficient of a^(n)_{i_n j}.
    """
    J = factors[n].shape[1]
    out = np.zeros((idx.shape[0], J))
    for j in range(J):
        f = [A.copy() for A in factors]
        f[n][:] = 0.0
        f[n][:, j] = 1.0
        out[:, j] = recon_at(idx, core, f)
    return out


def core_weights(idx, factors, beta):
    """w_beta(alpha) as B(alpha) of a core that is the indicator of beta."""
    ranks = [A.shape[1] for A in factors]
    g = np.zeros(ranks)
    g[tuple(beta)] = 1.0
    return recon_at(idx, g, factors)


def quad_argmin(fn, x0, h=0.5):
    """Exact minimiser of a function known to be quadratic, from 3 samples."""
    xs = np.array([x0 - h, x0, x0 + h])
    ys = np.array([fn(x) for x in xs])
    a, b, _ = np.polyfit(xs, ys, 2)
    return -b / (2 * a), a


def lasso_argmin(fn_smooth, lam):
    """argmin of q(x) + lam |x| where q is quadratic (sampled at -1, 0, 1)."""
    xs = np.array([-1.0, 0.0, 1.0])
    ys = np.array([fn_smooth(x) for x in xs])
    a, b, _ = np.polyfit(xs, ys, 2)
    cands = [0.0]
    xp = (-b - lam) / (2 * a)
    if xp > 0:
        cands.append(xp)
    xm = (-b + lam) / (2 * a)
    if xm < 0:
        cands.append(xm)
    vals = [a * x * x + b * x + lam * abs(x) for x in cands]
    return cands[int(np.argmin(vals))]
