"""Reference minimisers for the minimiser tests: scipy's BFGS over vech(L),
H = L L^T, on an objective from the oracle (value and exact gradient)."""
import numpy as np
from scipy import optimize


def unvech(v, d):
    """Lower-triangular L from vech (columns of the lower triangle stacked)."""
    L = np.zeros((d, d))
    k = 0
    for j in range(d):
        L[j:, j] = v[k:k + d - j]
        k += d - j
    return L


def H_of(v, d):
    L = unvech(np.asarray(v, dtype=np.float64), d)
    return L @ L.T


def argmin_vech(fun, v0, d, gtol=1e-12):
    """fun(H) -> (value, d value / d vech(chol H)); minimised over vech(L) from
    v0.  The gradient is taken at L itself (the oracle's chain rule gives it
    for the Cholesky factor, which L stays while its diagonal is positive)."""
    def f(v):
        L = unvech(v, d)
        if np.any(np.diag(L) <= 0):
            return np.inf, np.zeros_like(v)
        o, g = fun(L @ L.T)
        return o, g
    res = optimize.minimize(f, np.asarray(v0, dtype=np.float64), jac=True, method="BFGS",
                            options={"gtol": gtol, "maxiter": 2000})
    return res.x, res.fun


def normal_scale_H(Sigma, n):
    """Minimiser of the normal-kernel AMISE when psi_4 is that of N(0, Sigma):
    (4 / (d + 2))^{2 / (d + 4)} n^{-2 / (d + 4)} Sigma."""
    d = Sigma.shape[0]
    return (4.0 / (d + 2)) ** (2.0 / (d + 4)) * n ** (-2.0 / (d + 4)) * Sigma
