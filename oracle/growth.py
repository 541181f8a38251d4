"""Linear and approximate second-order growth factors D1(k,a), D2(k,a) (Secs. 3-4, App. B).

Per Fourier mode k (primes are d/dtau, kappa = 1.5 Omega_m a):

  D1'' = kappa mu(k,a) D1                                                (Sec. 4.1)
  D2'' = kappa mu D2 - kappa mu D1^2 [1 + 2 a^4 H^2 gamma_2(k, k/sqrt2, k/sqrt2, a)
                                          / (kappa mu)]                  (Sec. 4.2, eq. fofrapprox)

with the Einstein-de Sitter growing-mode initial conditions at a_ini (Secs. 3.1-3.2):
D1 = 1, D1' = (a^-1 da/dtau)_ini, D2 = -3/7, D2' = -(6/7)(a^-1 da/dtau)_ini.
The system is integrated in a, with d/da = (a^3 E)^-1 d/dtau, by scipy's DOP853.
"""

import numpy as np
from scipy import integrate

from .background import E, kappa, dlna_dtau
from .params import MODEL_SYMMETRON, READ_D2_HALF_K


def solve_growth(k, a_out, om, mu_fn, g2_fn, a_ini, rtol=1e-12, atol=1e-14, breaks=(),
                 half_k=False):
    """Return an array G[len(a_out), len(k), 6] of (D1, D1', D1'', D2, D2', D2'')
    at the requested scale factors (a_out sorted ascending, a_out[0] >= a_ini).

    mu_fn(k, a) and g2_fn(k, a) give mu and gamma_2 at the orthogonal triangle.
    D'' is taken from the right-hand side of the ODE at each output time.
    breaks: scale factors where the right-hand side is not smooth (the symmetron's
    switch-on at a_*, App. C); the integration restarts there with a tiny first step, so
    that the narrow feature that follows is resolved rather than stepped over.
    half_k: the alternative reading of the D2 source, D1(k/sqrt2, a)^2 in place of the
    printed D1(k, a)^2 (k1 = k2 = k/sqrt2 is the triangle gamma_2 is taken at); D1 at
    k/sqrt2 is then integrated alongside.
    """
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    a_out = np.asarray(a_out, dtype=np.float64)
    K = k.size
    kh = k / np.sqrt(2.0)

    def rhs_tau(a, y):
        D1, dD1, D2, dD2 = y[:K], y[K:2 * K], y[2 * K:3 * K], y[3 * K:4 * K]
        kap = kappa(a, om)
        mu = mu_fn(k, a)
        g2 = g2_fn(k, a)
        Ea = E(a, om)
        dd1 = kap * mu * D1
        Ds = y[4 * K:5 * K] if half_k else D1   # the growth factor squared in the D2 source
        dd2 = kap * mu * D2 - kap * mu * Ds * Ds - 2.0 * a ** 4 * Ea * Ea * g2 * Ds * Ds
        if not half_k:
            return dD1, dd1, dD2, dd2
        return dD1, dd1, dD2, dd2, y[5 * K:], kap * mu_fn(kh, a) * y[4 * K:5 * K]

    def rhs(a, y):
        f = 1.0 / (a ** 3 * E(a, om))
        return np.concatenate([d * f for d in rhs_tau(a, y)])

    g0 = dlna_dtau(a_ini, om)
    y0 = np.concatenate([np.ones(K), np.full(K, g0), np.full(K, -3.0 / 7.0),
                         np.full(K, -6.0 / 7.0 * g0)]
                        + ([np.ones(K), np.full(K, g0)] if half_k else []))
    out = np.empty((a_out.size, K, 6))
    need = a_out > a_ini
    if np.any(need):
        Ys = iter(_integrate_pieces(rhs, y0, a_ini, a_out[need], breaks, rtol, atol))
    for i, a in enumerate(a_out):
        y = next(Ys) if need[i] else y0
        dD1, dd1, dD2, dd2 = rhs_tau(a, y)[:4]
        out[i, :, 0] = y[:K]
        out[i, :, 1] = dD1
        out[i, :, 2] = dd1
        out[i, :, 3] = y[2 * K:3 * K]
        out[i, :, 4] = dD2
        out[i, :, 5] = dd2
    return out


def _integrate_pieces(rhs, y0, a0, a_eval, breaks, rtol, atol):
    """DOP853 from a0 through the sorted a_eval, restarted at every break point inside;
    returns the states at a_eval."""
    a_end = float(a_eval[-1])
    cuts = [a0] + sorted(b for b in breaks if a0 < b < a_end) + [a_end]
    ys, y = [], y0
    for j in range(len(cuts) - 1):
        lo, hi = cuts[j], cuts[j + 1]
        sel = a_eval[(a_eval > lo) & (a_eval <= hi)]
        t_eval = np.unique(np.concatenate([sel, [hi]]))
        kw = dict(first_step=1e-12 * hi) if j > 0 else {}
        sol = integrate.solve_ivp(rhs, (lo, hi), y, method="DOP853", t_eval=t_eval, rtol=rtol,
                                  atol=atol, **kw)
        if not sol.success:
            raise RuntimeError(sol.message)
        for t, col in zip(sol.t, sol.y.T):
            if np.any(sel == t):
                ys.append(col)
        y = sol.y[:, -1]
    return ys


def distinct_n2(n):
    """Distinct integer |nu|^2 = nx^2 + ny^2 + nz^2 on an n^3 FFT grid with
    nu_i in [-n/2, n/2 - 1] (n even): the values 0 .. 3 (n/2)^2."""
    return np.arange(3 * (n // 2) ** 2 + 1, dtype=np.int64)


def growth_table(p, model, a_out):
    """Growth factors for a run on the particle grid, indexed by integer |nu|^2.

    Scale-independent runs (LCDM, nDGP, or growth_mode 1) solve one ODE and
    broadcast it; scale-dependent runs (f(R)) solve one ODE per integer |nu|^2 with
    k = 2 pi sqrt(|nu|^2) / L, so no interpolation in k is ever needed.
    Returns G[len(a_out), n_k, 6] and a flag saying whether it is k-dependent.
    """
    breaks = growth_breaks(p, model)
    half = bool(p.readings & READ_D2_HALF_K)
    if not p.scale_dependent:
        G = solve_growth(np.array([0.0]), a_out, p.omega_m, model.mu, model.gamma2_orth,
                         p.a_ini, breaks=breaks, half_k=half)
        return G, False
    n2 = distinct_n2(p.np1d)
    k = 2.0 * np.pi * np.sqrt(n2.astype(np.float64)) / p.box
    G = solve_growth(k, a_out, p.omega_m, model.mu, model.gamma2_orth, p.a_ini, breaks=breaks,
                     half_k=half)
    return G, True


def growth_breaks(p, model):
    """Scale factors where the growth equations' right-hand side is not smooth: a_* of the
    symmetron run with its own growth factors (App. C)."""
    return (p.sym_astar,) if (model.kind == MODEL_SYMMETRON and not model.lcdm_growth) else ()
