"""Chebyshev smoothers (paper, Sec. 2).

* 1st kind, Algorithm 1 ("Chebyshev smoother, 1st-kind"): three-term recurrence
  on the interval [lambda_min, lambda_max] with S applied to the residual.
  lambda_min = 0.1 lambda_max ("1st-Cheb"), or the correlation of eq.
  opt-lambda-min, lambda_min* = 1.69 / (k^1.68 + 2.11 k + 1.98) (as a fraction of
  lambda_max), for "1st-Cheb, lambda_min^opt".
* 4th kind and optimised 4th kind, Algorithm 2 ("Chebyshev smoother, (Opt.)
  4th-kind"); beta_i = 1 for the plain 4th kind, the supplementary Table
  beta_coef for the optimised one (k <= 16).

S is a diagonal (Jacobi) smoother given as a vector of diag(A)^{-1}.
"""
from __future__ import annotations

import numpy as np

CHEB1 = "cheb1"          # 1st kind, lambda_min = 0.1 lambda_max
CHEB1_OPT = "cheb1opt"   # 1st kind, lambda_min from eq. opt-lambda-min
CHEB4 = "cheb4"          # 4th kind, beta = 1
CHEB4_OPT = "cheb4opt"   # optimised 4th kind, beta from Table beta_coef
KINDS = (CHEB1, CHEB1_OPT, CHEB4, CHEB4_OPT)

# Supplementary material, Table beta_coef: beta_i^{(k)} for k = 1..16.
BETA = {
    1: [1.12500000000000],
    2: [1.02387287570313, 1.26408905371085],
    3: [1.00842544782028, 1.08867839208730, 1.33753125909618],
    4: [1.00391310427285, 1.04035811188593, 1.14863498546254, 1.38268869241000],
    5: [1.00212930146164, 1.02173711549260, 1.07872433192603, 1.19810065292663,
        1.41322542791682],
    6: [1.00128517255940, 1.01304293035233, 1.04678215124113, 1.11616489419675,
        1.23829020218444, 1.43524297106744],
    7: [1.00083464397912, 1.00843949430122, 1.03008707768713, 1.07408384092003,
        1.15036186707366, 1.27116474046139, 1.45186658649364],
    8: [1.00057246631197, 1.00577427662415, 1.02050187922941, 1.05019803444565,
        1.10115572984941, 1.18086042806856, 1.29838585382576, 1.46486073151099],
    9: [1.00040960072832, 1.00412439506106, 1.01460212148266, 1.03561113626671,
        1.07139972529194, 1.12688273710962, 1.20785219140729, 1.32121930716746,
        1.47529642820699],
    10: [1.00030312229652, 1.00304840660796, 1.01077022715387, 1.02619011597640,
         1.05231724933755, 1.09255743207549, 1.15083376663972, 1.23172250870894,
         1.34060802024460, 1.48386124407011],
    11: [1.00023058595209, 1.00231675024028, 1.00817245396304, 1.01982986566342,
         1.03950210235324, 1.06965042700541, 1.11305754295742, 1.17290876275564,
         1.25288300576792, 1.35725579919519, 1.49101672564139],
    12: [1.00017947200828, 1.00180189139619, 1.00634861907307, 1.01537864566306,
         1.03056942830760, 1.05376019693943, 1.08699862592072, 1.13259183097913,
         1.19316273358172, 1.27171293675110, 1.37169337969799, 1.49708418575562],
    13: [1.00014241921559, 1.00142906932629, 1.00503028986298, 1.01216910518495,
         1.02414874342792, 1.04238158880820, 1.06842008128700, 1.10399010936759,
         1.15102748242645, 1.21171811910125, 1.28854264865128, 1.38432619380991,
         1.50229418757368],
    14: [1.00011490538261, 1.00115246376914, 1.00405357333264, 1.00979590573153,
         1.01941300472994, 1.03401425035436, 1.05480599606629, 1.08311420301813,
         1.12040891660892, 1.16833095655446, 1.22872122288238, 1.30365305707817,
         1.39546814053678, 1.50681646209583],
    15: [1.00009404750752, 1.00094291696343, 1.00331449056444, 1.00800294833816,
         1.01584236259140, 1.02772083317705, 1.04459535422831, 1.06750761206125,
         1.09760092545889, 1.13613855366157, 1.18452361426236, 1.24432087304475,
         1.31728069083392, 1.40536543893560, 1.51077872501845],
    16: [1.00007794828179, 1.00078126847253, 1.00274487974401, 1.00662291017015,
         1.01309858836971, 1.02289448329337, 1.03678321409983, 1.05559875719896,
         1.08024848405560, 1.11172607131497, 1.15112543431072, 1.19965584614973,
         1.25865841744946, 1.32962412656664, 1.41421360695576, 1.51427891730346],
}


MAX_OPT_ORDER = 32  # optimised 4th kind: the table up to 16, computed beta up to this order


def fourth_kind_polynomials(k: int, lam: np.ndarray):
    """p_i(lam) = W_i(1 - 2 lam) / (2i + 1), i = 0..k, and their first derivatives
    (eq. fourth-kind-polynomial-iterate with the recurrence of eq. fourth-kind-chebyshev:
    W_0 = 1, W_1 = 2x + 1, W_n = 2x W_{n-1} - W_{n-2})."""
    x = 1.0 - 2.0 * np.asarray(lam, dtype=np.float64)
    W = [np.ones_like(x), 2.0 * x + 1.0]
    dW = [np.zeros_like(x), np.full_like(x, 2.0)]
    for n in range(2, k + 1):
        W.append(2.0 * x * W[n - 1] - W[n - 2])
        dW.append(2.0 * W[n - 1] + 2.0 * x * dW[n - 1] - dW[n - 2])
    p = [W[n] / (2 * n + 1) for n in range(k + 1)]
    dp = [-2.0 * dW[n] / (2 * n + 1) for n in range(k + 1)]   # d/dlam, x = 1 - 2 lam
    return p, dp


def _gamma_terms(beta, lam):
    """f(lam) = lam p^2 / (1 - p^2) of eq. gamma-defn and df/dlam for the optimised
    polynomial p = 1 + sum_i beta_i (p_i - p_{i-1}) (the error polynomial of Algorithm 2:
    its iterate adds beta_i times the plain 4th-kind increments)."""
    k = len(beta)
    P, dP = fourth_kind_polynomials(k, lam)
    p = 1.0 + sum(beta[i - 1] * (P[i] - P[i - 1]) for i in range(1, k + 1))
    dp = sum(beta[i - 1] * (dP[i] - dP[i - 1]) for i in range(1, k + 1))
    g = 1.0 - p * p
    f = lam * p * p / g
    df = (p * p + 2.0 * lam * p * dp) / g + lam * p * p * (2.0 * p * dp) / (g * g)
    return f, df


def minimax_betas(kmax: int) -> dict:
    """beta^{(k)}, k = 1..kmax, minimising gamma (eq. gamma-defn) over the coefficients of
    Algorithm 2 (paper, Sec. 2: the beta_i come from optimising eq. gamma-defn).

    Characterisation used: at the minimum, f(lam) = lam p^2 / (1 - p^2) attains its
    supremum gamma at k+1 points: lam -> 0 (where f tends to 3 / (8 sum_i i beta_i),
    since p'(0) = -(4/3) sum_i i beta_i), k-1 interior maxima (f = gamma, f' = 0) and
    lam = 1. Those 2k equations in (beta, gamma, interior maxima) are solved by Newton's
    method (Jacobian by central differences), continued in k from beta^{(1)}: the start
    for order k spreads beta^{(k-1)} over k indices and takes the maxima of f on a grid."""
    out = {}
    grid = np.linspace(1e-9, 1.0, 100001)

    def residual(z, k):
        beta, gam, lam = z[:k], z[k], z[k + 1:]
        f, df = _gamma_terms(beta, lam)
        f1, _ = _gamma_terms(beta, np.array([1.0]))
        f0 = 3.0 / (8.0 * float(np.dot(np.arange(1, k + 1), beta)))
        return np.concatenate([f - gam, df, [f1[0] - gam, f0 - gam]])

    beta = np.array([1.0])
    for k in range(1, kmax + 1):
        if k > 1:   # spread the previous coefficients over k indices
            t_old = (np.arange(1, k) - 0.5) / (k - 1)
            t_new = (np.arange(1, k + 1) - 0.5) / k
            beta = np.interp(t_new, t_old, beta)
        f, _ = _gamma_terms(beta, grid)
        inner = np.nonzero((f[1:-1] >= f[:-2]) & (f[1:-1] >= f[2:]))[0] + 1
        if len(inner) != k - 1:
            raise RuntimeError(f"order {k}: the start has {len(inner)} interior maxima, not {k - 1}")
        z = np.concatenate([beta, [float(f[-1])], grid[inner]])
        close = False
        for _ in range(40):
            F = residual(z, k)
            J = np.empty((len(F), len(z)))
            for c in range(len(z)):
                h = 1e-7 * max(1.0, abs(z[c]))
                zp, zm = z.copy(), z.copy()
                zp[c] += h
                zm[c] -= h
                J[:, c] = (residual(zp, k) - residual(zm, k)) / (2.0 * h)
            dz = np.linalg.solve(J, -F)
            z = z + dz
            if close:            # one step after the update fell below 1e-12: converged
                break
            close = np.max(np.abs(dz)) < 1e-12
        beta = z[:k]
        out[k] = [float(v) for v in beta]
    return out


_COMPUTED: dict = {}


def lambda_min_fraction(kind: str, k: int) -> float:
    """lambda_min / lambda_max for the 1st-kind smoothers."""
    if kind == CHEB1:
        return 0.1
    if kind == CHEB1_OPT:
        return 1.69 / (k ** 1.68 + 2.11 * k + 1.98)
    raise ValueError(kind)


def betas(kind: str, k: int) -> list:
    if kind == CHEB4:
        return [1.0] * k
    if kind == CHEB4_OPT:
        if k in BETA:                         # the printed Table beta_coef
            return list(BETA[k])
        if not 1 <= k <= MAX_OPT_ORDER:
            raise ValueError(f"optimised 4th-kind coefficients exist for k <= {MAX_OPT_ORDER}")
        if k not in _COMPUTED:                # beyond the table: minimise eq. gamma-defn
            _COMPUTED.update(minimax_betas(k))
        return list(_COMPUTED[k])
    raise ValueError(kind)


class ApplyCounter:
    """Wraps an operator to count its applications."""

    def __init__(self, A):
        self.A = A
        self.count = 0

    def __call__(self, x):
        self.count += 1
        return self.A(x)


def smooth(kind: str, k: int, A, Sinv, lmax: float, b: np.ndarray,
           x0: np.ndarray | None = None) -> np.ndarray:
    """Order-k Chebyshev smoothing of A x = b starting from x0 (None means x0 = 0).

    From a zero initial guess the first residual is b itself, so the smoother
    applies A k-1 times; from a nonzero guess it applies A k times. Sinv is the
    Jacobi diag(A)^{-1} as an array, or any linear smoother S as a callable r -> S r
    (the Schwarz smoothers of Sec. 4.1 enter Algorithms 1 and 2 the same way).
    """
    if k <= 0:
        return np.zeros_like(b) if x0 is None else x0.copy()
    if callable(Sinv):
        S = Sinv
    else:
        S = lambda r: Sinv * r  # noqa: E731
    if kind in (CHEB1, CHEB1_OPT):
        return _cheb1(k, A, S, lmax, lambda_min_fraction(kind, k) * lmax, b, x0)
    return _cheb4(k, A, S, lmax, betas(kind, k), b, x0)


def _cheb1(k, A, S, lmax, lmin, b, x0):
    # Algorithm 1
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(b)
        r = S(b)
    else:
        x = x0.copy()
        r = S(b - A(x))
    d = r / theta
    for _ in range(1, k):
        x = x + d
        r = r - S(A(d))
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x + d


def _cheb4(k, A, S, lmax, beta, b, x0):
    # Algorithm 2
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - A(x)
    d = (4.0 / 3.0) * (1.0 / lmax) * S(r)
    for i in range(1, k):
        x = x + beta[i - 1] * d
        r = r - A(d)
        d = ((2 * i - 1) / (2 * i + 3)) * d + ((8 * i + 4) / (2 * i + 3)) * (1.0 / lmax) * S(r)
    return x + beta[k - 1] * d
