"""Pins of the Chebyshev smoothers and the smoother-quality analysis.

The smoothers (Alg. 1, Alg. 2) are run on the isotropic 2D finite-difference
Laplacian, whose Jacobi-scaled eigenvectors are sin(i pi x) sin(j pi y). With
b = 0 and x0 = v_ij one smoother application must return p_k(lambda_ij) v_ij,
with p_k the closed forms of the paper's Sec. 2:
  1st kind:  T_k((theta - lambda)/delta) / T_k(theta/delta)   (eq. 1st-kind-cheby-polynomials)
  4th kind:  W_k(1 - 2 lambda/lambda_max) / (2k + 1)            (eq. fourth-kind-polynomial-iterate)
  opt. 4th:  1 + sum_i beta_i (p_i - p_{i-1})
Chebyshev polynomials here come from their trigonometric definitions
(T_k(cos t) = cos(k t), W_k(cos t) = sin((k + 1/2) t) / sin(t/2)), not from the
recurrences the algorithms use.
"""
import numpy as np
import pytest

from oracle import chebyshev as cheb
from oracle import analysis as an
from oracle.fd2d import laplacian_5pt

GOLDEN = __file__.replace("test_oracle_chebyshev.py", "golden/beta_coef.txt")


def T(k, x):
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    a = np.abs(x) <= 1
    out[a] = np.cos(k * np.arccos(x[a]))
    b = ~a
    out[b] = np.sign(x[b]) ** k * np.cosh(k * np.arccosh(np.abs(x[b])))
    return out


def U(k, x):
    """Chebyshev polynomial of the 2nd kind for |x| > 1 via its closed form."""
    x = np.asarray(x, dtype=float)
    t = np.arccosh(np.abs(x))
    return np.sign(x) ** k * np.sinh((k + 1) * t) / np.sinh(t)


def W(k, x):
    t = np.arccos(np.clip(x, -1, 1))
    return np.sin((k + 0.5) * t) / np.sin(t / 2)


def p4(k, lam):
    return W(k, 1 - 2 * lam) / (2 * k + 1)


def p1(k, lam, lmin):
    theta, delta = (1 + lmin) / 2, (1 - lmin) / 2
    return T(k, (theta - lam) / delta) / T(k, np.array([theta / delta]))[0]


def p4opt(k, lam, beta=None):
    beta = cheb.betas(cheb.CHEB4_OPT, k) if beta is None else beta
    out = np.ones_like(lam)
    prev = np.ones_like(lam)
    for i in range(1, k + 1):
        cur = p4(i, lam)
        out = out + beta[i - 1] * (cur - prev)
        prev = cur
    return out


def test_beta_table_matches_golden():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, i, v = line.split()
        rows.setdefault(int(k), []).append(float(v))
    assert sorted(rows) == list(range(1, 17))
    for k, vals in rows.items():
        assert vals == cheb.BETA[k], k


@pytest.fixture(scope="module")
def fd_eig():
    n = 16
    A = laplacian_5pt(n)
    Sinv = 1.0 / A.diagonal()
    h = 1.0 / n
    xs = np.arange(1, n) * h
    modes = []
    for (i, j) in [(1, 1), (2, 5), (7, 3), (15, 15), (8, 9), (12, 1)]:
        v = np.outer(np.sin(j * np.pi * xs), np.sin(i * np.pi * xs)).ravel()
        lam = 1 - (np.cos(i * np.pi * h) + np.cos(j * np.pi * h)) / 2
        modes.append((v, lam))
    lmax = 1 + np.cos(np.pi * h)
    return A, Sinv, lmax, modes


@pytest.mark.parametrize("kind", cheb.KINDS)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 20])
def test_smoother_closed_form_on_eigenvectors(fd_eig, kind, k):
    A, Sinv, lmax, modes = fd_eig
    for v, lam in modes:
        x = cheb.smooth(kind, k, lambda y: A @ y, Sinv, lmax, np.zeros_like(v), v)
        t = lam / lmax
        if kind in (cheb.CHEB1, cheb.CHEB1_OPT):
            expect = p1(k, np.array([t]), cheb.lambda_min_fraction(kind, k))[0]
        elif kind == cheb.CHEB4:
            expect = p4(k, np.array([t]))[0]
        else:
            expect = p4opt(k, np.array([t]))[0]
        assert np.max(np.abs(x - expect * v)) < 1e-13 * np.max(np.abs(v))


def test_opt4_order1_is_weighted_jacobi():
    lam = np.linspace(0, 1, 101)
    assert np.max(np.abs(an.smoother_polynomial(cheb.CHEB4_OPT, 1, lam) - (1 - 1.5 * lam))) < 1e-15


@pytest.mark.parametrize("kind", cheb.KINDS)
def test_apply_counts(kind):
    A = laplacian_5pt(8)
    calls = cheb.ApplyCounter(lambda y: A @ y)
    b = np.ones(A.shape[0])
    cheb.smooth(kind, 5, calls, 1 / A.diagonal(), 2.0, b, None)
    assert calls.count == 4          # zero guess: k - 1 applies
    calls.count = 0
    cheb.smooth(kind, 5, calls, 1 / A.diagonal(), 2.0, b, b.copy())
    assert calls.count == 5          # nonzero guess: k applies


@pytest.mark.parametrize("k", range(1, 7))
def test_gamma_inv_fourth_kind(k):
    # eq. gamma-4th-kind: (4/3) k (k+1), exact
    g = an.gamma_inv(cheb.CHEB4, k)
    assert abs(g - 4 / 3 * k * (k + 1)) < 1e-5 * g


@pytest.mark.parametrize("k,exact", [(1, 3.000), (2, 9.472), (3, 19.196), (4, 32.163), (8, 116.461), (16, 440.689)])
def test_gamma_inv_opt_fourth_kind(k, exact):
    # the table's betas give gamma^{-1} close to eq. gamma-opt-4th-kind (approximate form)
    g = an.gamma_inv(cheb.CHEB4_OPT, k)
    assert abs(g - exact) < 1e-3
    approx = 4 / np.pi ** 2 * (2 * k + 1) ** 2 - 2 / 3
    assert abs(g - approx) < 0.01 * g


@pytest.mark.parametrize("k", [2, 3])
def test_beta_table_is_locally_optimal(k):
    base = an.gamma_inv(cheb.CHEB4_OPT, k)
    saved = list(cheb.BETA[k])
    try:
        for i in range(k):
            for eps in (2e-3, -2e-3):
                cheb.BETA[k] = list(saved)
                cheb.BETA[k][i] += eps
                assert an.gamma_inv(cheb.CHEB4_OPT, k) <= base + 1e-7
    finally:
        cheb.BETA[k] = saved


@pytest.mark.parametrize("omega", [0.5, 1.0, 1.5])
def test_gamma_inv_simple(omega):
    # eq. simple-smoother-iter-gamma: 2 omega k
    for k in (1, 2, 3):
        g = an.gamma_inv_of(lambda l: an.simple_polynomial(omega, k, l))
        assert abs(g - 2 * omega * k) < 1e-4 * g


@pytest.mark.parametrize("k", range(1, 7))
def test_gamma_inv_first_kind_branches(k):
    # eq. gamma-1st-kind with lambda_min = 0.1 and k* = 3
    lmin = 0.1
    x = np.array([(lmin + 1) / (lmin - 1)])
    if k <= 3:
        formula = T(k, x)[0] ** 2 - 1
    else:
        formula = 4 * k * U(k - 1, x)[0] / ((lmin - 1) * T(k, x)[0])
    g = an.gamma_inv(cheb.CHEB1, k)
    assert abs(g - formula) < 1e-4 * g


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12])
def test_lambda_min_correlation(k):
    # eq. opt-lambda-min: within 1% of the lambda_min that maximises gamma^{-1}
    import scipy.optimize as so

    def neg(lm):
        return -an.gamma_inv_of(lambda l: p1(k, l, lm))
    res = so.minimize_scalar(neg, bounds=(1e-4, 0.9), method="bounded", options={"xatol": 1e-7})
    corr = cheb.lambda_min_fraction(cheb.CHEB1_OPT, k)
    assert abs(corr - res.x) <= 0.01 * res.x + 1e-3


@pytest.mark.parametrize("k", range(1, 6))
def test_critical_C_closed_forms(k):
    # eq. 4th-kind-condition-C from the numerically computed gamma^{-1}
    c = an.critical_C(an.gamma_inv(cheb.CHEB4, k), an.gamma_inv(cheb.CHEB4, 2 * k))
    assert abs(c - 2 * (k + 1) ** 2 / 3) < 1e-4 * c
    # eq. opt-4th-kind-condition-C is the same construction with eq. gamma-opt-4th-kind
    g = lambda q: 4 / np.pi ** 2 * (2 * q + 1) ** 2 - 2 / 3
    printed = (2 * (6 * (2 * k + 1) ** 2 - np.pi ** 2) ** 2
               / (3 * np.pi ** 2 * (-12 * (2 * k + 1) ** 2 + 6 * (4 * k + 1) ** 2 + np.pi ** 2)))
    assert abs(an.critical_C(g(k), g(2 * k)) - printed) < 1e-12 * printed


# ---- optimised 4th kind beyond the printed table: beta minimising eq. gamma-defn
@pytest.fixture(scope="module")
def computed_betas():
    return cheb.minimax_betas(cheb.MAX_OPT_ORDER)


def test_minimax_betas_reproduce_the_printed_table(computed_betas):
    """The optimisation, run from beta^{(1)} by continuation and knowing nothing of the
    table, lands on every printed coefficient of Table beta_coef (k = 1..16, 15 digits)."""
    rows = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, i, v = line.split()
            rows.setdefault(int(k), []).append(float(v))
    for k, vals in rows.items():
        assert np.max(np.abs(np.array(computed_betas[k]) - np.array(vals))) < 1e-12, k


@pytest.mark.parametrize("k", [17, 18, 20, 24, 32])
def test_computed_betas_equioscillate(computed_betas, k):
    """For k > 16: lam p^2 / (1 - p^2), p evaluated with the trigonometric closed form of
    W_k, reaches the same maximum at lam -> 0, at k-1 interior points and at lam = 1 (the
    minimax characterisation), and that gamma^{-1} lies above the plain 4th kind's
    (4/3) k (k+1) and within 0.1 % of the approximation eq. gamma-opt-4th-kind."""
    beta = computed_betas[k]
    lam = np.linspace(1e-8, 1.0, 200001)
    p = p4opt(k, lam, beta)
    f = lam * p ** 2 / (1 - p ** 2)
    inner = np.nonzero((f[1:-1] >= f[:-2]) & (f[1:-1] >= f[2:]))[0] + 1
    assert len(inner) == k - 1
    gam = f[-1]
    # refine each interior maximum on a local grid; the grid maximum sits below the true one
    for i in inner:
        loc = np.linspace(lam[i - 1], lam[i + 1], 2001)
        pl = p4opt(k, loc, beta)
        fl = np.max(loc * pl ** 2 / (1 - pl ** 2))
        assert abs(fl - gam) <= 1e-9 * gam
    f0 = 3.0 / (8.0 * sum(i * b for i, b in enumerate(beta, start=1)))
    assert abs(f0 - gam) <= 1e-12 * gam       # f -> 3 / (8 sum_i i beta_i) as lam -> 0
    ginv = 1.0 / gam
    assert ginv > 4.0 / 3.0 * k * (k + 1)
    approx = 4.0 / np.pi ** 2 * (2 * k + 1) ** 2 - 2.0 / 3.0
    assert abs(ginv - approx) <= 1e-3 * ginv
    assert cheb.betas(cheb.CHEB4_OPT, k) == beta
