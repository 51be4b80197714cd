"""The polynomial starts of the mixed path's iterations, checked against the
mathematics they are built on (no GPU; the constants are read from the
kernel source, so a change there is checked here).

* Expansion start, degree 7: with K = b (h - mu), X0 = 1/2 - K/4 + a3 K^3 +
  a5 K^5 + a7 K^7 stays in (0, 1/2) for K in (0, 8] (odd about 1/2), and
  after n doublings (each mapping f(u) to f(2u), f the Fermi function) the
  occupation f(2^n u0(K)), u0 = log((1 - X0) / X0), is within 6.1e-8 of
  f(2^n K) for every K in (0, 8] and n = 5..9.
* Expansion start, cubic: X0 = 1/2 - K/4 + K^3/108 stays in [0, 1] for
  |K| <= 4 with its minimum 0 at K = 3, and its occupation error after n
  doublings is at most 1.4e-5 (n = 6).
* Inverse start in each doubling: y0(a) = (420 - 576 a + 256 a^2) / 99 has
  |1 - a y0(a)| <= 1/99 on [1/2, 1] (a Chebyshev T3 residual), attained
  with alternating signs at four points; the quartic y4 has the scaled T5 as
  its residual, |1 - a y4(a)| <= 1/3363, also with its FP32 coefficients and
  evaluated the way the kernel does (Q = c4 a^2 + c3 a + c2, y = Q a^2 +
  c1 a + c0).
* Inverse square root start: z0(x) = c0 + c1 x has |1 - x z0(x)^2| <= 0.417
  on [0.1, 1], the range of s / c.
* Last doubling's inverse: the same split start and steps, then FP64
  Newton-Schulz steps, each squaring the residual I - A Y exactly for any Y.
* The FP64 steps taken as corrections: X^2 A^-1 = I/2 + (X - I/2) A^-1,
  Y (2I - A Y) = Y + Y (I - A Y), and the refinement of Z leaving an O(E^3)
  residual (exact rational arithmetic).
"""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "paper_2606_03140_amd", "csrc", "mixed.hip")).read()


def fermi(u):
    return 0.5 * (1.0 - np.tanh(0.5 * u))


def logit(x):
    return np.log((1.0 - x) / x)


def start7():
    m = re.search(r"kStart7\[3\]\s*=\s*\{([^}]*)\}", SRC)
    return np.array([float(v.strip().rstrip("f")) for v in m.group(1).split(",")], dtype=np.float32).astype(np.float64)


def test_degree7_start_error_after_doublings():
    a3, a5, a7 = start7()
    K = np.linspace(1e-6, 8.0, 400001)
    X0 = 0.5 - K / 4 + a3 * K**3 + a5 * K**5 + a7 * K**7
    assert X0.min() > 0.0 and X0.max() < 0.5
    u0 = logit(X0)
    for n in range(5, 10):
        err = np.abs(fermi(2.0**n * u0) - fermi(2.0**n * K)).max()
        assert err < 6.2e-8, (n, err)
    # fewer doublings do not settle the states near |K| = 8: the reason the
    # library falls back to the cubic start below 5
    assert np.abs(fermi(16.0 * u0) - fermi(16.0 * K)).max() > 1e-5


def test_cubic_start_range_and_error():
    assert "1.0f / 108.0f" in SRC
    K = np.linspace(-4.0, 4.0, 400001)
    X0 = 0.5 - K / 4 + K**3 / 108
    assert X0.min() >= -1e-15 and X0.max() <= 1.0 + 1e-15
    assert abs(K[np.argmin(X0)] - 3.0) < 1e-4
    Kp = K[K > 1e-6]
    u0 = logit(np.clip(0.5 - Kp / 4 + Kp**3 / 108, 1e-300, 0.5))
    err = np.abs(fermi(64.0 * u0) - fermi(64.0 * Kp)).max()
    assert err < 1.45e-5


def test_quadratic_inverse_start_is_minimax():
    assert "256.0f / 99.0f, -576.0f / 99.0f, 420.0f / 99.0f" in SRC
    a = np.linspace(0.5, 1.0, 200001)
    r = 1.0 - a * (420.0 - 576.0 * a + 256.0 * a * a) / 99.0
    assert np.abs(r).max() <= 1.0 / 99.0 + 1e-15
    # equioscillation: the residual is the scaled Chebyshev T3 of 4a - 3
    x = 4.0 * a - 3.0
    assert np.allclose(r, (4 * x**3 - 3 * x) / -99.0, atol=1e-15)


def inv_start4():
    m = re.search(r"kInvStart4\[5\]\s*=\s*\{([^}]*)\}", SRC)
    out = []
    for v in m.group(1).split(","):
        num, den = v.strip().split("/")
        out.append(float(np.float32(float(num.strip().rstrip("f")) / float(den.strip().rstrip("f")))))
    return out


def chebyshev_t(n, x):
    return np.cos(n * np.arccos(np.clip(x, -1.0, 1.0)))


def test_quartic_inverse_start_is_minimax():
    c0, c1, c2, c3, c4 = inv_start4()
    # exact rational coefficients: a y4(a) = 1 + T5(4a - 3) / 3363, T5(-3) = -3363
    from fractions import Fraction as Fr
    num = [23780, -66240, 90880, -61440, 16384]
    a_r = [Fr(1, 2) + Fr(k, 16) for k in range(9)]
    for a in a_r:
        x = 4 * a - 3
        t5 = 16 * x**5 - 20 * x**3 + 5 * x
        assert a * sum(Fr(c, 3363) * a**i for i, c in enumerate(num)) == 1 + t5 / 3363
    a = np.linspace(0.5, 1.0, 200001)
    y = (c4 * a * a + c3 * a + c2) * a * a + c1 * a + c0       # the kernel's two products
    r = 1.0 - a * y
    # FP32 coefficients (|c| up to 27) move the residual by at most ~5e-6
    assert np.abs(r).max() <= 1.0 / 3363.0 + 5e-6
    assert np.allclose(r, chebyshev_t(5, 4.0 * a - 3.0) / -3363.0, atol=5e-6)
    # six alternating extrema of size 1/3363 at the Chebyshev points
    # (equioscillation of the minimax residual)
    a_ext = 0.5 + 0.25 * (1.0 + np.cos(np.pi * np.arange(6) / 5))
    r_ext = 1.0 - a_ext * np.polyval([c4, c3, c2, c1, c0], a_ext)
    assert np.all(np.abs(np.abs(r_ext) - 1.0 / 3363.0) < 5e-6)
    assert np.all(np.sign(r_ext[:-1]) != np.sign(r_ext[1:]))
    # one Newton-Schulz step squares it below the split products' rounding
    assert (np.abs(r).max()) ** 2 < 9.3e-8
    # plausible mistakes fail: a sign slip in c3, or the quadratic's scale
    y_bad = (c4 * a * a - c3 * a + c2) * a * a + c1 * a + c0
    assert np.abs(1.0 - a * y_bad).max() > 1e-2
    y_bad = (c4 * a * a + c3 * a + c2) * a * a + c1 * a + c0 * 99.0 / 3363.0
    assert np.abs(1.0 - a * y_bad).max() > 1e-2
    # the library's default: the quartic with one step
    assert "int mixed_inv_deg = 4;" in open(os.path.join(ROOT, "paper_2606_03140_amd", "csrc",
                                                        "gdm_internal.h")).read()


def test_inverse_sqrt_start_bound():
    m = re.search(r"kZ0a\s*=\s*([-0-9.e]+)f,\s*kZ0b\s*=\s*([-0-9.e]+)f", SRC)
    c0, c1 = float(np.float32(m.group(1))), float(np.float32(m.group(2)))
    x = np.linspace(0.1, 1.0, 200001)
    e = np.abs(1.0 - x * (c0 + c1 * x) ** 2)
    assert e.max() <= 0.417


def test_final_doubling_inverse_start():
    # the last doubling's inverse starts on the split products like the others
    # (the quadratic start y0 = (420 - 576 a + 256 a^2) / 99 and the split
    # Newton-Schulz steps), then FP64 steps: one for FP16 pairs, two for BF16
    body = SRC[SRC.index("static int last_doubling_f64"):SRC.index("// FP64 core traces of the last pass")]
    start = SRC[SRC.index("static int inv_start"):SRC.index("// Doubling history for the charge response")]
    assert "inv_start(ctx, As, Ys, Rs, Ysb, 0, skip)" in body
    assert "256.0f / 99.0f, -576.0f / 99.0f, 420.0f / 99.0f" in start and "kInvStart4" in start
    assert "final_ns = P.precision == GDM_MIXED_BF16 ? 2 : 1" in body
    assert "ctx->mixed_ns_inv" in body
    # a Newton-Schulz step Y' = Y (2I - A Y) maps the residual I - A Y to its
    # square exactly for any Y (no commutation assumed): check it on random
    # non-symmetric matrices in exact rational arithmetic
    from fractions import Fraction
    rng = np.random.default_rng(3)
    n = 4
    A = [[Fraction(int(x), 7) for x in row] for row in rng.integers(-9, 10, (n, n))]
    Y = [[Fraction(int(x), 5) for x in row] for row in rng.integers(-9, 10, (n, n))]

    def mul(X, Z):
        return [[sum(X[i][k] * Z[k][j] for k in range(n)) for j in range(n)] for i in range(n)]

    def sub(X, Z):
        return [[X[i][j] - Z[i][j] for j in range(n)] for i in range(n)]

    I2 = [[Fraction(2 if i == j else 0) for j in range(n)] for i in range(n)]
    I1 = [[Fraction(1 if i == j else 0) for j in range(n)] for i in range(n)]
    R = sub(I1, mul(A, Y))
    Yn = mul(Y, sub(I2, mul(A, Y)))
    assert sub(I1, mul(A, Yn)) == mul(R, R)
    # the split start and two split steps leave |1 - a y| <= 99^-4 in exact
    # arithmetic, below the split products' rounding (FP16 pairs ~1e-7 relative,
    # BF16 pairs ~1e-5); one FP64 step squares 2e-7 to 4e-14, two square 2e-5
    # to 1.6e-19: both below the 3.6e-12 of three FP64 steps from 4 - 5a + 2a^2
    a = np.linspace(0.5, 1.0, 200001)
    r = 1.0 - a * (420.0 - 576.0 * a + 256.0 * a * a) / 99.0
    assert np.abs(r).max() <= 1.0 / 99.0 + 1e-15
    assert (np.abs(r) ** 4).max() <= 99.0 ** -4 + 1e-20 and 99.0 ** -4 < 1.1e-8
    assert (2e-7) ** 2 < 3.6e-12 and ((2e-5) ** 2) ** 2 < 3.6e-12
    r_old = 1.0 - a * (4.0 - 5.0 * a + 2.0 * a * a)
    assert abs((np.abs(r_old) ** 8).max() - 27.0 ** -8) < 1e-20 and 27.0 ** -8 > 3.5e-12


def test_fp64_steps_taken_as_corrections():
    # The last doubling forms X^2 A^-1 as I/2 + (X - I/2) A^-1 with
    # A = 2 X^2 - 2 X + I, and takes its last Newton-Schulz step as
    # Y + Y (I - A Y); the refinement of Z uses T = 3/8 E^2 - E/2 so that
    # (I + T)(I + E)(I + T) = I + O(E^3).  Checked in exact rational
    # arithmetic on a symmetric X (A then commutes with X) and a symmetric E.
    from fractions import Fraction
    rng = np.random.default_rng(5)
    n = 3

    def mat(m):
        return [[Fraction(int(v), 11) for v in row] for row in m]

    def mul(X, Z):
        return [[sum(X[i][k] * Z[k][j] for k in range(n)) for j in range(n)] for i in range(n)]

    def add(X, Z, a=1, b=1):
        return [[a * X[i][j] + b * Z[i][j] for j in range(n)] for i in range(n)]

    I = [[Fraction(1 if i == j else 0) for j in range(n)] for i in range(n)]
    M = rng.integers(-5, 6, (n, n))
    X = mat(M + M.T)
    A = add(add(mul(X, X), X, 2, -2), I)
    # A^-1 by Gauss-Jordan in rationals
    aug = [row[:] + I[i][:] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[p] = aug[p], aug[c]
        piv = aug[c][c]
        aug[c] = [v / piv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    Ainv = [row[n:] for row in aug]
    half = [[Fraction(1, 2) if i == j else Fraction(0) for j in range(n)] for i in range(n)]
    assert mul(mul(X, X), Ainv) == add(half, mul(add(X, half, 1, -1), Ainv))
    # a plausible slip (I instead of I/2 in the shift) fails
    assert mul(mul(X, X), Ainv) != add(half, mul(add(X, I, 1, -1), Ainv))
    Y = mat(rng.integers(-5, 6, (n, n)))
    rho = add(I, mul(A, Y), 1, -1)
    assert add(Y, mul(Y, rho)) == mul(Y, add(add(I, I), mul(A, Y), 1, -1))
    # refinement: with E = t E0 the residual (I + T)(I + E)(I + T) - I has no
    # t and t^2 terms for T = 3/8 E^2 - E/2, so R(t) / t^2 -> 0
    M = rng.integers(-5, 6, (n, n))
    E0 = mat(M + M.T)

    def resid(t):
        E = [[t * v for v in row] for row in E0]
        T = add(mul(E, E), E, Fraction(3, 8), Fraction(-1, 2))
        return add(mul(mul(add(I, T), add(I, E)), add(I, T)), I, 1, -1)
    for i in range(n):
        for j in range(n):
            r1, r2 = resid(Fraction(1, 1000))[i][j], resid(Fraction(1, 2000))[i][j]
            assert abs(r1) * 1000**2 < Fraction(1, 10) and abs(r2) * 2000**2 < Fraction(1, 20)
    # T = -E/2 alone (second order) leaves a t^2 term
    E = [[Fraction(1, 1000) * v for v in row] for row in E0]
    T2 = [[-v / 2 for v in row] for row in E]
    R2 = add(mul(mul(add(I, T2), add(I, E)), add(I, T2)), I, 1, -1)
    assert max(abs(R2[i][j]) for i in range(n) for j in range(n)) * 1000**2 > Fraction(1, 10)
