"""Pins for the emulated reduced-precision pass (oracle/mixed.py), CPU only.

The paper analyses every step with one unit roundoff (Section 1, notation);
the split-bfloat16 arithmetic is this library's own reading of "A Z and the
Gram in reduced precision".  Its definition, which these tests hold the
emulation to:

* slices of x: s_0 = bf16(x), s_i = bf16(x - s_0 - ... - s_{i-1}), each a round
  to nearest even to 8 significant bits;
* a k-slice product keeps the slice pairs (i, j) with i + j < k (bf16x2:
  hi*hi + hi*lo + lo*hi; bf16x3: six pairs);
* the kept products of one tile of `kt` consecutive K indices are summed in
  FP32, the tile sums in FP64;
* the shift rule of the Cholesky step: a reduced-precision pass starts at
  s = c 2^-24 max_i G_ii, an FP64 pass starts unshifted and retries at
  c 2^-53 max_i G_ii, each further retry multiplies c by 10.

Nothing here calls the emulation to produce an expected value: references are
exact rational arithmetic (fractions.Fraction) on slices computed by an
independent rounding routine, or constructed inputs whose result is known in
closed form.  Planted mistakes (copies of the routine with one slip) must fail
the same checks.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import mixed

U32 = Fraction(1, 2 ** 24)
U64 = Fraction(1, 2 ** 53)


# ---- an independent exact model -------------------------------------------------------------

def _round_sig(x: Fraction, bits: int) -> Fraction:
    """x rounded to `bits` significant bits, ties to even (exact rational arithmetic)."""
    if x == 0:
        return Fraction(0)
    sgn = -1 if x < 0 else 1
    ax = abs(x)
    e = ax.numerator.bit_length() - ax.denominator.bit_length()
    if ax < Fraction(2) ** e:
        e -= 1                                   # now 2^e <= ax < 2^(e+1)
    scale = Fraction(2) ** (bits - 1 - e)
    y = ax * scale
    f = y.numerator // y.denominator
    rem = y - f
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return sgn * Fraction(f) / scale


def exact_slices(x: float, k: int):
    r = Fraction(float(x))
    out = []
    for _ in range(k):
        h = _round_sig(r, 8)
        out.append(h)
        r -= h
    return out


def kept_pairs(k: int):
    return [(i, j) for i in range(k) for j in range(k) if i + j < k]


def exact_tile_sums(a, b, k, kt):
    """Exact sums of the kept slice products, per output entry and per K tile, with the sum of their
    magnitudes: (S[t][r][c], M[t][r][c], N terms per tile)."""
    rows, K = a.shape
    cols = b.shape[1]
    sa = [[exact_slices(a[r, q], k) for q in range(K)] for r in range(rows)]
    sb = [[exact_slices(b[q, c], k) for c in range(cols)] for q in range(K)]
    pairs = kept_pairs(k)
    tiles = []
    for k0 in range(0, K, kt):
        k1 = min(K, k0 + kt)
        S = [[Fraction(0)] * cols for _ in range(rows)]
        M = [[Fraction(0)] * cols for _ in range(rows)]
        for r in range(rows):
            for c in range(cols):
                s = m = Fraction(0)
                for q in range(k0, k1):
                    for i, j in pairs:
                        p = sa[r][q][i] * sb[q][c][j]
                        s += p
                        m += abs(p)
                S[r][c], M[r][c] = s, m
        tiles.append((S, M, (k1 - k0) * len(pairs)))
    return tiles


def within_fp32_tile_bound(out, a, b, k, kt):
    """True if every entry of `out` lies within the error bound of FP32 summation inside each tile
    (gamma_{N-1} u32 times the sum of magnitudes, any order) plus FP64 summation across tiles."""
    tiles = exact_tile_sums(a, b, k, kt)
    rows, cols = out.shape
    T = len(tiles)
    for r in range(rows):
        for c in range(cols):
            exact = sum(t[0][r][c] for t in tiles)
            bound = Fraction(0)
            mag = Fraction(0)
            for S, M, N in tiles:
                g = (N - 1) * U32 / (1 - (N - 1) * U32)
                bound += g * M[r][c]
                mag += abs(S[r][c]) + g * M[r][c]
            bound += (T + 1) * U64 / (1 - (T + 1) * U64) * mag
            if abs(Fraction(float(out[r, c])) - exact) > bound:
                return False
    return True


# ---- the rounding itself ---------------------------------------------------------------------

def test_exact_slices_reproduce_known_splits():
    assert exact_slices(1 + 2 ** -10, 2) == [1, Fraction(1, 2 ** 10)]
    assert exact_slices(1 + 2 ** -10 + 2 ** -20, 3) == [1, Fraction(1, 2 ** 10), Fraction(1, 2 ** 20)]
    # a tie at the eighth bit rounds to even: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert exact_slices(1 + 2 ** -8, 1) == [1]
    assert exact_slices(1 + 3 * 2 ** -8, 1) == [1 + Fraction(1, 2 ** 6)]


def test_emulated_split_equals_exact_split():
    rng = np.random.default_rng(4242)
    x = rng.standard_normal(200).astype(np.float32).astype(np.float64) * 10.0 ** rng.integers(-5, 5, 200)
    x = x.astype(np.float32).astype(np.float64)           # FP32 inputs: the split is one rounding per slice
    for k in (2, 3):
        sl = mixed.split(x, k)
        for t in range(len(x)):
            assert [Fraction(float(s[t])) for s in sl] == exact_slices(x[t], k)


# ---- products: which slice pairs are kept ----------------------------------------------------

def test_bf16x2_keeps_hi_hi_hi_lo_lo_hi():
    """a = 1 + 2^-10, b = 1 + 2^-11: hi*hi = 1, hi*lo = 2^-11, lo*hi = 2^-10, lo*lo = 2^-21 (dropped).
    The kept sum is exact in FP32."""
    a = np.array([[1 + 2 ** -10]])
    b = np.array([[1 + 2 ** -11]])
    assert mixed.matmul(a, b, "bf16x2")[0, 0] == 1 + 2 ** -10 + 2 ** -11


def test_bf16x3_keeps_the_six_pairs_below_three():
    """Slices a = (1, 2^-10, 2^-20), b = (1, 2^-11, 2^-22); a second K term (-1) x 1 cancels the
    leading product, so that the pairs (1, 2) and (2, 1) (2^-32, 2^-31) would be visible if kept."""
    a = np.array([[1 + 2 ** -10 + 2 ** -20, -1.0]])
    b = np.array([[1 + 2 ** -11 + 2 ** -22], [1.0]])
    want = 2 ** -10 + 2 ** -11 + 2 ** -20 + 2 ** -21 + 2 ** -22
    assert mixed.matmul(a, b, "bf16x3")[0, 0] == want


def test_fp32_scheme_is_one_fp32_product():
    a = np.array([[1 + 2 ** -30]])           # rounds to 1 in FP32
    b = np.array([[3.0]])
    assert mixed.matmul(a, b, "fp32")[0, 0] == 3.0
    assert mixed.matmul(a, b, "fp64")[0, 0] == 3.0 * (1 + 2 ** -30)


# ---- products: FP32 inside a K tile, FP64 across tiles ----------------------------------------

def _tile_probe(kt, gap):
    """Row 0 of A times column 0 of B: a product 2^24 at K index 0 and a product 1 at K index `gap`;
    2^24 + 1 is not an FP32 number (the tie rounds to 2^24)."""
    K = 2 * kt
    a = np.zeros((1, K))
    b = np.zeros((K, 1))
    a[0, 0], b[0, 0] = 2.0 ** 12, 2.0 ** 12
    a[0, gap], b[gap, 0] = 1.0, 1.0
    return a, b


@pytest.mark.parametrize("scheme", ["fp32", "bf16x2", "bf16x3"])
def test_tile_sums_are_fp32_and_cross_tile_sums_fp64(scheme):
    """Default tile of 256 K indices."""
    a, b = _tile_probe(256, 255)             # both products in the first tile: FP32 loses the 1
    assert mixed.matmul(a, b, scheme)[0, 0] == 2.0 ** 24
    a, b = _tile_probe(256, 256)             # the 1 opens the second tile: FP64 keeps it
    assert mixed.matmul(a, b, scheme)[0, 0] == 2.0 ** 24 + 1


@pytest.mark.parametrize("gap,want", [(255, 2.0 ** 24), (256, 2.0 ** 24 + 1)])
def test_dense_gram_uses_the_same_tiles(gap, want):
    """G = Z^T (A Z) with A's row 0 = the probe, Z's column 0 = the probe: G_00 = 2^12 W_00."""
    a, b = _tile_probe(256, gap)
    A = np.zeros((512, 512))
    A[0] = a[0]
    g = mixed.gram(A, b, "bf16x2")
    assert g[0, 0] == 2.0 ** 12 * want


@pytest.mark.parametrize("gap,want", [(255, 2.0 ** 24), (256, 2.0 ** 24 + 1)])
def test_stencil_gram_and_pass_use_the_same_tiles(gap, want):
    """Stencil with centre 1 and no coupling (A = I): G = Z^T Z summed over 256-row tiles.  Through the
    pass, R_00^2 = G_00 + s with s = 2^-24 G_00, so the tile rounding shows in R as well."""
    import workloads as W_
    st = W_.Stencil7(512, 1, 1, 1.0, 0.0)
    z = np.zeros((512, 1))
    z[0, 0], z[gap, 0] = 2.0 ** 12, 1.0
    assert mixed.gram(st, z, "bf16x3")[0, 0] == want
    q, r, info, s = mixed.cholqr_pass(st, z, "bf16x3")
    assert info == 0 and s == want * 2.0 ** -24 and r[0, 0] == np.sqrt(want + s)


@pytest.mark.parametrize("scheme,k", [("bf16x2", 2), ("bf16x3", 3)])
def test_random_product_within_fp32_tile_bound(scheme, k):
    """Signed random inputs (FP32 numbers), three K tiles with a ragged last one, the default tile."""
    rng = np.random.default_rng(77 + k)
    a = rng.standard_normal((2, 600)).astype(np.float32).astype(np.float64)
    b = rng.standard_normal((600, 2)).astype(np.float32).astype(np.float64)
    assert within_fp32_tile_bound(mixed.matmul(a, b, scheme), a, b, k, 256)


# ---- planted mistakes ------------------------------------------------------------------------

def _mutant_matmul(a, b, scheme, kt=256, pairs=None, tile_dtype=np.float32, cross_dtype=np.float64):
    K = a.shape[1]
    k = mixed.NSLICE[scheme]
    a_s, b_s = mixed.split(a, k), mixed.split(b, k)
    pairs = pairs if pairs is not None else kept_pairs(k)
    out = np.zeros((a.shape[0], b.shape[1]), dtype=cross_dtype)
    for k0 in range(0, K, kt):
        k1 = min(K, k0 + kt)
        acc = np.zeros((a.shape[0], b.shape[1]), dtype=tile_dtype)
        for i, j in pairs:
            acc += a_s[i][:, k0:k1].astype(tile_dtype) @ b_s[j][k0:k1].astype(tile_dtype)
        out = (out + acc.astype(cross_dtype)).astype(cross_dtype)
    return out.astype(np.float64)


def _positive_case():
    rng = np.random.default_rng(5)
    a = (1.0 + rng.random((2, 300))).astype(np.float32).astype(np.float64)
    b = (1.0 + rng.random((300, 2))).astype(np.float32).astype(np.float64)
    return a, b


def test_mutant_without_lo_hi_fails():
    a = np.array([[1 + 2 ** -10]])
    b = np.array([[1 + 2 ** -11]])
    m = _mutant_matmul(a, b, "bf16x2", pairs=[(0, 0), (0, 1)])
    assert m[0, 0] != 1 + 2 ** -10 + 2 ** -11
    a, b = _positive_case()
    assert within_fp32_tile_bound(_mutant_matmul(a, b, "bf16x2"), a, b, 2, 256)       # the faithful copy passes
    assert not within_fp32_tile_bound(_mutant_matmul(a, b, "bf16x2", pairs=[(0, 0), (0, 1)]), a, b, 2, 256)


def test_mutant_with_lo_lo_fails():
    a = np.array([[1 + 2 ** -10]])
    b = np.array([[1 + 2 ** -11]])
    m = _mutant_matmul(a, b, "bf16x2", pairs=[(0, 0), (0, 1), (1, 0), (1, 1)])
    assert m[0, 0] != 1 + 2 ** -10 + 2 ** -11


def test_mutant_with_fp64_tile_sums_fails():
    a, b = _tile_probe(256, 255)
    assert _mutant_matmul(a, b, "bf16x2", tile_dtype=np.float64)[0, 0] != 2.0 ** 24


def test_mutant_with_fp32_cross_tile_sums_fails():
    a, b = _tile_probe(256, 256)
    assert _mutant_matmul(a, b, "bf16x2", cross_dtype=np.float32)[0, 0] != 2.0 ** 24 + 1


@pytest.mark.parametrize("kt", [128, 512])
def test_mutant_with_wrong_tile_length_fails(kt):
    ok = True
    for gap, want in ((255, 2.0 ** 24), (256, 2.0 ** 24 + 1)):
        a, b = _tile_probe(256, gap)
        ok &= _mutant_matmul(a, b, "bf16x2", kt=kt)[0, 0] == want
    assert not ok


# ---- Gram products ---------------------------------------------------------------------------

def test_dense_gram_is_fp64_zt_times_split_az():
    """Dense A: W = A Z in the split arithmetic, G = Z^T W in FP64.  Inputs with lo*lo = 9 * 2^-20 in
    every product, so that a Gram that took A Z in FP64 (lo*lo included) lands outside the bound."""
    rng = np.random.default_rng(11)
    m, n = 6, 2
    a = np.full((m, m), 1 + 3 * 2 ** -10)                 # hi = 1, lo = 3 * 2^-10
    a += np.diag(rng.integers(1, 4, m).astype(np.float64))
    a = (a + a.T) / 2
    z = (1 + 3 * 2 ** -10) * np.ones((m, n)) + np.arange(m * n).reshape(m, n) * 2.0 ** -3
    g = mixed.gram(a, z, "bf16x2")
    tiles = exact_tile_sums(a, z, 2, 256)
    W = [[sum(t[0][r][c] for t in tiles) for c in range(n)] for r in range(m)]
    Wb = [[sum((t[2] - 1) * U32 * t[1][r][c] for t in tiles) * (1 + U32) for c in range(n)] for r in range(m)]
    for i in range(n):
        for j in range(n):
            exact = sum(Fraction(float(z[r, i])) * W[r][j] for r in range(m))
            # FP32 tile error of W, then the FP64 sum of m products z_ri * W_rj (W itself within Wb)
            bnd = sum(abs(Fraction(float(z[r, i]))) * Wb[r][j] for r in range(m))
            bnd += (m + 1) * U64 * sum(abs(Fraction(float(z[r, i]))) * (abs(W[r][j]) + Wb[r][j]) for r in range(m))
            assert abs(Fraction(float(g[i, j])) - exact) <= bnd
            full = sum(Fraction(float(z[r, i])) * sum(Fraction(float(a[r, q])) * Fraction(float(z[q, j]))
                                                     for q in range(m)) for r in range(m))
            assert abs(Fraction(float(g[i, j])) - full) > bnd      # the dropped lo*lo products are visible


def test_stencil_gram_is_split_zt_times_fp64_stencil():
    """Stencil A: W = A Z exactly (integer Z, centre 6, off-diagonal -1), G = Z^T W in the split
    arithmetic: within the FP32 tile bound of the exact split product of Z^T and W."""
    import workloads as W_
    st = W_.Stencil7(4, 3, 2, 6.0, -1.0)
    rng = np.random.default_rng(13)
    z = rng.integers(-300, 300, (st.m, 3)).astype(np.float64) + 0.5
    from oracle import stencil
    w = stencil.apply(st, z)
    g = mixed.gram(st, z, "bf16x3")
    assert within_fp32_tile_bound(g, np.ascontiguousarray(z.T), w, 3, 256)


# ---- the symmetric formation (dense A read in its upper block triangle) ---------------------------

def _int_case(m=10, n=3, seed=21):
    """Small integers (bf16-exact, every sum exact in FP32 and FP64): both formations give Z^T A Z."""
    rng = np.random.default_rng(seed)
    b = rng.integers(-4, 5, (m, m)).astype(np.float64)
    a = b + b.T + np.diag(np.full(m, 20.0))
    z = rng.integers(-3, 4, (m, n)).astype(np.float64)
    return a, z


@pytest.mark.parametrize("blocks", [1, 3, 4, 10, 64])
def test_symmetric_formation_is_zt_a_z_on_exact_inputs(blocks):
    """Ragged and single blocks: W_sym = (U + D) Z and W_off^T Z add up to Z^T A Z exactly."""
    a, z = _int_case()
    want = (z.T @ a @ z).astype(np.int64)
    for scheme in ("fp64", "bf16x2", "bf16x3"):
        g = mixed.gram(a, z, scheme, symmetric_blocks=blocks)
        assert np.array_equal(g, want), (scheme, blocks)


def test_symmetric_formation_mutant_without_the_transposed_term_fails():
    a, z = _int_case()
    m = a.shape[0]
    u = np.triu(a, 4)                        # blocks of 4: everything right of the diagonal blocks
    for t0 in range(0, m, 4):
        u[t0:t0 + 4, t0:min(m, t0 + 4)] = 0.0
    d = a - u - u.T
    mutant = z.T @ (u @ z + d @ z)           # W_off^T Z forgotten
    assert not np.array_equal(mutant, z.T @ a @ z)


def test_symmetric_formation_diagonal_blocks_are_fp64():
    """A = x I with x = 1 + 3 2^-10 (hi = 1, lo = 3 2^-10) and Z = x I: one diagonal block, so
    G = x^3 exactly (31 bits); a split product of the diagonal block would drop lo * lo = 9 2^-20."""
    x = 1 + 3 * 2.0 ** -10
    a, z = x * np.eye(4), x * np.eye(4)
    g = mixed.gram(a, z, "bf16x2", symmetric_blocks=4)
    assert np.array_equal(g, x ** 3 * np.eye(4))
    assert not np.array_equal(mixed.gram(a, z, "bf16x2"), x ** 3 * np.eye(4))   # the full split product


def test_symmetric_formation_off_diagonal_blocks_are_split():
    """m = 2, blocks of 1: G_12 = z * split(x * z) with the lo * lo product dropped (bf16x2)."""
    x, zz = 0.5 * (1 + 3 * 2.0 ** -10), 1 + 5 * 2.0 ** -10
    a = np.array([[1.0, x], [x, 1.0]])
    z = zz * np.eye(2)
    g = mixed.gram(a, z, "bf16x2", symmetric_blocks=1)
    sx, sz = exact_slices(x, 2), exact_slices(zz, 2)
    kept = sx[0] * sz[0] + sx[0] * sz[1] + sx[1] * sz[0]
    assert Fraction(float(g[0, 1])) == Fraction(zz) * kept
    assert Fraction(float(g[0, 1])) != Fraction(zz) * Fraction(x) * Fraction(zz)


# ---- the shift rule --------------------------------------------------------------------------

def _gram_needing(delta):
    """2 x 2 Gram [[1, 1], [1, 1 - delta]] (max diagonal 1): with s added to the diagonal the second
    pivot is (1 - delta + s) - 1 / (1 + s) = 2 s - delta + O(s^2), so a shift s succeeds iff
    s > about delta / 2."""
    return np.array([[1.0, 1.0], [1.0, 1.0 - delta]])


@pytest.mark.parametrize("scheme,delta,attempt", [
    ("bf16x2", 0.0, 0),                  # singular Gram: the first shifted attempt already succeeds
    ("bf16x2", 2 * 30 * 2.0 ** -24, 2),  # needs s > 30 * 2^-24: c = 1 and 10 fail, 100 succeeds
    ("bf16x3", 2 * 3000 * 2.0 ** -24, 4),
    ("fp64", 2 * 3 * 2.0 ** -53, 2),     # FP64: 0, then 2^-53, 10 * 2^-53: the third retry
])
def test_shift_sequence(monkeypatch, scheme, delta, attempt):
    g = _gram_needing(delta)
    monkeypatch.setattr(mixed, "gram", lambda a, z, s, kt=256, sb=None: g.copy())
    z = np.eye(2)
    q, r, info, s = mixed.cholqr_pass(None, z, scheme, shift_c=1.0, max_retries=4)
    u = 2.0 ** -24 if scheme != "fp64" else 2.0 ** -53
    want = (10.0 ** attempt * u) if scheme != "fp64" else (10.0 ** (attempt - 1) * u if attempt else 0.0)
    assert info == 0 and s == want
    # R is the Cholesky factor of the shifted Gram (backward error of a 2 x 2 factorisation)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert np.abs(r.T @ r - (g + want * np.eye(2))).max() <= 8 * 2.0 ** -53


def test_shift_failure_reports_pivot(monkeypatch):
    g = np.array([[1.0, 0.0], [0.0, -1.0]])
    monkeypatch.setattr(mixed, "gram", lambda a, z, s, kt=256, sb=None: g.copy())
    q, r, info, s = mixed.cholqr_pass(None, np.eye(2), "bf16x2", shift_c=1.0, max_retries=3)
    assert q is None and info == 2 and s == 1e3 * 2.0 ** -24


def _mutant_cholqr_pass(g, scheme, shift_c=1.0, max_retries=4, factor=10.0, fp64_starts_shifted=False):
    """Copy of the shift-and-retry loop with one slip: another retry factor, or an FP64 pass that starts
    shifted like a reduced-precision one."""
    u = 2.0 ** -24 if scheme != "fp64" else 2.0 ** -53
    c = shift_c if (scheme != "fp64" or fp64_starts_shifted) else 0.0
    s = 0.0
    for _ in range(max_retries + 1):
        s = c * u * float(np.max(np.diag(g))) if c else 0.0
        if np.all(np.linalg.eigvalsh(g + s * np.eye(g.shape[0])) > 0):
            return s
        c = c * factor if c else shift_c
    return None


def test_shift_mutants_fail(monkeypatch):
    """The expectations of test_shift_sequence reject a retry factor of 2 and an FP64 pass that starts
    shifted; an FP64 pass on a well-conditioned Gram uses no shift at all, a split pass does."""
    g = _gram_needing(2 * 30 * 2.0 ** -24)
    assert _mutant_cholqr_pass(g, "bf16x2") == 100 * 2.0 ** -24       # a faithful copy agrees
    assert _mutant_cholqr_pass(g, "bf16x2", factor=2.0) != 100 * 2.0 ** -24
    g = np.array([[1.0, 0.5], [0.5, 1.0]])
    assert _mutant_cholqr_pass(g, "fp64", fp64_starts_shifted=True) != 0.0
    monkeypatch.setattr(mixed, "gram", lambda a, z, s, kt=256, sb=None: g.copy())
    assert mixed.cholqr_pass(None, np.eye(2), "fp64")[3] == 0.0
    assert mixed.cholqr_pass(None, np.eye(2), "bf16x2")[3] == 2.0 ** -24
