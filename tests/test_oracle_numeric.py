"""Pins for the numeric CPU oracle (no GPU).

Each check ties the oracle to something other than itself: exact rational
arithmetic on tiny inputs, closed forms (identity, rank-1 products, k=1 outer
products, integer data), an independent library routine (numpy.matmul in
float64), and format definitions for the decoders and the output rounding
(numpy's binary16, torch's bfloat16/float8 tables, hand-derived tie cases).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def op(x, dtype="f64", order="row", scale=None):
    return W.store(np.asarray(x, dtype=np.float64), dtype, order, scale)


# ---------------------------------------------------------------- decoders

def test_decode_f16_all_patterns_match_numpy():
    bits = np.arange(65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = oracle.decode(bits, "f16")
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(np.isinf(got), np.isinf(ref))


def test_decode_bf16_all_patterns_match_torch():
    bits = np.arange(65536, dtype=np.uint16)
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).double().numpy()
    got = oracle.decode(bits, "bf16")
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_decode_f8e4m3_format_points_and_torch_table():
    bits = np.arange(256, dtype=np.uint8)
    got = oracle.decode(bits, "f8e4m3")
    # OCP e4m3fn definition points
    assert got[0x7E] == 448.0 and got[0xFE] == -448.0
    assert np.isnan(got[0x7F]) and np.isnan(got[0xFF])
    assert got[0x38] == 1.0 and got[0xB8] == -1.0
    assert got[0x08] == 2.0 ** -6            # min normal
    assert got[0x01] == 2.0 ** -9            # min subnormal
    assert got[0x07] == 7 * 2.0 ** -9        # max subnormal
    assert got[0x00] == 0.0 and math.copysign(1, got[0x80]) == -1
    ref = torch.from_numpy(bits).view(torch.float8_e4m3fn).double().numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])


def test_decode_f32_matches_view():
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 2**32, size=20000, dtype=np.uint64).astype(np.uint32)
    ref = bits.view(np.float32).astype(np.float64)
    got = oracle.decode(bits, "f32")
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])


# ---------------------------------------------------------------- rounding

def test_round_bf16_hand_ties():
    vals = np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8, -(1 + 2.0**-8), 1 + 2.0**-8 + 2.0**-30,
                     3.0e38 * 1.2, 2.0**-133, 2.0**-134, 3 * 2.0**-134])
    got = oracle.decode(oracle.round_to(vals, "bf16"), "bf16")
    assert got[0] == 1.0                       # tie -> even (fraction 0)
    assert got[1] == 1 + 2.0**-6               # tie between 1+2^-7 and 1+2^-6 -> even
    assert got[2] == -1.0
    assert got[3] == 1 + 2.0**-7               # just above the tie rounds up
    assert math.isinf(got[4])
    assert got[5] == 2.0**-133                 # min subnormal is exact
    assert got[6] == 0.0                       # half of min subnormal: tie -> even (0)
    assert got[7] == 2 * 2.0**-133             # 1.5 ulp: tie -> even (2)


def test_round_bf16_matches_torch_on_float32_values():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(50000) * np.exp(rng.uniform(-30, 30, 50000))).astype(np.float32)
    x = x.astype(np.float64)    # exactly float32 values: one rounding either way
    got = oracle.round_to(x, "bf16")
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, ref)


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(8)
    x = rng.standard_normal(50000) * np.exp(rng.uniform(-20, 12, 50000))
    x = np.concatenate([x, [65504.0, 65519.99, 65520.0, 2.0**-24, 2.0**-25, 1.5 * 2.0**-24]])
    got = oracle.round_to(x, "f16")
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, ref)


def test_round_f32_matches_numpy():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(50000) * np.exp(rng.uniform(-80, 80, 50000))
    got = oracle.round_to(x, "f32")
    ref = x.astype(np.float32).view(np.uint32)
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- GEMM pins

def exact_gemm(A, B, C, alpha, beta):
    m, k = A.shape
    n = B.shape[1]
    out = [[None] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = sum((Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(k)), Fraction(0))
            v = Fraction(alpha) * s
            if beta != 0:
                v += Fraction(beta) * Fraction(C[i, j])
            out[i][j] = v
    return out


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_rational_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    m, n, k = (int(v) for v in rng.integers(1, 7, size=3))
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    C = rng.uniform(-1, 1, (m, n))
    alpha, beta = float(rng.uniform(-2, 2)), float(rng.choice([0.0, rng.uniform(-2, 2)]))
    got = oracle.gemm(m, n, k, op(A), op(B), op(C), alpha, beta)
    ex = exact_gemm(A, B, C, alpha, beta)
    u = 2.0 ** -53
    gamma = (k + 2) * u / (1 - (k + 2) * u)
    for i in range(m):
        for j in range(n):
            mag = abs(alpha) * float(np.abs(A[i]) @ np.abs(B[:, j])) + abs(beta) * abs(C[i, j])
            assert abs(got[i, j] - float(ex[i][j])) <= gamma * mag + 1e-300


def test_identity_closed_form():
    rng = np.random.default_rng(1)
    m, k, n = 37, 37, 23
    B = rng.uniform(-1, 1, (k, n))
    got = oracle.gemm(m, n, k, op(np.eye(m)), op(B))
    assert np.array_equal(got, B)
    A = rng.uniform(-1, 1, (m, k))
    got = oracle.gemm(m, k, k, op(A), op(np.eye(k)))
    assert np.array_equal(got, A)


def test_rank1_closed_form_integers():
    rng = np.random.default_rng(2)
    m, k, n = 19, 45, 31
    u = rng.integers(-3, 4, m).astype(float)
    v = rng.integers(-3, 4, k).astype(float)
    w = rng.integers(-3, 4, k).astype(float)
    z = rng.integers(-3, 4, n).astype(float)
    A, B = np.outer(u, v), np.outer(w, z)
    got = oracle.gemm(m, n, k, op(A), op(B))
    assert np.array_equal(got, float(v @ w) * np.outer(u, z))


def test_k1_outer_product_and_zero():
    rng = np.random.default_rng(3)
    a = rng.uniform(-1, 1, (13, 1))
    b = rng.uniform(-1, 1, (1, 11))
    got = oracle.gemm(13, 11, 1, op(a), op(b))
    assert np.array_equal(got, a * b)                    # one product each: exact
    got0 = oracle.gemm(13, 11, 9, op(np.zeros((13, 9))), op(rng.uniform(-1, 1, (9, 11))))
    assert np.array_equal(got0, np.zeros((13, 11)))


def test_alpha_beta_integers_exact():
    rng = np.random.default_rng(4)
    m, n, k = 21, 17, 40
    A = W.small_integers((m, k), rng)
    B = W.small_integers((k, n), rng)
    C = W.small_integers((m, n), rng)
    prod = np.zeros((m, n))
    for p in range(k):                                   # exact integer sums
        prod += np.outer(A[:, p], B[p, :])
    got = oracle.gemm(m, n, k, op(A), op(B), op(C), alpha=2.0, beta=-1.0)
    assert np.array_equal(got, 2.0 * prod - C)
    got_b0 = oracle.gemm(m, n, k, op(A), op(B), op(C * np.nan), alpha=1.0, beta=0.0)
    assert np.array_equal(got_b0, prod)                  # beta == 0: C is never read


def test_matches_numpy_matmul():
    rng = np.random.default_rng(6)
    for (m, n, k) in [(70, 130, 257), (128, 64, 1000), (5, 300, 77)]:
        A = rng.uniform(-1, 1, (m, k))
        B = rng.uniform(-1, 1, (k, n))
        got = oracle.gemm(m, n, k, op(A), op(B))
        ref = A @ B
        err = np.linalg.norm(got - ref) / (np.linalg.norm(A) * np.linalg.norm(B))
        assert err < 1e-15


def test_all_layouts_agree_bitwise():
    rng = np.random.default_rng(10)
    m, n, k = 33, 29, 71
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    C = rng.uniform(-1, 1, (m, n))
    base = oracle.gemm(m, n, k, op(A), op(B), op(C), 1.5, 0.5)
    for ao, bo, co in itertools.product(["row", "col"], repeat=3):
        got = oracle.gemm(m, n, k, op(A, order=ao), op(B, order=bo), op(C, order=co), 1.5, 0.5)
        assert np.array_equal(got, base), (ao, bo, co)
    # a transposed operand must not agree (catches a swapped index)
    At = op(A.T.copy(), order="row")
    At = W.Operand(At.tensor, m, k, "f64", "col", m)     # A^T bytes read as col-major A: same A
    assert np.array_equal(oracle.gemm(m, n, k, At, op(B), op(C), 1.5, 0.5), base)
    wrong = W.Operand(op(A).tensor, m, k, "f64", "col", m)  # row-major bytes read as col-major
    assert not np.array_equal(oracle.gemm(m, n, k, wrong, op(B), op(C), 1.5, 0.5), base)


def test_block_size_does_not_change_the_sum_order():
    rng = np.random.default_rng(11)
    m, n, k = 40, 50, 333
    A = op(rng.uniform(-1, 1, (m, k)))
    B = op(rng.uniform(-1, 1, (k, n)))
    base = oracle.gemm(m, n, k, A, B, blk=(64, 64, 64))
    for blk in [(1, 1, 1), (7, 13, 5), (128, 128, 16), (40, 50, 333)]:
        assert np.array_equal(oracle.gemm(m, n, k, A, B, blk=blk), base)


def test_elementwise_matches_full():
    rng = np.random.default_rng(12)
    m, n, k = 30, 20, 100
    A = op(rng.uniform(-1, 1, (m, k)), order="col")
    B = op(rng.uniform(-1, 1, (k, n)))
    C = op(rng.uniform(-1, 1, (m, n)), order="col")
    full = oracle.gemm(m, n, k, A, B, C, 0.75, -1.25)
    rows = rng.integers(0, m, 50)
    cols = rng.integers(0, n, 50)
    got = oracle.gemm_elems(rows, cols, k, A, B, C, 0.75, -1.25)
    assert np.array_equal(got, full[rows, cols])


@pytest.mark.parametrize("dtype", ["f16", "bf16", "f8e4m3"])
def test_narrow_inputs_use_exact_stored_values(dtype):
    rng = np.random.default_rng(13)
    m, n, k = 24, 18, 64
    A = op(rng.standard_normal((m, k)), dtype)
    B = op(rng.standard_normal((k, n)), dtype, "col")
    Ad = oracle.decode_operand(A)
    Bd = oracle.decode_operand(B)
    if dtype == "f8e4m3":
        assert A.scale != 1.0
        table = oracle.decode(np.arange(256, dtype=np.uint8), "f8e4m3")
        table = set(table[np.isfinite(table)].tolist())
        assert set((Ad / A.scale).ravel().tolist()) <= table   # every value is s * code
    got = oracle.gemm(m, n, k, A, B)
    ref = Ad @ Bd
    assert np.linalg.norm(got - ref) <= 1e-15 * np.linalg.norm(Ad) * np.linalg.norm(Bd)
    # the stored values are not the drawn ones, so a reference on the drawn
    # values would differ: the oracle must be fed the rounded inputs
    drawn = np.random.default_rng(13).standard_normal((m, k))
    assert not np.array_equal(Ad, drawn)


def test_fp8_integer_codes_scale_one_exact():
    rng = np.random.default_rng(14)
    m, n, k = 16, 16, 256
    A = W.small_integers((m, k), rng)
    B = W.small_integers((k, n), rng)
    got = oracle.gemm(m, n, k, op(A, "f8e4m3", scale=1.0), op(B, "f8e4m3", scale=1.0))
    prod = np.zeros((m, n))
    for p in range(k):
        prod += np.outer(A[:, p], B[p, :])
    assert np.array_equal(got, prod)
