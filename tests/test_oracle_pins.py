"""Pins for the FP64 oracle: each test checks it against something the
mathematics or the paper fixes (closed forms, brute force on tiny inputs,
exact integer arithmetic, invariants, special cases that reduce to a library
routine), chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them."""
import itertools
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import chain, evaluate, gepp, parse
from oracle.evaluate import OracleDimError
from oracle.parse import OracleSyntaxError


def loops_product(a, b):
    """(AB)_ij = sum_k A_ik B_kj with explicit loops (tiny sizes only)."""
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    out = np.zeros((m, n))
    for i in range(m):
        for j in range(n):
            s = 0.0
            for t in range(k):
                s += float(a[i, t]) * float(b[t, j])
            out[i, j] = s
    return out


# ------------------------------------------------------------------ parser

def test_parse_precedence_and_grouping():
    assert parse("A + B * C") == ("add", ("var", "A"), ("mul", ("var", "B"), ("var", "C")))
    # * % / share one level, grouped left to right (C++ operator rules)
    assert parse("A * B % C") == ("schur", ("mul", ("var", "A"), ("var", "B")), ("var", "C"))
    assert parse("A - B - C") == ("sub", ("sub", ("var", "A"), ("var", "B")), ("var", "C"))
    assert parse("-A*B") == ("mul", ("neg", ("var", "A")), ("var", "B"))
    assert parse("A.t()") == ("call", "trans", [("var", "A")])
    assert parse("solve(A*A.t(), b)")[1] == "solve"
    assert parse("0.5*exp(-(A%A))")[2] == ("call", "exp", [("neg", ("schur", ("var", "A"), ("var", "A")))])


@pytest.mark.parametrize("bad", ["A +", "foo(A)", "solve(A)", "(A", "A $ B", "trans(A, B)"])
def test_parse_errors(bad):
    with pytest.raises(OracleSyntaxError):
        parse(bad)


# ------------------------------------------------------------ element-wise

def test_paper_fusion_example_special_values():
    # Z = 0.4 X + 0.6 Y (Sec. II): X = Y gives X back; X alone scales by 0.4
    g = inputs.rng(1)
    x = inputs.normal(g, 7, 5)
    z = evaluate("0.4*X + 0.6*Y", {"X": x, "Y": x})
    assert np.allclose(z, x, rtol=4e-16, atol=0)
    z = evaluate("0.4*X + 0.6*Y", {"X": np.full((3, 2), 10.0), "Y": np.zeros((3, 2))})
    assert np.all(z == 4.0)
    z = evaluate("0.4*X + 0.6*Y", {"X": np.zeros((3, 2)), "Y": np.full((3, 2), 5.0)})
    assert np.all(z == 3.0)


def test_elementwise_expression_closed_forms():
    g = inputs.rng(2)
    b = inputs.normal(g, 6, 4)
    c = inputs.uniform(g, 6, 4, 1.0, 2.0)
    # A = 0: exp(0) = 1, so the result is 0.5 + B/C exactly
    y = evaluate("0.5*exp(-(A%A)) + B/C", {"A": np.zeros((6, 4)), "B": b, "C": c})
    assert np.array_equal(y, 0.5 + b / c)
    # A_ij^2 = k ln 2 gives exp(-A^2) = 2^-k; B = 0 isolates the first term
    k = np.arange(24, dtype=np.float64).reshape(6, 4) % 9
    a = np.sqrt(k * math.log(2.0))
    y = evaluate("0.5*exp(-(A%A)) + B/C", {"A": a, "B": np.zeros((6, 4)), "C": c})
    assert np.allclose(y, 0.5 * 2.0 ** -k, rtol=1e-14, atol=0)
    # division orientation and subtraction order
    assert evaluate("B/C", {"B": np.ones((1, 1)), "C": np.full((1, 1), 2.0)})[0, 0] == 0.5
    assert evaluate("A - B", {"A": np.full((1, 1), 3.0), "B": np.ones((1, 1))})[0, 0] == 2.0
    assert evaluate("-A + B", {"A": np.full((1, 1), 3.0), "B": np.ones((1, 1))})[0, 0] == -2.0
    assert evaluate("exp(A)", {"A": np.ones((1, 1))})[0, 0] == pytest.approx(math.e, rel=1e-15)


def test_elementwise_size_check():
    with pytest.raises(OracleDimError):
        evaluate("A + B", {"A": np.zeros((2, 3)), "B": np.zeros((3, 2))})


# ----------------------------------------------------------------- products

def test_products_against_explicit_loops():
    g = inputs.rng(3)
    a = inputs.normal(g, 4, 3)
    b = inputs.normal(g, 4, 5)
    c = inputs.normal(g, 5, 2)
    got = evaluate("trans(A)*B*C", {"A": a, "B": b, "C": c})
    ref = loops_product(loops_product(a.T.copy(), b), c)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    got = evaluate("2*A*trans(C)", {"A": b, "C": inputs.normal(inputs.rng(4), 3, 5)})
    assert got.shape == (4, 3)
    # a transposed operand must not be confused with the plain one
    sq = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert np.array_equal(evaluate("trans(A)*B", {"A": sq, "B": np.eye(2)}), sq.T)
    assert np.array_equal(evaluate("A*trans(B)", {"A": np.eye(2), "B": sq}), sq.T)


def test_small_integer_chain_all_orders_bitwise_equal():
    # entries in [-8, 8]: every partial sum is an exactly representable integer,
    # so every bracketing (and the oracle's own choice) must agree bit for bit
    g = inputs.rng(5)
    dims = [5, 3, 7, 2, 6, 4]
    mats = [inputs.small_ints(g, dims[i], dims[i + 1]) for i in range(5)]
    env = {f"M{i}": m for i, m in enumerate(mats)}
    got = evaluate("M0*M1*M2*M3*M4", env)
    results = []
    for t in chain.trees(0, 4):
        def run(node):
            if isinstance(node, int):
                return mats[node]
            return loops_product(run(node[0]), run(node[1]))
        results.append(run(t))
    assert len(results) == chain.catalan(4) == 14
    for r in results:
        assert np.array_equal(r, got)


def test_product_size_check():
    with pytest.raises(OracleDimError):
        evaluate("A*B", {"A": np.zeros((2, 3)), "B": np.zeros((2, 3))})


# ---------------------------------------------------------------- chain cost

def test_catalan_counts():
    for length, count in zip(range(1, 9), [1, 1, 2, 5, 14, 42, 132, 429]):
        assert len(chain.trees(0, length - 1)) == count == chain.catalan(length - 1)


def test_chain_golden_costs():
    # [2,1,3,10]: the paper's greedy pair rule takes (M1 M2) first: 6 + 60 = 66
    # multiply-adds; the cheapest order M1 (M2 M3) costs 30 + 20 = 50
    tree, cost = chain.greedy_smallest_result([2, 1, 3, 10])
    assert tree == ((0, 1), 2) and cost == 66
    assert chain.brute_force_min([2, 1, 3, 10])[0] == 50
    # expression (6) of Sec. III, m = 1000 (m/3, m/4 floored): the cheapest
    # order and the greedy order are both right-to-left
    dims = [1000, 1000, 500, 333, 250]
    best, trees = chain.brute_force_min(dims)
    assert chain.right_to_left(4) in trees
    assert chain.greedy_smallest_result(dims)[0] == chain.right_to_left(4)
    l2r = chain.tree_cost(chain.left_to_right(4), dims)
    assert l2r / best == pytest.approx(1.80, abs=0.01)
    # the FP32 5-factor chain: right-to-left is optimal at 1,476,395,008 MACs;
    # greedy with leftmost tie-break pays 4,999,610,368
    dims = [8192, 1024, 8192, 512, 4096, 64]
    best, trees = chain.brute_force_min(dims)
    assert best == 1_476_395_008 and chain.right_to_left(5) in trees
    assert chain.greedy_smallest_result(dims)[1] == 4_999_610_368
    # trans(A)*B*C*v: A^T (B (C v)) at 480,000 MACs
    dims = [300, 400, 600, 200, 1]
    best, trees = chain.brute_force_min(dims)
    assert best == 480_000 and trees == [chain.right_to_left(4)]


def test_symmetric_pair_cost():
    # X^T X with X 10 x 4: n(n+1)/2 * k = 4*5/2*10 = 100 instead of 160
    assert chain.tree_cost((0, 1), [4, 10, 4], frozenset({(0, 1)})) == 100
    assert chain.tree_cost((0, 1), [4, 10, 4]) == 160


# ------------------------------------------------------------------- GEPP

def test_lu_reconstruction_and_multiplier_bound():
    g = inputs.rng(6)
    s = inputs.normal(g, 60, 60)
    perm, lu = gepp.lu_partial_pivot(s)
    low, up = gepp.unpack_lu(lu)
    err = np.linalg.norm(s[perm] - low @ up, np.inf)
    assert err <= 60 * 2.0 ** -52 * np.linalg.norm(s, np.inf) * 4
    assert np.max(np.abs(np.tril(lu, -1))) <= 1.0
    assert sorted(perm) == list(range(60))


def test_pivot_tie_goes_to_lowest_row():
    s = np.array([[1.0, 0.0, 0.0], [-2.0, 1.0, 0.0], [2.0, 0.0, 1.0]])
    perm, _ = gepp.lu_partial_pivot(s)
    assert perm[0] == 1


def test_solve_special_cases_exact():
    n = 6
    assert np.array_equal(gepp.solve(np.eye(n), np.arange(n, dtype=float)), np.arange(n, dtype=float))
    d = np.diag([2.0, 4.0, 8.0, 0.5, 1.0, 16.0])
    b = np.array([2.0, 8.0, 8.0, 1.0, 3.0, 32.0])
    assert np.array_equal(gepp.solve(d, b), b / np.diag(d))
    p = np.eye(n)[[3, 0, 5, 1, 2, 4]]
    x = np.arange(1.0, n + 1)
    assert np.array_equal(gepp.solve(p, p @ x), x)
    # unit upper triangular integer matrix with integer solution: exact
    g = inputs.rng(7)
    u = np.triu(inputs.small_ints(g, n, n, -3, 3), 1) + np.eye(n)
    x = inputs.small_ints(g, n, 2, -5, 5)
    assert np.array_equal(gepp.solve(u, u @ x), x)


def test_solve_matches_lapack_and_inverse():
    g = inputs.rng(8)
    s = inputs.normal(g, 40, 40)
    b = inputs.normal(g, 40, 3)
    x = gepp.solve(s, b)
    assert np.allclose(x, np.linalg.solve(s, b), rtol=1e-11, atol=1e-12)
    inv = gepp.gauss_jordan_inverse(s)
    assert np.allclose(inv @ s, np.eye(40), atol=1e-11)
    assert np.allclose(evaluate("inv(S)*B", {"S": s, "B": b}), x, rtol=0, atol=1e-12)
    assert np.allclose(evaluate("inv(S)*B", {"S": s, "B": b}, explicit_inverse=True), x, atol=1e-10)
    assert np.allclose(evaluate("solve(S,B)", {"S": s, "B": b}), x, rtol=0, atol=0)
    # backward error of the solve at the level of unit roundoff
    r = np.linalg.norm(b - s @ x, np.inf)
    assert r / (np.linalg.norm(s, np.inf) * np.linalg.norm(x, np.inf)) < 40 * 2.0 ** -52


def test_gauss_jordan_integer_inverse_exact():
    # a unimodular integer matrix has an integer inverse
    l = np.array([[1.0, 0, 0], [2, 1, 0], [-1, 3, 1]])
    u = np.array([[1.0, 4, -2], [0, 1, 5], [0, 0, 1]])
    s = l @ u
    inv = gepp.gauss_jordan_inverse(s)
    assert np.allclose(inv, np.rint(inv), atol=1e-12)
    assert np.array_equal(np.rint(inv) @ s, np.eye(3))


def test_singular_detection():
    s = np.array([[1.0, 2.0], [2.0, 4.0]])
    with pytest.raises(gepp.SingularMatrix):
        gepp.lu_partial_pivot(s)
    with pytest.raises(gepp.SingularMatrix):
        gepp.lu_partial_pivot(np.zeros((3, 3)))


def test_chain_with_inverse_and_solve():
    g = inputs.rng(9)
    s = inputs.diag_dominant(g, 12)
    a = inputs.normal(g, 12, 12)
    b = inputs.normal(g, 12, 1)
    ref = gepp.gauss_jordan_inverse(s) @ (a @ b)
    got = evaluate("inv(S)*A*b", {"S": s, "A": a, "b": b})
    assert np.allclose(got, ref, atol=1e-12)
    got = evaluate("A*inv(S)*b", {"S": s, "A": a, "b": b})
    assert np.allclose(got, a @ np.linalg.solve(s, b), atol=1e-12)


# ------------------------------------------------------------- symmetric product

def test_gram_invariants_and_closed_form():
    x, u, sv, v = inputs.svd_matrix(10, 300, 20, 1e4)
    g = evaluate("trans(X)*X", {"X": x})
    assert np.array_equal(g, g.T) or np.allclose(g, g.T, rtol=0, atol=1e-15)
    assert np.allclose(np.diag(g), np.sum(x * x, axis=0), rtol=1e-13)
    assert np.min(np.linalg.eigvalsh(g)) > -1e-12
    assert np.allclose(g, (v * sv ** 2) @ v.T, atol=1e-13)
    assert np.allclose(np.sort(np.linalg.eigvalsh(g))[::-1], sv ** 2, rtol=1e-8, atol=1e-13)
    h = evaluate("X*trans(X)", {"X": x[:20, :]})
    assert np.allclose(h, loops_product(x[:20, :], x[:20, :].T.copy()), atol=1e-13)


# --------------------------------------- diagonals, traces and submatrices

def test_diagonal_functions_by_hand():
    x = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
    env = {"X": x, "W": x[:2, :], "v": np.array([[2.0], [-1.0], [0.5]])}
    assert oracle.evaluate("diag(X)", env).ravel().tolist() == [1.0, 5.0, 10.0]
    assert oracle.evaluate("diag(W)", env).ravel().tolist() == [1.0, 5.0]  # 2 x 3: two entries
    assert oracle.evaluate("trace(X)", env).tolist() == [[16.0]]
    assert oracle.evaluate("diagmat(X)", env).tolist() == [[1, 0, 0], [0, 5, 0], [0, 0, 10]]
    assert oracle.evaluate("diagmat(v)", env).tolist() == [[2, 0, 0], [0, -1, 0], [0, 0, 0.5]]
    assert oracle.evaluate("diagmat(trans(v))", env).tolist() == [[2, 0, 0], [0, -1, 0], [0, 0, 0.5]]
    # expression (3): diagmat(v) * X scales the rows of X
    assert oracle.evaluate("diagmat(v)*X", env).tolist() == [[2, 4, 6], [-4, -5, -6], [3.5, 4, 5]]
    # expression (7): a^T diagmat(B) c = sum_i a_i B_ii c_i = 1*1*2 + 1*5*(-1) + 1*10*0.5 = 2
    env["a"] = np.ones((3, 1))
    assert oracle.evaluate("trans(a)*diagmat(X)*v", env).tolist() == [[2.0]]


def test_paper_view_expression_by_hand():
    # expression (2): C = A(:,1) + B(2,:)^T, the first column of A plus the
    # transposed second row of B
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    b = np.array([[5.0, 6.0], [7.0, 8.0]])
    got = oracle.evaluate("col(A, 0) + trans(row(B, 1))", {"A": a, "B": b})
    assert got.tolist() == [[8.0], [11.0]]
    assert oracle.evaluate("submat(A, 1, 0, 1, 2)", {"A": a}).tolist() == [[3.0, 4.0]]
    with pytest.raises(oracle.OracleDimError):
        oracle.evaluate("col(A, 2)", {"A": a})


def test_trace_and_diagonal_identities():
    g = inputs.rng(33)
    a, b = inputs.normal(g, 5, 7), inputs.normal(g, 7, 5)
    env = {"A": a, "B": b, "u": inputs.normal(g, 5, 1), "w": inputs.normal(g, 5, 1),
           "S": inputs.normal(g, 5, 5), "one": np.ones((5, 1))}
    tab = oracle.evaluate("trace(A*B)", env)[0, 0]
    # trace(AB) = trace(BA) = sum(A % B^T) (the Frobenius inner product)
    assert tab == pytest.approx(oracle.evaluate("trace(B*A)", env)[0, 0], rel=1e-12)
    assert tab == pytest.approx(float(np.sum(oracle.evaluate("A % trans(B)", env))), rel=1e-12)
    # diag(AB) = row sums of A % B^T
    assert np.allclose(oracle.evaluate("diag(A*B)", env),
                       oracle.evaluate("(A % trans(B))*ones", dict(env, ones=np.ones((7, 1)))),
                       rtol=1e-12, atol=1e-12)
    # diagmat(AB) keeps exactly the diagonal of AB
    dm = oracle.evaluate("diagmat(A*B)", env)
    assert np.array_equal(np.diag(np.diag(dm)), dm)
    assert np.allclose(np.diag(dm), oracle.evaluate("diag(A*B)", env).ravel(), rtol=1e-12)
    # u^T diagmat(S) w = u^T (diag(S) % w); diagmat(u) * S = (u * one^T) % S
    assert oracle.evaluate("trans(u)*diagmat(S)*w", env)[0, 0] == pytest.approx(
        oracle.evaluate("trans(u)*(diag(S) % w)", env)[0, 0], rel=1e-12)
    assert np.allclose(oracle.evaluate("diagmat(u)*S", env),
                       oracle.evaluate("(u*trans(one)) % S", env), rtol=1e-14, atol=0)


def test_magnitude_of_diagonal_functions():
    a = np.array([[1.0, -2.0], [3.0, 4.0]])
    b = np.array([[-1.0, 1.0], [2.0, -3.0]])
    env = {"A": a, "B": b}
    # |A||B| = [[5, 7], [11, 15]]: its diagonal and trace
    assert oracle.magnitude("diag(A*B)", env).ravel().tolist() == [5.0, 15.0]
    assert oracle.magnitude("trace(A*B)", env).tolist() == [[20.0]]
    assert oracle.magnitude("col(A, 1)", env).ravel().tolist() == [2.0, 4.0]


def test_roofline_time_by_hand_and_golden_order():
    # one product 2 x 3 by 3 x 4: 48 flops, 6 + 12 + 8 = 26 elements
    assert chain.roofline_time((0, 1), [2, 3, 4], 4, 48.0, 26 * 4.0) == 1.0
    assert chain.roofline_time((0, 1), [2, 3, 4], 4, 24.0, 1e9) == 2.0   # flop-bound
    assert chain.roofline_time((0, 1), [2, 3, 4], 8, 1e9, 26 * 4.0) == 2.0  # byte-bound at 8 B
    # [1, 4, 8192, 4] in FP32 at 157.3 TFLOP/s and 8 TB/s: the fewest
    # multiply-adds first make a 1 x 8192 row (65,536 MACs); the roofline
    # order forms the 4 x 4 product of the two large factors first (131,088
    # MACs) and moves (65,552 + 24) * 4 = 262,304 bytes instead of
    # (40,964 + 40,964) * 4 = 327,712
    dims = [1, 4, 8192, 4]
    assert chain.brute_force_min(dims)[1] == [((0, 1), 2)]
    t, best = chain.brute_force_min_time(dims, 4, 157.3e12, 8e12)
    assert best == [(0, (1, 2))]
    assert t == pytest.approx(262304 / 8e12, rel=1e-12)
    assert chain.roofline_time(((0, 1), 2), dims, 4, 157.3e12, 8e12) == pytest.approx(327712 / 8e12,
                                                                                     rel=1e-12)
