"""The oracle's Cash-Karp coefficients in exact rationals: the stage matrix
has the published nodes as row sums, the fifth-order weights satisfy all 17
order conditions up to order five, and the embedded weights b* = b - e all
eight up to order four but not those of order five (rooted-tree conditions,
Butcher; the method of Cash & Karp 1990)."""
import os
import re
from fractions import Fraction as F

ORACLE_C = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                        "raytrace_oracle.c")


def _array(name):
    src = open(ORACLE_C).read()
    m = re.search(name + r"\s*(\[[^=]*\])?\s*=\s*\{(.*?)\};", src, re.S)
    body = m.group(2).replace("{", " ").replace("}", " ")
    vals = []
    for tok in body.split(","):
        tok = tok.strip()
        if not tok:
            continue
        if "/" in tok:
            p, q = tok.split("/")
            vals.append(F(p.strip().replace(".0", "")) / F(q.strip().replace(".0", "")))
        else:
            vals.append(F(tok.replace(".0", "")))
    return vals


def tableau():
    a = _array("CK_A")
    A = [a[5 * i:5 * i + 5] + [F(0)] for i in range(6)]
    return A, _array("CK_B"), _array("CK_E")


def _conditions(A, b):
    n = len(b)
    c = [sum(A[i]) for i in range(n)]
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    Av = lambda v: [dot(A[i], v) for i in range(n)]
    pw = lambda k: [ci ** k for ci in c]
    mul = lambda u, v: [x * y for x, y in zip(u, v)]
    Ac, Ac2, Ac3 = Av(c), Av(pw(2)), Av(pw(3))
    AAc = Av(Ac)
    return {
        1: [(sum(b), F(1))],
        2: [(dot(b, c), F(1, 2))],
        3: [(dot(b, pw(2)), F(1, 3)), (dot(b, Ac), F(1, 6))],
        4: [(dot(b, pw(3)), F(1, 4)), (dot(b, mul(c, Ac)), F(1, 8)), (dot(b, Ac2), F(1, 12)),
            (dot(b, AAc), F(1, 24))],
        5: [(dot(b, pw(4)), F(1, 5)), (dot(b, mul(pw(2), Ac)), F(1, 10)),
            (dot(b, mul(c, Ac2)), F(1, 15)), (dot(b, mul(c, AAc)), F(1, 30)),
            (dot(b, mul(Ac, Ac)), F(1, 20)), (dot(b, Ac3), F(1, 20)),
            (dot(b, Av(mul(c, Ac))), F(1, 40)), (dot(b, Av(Ac2)), F(1, 60)),
            (dot(b, Av(AAc)), F(1, 120))],
    }


def test_nodes():
    A, b, e = tableau()
    c = [sum(row) for row in A]
    assert c == [F(0), F(1, 5), F(3, 10), F(3, 5), F(1), F(7, 8)]
    assert all(A[i][j] == 0 for i in range(6) for j in range(i, 6))  # explicit


def test_fifth_order_weights():
    A, b, e = tableau()
    cond = _conditions(A, b)
    assert sum(len(v) for v in cond.values()) == 17
    for order, items in cond.items():
        for got, want in items:
            assert got == want, (order, got, want)


def test_embedded_fourth_order_weights():
    A, b, e = tableau()
    bs = [x - y for x, y in zip(b, e)]
    cond = _conditions(A, bs)
    for order in (1, 2, 3, 4):
        for got, want in cond[order]:
            assert got == want, (order, got, want)
    assert any(got != want for got, want in cond[5])
