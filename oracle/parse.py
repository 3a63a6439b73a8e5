"""Parser for the expression language the oracle evaluates (test infrastructure).

The language is the user-facing notation of the paper (Sec. I, Sec. II, Fig. 2):
matrices and vectors are named operands, ``*`` is the matrix product (or a
scalar multiple when one side is a number), ``+``/``-`` are element-wise,
``%`` is the element-wise (Schur) product and ``/`` element-wise division,
``trans(X)`` / ``X.t()`` transpose, ``inv(X)`` the inverse, ``solve(A,B)`` the
solution of A X = B and ``exp(X)`` the element-wise exponential.
``diag(X)`` is the main diagonal as a column vector, ``diagmat(X)`` the
diagonal matrix of a vector (or a matrix's diagonal part), ``trace(X)`` the
sum of the diagonal (the functions of Sec. III's expressions (3)-(5), (7)).
``col(X, j)``, ``row(X, i)`` and ``submat(X, r0, c0, rows, cols)`` are
submatrices with 0-based integer indices (expression (2): the paper's first
column A(:,1) is col(A, 0), its second row B(2,:) is row(B, 1)).

``*``, ``%`` and ``/`` share one precedence level and group left to right, as
the C++ operators they overload do; ``+`` and ``-`` bind looser; unary minus
binds tighter than all of them.

AST nodes are tuples:
  ('num', value) ('var', name) ('neg', x) ('add', a, b) ('sub', a, b)
  ('mul', a, b) ('schur', a, b) ('div', a, b) ('call', fname, [args])
"""
from __future__ import annotations

import re

FUNCTIONS = {"trans": 1, "inv": 1, "exp": 1, "solve": 2, "diag": 1, "diagmat": 1, "trace": 1,
             "col": 2, "row": 2, "submat": 5}

_TOKEN = re.compile(
    r"\s*(?:(?P<num>(?:\d+\.\d*|\.\d+|\d+)(?:[eE][+-]?\d+)?)"
    r"|(?P<name>[A-Za-z_][A-Za-z0-9_]*)"
    r"|(?P<dott>\.t\(\))"
    r"|(?P<op>[-+*%/(),]))")


class OracleSyntaxError(ValueError):
    pass


def tokenize(text: str) -> list:
    pos, out = 0, []
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if m is None or m.end() == pos:
            raise OracleSyntaxError(f"bad character at {pos}: {text[pos:pos + 10]!r}")
        kind = m.lastgroup
        out.append((kind, m.group(kind)))
        pos = m.end()
    return out


class _Parser:
    def __init__(self, toks):
        self.toks, self.i = toks, 0

    def peek(self):
        return self.toks[self.i] if self.i < len(self.toks) else (None, None)

    def take(self, value=None):
        tok = self.peek()
        if tok[0] is None or (value is not None and tok[1] != value):
            raise OracleSyntaxError(f"expected {value!r}, found {tok[1]!r}")
        self.i += 1
        return tok

    def expr(self):
        node = self.term()
        while self.peek()[1] in ("+", "-"):
            op = self.take()[1]
            node = ("add" if op == "+" else "sub", node, self.term())
        return node

    def term(self):
        node = self.unary()
        while self.peek()[1] in ("*", "%", "/"):
            op = self.take()[1]
            kind = {"*": "mul", "%": "schur", "/": "div"}[op]
            node = (kind, node, self.unary())
        return node

    def unary(self):
        if self.peek()[1] == "-":
            self.take()
            return ("neg", self.unary())
        return self.postfix()

    def postfix(self):
        node = self.primary()
        while self.peek()[0] == "dott":
            self.take()
            node = ("call", "trans", [node])
        return node

    def primary(self):
        kind, val = self.peek()
        if kind == "num":
            self.take()
            return ("num", float(val))
        if kind == "name":
            self.take()
            if self.peek()[1] == "(":
                if val not in FUNCTIONS:
                    raise OracleSyntaxError(f"unknown function {val!r}")
                self.take("(")
                args = [self.expr()]
                while self.peek()[1] == ",":
                    self.take(",")
                    args.append(self.expr())
                self.take(")")
                if len(args) != FUNCTIONS[val]:
                    raise OracleSyntaxError(f"{val} takes {FUNCTIONS[val]} argument(s)")
                return ("call", val, args)
            return ("var", val)
        if val == "(":
            self.take("(")
            node = self.expr()
            self.take(")")
            return node
        raise OracleSyntaxError(f"unexpected token {val!r}")


def parse(text: str):
    p = _Parser(tokenize(text))
    node = p.expr()
    if p.peek()[0] is not None:
        raise OracleSyntaxError(f"trailing input at token {p.peek()[1]!r}")
    return node
