"""FP64 CPU oracle for compound linear-algebra expressions.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
run anything in this package; only the tests, the smoke check and the bench's
CPU-baseline leg use it. It shares no code with the HIP evaluator: it parses the
expression text itself and evaluates every step with plain definitions in
float64, the precision the paper's own evaluation uses (Sec. III, the ``mat``
type of Fig. 2 and the ``double`` element type of Fig. 3).

Modules
-------
parse     recursive-descent parser for the expression language
evaluate  plain evaluation of a parsed expression (definitions, no rewrites),
          and the componentwise error scale of its result
chain     parenthesisation enumeration, cost counts, the paper's greedy rule
gepp      Gaussian elimination with partial pivoting, substitution, inverse
bf16      bfloat16 round-to-nearest-even and hi/lo splitting
refine    mixed-precision iterative refinement, step by step
mlp       small ReLU network: forward, backward, MSE, Adam
"""
from .parse import parse, OracleSyntaxError
from .evaluate import evaluate, magnitude, OracleDimError
from .gepp import SingularMatrix

__all__ = ["parse", "evaluate", "magnitude", "OracleSyntaxError", "OracleDimError",
           "SingularMatrix"]
