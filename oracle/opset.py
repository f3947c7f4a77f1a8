"""Symbol codes and operator semantics, float64.

Codes: the paper's array encoding (Fig. 1, value row) numbers the operators
+ - x / sin as 0..4; the remaining operators of Tab. 2's set follow in the
order listed there: cos 5, square 6, sqrt 7, exp 8, log 9, pow 10.  A constant
is 32 and variable k is 64+k; -1 ends / pads a program.  (The paper keeps the
node type in a separate array T; one signed byte carries both here.)

Protection is a reading: Tab. 2 lists plain / sqrt exp log pow and the paper
never says how they are protected.  The reading used everywhere:

  DIV_P(a, b)  = 1                       if |b| < GUARD, else a / b
  SQRT_P(a)    = sqrt(|a|)
  EXP_C(a)     = exp(clamp(a, -80, 80))  (clamp passes NaN through)
  LOG_P(a)     = 0                       if |a| < GUARD, else ln|a|
  POW_P(a, b)  = 0                       if |a| < GUARD, else exp(clamp(b ln|a|, -80, 80))

GUARD is the binary32 number nearest to 1e-6 (so a float32 input is compared
against the same threshold on every side).

Range: the paper's GPU evaluates in single precision (Section 5).  When
``rng == "f32"`` every node value whose magnitude would round to infinity in
binary32 becomes +-inf, so that overflow, and what later operators do with an
infinite operand, matches a float32 evaluation; precision is not emulated.
"""
import numpy as np

ADD, SUB, MUL, DIV, SIN, COS, SQ, SQRT, EXP, LOG, POW = range(11)
CONST = 32
VAR0 = 64
END = -1

NAMES = {ADD: "+", SUB: "-", MUL: "*", DIV: "/", SIN: "sin", COS: "cos", SQ: "sq",
         SQRT: "sqrt", EXP: "exp", LOG: "log", POW: "pow"}
ARITY = {ADD: 2, SUB: 2, MUL: 2, DIV: 2, POW: 2, SIN: 1, COS: 1, SQ: 1, SQRT: 1, EXP: 1, LOG: 1}

GUARD = float(np.float32(1e-6))
CLAMP = 80.0
F32_MAX = float(np.finfo(np.float32).max)
#: smallest magnitude that rounds to infinity in binary32 (round to nearest even)
F32_OVERFLOW = (2.0 - 2.0 ** -24) * 2.0 ** 127


def is_function(sym: int) -> bool:
    return int(sym) in ARITY


def is_terminal(sym: int) -> bool:
    s = int(sym)
    return s == CONST or s >= VAR0


def arity(sym: int) -> int:
    return ARITY.get(int(sym), 0)


def to_range(v, rng: str):
    """Round a float64 array's magnitude to the node precision's range."""
    if rng == "f32":
        big = np.abs(v) >= F32_OVERFLOW
        if np.any(big):
            v = np.where(big, np.copysign(np.inf, v), v)
    return v


def _clamp(t, clamp=CLAMP):
    # NaN compares false on both sides and is passed through unchanged
    return np.where(t < -clamp, -clamp, np.where(t > clamp, clamp, t))


def apply(op: int, a, b=None, guard=GUARD, clamp=CLAMP):
    """Value of operator ``op`` on float64 arrays (same shape).  ``guard`` and
    ``clamp`` default to the protection thresholds; other values serve only
    the conditioning check (mca), which moves them to find the decisions an
    input sits next to."""
    with np.errstate(all="ignore"):
        if op == ADD:
            return a + b
        if op == SUB:
            return a - b
        if op == MUL:
            return a * b
        if op == DIV:
            g = np.abs(b) < guard
            return np.where(g, 1.0, a / np.where(g, 1.0, b))
        if op == SIN:
            return np.sin(a)
        if op == COS:
            return np.cos(a)
        if op == SQ:
            return a * a
        if op == SQRT:
            return np.sqrt(np.abs(a))
        if op == EXP:
            return np.exp(_clamp(a, clamp))
        if op == LOG:
            g = np.abs(a) < guard
            return np.where(g, 0.0, np.log(np.where(g, 1.0, np.abs(a))))
        if op == POW:
            g = np.abs(a) < guard
            t = b * np.log(np.where(g, 1.0, np.abs(a)))
            return np.where(g, 0.0, np.exp(_clamp(t, clamp)))
    raise ValueError(f"not an operator: {op}")


def partials(op: int, a, b, v, guard=GUARD, clamp=CLAMP):
    """(d v / d a, d v / d b) of ``v = apply(op, a, b)``; b-partial is None
    for unary operators.  A guarded branch or a clamp in its saturated range
    has derivative 0; sqrt(|a|) has derivative sign(a)/(2 sqrt|a|), taken as 0
    at a = 0."""
    with np.errstate(all="ignore"):
        one = np.ones_like(a)
        if op == ADD:
            return one, one
        if op == SUB:
            return one, -one
        if op == MUL:
            return b, a
        if op == DIV:
            g = np.abs(b) < guard
            bs = np.where(g, 1.0, b)
            return np.where(g, 0.0, 1.0 / bs), np.where(g, 0.0, -a / (bs * bs))
        if op == SIN:
            return np.cos(a), None
        if op == COS:
            return -np.sin(a), None
        if op == SQ:
            return 2.0 * a, None
        if op == SQRT:
            r = np.sqrt(np.abs(a))
            return np.where(a == 0, 0.0, np.sign(a) / (2.0 * np.where(a == 0, 1.0, r))), None
        if op == EXP:
            inside = (a >= -clamp) & (a <= clamp)
            return np.where(inside, np.exp(np.where(inside, a, 0.0)), 0.0), None
        if op == LOG:
            g = np.abs(a) < guard
            return np.where(g, 0.0, 1.0 / np.where(g, 1.0, a)), None
        if op == POW:
            g = np.abs(a) < guard
            la = np.log(np.where(g, 1.0, np.abs(a)))
            t = b * la
            live = (~g) & (t >= -clamp) & (t <= clamp)
            r = np.exp(np.where(live, t, 0.0))
            da = np.where(live, r * b / np.where(g, 1.0, a), 0.0)
            db = np.where(live, r * la, 0.0)
            return da, db
    raise ValueError(f"not an operator: {op}")


def decision_inputs(op: int, a, b, guard=GUARD, clamp=CLAMP):
    """Inputs of the discrete decisions an operator takes, with thresholds:
    a list of (array, threshold) pairs compared as |array| vs threshold."""
    with np.errstate(all="ignore"):
        if op == DIV:
            return [(b, guard)]
        if op == LOG:
            return [(a, guard)]
        if op == EXP:
            return [(a, clamp)]
        if op == POW:
            g = np.abs(a) < guard
            t = b * np.log(np.where(g, 1.0, np.abs(a)))
            return [(a, guard), (np.where(g, 0.0, t), clamp)]
    return []
