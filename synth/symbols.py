"""Integer symbol codes of the genotype alphabet, as the generators need them.

The numbering follows the value row of the paper's array-encoding example
(Fig. 1: + - x / sin = 0..4), continued in the order of the operator set of
Tab. 2 (cos, square, sqrt, exp, log, pow = 5..10).  CONST = 32, VAR k = 64 + k,
PAD = -1.  Only the codes live here; what the symbols compute is defined on the
oracle side and on the library side independently.
"""
ADD, SUB, MUL, DIV, SIN, COS, SQ, SQRT, EXP, LOG, POW = range(11)
CONST = 32
VAR0 = 64
PAD = -1

#: operator subsets used by the workloads
FUNCS_BASIC = (ADD, SUB, MUL, DIV)
FUNCS_8 = (ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG)
FUNCS_ALL = (ADD, SUB, MUL, DIV, SIN, COS, SQ, SQRT, EXP, LOG, POW)
#: operator set of the formula-ladder experiment (Tab. 2, Experiment III column)
FUNCS_LADDER = (ADD, SUB, MUL, DIV, SQ, SQRT)
#: operators with one operand (the others take two)
UNARY = (SIN, COS, SQ, SQRT, EXP, LOG)
