"""Genotype <-> postfix program, following Section 3.2 ("Data Structure of
Individuals") and Fig. 1.

encode: post-order traversal of the active nodes only (introns dropped).  Each
node becomes one signed-byte symbol; a constant additionally takes the next
entry of the individual's constant list, so constants are listed in order of
appearance in the postfix program.  The program is padded with END (-1) to the
fixed stride L_max, and the constant list with zeros to C_max (the padding to a
common length that makes a population one dense array, Section 3.2).

decode: rebuild the tree from the postfix program with a stack of subtrees and
lay it out from heap slot 0 (left child first, a unary operator's operand in the
left child); all other slots become PAD (-1) with constant 0.

The paper's two arrays (type T, value V) map onto (symbol byte, constant list):
type 0 = variable (symbol 64+k), type 1 = constant (symbol 32, value in the
constant list), type 2 = operator (symbol = operator index).
"""
import numpy as np

from . import opset as O
from .tree import depth_of

PAD = -1


def encode_one(genes_row, gconst_row, height: int):
    """(list of symbols, list of float32 constants) of one genotype."""
    T = 2 ** (height + 1) - 1
    syms, consts = [], []

    def walk(i):
        if i >= T:
            raise ValueError("active node outside the template")
        g = int(genes_row[i])
        k = O.arity(g)
        if k:
            if depth_of(i) == height:
                raise ValueError(f"active operator at leaf slot {i}")
            for c in range(k):
                walk(2 * i + 1 + c)
        elif not O.is_terminal(g):
            raise ValueError(f"active slot {i} holds no symbol ({g})")
        syms.append(g)
        if g == O.CONST:
            consts.append(np.float32(gconst_row[i]))

    walk(0)
    return syms, consts


def encode(genes, gconst, heights, L_max: int, C_max: int):
    """Batch encoder.  ``heights`` is an int or a per-individual array.

    Returns ops int8 [M, L_max], consts float32 [M, C_max], lens int16 [M],
    nconst int16 [M]."""
    genes = np.asarray(genes)
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    ops = np.full((M, L_max), PAD, dtype=np.int8)
    cs = np.zeros((M, C_max), dtype=np.float32)
    lens = np.zeros(M, dtype=np.int16)
    ncs = np.zeros(M, dtype=np.int16)
    for m in range(M):
        s, c = encode_one(genes[m], gconst[m], int(hs[m]))
        if len(s) > L_max or len(c) > C_max:
            raise ValueError(f"individual {m}: program does not fit (L={len(s)}, C={len(c)})")
        ops[m, : len(s)] = s
        cs[m, : len(c)] = c
        lens[m] = len(s)
        ncs[m] = len(c)
    return ops, cs, lens, ncs


def parse(ops_row, consts_row):
    """Parse one postfix program into nested tuples (sym, const, children...).
    Raises ValueError on a malformed program."""
    stack = []
    j = 0
    for t in ops_row:
        t = int(t)
        if t == PAD:
            break
        if t == O.CONST:
            stack.append((t, float(np.float32(consts_row[j])),))
            j += 1
        elif t >= O.VAR0:
            stack.append((t, 0.0))
        elif O.is_function(t):
            k = O.arity(t)
            if len(stack) < k:
                raise ValueError("stack underflow")
            kids = stack[len(stack) - k:]
            del stack[len(stack) - k:]
            stack.append((t, 0.0, *kids))
        else:
            raise ValueError(f"bad symbol {t}")
    if len(stack) != 1:
        raise ValueError(f"program leaves {len(stack)} values on the stack")
    return stack[0]


def tree_height(node) -> int:
    kids = node[2:]
    return 0 if not kids else 1 + max(tree_height(k) for k in kids)


def decode_one(ops_row, consts_row, height: int):
    T = 2 ** (height + 1) - 1
    genes = np.full(T, PAD, dtype=np.int8)
    gc = np.zeros(T, dtype=np.float32)
    root = parse(ops_row, consts_row)
    if tree_height(root) > height:
        raise ValueError("program is taller than the template")

    def place(node, i):
        genes[i] = node[0]
        gc[i] = node[1]
        for c, kid in enumerate(node[2:]):
            place(kid, 2 * i + 1 + c)

    place(root, 0)
    return genes, gc


def decode(ops, consts, height: int):
    """Batch decoder: genes int8 [M, 2^(h+1)-1], gene constants float32."""
    M = ops.shape[0]
    T = 2 ** (height + 1) - 1
    genes = np.full((M, T), PAD, dtype=np.int8)
    gc = np.zeros((M, T), dtype=np.float32)
    for m in range(M):
        genes[m], gc[m] = decode_one(ops[m], consts[m], height)
    return genes, gc


def infix(ops_row, consts_row) -> str:
    """Readable infix string of a postfix program (for messages)."""
    def show(n):
        s = n[0]
        if s == O.CONST:
            return repr(n[1])
        if s >= O.VAR0:
            return f"x{s - O.VAR0}"
        kids = [show(k) for k in n[2:]]
        if len(kids) == 2 and s in (O.ADD, O.SUB, O.MUL, O.DIV):
            return f"({kids[0]} {O.NAMES[s]} {kids[1]})"
        return f"{O.NAMES[s]}({', '.join(kids)})"
    return show(parse(ops_row, consts_row))
