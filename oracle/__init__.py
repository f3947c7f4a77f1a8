"""Plain, slow, float64 CPU oracle for GP-GOMEA fitness evaluation.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code, table or constant with the HIP library;
it is written from the paper and from the stated readings of the points the
paper leaves open.

Modules
-------
opset    symbol codes and protected operator semantics in float64
tree     active-node set and recursive tree walk over heap-ordered genotypes
codec    genotype <-> postfix (Reverse Polish) encoder / decoder
fitness  MSE (Eq. 1), NMSE (Eq. 2) and the linearly scaled MSE
grad     d(fitness)/d(constants) by forward-mode dual numbers; central FD
mca      Monte-Carlo-arithmetic conditioning flags (which results are gradeable)

Pins: every function is checked in ``tests/test_oracle_*.py`` against values
fixed by the paper (the Fig. 1 worked example), closed forms, invariants and
brute force.  The protected-operator constants are a reading (the paper never
defines protection), so their values are "parity unpinned" in the sense that
nothing in the paper fixes them; their invariants (guards, clamps) are pinned.
"""
from . import opset, tree, codec, fitness, grad, mca  # noqa: F401
