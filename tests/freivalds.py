"""Freivalds' check of a whole product, with the oracle as the checker.

For a seeded x in [0, p)^n the oracle forms A (B x) and C x mod p (products
with a single column, O(mk + kn + mn) work) and they must agree.  A row of C
with a wrong entry passes one trial with probability at most 1/p (p prime).
"""
import numpy as np

import mmp_inputs as gen
import oracle


def check(p, A, B, C, seed, trials=2):
    """Raises AssertionError naming the first row of C that fails."""
    C = np.asarray(C)
    n = C.shape[1]
    for t in range(trials):
        x = gen.uniform_mod(seed, 90 + t, n, p).reshape(n, 1)
        lhs = oracle.mm_modp(p, A, oracle.mm_modp(p, B, x))
        rhs = oracle.mm_modp(p, C, x)
        bad = np.nonzero(lhs[:, 0] != rhs[:, 0])[0]
        assert bad.size == 0, f"Freivalds trial {t}: {bad.size} rows of C wrong, first row {bad[0]}"
