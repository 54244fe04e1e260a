"""Chinese remainder reconstruction and the product counts of Section 5.2.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the GPU
library or its Python binding, and nothing here imports them.

Section 5.2 (the comparison with multimodular approaches) computes the
products A_i B_i modulo coprime moduli m_1 ... m_s and recovers the integer
product by the Chinese remainder theorem: there is a unique C with entries in
[0, M), M = m_1 ... m_s, such that C = A B mod M, and when M exceeds
k (p - 1)^2 (eq. CRT2) that C is the integer product itself.

* ``crt_reconstruct``: that unique integer for one entry, written as the
  textbook sum X = sum_i r_i M_i (M_i^{-1} mod m_i) mod M with M_i = M / m_i,
  in Python integers.
* ``crt_matrix``: the same for every entry of s residue matrices.
* ``moduli_needed``: the shortest prefix of a list of moduli whose product
  exceeds k (2^bits - 1)^2, the bound of eq. CRT2 for entries below 2^bits.
* ``numprod_mm``: eq. numprodMM, the least number of moduli (hence products)
  of the multimodular approach.
* ``numprod_mw``: the least uv over the word pairs whose uv satisfies eq.
  numprodMW's relation uv >= (u + v) log2(p) / (t - log2(lambda)) (the
  paper's count with the p - 1 term neglected).
"""

from __future__ import annotations

import math

import numpy as np

T_BITS = 53

# The word pairs of Section 3.3 (Table tab.summary and their transposes).
WORD_PAIRS = [(1, 1), (1, 2), (2, 1), (1, 3), (3, 1), (1, 4), (4, 1), (2, 2), (2, 3), (3, 2)]


def crt_reconstruct(residues, moduli) -> int:
    """The unique X in [0, prod(moduli)) with X = residues[i] mod moduli[i]."""
    moduli = [int(m) for m in moduli]
    residues = [int(r) for r in residues]
    if len(moduli) != len(residues) or not moduli:
        raise ValueError("one residue per modulus")
    for i in range(len(moduli)):
        for j in range(i + 1, len(moduli)):
            if math.gcd(moduli[i], moduli[j]) != 1:
                raise ValueError("moduli must be pairwise coprime")
    M = 1
    for m in moduli:
        M *= m
    X = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        X += r * Mi * pow(Mi, -1, m)
    return X % M


def crt_matrix(residue_matrices, moduli) -> np.ndarray:
    """Entry-wise crt_reconstruct of s equally shaped residue matrices;
    returns an object array of Python integers."""
    mats = [np.asarray(c) for c in residue_matrices]
    shape = mats[0].shape
    out = np.empty(shape, dtype=object)
    for idx in np.ndindex(shape):
        out[idx] = crt_reconstruct([int(c[idx]) for c in mats], moduli)
    return out


def moduli_needed(moduli, k: int, bits: int) -> int:
    """Length of the shortest prefix of ``moduli`` whose product exceeds
    k (2^bits - 1)^2 (eq. CRT2 for entries below 2^bits); 0 if none does."""
    bound = int(k) * ((1 << bits) - 1) ** 2
    M = 1
    for i, m in enumerate(moduli):
        M *= int(m)
        if M > bound:
            return i + 1
    return 0


def numprod_mm(log2p: float, k: int, lam: int, t: int = T_BITS) -> int:
    """eq. numprodMM: s = ceil((4 log2 p + 2 log2 k) / (t - log2 lambda))."""
    return math.ceil((4.0 * log2p + 2.0 * math.log2(k)) / (t - math.log2(lam)))


def numprod_mw(log2p: float, lam: int, t: int = T_BITS) -> int:
    """Least uv over WORD_PAIRS with uv >= (u + v) log2 p / (t - log2 lambda)
    (eq. numprodMW, the p - 1 term neglected); 0 if no pair qualifies."""
    best = 0
    for u, v in WORD_PAIRS:
        if u * v >= (u + v) * log2p / (t - math.log2(lam)) and (best == 0 or u * v < best):
            best = u * v
    return best
