"""Pins of the oracle's SAI preconditioner and RWG-pair entries (CPU).

The paper builds its SAI preconditioner from the BI block C alone (Sec.
III, dielectric-plate example) and gives no formula; the oracle takes the
Frobenius-norm definition of the cited SAI literature over the near field.
These tests pin that definition by what the mathematics fixes: the pair
entries against the product oracle's near part, the least-squares optimality
(normal equations) of every column against an independently assembled
C_near, the inverse when the pattern is everything, and the nearest-RWG
pattern against its defining property.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import sai

K0 = 2 * np.pi
LEAF = 0.25


def _dense_classes(v, t, op):
    """Near part (class 0) and whole matrix of op, column by column from
    the product oracle; columns in the product's order (J of all RWGs, then M)."""
    N = 3 * len(t) // 2
    X = np.eye(2 * N, dtype=complex)
    y = oracle.matvec(v, t, K0, X, op=op, leaf=LEAF, classes=True)
    return y[0], y.sum(axis=0)


def _to_pair_order(A, N):
    """Reorder columns (h N + i) -> (2 i + h)."""
    return A[:, [h * N + i for i in range(N) for h in range(2)]]


@pytest.fixture(scope="module")
def small():
    v, t = synth.icosphere(2, 0.5)          # 80 triangles, N = 120, 3 levels at leaf 0.25
    N = 3 * len(t) // 2
    near_c, full_c = _dense_classes(v, t, oracle.OP_C)
    return v, t, N, near_c, full_c


def test_entries_match_product_near_part(small):
    """oracle_entries summed per RWG pair (op C blocks, eqs. 43-46) equals the
    product oracle's near class applied to unit vectors; the near part is a
    strict part of the whole matrix on this mesh."""
    v, t, N, near_c, full_c = small
    cols = list(range(0, N, 6))
    A = sai.near_columns(v, t, K0, LEAF, cols)
    ref = _to_pair_order(near_c, N)[:, [2 * i + h for i in cols for h in range(2)]]
    assert np.abs(A - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.linalg.norm(full_c - near_c) > 1e-3 * np.linalg.norm(full_c)


def test_entries_em_blocks():
    """op EM blocks [[T, -K], [K, T]] from the entries equal the product
    oracle's op EM on unit vectors (tiny mesh, every pair near)."""
    v, t = synth.octahedron(0.1)
    N = 3 * len(t) // 2
    pairs = np.array([(m, n) for m in range(N) for n in range(N)], np.int32)
    B = oracle.blocks(oracle.entries(v, t, K0, pairs), oracle.OP_EM)
    X = np.eye(2 * N, dtype=complex)
    ref = oracle.matvec(v, t, K0, X, op=oracle.OP_EM)
    for (m, n), blk in zip(pairs, B):
        for hr in range(2):
            for hc in range(2):
                assert abs(blk[hr, hc] - ref[hr * N + m, hc * N + n]) <= 1e-14 * np.abs(ref).max()


def test_pattern_defining_property(small):
    """pattern(n) holds n, lies in leaf boxes adjacent to n's, has at least k
    members (or every candidate), and every candidate left out is farther
    than every member."""
    v, t, N, _, _ = small
    coords, _ = oracle.leaf_boxes(v, t, LEAF)
    e, _ = oracle.rwg_table(v, t)
    c = 0.5 * (v[e[:, 0]] + v[e[:, 1]])
    for k in (1, 6, 16):
        pats = sai.pattern(v, t, LEAF, k)
        for n, P in enumerate(pats):
            cand = set(np.nonzero(np.max(np.abs(coords - coords[n]), axis=1) <= 1)[0])
            assert n in P and set(P) <= cand
            assert len(P) >= min(k, len(cand))
            dist = np.linalg.norm(c - c[n], axis=1)
            out = cand - set(P)
            if out:
                assert min(dist[list(out)]) > max(dist[P]) * (1 + 1e-12)


def test_sai_columns_satisfy_normal_equations(small):
    """Each SAI column m minimises ||C_near m - e||: it vanishes off the
    pattern and the residual is orthogonal to the pattern's columns of
    C_near (assembled independently, by the product oracle)."""
    v, t, N, near_c, _ = small
    rwgs = [0, 17, 59, 119]
    k = 6
    M = sai.columns(v, t, K0, LEAF, k, rwgs)
    pats = sai.pattern(v, t, LEAF, k, rwgs)
    for i, (n, P) in enumerate(zip(rwgs, pats)):
        sup = np.concatenate([P, N + np.asarray(P)])
        off = np.setdiff1d(np.arange(2 * N), sup)
        for h in range(2):
            m = M[:, 2 * i + h]
            assert np.all(m[off] == 0)
            e = np.zeros(2 * N, complex)
            e[h * N + n] = 1
            r = near_c @ m - e
            g = near_c[:, sup].conj().T @ r
            assert np.abs(g).max() <= 1e-10 * np.linalg.norm(near_c[:, sup], 2) * np.linalg.norm(r)
            # and strictly better than the unpreconditioned column e itself
            assert np.linalg.norm(r) < np.linalg.norm(near_c @ e - e)


def test_full_pattern_gives_the_inverse():
    """With every RWG near and in the pattern, the SAI is C^-1 exactly."""
    v, t = synth.octahedron(0.1)
    N = 3 * len(t) // 2
    X = np.eye(2 * N, dtype=complex)
    C = oracle.matvec(v, t, K0, X, op=oracle.OP_C)
    M = sai.columns(v, t, K0, LEAF, N, list(range(N)))
    Mp = np.zeros_like(M)
    for i in range(N):
        for h in range(2):
            Mp[:, h * N + i] = M[:, 2 * i + h]
    assert np.abs(C @ Mp - np.eye(2 * N)).max() <= 1e-9
