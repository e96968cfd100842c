"""Sparse approximate inverse (SAI) of the BI block's near field, written
plainly (test infrastructure only: only tests may import it; it shares no
code with the GPU library).

The paper preconditions GMRES with an SAI built from the BI block C alone
(Sec. III, dielectric-plate example, citing Lee et al. 2004) and gives no
formula; the reading used here is the Frobenius-norm SAI of those
references restricted to the near field:

  * C_near = the entries of C (eqs. 43-46, alpha = 1/2) of the RWG pairs
    whose leaf boxes are at Chebyshev distance <= 1 (the near-field part
    the MLFMA stores), all other entries zero;
  * pattern(n) = the k RWGs nearest to RWG n (centres = edge midpoints)
    among those whose leaf box is adjacent to n's, every RWG tied with the
    k-th distance (relative 1e-9) included; both halves (J, M) of each;
  * the columns (n, J) and (n, M) of the preconditioner M solve
    min || C_near m - e ||_2 over vectors m supported on pattern(n), so that
    || I - C_near M ||_F is minimal column by column.

Everything is dense numpy on small meshes; the least-squares problems use
numpy's lstsq (an SVD), over all rows of C_near.
"""
import numpy as np

from . import oracle as _o

TIE = 1e-9


def _centres(verts, tris):
    e, _ = _o.rwg_table(verts, tris)
    v = np.asarray(verts, np.float64)
    return 0.5 * (v[e[:, 0]] + v[e[:, 1]])


def pattern(verts, tris, leaf, k_nearest, rwgs=None):
    """Pattern (sorted RWG indices) of every RWG in rwgs (default: all)."""
    coords, _ = _o.leaf_boxes(verts, tris, leaf)
    c = _centres(verts, tris)
    N = len(c)
    out = []
    for n in (range(N) if rwgs is None else rwgs):
        cand = np.nonzero(np.max(np.abs(coords - coords[n]), axis=1) <= 1)[0]
        d = c[cand] - c[n]
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        if len(cand) <= k_nearest:
            out.append(np.sort(cand))
            continue
        kth = np.sort(d2)[k_nearest - 1]
        out.append(np.sort(cand[d2 <= kth * (1 + TIE)]))
    return out


def near_columns(verts, tris, k, leaf, cols, op=_o.OP_C):
    """Columns `cols` (RWG indices) of C_near, both halves: dense array
    (2N, 2 len(cols)) with column 2 i + h = unknown (cols[i], h), h = 0 (J)
    or 1 (M); rows J of all RWGs, then M."""
    coords, _ = _o.leaf_boxes(verts, tris, leaf)
    N = len(coords)
    pairs = []
    for p in cols:
        rows = np.nonzero(np.max(np.abs(coords - coords[p]), axis=1) <= 1)[0]
        pairs += [(m, p) for m in rows]
    pairs = np.array(pairs, np.int32).reshape(-1, 2)
    B = _o.blocks(_o.entries(verts, tris, k, pairs), op)
    pos = {p: i for i, p in enumerate(cols)}
    A = np.zeros((2 * N, 2 * len(cols)), np.complex128)
    for (m, p), blk in zip(pairs, B):
        i = pos[p]
        for hr in range(2):
            for hc in range(2):
                A[hr * N + m, 2 * i + hc] = blk[hr, hc]
    return A


def columns(verts, tris, k, leaf, k_nearest, rwgs, op=_o.OP_C):
    """SAI columns (n, J) and (n, M) for each n in rwgs: dense (2N, 2 len(rwgs)),
    column 2 i + h = unknown (rwgs[i], h)."""
    pats = pattern(verts, tris, leaf, k_nearest, rwgs)
    N = 3 * len(tris) // 2
    union = sorted(set(int(p) for P in pats for p in P))
    pos = {p: i for i, p in enumerate(union)}
    A_all = near_columns(verts, tris, k, leaf, union, op)        # (2N, 2 |union|)
    out = np.zeros((2 * N, 2 * len(rwgs)), np.complex128)
    for i, (n, P) in enumerate(zip(rwgs, pats)):
        sel = [2 * pos[int(p)] + h for p in P for h in range(2)]
        A = A_all[:, sel]                                         # (2N, 2|P|), column 2 j + h
        E = np.zeros((2 * N, 2), np.complex128)
        E[n, 0] = 1
        E[N + n, 1] = 1
        sol = np.linalg.lstsq(A, E, rcond=None)[0]                # (2|P|, 2)
        for j, p in enumerate(P):
            for hc in range(2):
                out[hc * N + p, 2 * i:2 * i + 2] = sol[2 * j + hc]
    return out
