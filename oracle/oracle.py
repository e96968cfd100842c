"""ctypes wrapper of bi_oracle.c (test infrastructure only; see bi_oracle.c)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bi_oracle.c")
_LIB = os.path.join(_HERE, "_bi_oracle.so")

OP_C, OP_EM, OP_BOTH = 0, 1, 8
PRIM = {"T": 2, "K": 3, "Tx": 4, "Kx": 5, "Gram": 6, "Gx": 7}
KERNELS = {"full": 0, "static": 1, "sin": 2}

_lib = None


def build():
    """Compile the oracle (gcc, OpenMP, IEEE double arithmetic)."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                           "-o", _LIB + ".tmp", _SRC, "-lm"])
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_rwg.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P]
        lib.oracle_pair.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int, P]
        lib.oracle_pair_sub.argtypes = [P, P, P, P, ctypes.c_double, P, P]
        lib.oracle_matvec.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, P, P, ctypes.c_int, P, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int]
        lib.oracle_boxes.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, P, P]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_class_box_pairs.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, P, ctypes.c_int]
        lib.oracle_far_field.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P,
                                         ctypes.c_int, P, P]
        lib.oracle_entries.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P, P]
        lib.oracle_plane_wave_rhs.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                              P, P, P]
        _lib = lib
    return _lib


def _mesh(verts, tris):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    return v, t


def threads():
    return _load().oracle_threads()


def rwg_table(verts, tris):
    """(edges (N,2) with a < b, tri_pm (N,2) = (T+, T-))."""
    v, t = _mesh(verts, tris)
    n = 3 * len(t) // 2
    e = np.zeros((n, 2), np.int32)
    pm = np.zeros((n, 2), np.int32)
    rc = _load().oracle_rwg(len(v), v.ctypes.data, len(t), t.ctypes.data, e.ctypes.data, pm.ctypes.data)
    if rc < 0:
        raise ValueError("oracle rejected the mesh (code %d)" % rc)
    return e[:rc], pm[:rc]


def entries(verts, tris, k, pairs):
    """Primitive entries of RWG pairs (test m, source n) = rows of `pairs`
    (npairs, 2): array (npairs, 6) complex with columns T, K, Tx, Kx, Gram, Gx."""
    v, t = _mesh(verts, tris)
    pr = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    out = np.zeros((len(pr), 6), np.complex128)
    rc = _load().oracle_entries(len(v), v.ctypes.data, len(t), t.ctypes.data, k, len(pr), pr.ctypes.data,
                                out.ctypes.data)
    if rc < 0:
        raise ValueError("oracle_entries failed (code %d)" % rc)
    return out


def blocks(E, op=OP_C):
    """2 x 2 blocks [[JJ, JM], [MJ, MM]] of each pair, shape (npairs, 2, 2),
    from primitive entries E (npairs, 6).  op C: eqs. 43-46 with alpha = 1/2;
    op EM: [[T, -K], [K, T]] (eqs. 22/24)."""
    T, K, Tx, Kx, G, Gx = (E[:, i] for i in range(6))
    if op == OP_C:
        b = [[G - T / 2 - Kx / 2, Gx / 2 - Tx / 2 + K / 2], [Tx / 2 - K / 2, G / 2 - T / 2 - Kx / 2]]
    elif op == OP_EM:
        b = [[T, -K], [K, T]]
    else:
        raise ValueError("op must be OP_C or OP_EM")
    return np.stack([np.stack(r, axis=-1) for r in b], axis=-2)


def plane_wave_rhs(verts, tris, k, khat, pol):
    """[b^J; b^M] of eqs. 49-50 for plane waves (khat, pol: (nrhs, 3)); (2N, nrhs)."""
    v, t = _mesh(verts, tris)
    kh = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
    po = np.ascontiguousarray(np.atleast_2d(pol), np.float64)
    N = 3 * len(t) // 2
    out = np.zeros((len(kh), 2 * N), np.complex128)
    rc = _load().oracle_plane_wave_rhs(len(v), v.ctypes.data, len(t), t.ctypes.data, k, len(kh), kh.ctypes.data,
                                       po.ctypes.data, out.ctypes.data)
    if rc < 0:
        raise ValueError("oracle rejected the mesh (code %d)" % rc)
    return out.T


def far_field(verts, tris, k, x, dirs):
    """(F . theta_hat, F . phi_hat) of the far field of the currents x
    (2N x nrhs, J rows then M rows) in the directions dirs (ndir x 3):
    array (ndir, 2, nrhs).  F = (-jk/4pi)[P_J - khat(khat.P_J) - khat x P_M]."""
    v, t = _mesh(verts, tris)
    X = np.asfortranarray(np.atleast_2d(np.asarray(x, np.complex128).T).T)
    d = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
    out = np.zeros((len(d), 2, X.shape[1]), np.complex128)
    rc = _load().oracle_far_field(len(v), v.ctypes.data, len(t), t.ctypes.data, k, X.shape[1], X.ctypes.data,
                                  len(d), d.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_far_field failed (%d)" % rc)
    return out


def leaf_boxes(verts, tris, leaf):
    v, t = _mesh(verts, tris)
    n = 3 * len(t) // 2
    coords = np.zeros((n, 3), np.int32)
    lev = ctypes.c_int(0)
    rc = _load().oracle_boxes(len(v), v.ctypes.data, len(t), t.ctypes.data, leaf, coords.ctypes.data,
                              ctypes.byref(lev))
    if rc < 0:
        raise ValueError("oracle rejected the mesh (code %d)" % rc)
    return coords, lev.value


def class_box_pairs(verts, tris, leaf):
    """{level: number of distinct ordered box pairs (A, B) at that level that
    hold an RWG pair of that interaction class} for levels >= 2."""
    v, t = _mesh(verts, tris)
    out = np.zeros(32, np.int64)
    rc = _load().oracle_class_box_pairs(len(v), v.ctypes.data, len(t), t.ctypes.data, leaf, out.ctypes.data, 32)
    if rc < 0:
        raise ValueError("oracle rejected the mesh (code %d)" % rc)
    return {l: int(out[l]) for l in range(2, rc)}


def pair_integrals(ti, P, si, Q, k, nq=0, kernel="full", return_order=False):
    """Local 4x3x3 integrals (T, K, Tx, Kx) of one triangle pair without RWG
    coefficients; vertex ids ti/si decide which vertices are shared.
    nq = 0 selects the converged order search (the order used is returned
    with return_order=True)."""
    ti = np.ascontiguousarray(ti, np.int32)
    si = np.ascontiguousarray(si, np.int32)
    P = np.ascontiguousarray(P, np.float64)
    Q = np.ascontiguousarray(Q, np.float64)
    out = np.zeros(72, np.float64)
    rc = _load().oracle_pair(ti.ctypes.data, P.ctypes.data, si.ctypes.data, Q.ctypes.data,
                             KERNELS[kernel], k, nq, out.ctypes.data)
    if rc < 0 and nq > 0:
        raise ValueError("bad arguments")
    res = (out[0::2] + 1j * out[1::2]).reshape(4, 3, 3)
    return (res, rc) if return_order else res


# Test-triangle and remainder rules of the singularity-subtraction route:
# grading ratio, levels and points towards the singular set, points and
# levels along the sweep base, remainder points per source-triangle axis.
SUB_DEFAULT = (0.35, 24, 10, 6, 8, 12)


def pair_integrals_sub(ti, P, si, Q, k, params=SUB_DEFAULT):
    """Local 4x3x3 integrals (T, K, Tx, Kx) of one touching triangle pair by
    the second route: singularity subtraction with closed-form static
    integrals over the source triangle and graded Gauss rules over the test
    triangle (independent of pair_integrals' relative-coordinate rules).
    params = (sigma, levels, n, n_inner, n_s, s_levels)."""
    ti = np.ascontiguousarray(ti, np.int32)
    si = np.ascontiguousarray(si, np.int32)
    P = np.ascontiguousarray(P, np.float64)
    Q = np.ascontiguousarray(Q, np.float64)
    pr = np.ascontiguousarray(params, np.float64)
    out = np.zeros(72, np.float64)
    rc = _load().oracle_pair_sub(ti.ctypes.data, P.ctypes.data, si.ctypes.data, Q.ctypes.data, k, pr.ctypes.data,
                                 out.ctypes.data)
    if rc < 0:
        raise ValueError("bad arguments")
    return (out[0::2] + 1j * out[1::2]).reshape(4, 3, 3)


def matvec(verts, tris, k, x, op=OP_C, rows=None, leaf=None, nq=0, classes=False, route="duffy"):
    """Dense Galerkin product.

    x: (2N, nrhs) or (2N,) complex.  Returns y with shape (2*len(rows), nrhs)
    (or (2N, nrhs)); rows [0, nr) are J/E-tested, [nr, 2nr) are M/H-tested.
    op: OP_C, OP_EM, OP_BOTH (returns the pair (y_C, y_EM)), or a key of PRIM
    (then only the J half of x is used and only the J half of y is filled).
    With classes=True (needs leaf), returns (ncls, 2nr, nrhs): class 0 is the
    near part (leaf boxes adjacent), class l >= 2 the part translated at level l.
    route: "duffy" (relative-coordinate transformations, order search or the
    fixed order nq) or "subtraction" (pair_integrals_sub) for the triangle
    pairs that share a vertex, an edge or the triangle.
    """
    if route == "subtraction":
        nq = -1
    elif route != "duffy":
        raise ValueError("route must be 'duffy' or 'subtraction'")
    v, t = _mesh(verts, tris)
    N = 3 * len(t) // 2
    x = np.asarray(x, dtype=np.complex128)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[:, None]
    if x.shape[0] != 2 * N:
        raise ValueError("x must have 2N rows")
    nrhs = x.shape[1]
    xf = np.asfortranarray(x)
    opcode = PRIM[op] if isinstance(op, str) else int(op)
    if rows is None:
        rows_arr, nr = None, N
    else:
        rows_arr = np.ascontiguousarray(rows, np.int32)
        nr = len(rows_arr)
    if leaf is not None:
        levels = leaf_boxes(verts, tris, leaf)[1]
        ncls = max(levels, 1)
    else:
        ncls = 1
    nops = 2 if opcode == OP_BOTH else 1
    y = np.zeros((nops * ncls, nrhs, 2 * nr), np.complex128)
    rc = _load().oracle_matvec(len(v), v.ctypes.data, len(t), t.ctypes.data, k, opcode, nrhs,
                               xf.ctypes.data, None if rows_arr is None else rows_arr.ctypes.data,
                               nr, y.ctypes.data, -1.0 if leaf is None else float(leaf), ncls, nq)
    if rc < 0:
        raise ValueError("oracle_matvec failed (code %d)" % rc)
    y = np.transpose(y, (0, 2, 1))           # (nops*ncls, 2nr, nrhs)
    res = []
    for o in range(nops):
        yo = y[o * ncls:(o + 1) * ncls]
        if not classes:
            yo = yo.sum(axis=0)
            if squeeze:
                yo = yo[:, 0]
        elif squeeze:
            yo = yo[:, :, 0]
        res.append(yo)
    return tuple(res) if nops == 2 else res[0]
