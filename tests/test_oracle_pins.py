"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test names the passage of arXiv 2210.04892 or the identity it rests on.
Together they are chosen so that a dropped term, a wrong sign, a wrong
Jacobian or a transposed operand anywhere in the oracle fails one of them.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from pinmath import (K0, tri_area, tri_normal, tri_gauss, tri_radon7, linear_moment, potential,
                     sph_j1, sph_y1, sphere_rule, rwg_coefficients)

# two fixed, well-shaped but non-symmetric triangles sharing an edge (v0, v1)
V0 = np.array([0.0, 0.0, 0.0])
V1 = np.array([0.1, 0.0, 0.0])
VA = np.array([0.03, 0.08, 0.01])
VB = np.array([0.05, -0.07, 0.03])
VC = np.array([-0.06, 0.02, 0.05])
CASES = {
    "coincident": ([0, 1, 2], np.array([V0, V1, VA]), [0, 1, 2], np.array([V0, V1, VA])),
    "edge": ([0, 1, 2], np.array([V0, V1, VA]), [1, 0, 3], np.array([V1, V0, VB])),
    "edge_coplanar": ([0, 1, 2], np.array([V0, V1, [0.03, 0.08, 0]]), [1, 0, 3],
                      np.array([V1, V0, [0.05, -0.07, 0]])),
    "vertex": ([0, 1, 2], np.array([V0, V1, VA]), [3, 4, 0], np.array([VB, VC, V0])),
}


def _dense(verts, tris, op):
    """Primitive matrix from the oracle, column by column (tiny meshes)."""
    N = 3 * len(tris) // 2
    X = np.zeros((2 * N, N), complex)
    X[:N] = np.eye(N)
    return oracle.matvec(verts, tris, K0, X, op=op)[:N]


# ------------------------------------------------------------------ RWG / mesh
def test_rwg_convention_tetrahedron():
    """RWG table convention: edges (a<b) in lexicographic order, T+ holds a->b
    counter-clockwise (reading of the RWG pairs of the weak forms eqs. 32-33)."""
    v, t = synth.tetrahedron()
    e, pm = oracle.rwg_table(v, t)
    assert len(e) == 6
    assert [tuple(x) for x in e] == sorted(tuple(x) for x in e)
    assert np.all(e[:, 0] < e[:, 1])
    for (a, b), (tp, tm) in zip(e, pm):
        cyc = lambda tr: [(tr[i], tr[(i + 1) % 3]) for i in range(3)]
        assert (a, b) in cyc(list(t[tp]))
        assert (b, a) in cyc(list(t[tm]))


def test_mesh_rejections():
    v, t = synth.octahedron()
    flipped = t.copy()
    flipped[0] = flipped[0][::-1]
    with pytest.raises(ValueError):
        oracle.rwg_table(v, flipped)           # inconsistent orientation
    with pytest.raises(ValueError):
        oracle.rwg_table(v, t[:, ::-1])        # inward normals
    with pytest.raises(ValueError):
        oracle.rwg_table(v, t[:-1])            # open surface


def test_disconnected_surfaces():
    """Disconnected scatterers in one mesh (Sec. II-E remarks: BI equations
    on each surface): accepted when every closed surface is outward; one
    inward surface is rejected even where the total enclosed volume is
    positive.  RWGs never join two surfaces."""
    a = synth.icosphere(2, 0.5)
    b = synth.octahedron(0.2)
    v, t = synth.scene((a[0], a[1], (0, 0, 0)), (b[0], b[1], (1.5, 0, 0)))
    e, pm = oracle.rwg_table(v, t)
    na = len(a[1])
    assert len(e) == 3 * len(t) // 2
    assert np.all((pm[:, 0] < na) == (pm[:, 1] < na))
    v2, t2 = synth.scene((a[0], a[1], (0, 0, 0)), (b[0], b[1][:, ::-1], (1.5, 0, 0)))
    with pytest.raises(ValueError):
        oracle.rwg_table(v2, t2)


# ------------------------------------------------------------------ P-H Gram
@pytest.mark.parametrize("mesh", [synth.tetrahedron, synth.octahedron, synth.icosahedron])
def test_gram_closed_form(mesh):
    """Gram and twisted Gram (identity terms of eqs. 43, 44, 46) against the
    exact moments of linear functions over a triangle."""
    v, t = mesh()
    e, pm = oracle.rwg_table(v, t)
    N = len(e)
    co = rwg_coefficients(v, t, e, pm)
    G = np.zeros((N, N))
    Gx = np.zeros((N, N))
    for m in range(N):
        for n in range(N):
            for tm_, pmv, cm in co[m]:
                for tn_, pnv, cn in co[n]:
                    if tm_ != tn_:
                        continue
                    P = v[t[tm_]]
                    G[m, n] += cm * cn * linear_moment(P, pmv, pnv)
                    Gx[m, n] += cm * cn * linear_moment(P, pmv, pnv, twist=tri_normal(P))
    Go = _dense(v, t, "Gram")
    Gxo = _dense(v, t, "Gx")
    assert np.abs(Go - G).max() <= 1e-13 * np.abs(G).max()
    assert np.abs(Gxo - Gx).max() <= 1e-13 * np.abs(G).max()
    assert np.all(np.linalg.eigvalsh(G) > 0)


# ---------------------------------------------- transformations (smooth kernel)
def _product_rule_sin(P, Q, k=K0, n=22):
    """Reference local integrals with the entire kernel sin(kR)/(4 pi R) by
    a plain product Gauss rule over the two triangles."""
    x, wx = tri_gauss(P, n)
    y, wy = tri_gauss(Q, n + 1)
    nt = tri_normal(P)
    d = x[:, None, :] - y[None, :, :]
    R = np.linalg.norm(d, axis=2)
    G = np.sin(k * R) / (4 * np.pi * R)
    g1 = (k * R * np.cos(k * R) - np.sin(k * R)) / (4 * np.pi * R ** 3)
    W = wx[:, None] * wy[None, :]
    gG = g1[..., None] * d
    out = np.zeros((4, 3, 3), complex)
    for i in range(3):
        a = x - P[i]
        g = np.cross(nt, a)
        for j in range(3):
            b = y - Q[j]
            c = np.cross(gG, b[None, :, :])
            out[0, i, j] = np.sum(W * (-1j * k * (a @ b.T - 4 / k ** 2) * G))
            out[1, i, j] = np.sum(W * np.einsum("pc,pqc->pq", a, c))
            out[2, i, j] = np.sum(W * (-(-1j * k * (g @ b.T) * G - (2j / k) * np.einsum("pc,pqc->pq", g, gG))))
            out[3, i, j] = np.sum(W * (-np.einsum("pc,pqc->pq", g, c)))
    return out


@pytest.mark.parametrize("case", ["coincident", "edge", "edge_coplanar", "vertex"])
def test_touching_transformations_exact_for_smooth_kernel(case):
    """The relative-coordinate transformations of touching pairs are exact
    changes of variables: with an entire kernel they reproduce a plain
    product rule to rounding (pins every Jacobian and sub-domain)."""
    ti, P, si, Q = CASES[case]
    ref = _product_rule_sin(P, Q)
    got = oracle.pair_integrals(ti, P, si, Q, K0, nq=14, kernel="sin")
    for op in range(4):
        if case == "coincident" and op in (1, 3):
            continue          # set to zero by definition on a flat triangle
        assert np.abs(got[op] - ref[op]).max() <= 1e-12 * np.abs(ref[0]).max(), op


# ------------------------------------------------ static singular closed forms
def _split_static(ti, P, si, Q):
    """Separate the two parts of the static-kernel T and Tx entries using two
    wavenumbers: T/(-jk) = S_ab - 4 S_1 / k^2 and Tx/j = k U + (2/k) V."""
    k1, k2 = 1.0, 3.0
    o1 = oracle.pair_integrals(ti, P, si, Q, k1, kernel="static")
    o2 = oracle.pair_integrals(ti, P, si, Q, k2, kernel="static")
    X1, X2 = o1[0] / (-1j * k1), o2[0] / (-1j * k2)
    S1 = (X1 - X2) / (4 / k2 ** 2 - 4 / k1 ** 2)
    Y1, Y2 = o1[2] / 1j, o2[2] / 1j
    # [k1 2/k1; k2 2/k2] [U V]^T = [Y1 Y2]^T
    det = k1 * 2 / k2 - k2 * 2 / k1
    V = (k1 * Y2 - k2 * Y1) / det
    return S1.real, V.real


def _outer_potential(P, Q):
    """Int_P Int_Q 1/(4 pi R): closed-form inner potential, adaptive outer."""
    A2 = 2 * tri_area(P)
    f = lambda v_, u_: potential(P[0] + u_ * (P[1] - P[0]) + v_ * (P[2] - P[0]), Q)
    val, _ = integrate.dblquad(f, 0, 1, 0, lambda u_: 1 - u_, epsabs=0, epsrel=1e-12)
    return val * A2 / (4 * np.pi)


def _contour_potential(P, Q, i):
    """Int_P g_i . grad Phi_Q dA = sum over edges of P of Int Phi_Q (g_i . nu) dl
    (divergence theorem; the surface divergence of n x (r - p_i) vanishes)."""
    n = tri_normal(P)
    tot = 0.0
    for e in range(3):
        A, B = P[e], P[(e + 1) % 3]
        L = np.linalg.norm(B - A)
        nu = np.cross(B - A, n) / L                      # outward in-plane normal
        f = lambda s: potential(A + s * (B - A), Q) * np.dot(np.cross(n, A + s * (B - A) - P[i]), nu)
        val, _ = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=200)
        tot += val * L
    return tot / (4 * np.pi)


def test_potential_closed_form_is_right():
    """The closed-form potential used below against brute force off the triangle."""
    Q = CASES["edge"][3]
    for x in ([0.05, 0.03, 0.2], [0.3, -0.2, -0.05], [0.02, 0.01, 0.015]):
        y, w = tri_gauss(Q, 120)
        brute = np.sum(w / np.linalg.norm(y - np.array(x), axis=1))
        assert abs(potential(x, Q) - brute) <= 1e-10 * abs(brute)


@pytest.mark.parametrize("case", ["coincident", "edge", "edge_coplanar", "vertex"])
def test_static_singular_integrals(case):
    """Singular parts of touching pairs against closed forms: the 1/R double
    integral and the 1/R^2 (grad G) term of Tx reduced to a contour integral."""
    ti, P, si, Q = CASES[case]
    S1, V = _split_static(ti, P, si, Q)
    ref1 = _outer_potential(P, Q)
    assert np.abs(S1 - ref1).max() <= 1e-9 * abs(ref1)
    for i in range(3):
        refV = _contour_potential(P, Q, i)
        assert np.abs(V[i] - refV).max() <= 1e-8 * abs(ref1) * 10, (i, V[i], refV)


# ------------------------------------------------------------- P-G coplanar
def test_coplanar_K_vanishes():
    """K and Kx vanish for coplanar triangle pairs: (x - y) x f_n is normal to
    the plane while f_m and n x f_m are tangential (flat-plate pairs)."""
    v, t = synth.flat_plate(0.3, 3)
    for si in range(len(t)):
        o = oracle.pair_integrals(t[0], v[t[0]], t[si], v[t[si]], K0)
        scale = np.abs(o[0]).max()
        assert np.abs(o[1]).max() <= 1e-14 * scale
        assert np.abs(o[3]).max() <= 1e-14 * scale


# ----------------------------------------------------------- P-F convergence
@pytest.mark.parametrize("rel", [1, 2, 3])
def test_touching_pairs_converged(rel):
    """The order search returns values that a much higher fixed order confirms."""
    v, t = synth.icosphere(8, 0.5)
    t0 = t[37]
    j = next(j for j in range(len(t)) if len(set(t0) & set(t[j])) == rel)
    P, Q = v[t0], v[t[j]]
    auto = oracle.pair_integrals(t0, P, t[j], Q, K0)
    hi = oracle.pair_integrals(t0, P, t[j], Q, K0, nq=40)
    for op in range(4):
        scale = np.abs(hi[op]).max()
        if scale > 0:
            assert np.abs(auto[op] - hi[op]).max() <= 2e-12 * scale


# ----------------------------------------- P-F: the two touching-pair routes
def _touching_sample(v, t, seed, ntest=3):
    """Seeded test triangles (one of them where the surface is curved, when
    it has curved parts) with their coincident pair, one edge-adjacent and
    two vertex-adjacent source triangles."""
    rng = np.random.default_rng(seed)
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    curved = np.where(np.abs(nrm).max(axis=1) < 0.99)[0]
    picks = list(rng.choice(len(t), ntest - 1, replace=False))
    picks.append(int(rng.choice(curved)) if len(curved) else int(rng.integers(len(t))))
    out = []
    for ti in picks:
        sets = {1: [], 2: [], 3: []}
        for j in range(len(t)):
            c = len(set(t[ti]) & set(t[j]))
            if c:
                sets[c].append(j)
        out += [(ti, sets[3][0], 3), (ti, sets[2][rng.integers(len(sets[2]))], 2)]
        out += [(ti, j, 1) for j in rng.choice(sets[1], 2, replace=False)]
    return out


@pytest.mark.parametrize("name", ["icosphere", "rounded_box"])
def test_touching_routes_agree(name):
    """The oracle's two independent routes for pairs that share the
    triangle, an edge or a vertex agree to 1e-11 of the pair's largest entry
    for every operator: relative-coordinate (Duffy-type) transformations with
    the order search, and singularity subtraction with closed-form static
    integrals over the source triangle and graded rules over the test
    triangle."""
    if name == "icosphere":
        v, t = synth.icosphere(8, 0.5)
    else:
        v, t = synth.rounded_box((1.0, 1.0, 0.5), 0.2, 0.073)
    worst = {1: 0.0, 2: 0.0, 3: 0.0}
    for ti, sj, kind in _touching_sample(v, t, 91):
        a = oracle.pair_integrals(t[ti], v[t[ti]], t[sj], v[t[sj]], K0)
        b = oracle.pair_integrals_sub(t[ti], v[t[ti]], t[sj], v[t[sj]], K0)
        scale = np.abs(a).max()
        worst[kind] = max(worst[kind], float(np.abs(a - b).max() / scale))
    print("routes: max |diff| / pair scale by shared vertices:", worst)
    assert max(worst.values()) <= 1e-11


def test_subtraction_route_in_the_product():
    """oracle.matvec with route="subtraction" equals the default route's
    product on unit columns (the near field of two RWGs, touching pairs
    included) to the routes' agreement."""
    v, t = synth.icosphere(4, 0.5)
    N = 3 * len(t) // 2
    x = np.zeros((2 * N, 2), complex)
    x[5, 0] = 1.0
    x[N + 77, 1] = 1.0j
    for op in (oracle.OP_C, oracle.OP_EM):
        a = oracle.matvec(v, t, K0, x, op=op)
        b = oracle.matvec(v, t, K0, x, op=op, route="subtraction")
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


# ------------------------------------------------------------ P-B symmetry
@pytest.mark.parametrize("mesh", [synth.tetrahedron, synth.octahedron, synth.icosahedron])
def test_T_and_K_symmetric(mesh):
    """<f_m, L f_n> and <f_m, Kbar f_n> are symmetric (symmetric kernel; grad G
    odd under r <-> r'); touching pairs are computed with the test triangle
    first, so this also cross-checks the singular rules against themselves."""
    v, t = mesh()
    T = _dense(v, t, "T")
    Kk = _dense(v, t, "K")
    assert np.abs(T - T.T).max() <= 1e-11 * np.abs(T).max()
    assert np.abs(Kk - Kk.T).max() <= 1e-11 * np.abs(Kk).max()


# -------------------------------------------------------- P-E radiating part
def test_radiating_parts_equal_plane_wave_sums():
    """sin(kR)/(4 pi R) = k/(16 pi^2) Int exp(-jk khat.(r - r')) dOmega, exactly.
    Hence Re T, Im K, Re Tx and Im Kx of every entry are sphere sums of
    radiation patterns, independent of the singular quadrature.  Non-touching
    triangle pairs use the 7-point points (the matrix definition), touching
    pairs converged patterns."""
    v, t = synth.icosahedron(0.3)
    e, pm = oracle.rwg_table(v, t)
    N = len(e)
    co = rwg_coefficients(v, t, e, pm)
    khat, w = sphere_rule(20)
    k = K0

    def pats(P, rule):
        x, wq = rule
        ph = np.exp(1j * k * x @ khat.T)                      # (q, K)
        nt = tri_normal(P)
        vec = np.stack([np.einsum("q,qc,qK->Kc", wq, x - P[i], ph) for i in range(3)])
        twv = np.stack([np.einsum("q,qc,qK->Kc", wq, np.cross(nt, x - P[i]), ph) for i in range(3)])
        chg = np.einsum("q,qK->K", wq, ph)
        return vec, twv, chg

    p7 = [pats(v[tr], tri_radon7(v[tr])) for tr in t]
    pc = [pats(v[tr], tri_gauss(v[tr], 14)) for tr in t]
    c = k / (16 * np.pi ** 2)
    kx = lambda R: np.cross(khat, R)

    def block(A, B):
        """(T, K, Tx, Kx) radiating parts between test pattern A[i] and
        source pattern B[j] (vec (K,3), twisted vec (K,3), charge (K,))."""
        Sm, Sgm, rm = np.conj(A[0]), np.conj(A[1]), 2 * np.conj(A[2])
        Rn, rn = B[0], 2 * B[2]
        T_ = -k * c * np.sum(w * (np.sum(Sm * Rn, -1) - rm * rn / k ** 2), -1)
        K_ = -c * np.sum(w * np.sum(Sm * (-1j * k) * kx(Rn), -1), -1)
        Tx_ = c * np.sum(w * (k * np.sum(Sgm * Rn, -1) - 1j * np.sum(Sgm * khat, -1) * rn), -1)
        Kx_ = c * np.sum(w * np.sum(Sgm * (-1j * k) * kx(Rn), -1), -1)
        return T_.real, K_.real, Tx_.real, Kx_.real

    # local edge index of each RWG on each of its triangles
    ref = {op: np.zeros((N, N)) for op in ("T", "K", "Tx", "Kx")}
    loc = []
    for lst in co:
        loc.append([(tri, int(np.argmin(np.linalg.norm(v[t[tri]] - p, axis=1))), cf) for tri, p, cf in lst])
    for m in range(N):
        for n in range(N):
            acc = np.zeros(4)
            for tm_, i, cm in loc[m]:
                for tn_, j, cn in loc[n]:
                    touch = len(set(t[tm_]) & set(t[tn_])) > 0
                    A, B = (pc[tm_], pc[tn_]) if touch else (p7[tm_], p7[tn_])
                    acc += cm * cn * np.array(block((A[0][i], A[1][i], A[2]), (B[0][j], B[1][j], B[2])))
            for key, val in zip(("T", "K", "Tx", "Kx"), acc):
                ref[key][m, n] = val
    T = _dense(v, t, "T")
    Kk = _dense(v, t, "K")
    Tx = _dense(v, t, "Tx")
    Kx = _dense(v, t, "Kx")
    assert np.abs(T.real - ref["T"]).max() <= 1e-11 * np.abs(T).max()
    assert np.abs(Kk.imag - ref["K"]).max() <= 1e-11 * np.abs(Kk).max()
    assert np.abs(Tx.real - ref["Tx"]).max() <= 1e-11 * np.abs(Tx).max()
    assert np.abs(Kx.imag - ref["Kx"]).max() <= 1e-11 * np.abs(Kx).max()


# ------------------------------------------------- P-D / P-C sphere physics
def _project(v, t, field, order=8):
    """b_m = <f_m, F> with a converged triangle rule (F: (q,3) -> (q,3))."""
    e, pm = oracle.rwg_table(v, t)
    co = rwg_coefficients(v, t, e, pm)
    b = np.zeros(len(e), complex)
    for m, lst in enumerate(co):
        for tri, p, cm in lst:
            x, wq = tri_gauss(v[t[tri]], order)
            F = field(x, tri_normal(v[t[tri]]))
            b[m] += cm * np.sum(wq[:, None] * (x - p) * F)
    return b


def _gram(v, t):
    return _dense(v, t, "Gram").real


@pytest.mark.slow
def test_sphere_TE_eigenvalue():
    """On a sphere of radius a, L maps the TE degree-1 current z x r to
    -(ka)^2 j1(ka) h1(ka) times itself (addition theorem of G); at ka = pi this
    is -1 + j/pi.  Rayleigh quotient of the Galerkin T; error O(h^2)."""
    a = 0.5
    exact = -(K0 * a) ** 2 * sph_j1(K0 * a) * (sph_j1(K0 * a) - 1j * sph_y1(K0 * a))
    errs = []
    for m in (4, 8):
        v, t = synth.icosphere(m, a)
        N = 3 * len(t) // 2
        b = _project(v, t, lambda x, n: np.cross([0, 0, 1.0], x) / a)
        x = np.linalg.solve(_gram(v, t), b)
        X = np.zeros(2 * N, complex)
        X[:N] = x
        Tx_ = oracle.matvec(v, t, K0, X, op="T")[:N]
        Gx_ = oracle.matvec(v, t, K0, X, op="Gram")[:N]
        q = np.vdot(x, Tx_) / np.vdot(x, Gx_)
        errs.append(abs(q - exact) / abs(exact))
    print("TE eigenvalue relative errors (m=4, m=8):", errs)
    assert errs[1] < 0.02 and errs[1] < errs[0]


@pytest.mark.slow
def test_extinction_plane_wave():
    """Currents of an incident plane wave (J = n x H, M = -n x E) radiate -E,-H
    inside and 0 outside, so on the surface the principal-value operators give
    the average: T xJ - K xM = -<f,E>/2 and T xM + K xJ = -<f,H>/2 (eqs. 22,
    24).  For the C block (eqs. 43-46, alpha = 1/2) the same identities give
    C^JJ xJ + C^JM xM = <f, 3E/4 + 5 n x H/4> and
    C^MJ xJ + C^MM xM = <f, H/4 - 3 n x E/4>: all K terms cancel, so any sign
    error in the combination shows.  Discretisation error O(h)."""
    khat = np.array([0.0, 0.0, 1.0])
    pol = np.array([1.0, 0.0, 0.0])
    Ei = lambda x: pol[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    Hi = lambda x: np.cross(khat, pol)[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    errs = []
    for m in (4, 8):
        v, t = synth.icosphere(m, 0.5)
        N = 3 * len(t) // 2
        G = _gram(v, t)
        xJ = np.linalg.solve(G, _project(v, t, lambda x, n: np.cross(n, Hi(x))))
        xM = np.linalg.solve(G, _project(v, t, lambda x, n: -np.cross(n, Ei(x))))
        X = np.concatenate([xJ, xM])
        yC, yEM = oracle.matvec(v, t, K0, X, op=oracle.OP_BOTH)
        refs = [(yEM[:N], -0.5 * _project(v, t, lambda x, n: Ei(x))),
                (yEM[N:], -0.5 * _project(v, t, lambda x, n: Hi(x))),
                (yC[:N], _project(v, t, lambda x, n: 0.75 * Ei(x) + 1.25 * np.cross(n, Hi(x)))),
                (yC[N:], _project(v, t, lambda x, n: 0.25 * Hi(x) - 0.75 * np.cross(n, Ei(x))))]
        errs.append([np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in refs])
    errs = np.array(errs)
    print("extinction relative errors [E, H, C-J, C-M] at m=4 / m=8:", errs)
    assert np.all(errs[1] < 0.06), errs
    assert np.all(errs[1] < errs[0]), errs


# ------------------------------------------------------------- box rule
@pytest.mark.parametrize("m,r,levels,boxes,near", [(8, 0.5, 3, 56, 846744)])
def test_box_rule_counts(m, r, levels, boxes, near):
    """Leaf boxes of the RWG centres (0.25 wavelength leaves): level count,
    non-empty leaf boxes and near RWG pairs (Chebyshev distance <= 1)."""
    v, t = synth.icosphere(m, r)
    coords, lev = oracle.leaf_boxes(v, t, 0.25)
    assert lev == levels
    assert len({tuple(c) for c in coords}) == boxes
    d = np.abs(coords[:, None, :] - coords[None, :, :]).max(axis=2)
    assert int((d <= 1).sum()) == near


# Translations per level (levels >= 2, finest first) of the quarter-wavelength
# octree, counted from generated meshes before any code of this repository
# existed: icosphere r = 0.5 (frequency 8), r = 3 (frequency 36), r = 8
# (frequency 96).
TRANSLATION_COUNTS = [
    (8, 0.5, {2: 2504}),
    (36, 3.0, {5: 104448, 4: 28176, 3: 3632, 2: 2256}),
    (96, 8.0, {6: 754008, 5: 210960, 4: 54000, 3: 12216, 2: 2504}),
]


@pytest.mark.parametrize("m,r,counts", TRANSLATION_COUNTS)
def test_interaction_class_counts(m, r, counts):
    """The oracle's interaction class of an RWG pair (near, or the level at
    which their boxes are first well separated: the split of the per-level
    error), aggregated to box pairs per level, reproduces the recorded
    translation counts of the three spheres."""
    v, t = synth.icosphere(m, r)
    assert oracle.class_box_pairs(v, t, 0.25) == counts


def _interaction_lists_brute_force(coords, levels):
    """Translations per level straight from the definition: B is in the
    interaction list of A at level l when both hold RWGs, their parents are
    adjacent (Chebyshev distance <= 1) and A and B are not."""
    out = {}
    for l in range(2, levels):
        sh = levels - 1 - l
        boxes = np.unique(coords >> sh, axis=0)
        d = np.abs(boxes[:, None, :] - boxes[None, :, :]).max(axis=2)
        dp = np.abs((boxes[:, None, :] >> 1) - (boxes[None, :, :] >> 1)).max(axis=2)
        out[l] = int(((d >= 2) & (dp <= 1)).sum())
    return out


@pytest.mark.parametrize("name", ["sphere_r0.5", "box", "two_bodies"])
def test_interaction_classes_match_definition(name):
    """Same aggregation against the interaction lists computed by brute force
    over the occupied boxes of every level, on surfaces without recorded
    counts (the rounded box, two disjoint spheres)."""
    if name == "sphere_r0.5":
        v, t = synth.icosphere(8, 0.5)
    elif name == "box":
        v, t = synth.rounded_box((2.0, 2.0, 0.5), 0.1, 0.1)
    else:
        v, t = synth.scene(synth.icosphere(6, 0.5) + ((0, 0, 0),), synth.icosphere(4, 0.3) + ((1.4, 0.2, -0.1),))
    coords, levels = oracle.leaf_boxes(v, t, 0.25)
    want = _interaction_lists_brute_force(coords, levels)
    assert levels >= 4 or name == "sphere_r0.5"
    assert oracle.class_box_pairs(v, t, 0.25) == want


def test_plane_wave_rhs_matches_projection():
    """Right-hand sides of eqs. 49-50 for a plane wave (Sec. III excitation):
    the oracle's 7-point values against an independent high-order projection
    of E/2 + n x H/2 and H/2 - n x E/2 (agreement to the 7-point rule's error)."""
    v, t = synth.icosphere(6, 0.5)
    N = 3 * len(t) // 2
    khat = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    khat /= np.linalg.norm(khat)
    pol = np.cross(khat, [0.0, 0.0, 1.0])
    pol /= np.linalg.norm(pol)
    Ei = lambda x: pol[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    Hi = lambda x: np.cross(khat, pol)[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    bJ = _project(v, t, lambda x, n: 0.5 * Ei(x) + 0.5 * np.cross(n, Hi(x)))
    bM = _project(v, t, lambda x, n: 0.5 * Hi(x) - 0.5 * np.cross(n, Ei(x)))
    got = oracle.plane_wave_rhs(v, t, K0, khat[None, :], pol[None, :])[:, 0]
    ref = np.concatenate([bJ, bM])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


# ------------------------------------------------------------- far field
def _sph_units(kh):
    th, ph = np.arccos(np.clip(kh[2], -1, 1)), np.arctan2(kh[1], kh[0])
    return (np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)]),
            np.array([-np.sin(ph), np.cos(ph), 0.0]))


def test_far_field_dipole_limit():
    """As k -> 0 the far field of one RWG tends to (-jk/4pi) times the
    transverse part of its moment m = Int f ds = sum over its triangles of
    sigma l/(2A) * A (centroid - free vertex) for an electric current, and
    to (-jk/4pi) (-khat x m) for a magnetic one (closed form, independent of
    the quadrature)."""
    v, t = synth.octahedron(0.4)
    e, pm = oracle.rwg_table(v, t)
    co = rwg_coefficients(v, t, e, pm)
    N = len(e)
    k = 1e-9
    dirs = synth.fibonacci_directions(9, 3)[0]
    for n in (0, 5):
        m = sum(cm * tri_area(v[t[tri]]) * (v[t[tri]].mean(axis=0) - p) for tri, p, cm in co[n])
        for half in (0, 1):
            x = np.zeros((2 * N, 1), complex)
            x[half * N + n] = 1.0
            F = oracle.far_field(v, t, k, x, dirs)[:, :, 0] / (-1j * k / (4 * np.pi))
            for d, kh in enumerate(dirs):
                vec = m - kh * (kh @ m) if half == 0 else -np.cross(kh, m)
                tv, pv = _sph_units(kh)
                ref = np.array([tv @ vec, pv @ vec])
                assert np.allclose(F[d], ref, rtol=1e-9, atol=1e-9 * np.linalg.norm(m)), (n, half, d, F[d], ref)


@pytest.mark.slow
def test_far_field_extinction():
    """The equivalent currents of an incident plane wave (J = n x H,
    M = -n x E) radiate nothing outside the surface (the same extinction as
    on the surface), so their far field vanishes up to discretisation
    error, while the fields of J and of M alone do not.  Checks the relative
    sign and scale of the J and M terms and the sign of the phase."""
    khat = np.array([0.0, 0.0, 1.0])
    pol = np.array([1.0, 0.0, 0.0])
    Ei = lambda x: pol[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    Hi = lambda x: np.cross(khat, pol)[None, :] * np.exp(-1j * K0 * x @ khat)[:, None]
    dirs = synth.fibonacci_directions(40, 7)[0]
    ratios = []
    for m in (4, 8):
        v, t = synth.icosphere(m, 0.5)
        N = 3 * len(t) // 2
        G = _gram(v, t)
        xJ = np.linalg.solve(G, _project(v, t, lambda x, n: np.cross(n, Hi(x))))
        xM = np.linalg.solve(G, _project(v, t, lambda x, n: -np.cross(n, Ei(x))))
        X = np.stack([np.concatenate([xJ, xM]), np.concatenate([xJ, 0 * xM])], axis=1)
        F = oracle.far_field(v, t, K0, X, dirs)
        ratios.append(np.linalg.norm(F[:, :, 0]) / np.linalg.norm(F[:, :, 1]))
    print("far-field extinction |F(J,M)| / |F(J)| at m=4 / m=8:", ratios)
    assert ratios[1] < 0.05 and ratios[1] < ratios[0]
