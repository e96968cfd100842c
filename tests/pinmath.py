"""Independent mathematics used to pin the oracle (test side only).

Closed forms and textbook quadrature written from their published
definitions: the collapsed Gauss product rule on a triangle, the analytic
potential of a uniform source on a flat triangle (Wilton, Rao, Glisson,
Schaubert, Al-Bundak and Butler, IEEE TAP 1984), exact moments of linear
functions over a triangle, the spherical Bessel closed forms of degree 1,
and a Gauss-Legendre x uniform rule on the unit sphere.
"""
import numpy as np

K0 = 2.0 * np.pi


def tri_area(P):
    P = np.asarray(P, float)
    return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))


def tri_normal(P):
    P = np.asarray(P, float)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    return n / np.linalg.norm(n)


def tri_gauss(P, n):
    """Collapsed (Duffy) Gauss-Legendre product rule with n x n points:
    exact for polynomials of degree <= 2n-2 on the triangle."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = (x + 1) / 2
    w = w / 2
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    b0, b1, b2 = 1 - u, u * (1 - v), u * v
    P = np.asarray(P, float)
    pts = b0.ravel()[:, None] * P[0] + b1.ravel()[:, None] * P[1] + b2.ravel()[:, None] * P[2]
    return pts, (wu * wv * u).ravel() * 2 * tri_area(P)


def tri_radon7(P):
    """Radon's 7-point degree-5 rule (the published constants)."""
    s15 = np.sqrt(15.0)
    a, b = (6 - s15) / 21, (6 + s15) / 21
    wa, wb = (155 - s15) / 1200, (155 + s15) / 1200
    bary = np.array([[1 / 3, 1 / 3, 1 / 3], [a, a, 1 - 2 * a], [a, 1 - 2 * a, a], [1 - 2 * a, a, a],
                     [b, b, 1 - 2 * b], [b, 1 - 2 * b, b], [1 - 2 * b, b, b]])
    w = np.array([9 / 40, wa, wa, wa, wb, wb, wb])
    P = np.asarray(P, float)
    return bary @ P, w * tri_area(P)


def linear_moment(P, p, q, twist=None):
    """Exact Int_T (r - p) . M (r - q) dA for M = I (twist None) or M = n x (.)
    using Int lambda_i lambda_j = A (1 + delta_ij) / 12."""
    P = np.asarray(P, float)
    A = tri_area(P)
    tot = 0.0
    for i in range(3):
        for j in range(3):
            a = P[i] - p
            b = P[j] - q
            if twist is not None:
                b = np.cross(twist, b)
            tot += (1 + (i == j)) * np.dot(a, b)
    return A * tot / 12.0


def potential(x, Q):
    """Int_Q 1/|x - y| dA(y) over the flat triangle Q, closed form."""
    Q = np.asarray(Q, float)
    x = np.asarray(x, float)
    n = tri_normal(Q)
    h = np.dot(x - Q[0], n)
    rho = x - h * n
    tot = 0.0
    for i in range(3):
        A, B = Q[i], Q[(i + 1) % 3]
        lhat = (B - A) / np.linalg.norm(B - A)
        mhat = np.cross(lhat, n)
        lp, lm = np.dot(B - rho, lhat), np.dot(A - rho, lhat)
        P0 = np.dot(A - rho, mhat)
        R0sq = P0 * P0 + h * h
        Rp, Rm = np.sqrt(lp * lp + R0sq), np.sqrt(lm * lm + R0sq)
        if abs(P0) > 1e-15:
            # ln((R+ + l+)/(R- + l-)) = ln((R- - l-)/(R+ - l+)); take the form
            # without cancellation
            if lm >= 0:
                tot += P0 * np.log((Rp + lp) / (Rm + lm))
            else:
                tot += P0 * np.log((Rm - lm) / (Rp - lp))
            if abs(h) > 0:
                tot -= abs(h) * (np.arctan(P0 * lp / (R0sq + abs(h) * Rp))
                                 - np.arctan(P0 * lm / (R0sq + abs(h) * Rm)))
    return tot


def sph_j1(x):
    return np.sin(x) / x ** 2 - np.cos(x) / x


def sph_y1(x):
    return -np.cos(x) / x ** 2 - np.sin(x) / x


def sphere_rule(L):
    """(L+1) Gauss-Legendre nodes in cos(theta) x (2L+2) uniform azimuths:
    exact for spherical harmonics of degree <= 2L+1."""
    ct, wt = np.polynomial.legendre.leggauss(L + 1)
    ph = 2 * np.pi * np.arange(2 * L + 2) / (2 * L + 2)
    C, PH = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - C ** 2)
    khat = np.stack([S * np.cos(PH), S * np.sin(PH), C], axis=-1).reshape(-1, 3)
    w = (wt[:, None] * np.full(ph.shape, 2 * np.pi / (2 * L + 2))[None, :]).ravel()
    return khat, w


def rwg_coefficients(verts, tris, edges, tri_pm):
    """Per RWG n and each of its two triangles: (triangle, free vertex
    coords, coefficient sigma*l/(2A)) from the published RWG definition."""
    out = []
    for n, (a, b) in enumerate(edges):
        l = np.linalg.norm(verts[b] - verts[a])
        lst = []
        for sgn, t in ((1.0, tri_pm[n, 0]), (-1.0, tri_pm[n, 1])):
            tv = tris[t]
            p = [v for v in tv if v != a and v != b][0]
            A = tri_area(verts[tv])
            lst.append((int(t), verts[p], sgn * l / (2 * A)))
        out.append(lst)
    return out
