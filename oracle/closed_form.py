"""Closed forms for the honeycomb lattice with space-uniform fields.

TEST INFRASTRUCTURE ONLY.

If phi_{t,x} = c_t for every site, diag(exp(i phi_t)) = exp(i c_t) commutes
with everything and the product of Sec. 2 collapses to
    B_{N_t} ... B_1 = exp(i theta) exp(beta kappa K),   theta = sum_t c_t,
since N_t * delta = beta.  The honeycomb hopping matrix is diagonal in
momentum space: with unit cells (i, j), k = 2 pi (n1, n2) / L and
f(k) = 1 + exp(-i k1) + exp(-i k2), the 2 x 2 Bloch matrix is
h(k) = [[0, f], [f*, 0]] with eigenvalues +-|f(k)|.  Everything below is
written from these facts with no dense linear algebra:

  log det M = sum_k [ i theta + log(2 cos theta + 2 cosh(beta kappa |f|)) ],
  G(k)      = sum_+- Pi_+-(k) / (1 + exp(i theta) exp(+-beta kappa |f|)),
              Pi_+- = (1 +- h/|f|) / 2  (G(k) = 1/(1+exp(i theta)) if f = 0),
  F_{t,x}   = i/2 - (1/N) sum_k sin theta / (cos theta + cosh(beta kappa |f|)).
"""
from __future__ import annotations

import cmath
import math

import numpy as np


def _momenta(L):
    for n1 in range(L):
        for n2 in range(L):
            yield 2.0 * math.pi * n1 / L, 2.0 * math.pi * n2 / L


def honeycomb_dispersion(L: int) -> np.ndarray:
    """f(k) for every momentum k (complex, L*L values, n1-major)."""
    return np.array([1.0 + cmath.exp(-1j * k1) + cmath.exp(-1j * k2)
                     for k1, k2 in _momenta(L)])


def _wrap(z: complex) -> complex:
    im = math.remainder(z.imag, 2.0 * math.pi)
    if im <= -math.pi:
        im += 2.0 * math.pi
    return complex(z.real, im)


def uniform_field_logdet(L: int, bk: float, theta: float) -> complex:
    """log det M for phi_{t,x} = c_t, theta = sum_t c_t, bk = beta * kappa.

    Each +-|f| pair contributes (1 + e^{i th} e^{a})(1 + e^{i th} e^{-a})
    = e^{i th} (2 cos th + 2 cosh a), a = bk |f|.  For large a the log is
    evaluated as a + log(1 + 2 cos th e^{-a} + e^{-2a}) to avoid overflow.
    """
    total = 0.0 + 0.0j
    for f in honeycomb_dispersion(L):
        a = bk * abs(f)
        inner = 2.0 * math.cos(theta) * math.exp(-a) + math.exp(-2.0 * a)
        total += 1j * theta + a + math.log1p(inner)
    return _wrap(total)


def uniform_field_greens(L: int, bk: float, theta: float) -> np.ndarray:
    """Real-space G for a uniform field, by Fourier synthesis of G(k).

    Site index 2 (i L + j) + sigma; G_{(r,s),(r',s')} =
    (1/L^2) sum_k exp(i k.(r - r')) G(k)_{s s'}.
    """
    N = 2 * L * L
    G = np.zeros((N, N), dtype=np.complex128)
    eith = cmath.exp(1j * theta)
    idx = np.arange(L)
    for (k1, k2), f in zip(_momenta(L), honeycomb_dispersion(L)):
        af = abs(f)
        if af < 1e-14:
            Gk = np.eye(2, dtype=np.complex128) / (1.0 + eith)
        else:
            h = np.array([[0.0, f], [np.conj(f), 0.0]], dtype=np.complex128)
            Gk = np.zeros((2, 2), dtype=np.complex128)
            for sgn in (1.0, -1.0):
                proj = 0.5 * (np.eye(2) + sgn * h / af)
                x = sgn * bk * af
                # 1 / (1 + e^{i th} e^{x}), written to avoid overflow for x >> 0
                if x > 0:
                    w = cmath.exp(-x) / (cmath.exp(-x) + eith)
                else:
                    w = 1.0 / (1.0 + eith * cmath.exp(x))
                Gk += w * proj
        # phase e^{i k.(r - r')} over unit cells
        ph_i = np.exp(1j * k1 * idx)
        ph_j = np.exp(1j * k2 * idx)
        cell = np.outer(ph_i, ph_j).reshape(-1)          # e^{i k.r}, r = i*L + j
        phase = np.outer(cell, np.conj(cell)) / (L * L)  # (r, r')
        for s in range(2):
            for sp in range(2):
                G[s::2, sp::2] += Gk[s, sp] * phase
    return G


def uniform_field_force(L: int, bk: float, theta: float) -> complex:
    """F_{t,x} for a uniform field (the same for every t and x)."""
    N = 2 * L * L
    acc = 0.0
    for f in honeycomb_dispersion(L):
        a = bk * abs(f)
        acc += math.sin(theta) / (math.cos(theta) + math.cosh(a))
    return complex(-acc / N, 0.5)


def _taylor(x: float, n: int) -> float:
    """sum_{j <= n} x^j / j! by Horner's rule."""
    acc = 1.0
    for j in range(n, 0, -1):
        acc = 1.0 + acc * x / j
    return acc


def uniform_field_taylor_logdet_greens(L: int, dk: float, Nt: int, theta: float, n: int):
    """log det M~ and G~ = M~^{-1} for a uniform field when every slice uses
    the degree-n Taylor polynomial p_n of exp in place of exp(dk K) (the
    product form of Sec. 8 is that polynomial).  p_n(dk K) is diagonal in
    momentum space with eigenvalues p_n(+-dk |f|), so the product of the N_t
    slices has eigenvalues e^{i theta} p_n(+-dk |f|)^{N_t}; with
    a = N_t log p_n(+-dk |f|) (p_n > 0 on the range used here)
        log det M~ = sum_k sum_+- log(1 + e^{i theta} e^{a}),
        G~(k)      = sum_+- Pi_+-(k) / (1 + e^{i theta} e^{a}).
    Both are evaluated without forming e^{a} for large a."""
    N = 2 * L * L
    eith = cmath.exp(1j * theta)
    total = 0.0 + 0.0j
    G = np.zeros((N, N), dtype=np.complex128)
    idx = np.arange(L)
    for (k1, k2), f in zip(_momenta(L), honeycomb_dispersion(L)):
        af = abs(f)
        Gk = np.zeros((2, 2), dtype=np.complex128)
        for sgn in (1.0, -1.0):
            p = _taylor(sgn * dk * af, n)
            if not p > 0.0:
                raise ValueError("p_n(dk lambda) must be positive here")
            a = Nt * math.log(p)
            if a > 0:
                total += a + cmath.log(cmath.exp(-a) + eith)
                w = cmath.exp(-a) / (cmath.exp(-a) + eith)
            else:
                total += cmath.log(1.0 + eith * cmath.exp(a))
                w = 1.0 / (1.0 + eith * cmath.exp(a))
            if af < 1e-14:
                Gk += 0.5 * w * np.eye(2)
            else:
                h = np.array([[0.0, f], [np.conj(f), 0.0]], dtype=np.complex128)
                Gk += w * 0.5 * (np.eye(2) + sgn * h / af)
        cell = np.outer(np.exp(1j * k1 * idx), np.exp(1j * k2 * idx)).reshape(-1)
        phase = np.outer(cell, np.conj(cell)) / (L * L)
        for s_ in range(2):
            for sp in range(2):
                G[s_::2, sp::2] += Gk[s_, sp] * phase
    return _wrap(total), G


# ---------------------------------------------------------------------------
# Two sites with one bond: K = [[0, 1], [1, 0]], so K^2 = 1 and
# exp(dk K) = cosh(dk) 1 + sinh(dk) K.  The slice matrices, their product and
# 1 + P are 2 x 2; their determinant and inverse are written out, with no
# linear-algebra library: M = 1 + B_{N_t} ... B_1 (Sec. 2), G = M^{-1}, and
# F_{t,x} = i (1 - G~_t)_{xx} with G~_t = (1 + B_{t-1} ... B_1 B_{N_t} ... B_t)^{-1}
# (Sec. 4 response formula, phi_{t,x} entering B_t = E diag(e^{i phi_t})).
# The time-displaced G(t, t0) follows from the rows of the block fermion
# matrix instead of eq. sausage_all_in_denominator: G(t0, t0) = G~_{t0}, and
# each block row says G(t + 1, t0) = B_t G(t, t0) for t + 1 != t0, with the
# sign of the anti-periodic corner when the propagation wraps past slice N_t.
# ---------------------------------------------------------------------------

def _mul2(a, b):
    return [[a[0][0] * b[0][0] + a[0][1] * b[1][0], a[0][0] * b[0][1] + a[0][1] * b[1][1]],
            [a[1][0] * b[0][0] + a[1][1] * b[1][0], a[1][0] * b[0][1] + a[1][1] * b[1][1]]]


def _inv_one_plus2(p):
    """(1 + p)^{-1} and det(1 + p) of a 2 x 2 complex matrix."""
    a, b, c, d = 1.0 + p[0][0], p[0][1], p[1][0], 1.0 + p[1][1]
    det = a * d - b * c
    return [[d / det, -b / det], [-c / det, a / det]], det


def two_site(dk: float, phi) -> tuple:
    """(log det M, G, F) of the two-site system; phi is (N_t, 2), row t-1 = slice t.
    log det has its imaginary part in (-pi, pi]; G is 2 x 2, F is (N_t, 2)."""
    ch, sh = math.cosh(dk), math.sinh(dk)
    nt = len(phi)
    slices = []
    for t in range(nt):
        e0, e1 = cmath.exp(1j * phi[t][0]), cmath.exp(1j * phi[t][1])
        slices.append([[ch * e0, sh * e1], [sh * e0, ch * e1]])
    one = [[1.0 + 0j, 0j], [0j, 1.0 + 0j]]

    def prod(ts):
        # B_{ts[-1]} ... B_{ts[0]}: later slices on the left
        m = one
        for t in ts:
            m = _mul2(slices[t], m)
        return m

    g, det = _inv_one_plus2(prod(range(nt)))
    logdet = _wrap(cmath.log(det))
    force = []
    for t in range(nt):
        # cyclic product starting at slice t+1 (0-based t): B_t ... B_1 B_{N_t} ... B_{t+1}
        c = prod(list(range(t, nt)) + list(range(0, t)))
        gt, _ = _inv_one_plus2(c)
        force.append([1j * (1.0 - gt[0][0]), 1j * (1.0 - gt[1][1])])
    return logdet, np.array(g, dtype=complex), np.array(force, dtype=complex)


def uniform_field_displaced_greens(K: np.ndarray, dk: float, c, t: int, t0: int) -> np.ndarray:
    """G(t, t0) for a field constant in space, phi_{t,x} = c_t (every slice
    is e^{i c_t} E and the slices commute): with theta = sum c and, for
    t >= t0, the n = t - t0 slices of rows t0-1 .. t-2 carrying phase a,
        G(t, t0) = U diag(e^{i a} e^{dk lam n} / (1 + e^{i theta} e^{dk lam N_t})) U^T,
    and for t < t0, with n = t0 - t slices of rows t-1 .. t0-2 carrying a,
        G(t, t0) = -U diag(e^{i (theta - a)} e^{dk lam (N_t - n)}
                             / (1 + e^{i theta} e^{dk lam N_t})) U^T,
    K = U diag(lam) U^T (numpy.linalg.eigh).  Each fraction is evaluated in
    the form that cannot overflow."""
    c = np.asarray(c, dtype=float)
    Nt = len(c)
    theta = float(c.sum())
    lam, U = np.linalg.eigh(K)
    if t >= t0:
        n, a, pre = t - t0, float(c[t0 - 1:t - 1].sum()), 1.0
        m = n
    else:
        n = t0 - t
        a, pre = theta - float(c[t - 1:t0 - 1].sum()), -1.0
        m = Nt - n
    x = dk * lam
    big = x > 0
    num = np.where(big, np.exp(x * (m - Nt)), np.exp(x * m))
    den = np.where(big, np.exp(-x * Nt) + np.exp(1j * theta), 1.0 + np.exp(1j * theta) * np.exp(x * Nt))
    d = pre * np.exp(1j * a) * num / den
    return (U * d[None, :]) @ U.T


def _two_site_slices(cosh_part: float, sinh_part: float, phi):
    """B_t = (c 1 + s K) diag(e^{i phi_t}) for K = [[0, 1], [1, 0]]."""
    out = []
    for row in phi:
        e0, e1 = cmath.exp(1j * row[0]), cmath.exp(1j * row[1])
        out.append([[cosh_part * e0, sinh_part * e1], [sinh_part * e0, cosh_part * e1]])
    return out


def _two_site_prod(slices, ts):
    m = [[1.0 + 0j, 0j], [0j, 1.0 + 0j]]
    for t in ts:   # later slices on the left
        m = _mul2(slices[t], m)
    return m


def two_site_displaced(dk: float, phi, t: int, t0: int) -> np.ndarray:
    """G(t, t0) of the two-site system (1-based slices): G~_{t0} of the
    cyclic product from slice t0, propagated by the slices between t0 and t:
    G(t, t0) = B_{t-1} ... B_{t0} G~_{t0} for t > t0, and
    G(t, t0) = -B_{t-1} ... B_1 B_{N_t} ... B_{t0} G~_{t0} for t < t0."""
    nt = len(phi)
    sl = _two_site_slices(math.cosh(dk), math.sinh(dk), phi)
    r0 = t0 - 1
    gt, _ = _inv_one_plus2(_two_site_prod(sl, list(range(r0, nt)) + list(range(0, r0))))
    if t == t0:
        g = gt
    elif t > t0:
        g = _mul2(_two_site_prod(sl, range(r0, t - 1)), gt)
    else:
        p = _mul2(_two_site_prod(sl, list(range(r0, nt)) + list(range(0, t - 1))), gt)
        g = [[-p[0][0], -p[0][1]], [-p[1][0], -p[1][1]]]
    return np.array(g, dtype=complex)


def two_site_taylor(dk: float, phi, n: int) -> tuple:
    """(log det, G) of the two-site system with the slices of Sec. 8: the
    degree-n Taylor polynomial of exp(dk K) is c 1 + s K with c the even and
    s the odd terms of sum_{j <= n} dk^j / j! (K^2 = 1)."""
    c = sum(dk ** j / math.factorial(j) for j in range(0, n + 1, 2))
    s_ = sum(dk ** j / math.factorial(j) for j in range(1, n + 1, 2))
    sl = _two_site_slices(c, s_, phi)
    g, det = _inv_one_plus2(_two_site_prod(sl, range(len(phi))))
    return _wrap(cmath.log(det)), np.array(g, dtype=complex)


def two_site_slice_response(dk: float, phi, a) -> np.ndarray:
    """tr((1 - G~_t) A) for every slice t of the two-site system, A 2 x 2."""
    nt = len(phi)
    sl = _two_site_slices(math.cosh(dk), math.sinh(dk), phi)
    out = []
    for t in range(nt):
        gt, _ = _inv_one_plus2(_two_site_prod(sl, list(range(t, nt)) + list(range(0, t))))
        acc = 0j
        for x in range(2):
            for y in range(2):
                acc += ((1.0 if x == y else 0.0) - gt[x][y]) * a[y][x]
        out.append(acc)
    return np.array(out, dtype=complex)
