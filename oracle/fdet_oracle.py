"""CPU FP64 oracle: brute force and stabilised determinant, Green's function, force.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module.

Notation (paper Sec. 2): V = N spatial sites, N_t time slices, slice matrices
B_t = E diag(exp(i phi_t)) with E = exp(delta kappa K), the "sausage"
M = 1 + B_{N_t} ... B_1 (later times to the left, which is what the block
fermion matrix of Sec. 2 reduces to), log det M and the Green's function
G = M^{-1}.  phi is an (N_t, N) array whose row t-1 holds phi_t.

Three independent tiers:
  * brute force on the full (N N_t)^2 block fermion matrix (Sec. 2 and the
    matrix-element derivatives of Sec. 4, eq. sausage_all_in_denominator);
  * dense product followed by LU, valid only while the product is well
    conditioned (Sec. 6 spirit; used for N_t = 1 and tiny beta);
  * the stabilised UDV method of Sec. 7 (eqs. def_matrix_as_product,
    prod_2_mat_stab .. res_2_mat_stab, steps 1-6), its sporadic variant of
    Sec. 9, and the stabilised prefix/suffix force of Sec. 5
    (subsection "Stabilised dense pre- and suffix calculations").
Closed forms for the free and uniform-field honeycomb live in closed_form.py.

Readings taken where the paper is silent (listed in the design notes too):
  * QR decompositions use column pivoting (LAPACK zgeqp3) so that D is sorted
    by magnitude (Sec. 7 requires D sorted; it never names pivoting).
  * D = |diag R|; the unit-modulus phase of diag R goes into X.
  * log det Q is evaluated as i*arg(det Q) (|det Q| = 1, Sec. 7 step 5), the
    pivot permutation contributes i*pi*parity, Im log det is wrapped to
    (-pi, pi].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------------------
# elementary pieces
# ---------------------------------------------------------------------------

def wrap_phase(z: complex) -> complex:
    """Return z with its imaginary part mapped into (-pi, pi]."""
    im = math.remainder(z.imag, 2.0 * math.pi)   # in [-pi, pi]
    if im <= -math.pi:
        im += 2.0 * math.pi
    return complex(z.real, im)


def _perm_parity(piv: np.ndarray) -> int:
    """Parity (0 even, 1 odd) of the permutation i -> piv[i]."""
    piv = np.asarray(piv)
    seen = np.zeros(len(piv), dtype=bool)
    parity = 0
    for i in range(len(piv)):
        if seen[i]:
            continue
        j, length = i, 0
        while not seen[j]:
            seen[j] = True
            j = piv[j]
            length += 1
        parity ^= (length - 1) & 1
    return parity


def slice_exponential(K: np.ndarray, dk: float) -> np.ndarray:
    """E = exp(dk K) for real symmetric K by diagonalisation (Sec. 6 steps 1-2)."""
    lam, U = np.linalg.eigh(K)
    return (U * np.exp(dk * lam)) @ U.T


def slice_matrices(K: np.ndarray, dk: float, phi: np.ndarray) -> list[np.ndarray]:
    """[B_1, ..., B_{N_t}] with B_t = exp(dk K) diag(exp(i phi_t)) (Sec. 2)."""
    E = slice_exponential(K, dk)
    return [E * np.exp(1j * phi[t])[None, :] for t in range(phi.shape[0])]


# ---------------------------------------------------------------------------
# tier 1: brute force on the block fermion matrix (Sec. 2)
# ---------------------------------------------------------------------------

def block_fermion_matrix(K: np.ndarray, dk: float, phi: np.ndarray) -> np.ndarray:
    """The (N N_t) x (N N_t) fermion matrix of Sec. 2.

    Identity blocks on the diagonal, -B_t at block (t, t-1) for t = 1..N_t-1
    (0-based block indices, B_t acting between slice t-1 and t) and +B_{N_t}
    in the corner block (0, N_t-1) (anti-periodic time boundary).
    """
    return block_matrix_of_slices(slice_matrices(K, dk, phi))


def block_matrix_of_slices(B) -> np.ndarray:
    """The block fermion matrix of Sec. 2 for given slice matrices
    [B_1, ..., B_{N_t}] (the layout of block_fermion_matrix)."""
    Nt, N = len(B), B[0].shape[0]
    M = np.eye(N * Nt, dtype=np.complex128)
    for p in range(Nt - 1):
        M[(p + 1) * N:(p + 2) * N, p * N:(p + 1) * N] = -B[p]
    M[0:N, (Nt - 1) * N:Nt * N] += B[Nt - 1]
    return M


def bruteforce_logdet_greens(K, dk, phi):
    """(log det M, G) from the block matrix: det of the block matrix equals
    det(1 + B_{N_t}...B_1) and G is its (0, 0) block of the inverse (Sec. 2)."""
    Mb = block_fermion_matrix(K, dk, phi)
    sign, logabs = np.linalg.slogdet(Mb)
    Minv = np.linalg.inv(Mb)
    N = phi.shape[1]
    return wrap_phase(complex(logabs, np.angle(sign))), Minv[:N, :N].copy()


def bruteforce_force(K, dk, phi):
    """F[t-1, x] = d log det M / d phi_{t,x} by Jacobi's formula on the block
    matrix (Sec. 4, "Matrix element derivatives": d log det / dM_ij = (M^-1)_ji).

    phi_{t,x} enters only column x of B_t: dB_t/dphi_{t,x} = i B_t e_x e_x^T.
    B_t sits at block (t, t-1) with sign -1 for t < N_t and at the corner block
    (0, N_t-1) with sign +1 for t = N_t, so
        F[t-1, x] = -/+ i sum_y (M^-1)_{(t-1, x), (t mod N_t, y)} (B_t)_{y, x}.
    Returns the complex array F (N_t, N).
    """
    Mb = block_fermion_matrix(K, dk, phi)
    Minv = np.linalg.inv(Mb)
    B = slice_matrices(K, dk, phi)
    Nt, N = phi.shape
    F = np.zeros((Nt, N), dtype=np.complex128)
    for p in range(Nt):
        r = (p + 1) % Nt
        sgn = -1.0 if p < Nt - 1 else 1.0
        blk = Minv[p * N:(p + 1) * N, r * N:(r + 1) * N]      # (x, y)
        # sum_y blk[x, y] * B_p[y, x]
        F[p] = sgn * 1j * np.einsum("xy,yx->x", blk, B[p])
    return F


# ---------------------------------------------------------------------------
# tier 2: dense product and LU (only for well-conditioned products)
# ---------------------------------------------------------------------------

def dense_logdet_greens(K, dk, phi):
    """Form P = B_{N_t}...B_1, then log det(1 + P) and (1 + P)^{-1} by LU.

    This is the plain definition; it is useless once cond(P) is large and is
    used only for N_t = 1 and small beta.
    """
    B = slice_matrices(K, dk, phi)
    N = phi.shape[1]
    P = np.eye(N, dtype=np.complex128)
    for Bt in B:
        P = Bt @ P
    A = np.eye(N) + P
    sign, logabs = np.linalg.slogdet(A)
    return wrap_phase(complex(logabs, np.angle(sign))), np.linalg.inv(A)


# ---------------------------------------------------------------------------
# tier 3: stabilised UDV method (Sec. 7)
# ---------------------------------------------------------------------------
# A matrix is kept as the triple (X, D, Yinv) with A = X diag(D) Yinv
# (eq. def_matrix_as_product): D real, non-negative and sorted decreasing,
# X unitary, |det Yinv| = 1.

def udv_identity(N: int):
    """The identity as a UDV triple (the product starts from P_0 = 1)."""
    return (np.eye(N, dtype=np.complex128), np.ones(N), np.eye(N, dtype=np.complex128))


def _qr_udv(W):
    """Pivoted QR of W: returns (Q', D, Rn_Pt) with W = Q' diag(D) Rn_Pt.

    W Pi = Q R (column pivoting), D = |diag R|, Q' = Q diag(phase(diag R)),
    Rn = D^-1 phase^-1 R (unit diagonal), Rn_Pt = Rn Pi^T.
    """
    Q, R, piv = sla.qr(W, pivoting=True)
    d = np.diag(R).copy()
    D = np.abs(d)
    ph = np.where(D > 0, d / np.where(D > 0, D, 1.0), 1.0)
    Rn = R / np.where(d != 0, d, 1.0)[:, None]
    RnPt = np.empty_like(Rn)
    RnPt[:, piv] = Rn
    return Q * ph[None, :], D, RnPt


def udv_product(A1, A2):
    """Stabilised product of two UDV triples (eqs. prod_2_mat_stab .. res_2_mat_stab).

    A1 A2 = X1 [D1 (Y1^-1 X2) D2] Y2^-1; the bracket is contracted and
    decomposed by QR into X' D Y'^-1, giving X = X1 X', Y^-1 = Y'^-1 Y2^-1.
    """
    X1, D1, Y1inv = A1
    X2, D2, Y2inv = A2
    bracket = D1[:, None] * (Y1inv @ X2) * D2[None, :]
    Xp, D, Ypinv = _qr_udv(bracket)
    return (X1 @ Xp, D, Ypinv @ Y2inv)


def _slice_udv(U, lam_desc, Bphase):
    """B_t = U diag(exp(dk lam)) U^T diag(exp(i phi_t)) as an uncontracted UDV
    triple (Sec. 7 step 2): X = U, D = exp(dk lam) sorted decreasing,
    Y^-1 = U^T diag(exp(i phi_t))."""
    return (U.astype(np.complex128), lam_desc, U.T * Bphase[None, :])


def _slice_factors(K, dk):
    lam, U = np.linalg.eigh(K)
    order = np.argsort(-lam, kind="stable")
    return U[:, order], np.exp(dk * lam[order])


def stabilised_chain(K, dk, phi):
    """UDV of B_{N_t} ... B_1 by multiplying one uncontracted slice at a time
    with the stabilised product (Sec. 7 steps 1-3)."""
    Nt, N = phi.shape
    U, e = _slice_factors(K, dk)
    P = udv_identity(N)
    for t in range(Nt):
        P = udv_product(_slice_udv(U, e, np.exp(1j * phi[t])), P)
    return P


def udv_close(P):
    """log det(1 + P) and (1 + P)^{-1} for P = X D Y^-1 (Sec. 7 steps 4-6).

    1 + D Y^-1 X = Q^ D^ R^ (pivoted QR, diag R^ = 1 after scaling), so
    1 + P = X Q^ D^ R^ Pi^T X^-1,
    log det = log det Q^ + sum log D^ (+ i pi for an odd pivot permutation),
    (1 + P)^-1 = (X Pi R^-1) D^-1 (Q^H X^-1), with X^-1 = X^H for unitary X.
    """
    X, D, Yinv = P
    N = len(D)
    A = np.eye(N, dtype=np.complex128) + D[:, None] * (Yinv @ X)
    Q, R, piv = sla.qr(A, pivoting=True)
    Dh = np.diag(R).copy()
    if np.any(Dh == 0) or not np.all(np.isfinite(Dh)):
        raise np.linalg.LinAlgError("1 + P is singular")
    Rh = R / Dh[:, None]
    sQ, _ = np.linalg.slogdet(Q)
    logdet = 1j * np.angle(sQ) + np.sum(np.log(Dh.astype(np.complex128)))
    if _perm_parity(piv):
        logdet += 1j * math.pi
    Z = (Q.conj().T @ X.conj().T) / Dh[:, None]
    Z = sla.solve_triangular(Rh, Z, lower=False, unit_diagonal=True)
    G = X[:, piv] @ Z
    return wrap_phase(complex(logdet)), G


def logdet_close(P):
    """log det(1 + P) only (Sec. 7 steps 4-5)."""
    return udv_close(P)[0]


def stabilised_logdet_greens(K, dk, phi):
    """log det M and G by the stabilised small-volume method of Sec. 7."""
    return udv_close(stabilised_chain(K, dk, phi))


def sporadic_logdet_greens(K, dk, phi, s):
    """Sec. 9 variant: the accumulated P = X D Y^-1 is re-decomposed only every
    s slices; in between the contracted slices multiply X from the left.

    For a chunk C = B_{t+s} ... B_{t+1}: W = C X D, W = X' D' Y'^-1 (pivoted
    QR), P <- X' D' (Y'^-1 Y^-1).  A last partial chunk handles N_t mod s.
    """
    Nt, N = phi.shape
    B = slice_matrices(K, dk, phi)
    X, D, Yinv = udv_identity(N)
    t = 0
    while t < Nt:
        C = X
        for b in B[t:t + s]:
            C = b @ C
        t += s
        Xp, D, Ypinv = _qr_udv(C * D[None, :])
        X, Yinv = Xp, Ypinv @ Yinv
    return udv_close((X, D, Yinv))


def dsplit_logdet_greens(K, dk, phi, s=1):
    """Cross-check close (an algebraic identity, not from the paper):
    with D_b = max(D, 1), D_s = min(D, 1),
        1 + X D T = X D_b (D_b^-1 X^H T^-1 + D_s) T,
        G = T^-1 (D_b^-1 X^H T^-1 + D_s)^-1 D_b^-1 X^H.
    The chain is the same sporadic chain as above, but the close uses LU.
    """
    Nt, N = phi.shape
    B = slice_matrices(K, dk, phi)
    X, D, T = udv_identity(N)
    t = 0
    while t < Nt:
        C = X
        for b in B[t:t + s]:
            C = b @ C
        t += s
        Xp, D, Tp = _qr_udv(C * D[None, :])
        X, T = Xp, Tp @ T
    Db = np.maximum(D, 1.0)
    Ds = np.minimum(D, 1.0)
    Tinv = np.linalg.inv(T)
    Mid = (X.conj().T @ Tinv) / Db[:, None] + np.diag(Ds)
    sX, lX = np.linalg.slogdet(X)
    sT, lT = np.linalg.slogdet(T)
    sM, lM = np.linalg.slogdet(Mid)
    logdet = (lX + lT + lM + np.sum(np.log(Db))) + 1j * (np.angle(sX) + np.angle(sT) + np.angle(sM))
    G = Tinv @ np.linalg.solve(Mid, X.conj().T / Db[:, None])
    return wrap_phase(complex(logdet)), G


# ---------------------------------------------------------------------------
# force: stabilised prefix / suffix (Sec. 5, dense stabilised pre- and suffix;
# Sec. 4 response formula with t1 = t2)
# ---------------------------------------------------------------------------

def _prefix_suffix(K, dk, phi):
    """prefix[t] = UDV of B_t ... B_1 (prefix[0] = 1);
    suffix[t] = UDV of B_{N_t} ... B_t (suffix[N_t+1] = 1), 1-based t."""
    Nt, N = phi.shape
    U, e = _slice_factors(K, dk)
    slices = [_slice_udv(U, e, np.exp(1j * phi[t])) for t in range(Nt)]
    prefix = [udv_identity(N)]
    for t in range(Nt):
        prefix.append(udv_product(slices[t], prefix[-1]))
    suffix = [None] * (Nt + 2)
    suffix[Nt + 1] = udv_identity(N)
    for t in range(Nt, 0, -1):
        suffix[t] = udv_product(suffix[t + 1], slices[t - 1])
    return prefix, suffix


def stabilised_force_rows(K, dk, phi, rows):
    """Complex force rows F[t-1, :] for the 1-based slice indices in `rows`.

    F_{t,x} = d log det M / d phi_{t,x} = i (1 - G~_t)_{xx} with
    G~_t = (1 + B_{t-1}...B_1 B_{N_t}...B_t)^{-1}: the response formula of
    Sec. 4 for the field of slice t, whose derivative is exactly
    dB_t/dphi_{t,x} = i B_t e_x e_x^T.  Each G~_t gets its own stabilised
    inversion of the cyclically shifted product (Sec. 5, stabilised dense
    pre- and suffix; no wrapping between time slices).
    """
    prefix, suffix = _prefix_suffix(K, dk, phi)
    out = []
    for t in rows:
        _, Gt = udv_close(udv_product(prefix[t - 1], suffix[t]))
        out.append(1j * (1.0 - np.diag(Gt)))
    return np.array(out)


def stabilised_force(K, dk, phi):
    """Complex force F (N_t, N) for every slice (see stabilised_force_rows)."""
    return stabilised_force_rows(K, dk, phi, range(1, phi.shape[0] + 1))


# ---------------------------------------------------------------------------
# observables
# ---------------------------------------------------------------------------

def response_trace(G, A=None):
    """Equal-time response tr((1 - G) A) of one Green's function G = M^{-1}.

    Sec. 4, shortcut for simple operators: the expectation value of an
    operator A is the trace of A against prod_{t'' > t} B M^{-1} prod_{t' <= t} B;
    at the slice where the left product is empty that matrix is
    M^{-1} P = 1 - G (P = M - 1).  A = None stands for A = 1 / V, which gives
    the fermion number n = 1 - tr G / V (eq. fermion_number).  G and A are
    (N, N) arrays; the result is complex.
    """
    G = np.asarray(G, dtype=np.complex128)
    N = G.shape[0]
    if A is None:
        return complex(1.0 - np.trace(G) / N)
    A = np.asarray(A, dtype=np.complex128)
    return complex(np.trace((np.eye(N) - G) @ A))


def slice_response(K, dk, phi, A, rows=None):
    """Per-slice response tr((1 - G~_t) A) to a general operator A (Sec. 4,
    shortcut for simple operators, eq. response_simple before the average
    over t): the matrix inside its trace at slice t is 1 - G~ of the slice
    next to t, with G~_t = (1 + B_{t-1}...B_1 B_{N_t}...B_t)^{-1}, so that
    over all slices the traces are those of the 1 - G~_t, t = 1..N_t.
    Each G~_t is its own stabilised inversion, as in stabilised_force_rows.
    A is an (N, N) array shared by every slice; returns the complex traces
    for the 1-based slices in `rows` (all slices when None); their mean is
    the slice-averaged response."""
    Nt, N = phi.shape
    A = np.asarray(A, dtype=np.complex128)
    rows = range(1, Nt + 1) if rows is None else rows
    prefix, suffix = _prefix_suffix(K, dk, phi)
    out = []
    for t in rows:
        _, Gt = udv_close(udv_product(prefix[t - 1], suffix[t]))
        out.append(np.trace((np.eye(N) - Gt) @ A))
    return np.array(out, dtype=np.complex128)


# ---------------------------------------------------------------------------
# intermediate volume, low temperature: slices in the product form of
# Sec. 8, re-decomposed every s slices (Sec. 9)
# ---------------------------------------------------------------------------

def taylor_product_coefficients(n: int) -> np.ndarray:
    """gamma_1 .. gamma_n with prod_k (1 + gamma_k x) = sum_{j <= n} x^j / j!
    (Sec. 8).  Both sides are degree-n polynomials with constant term 1, so
    the factors vanish where the Taylor polynomial does: gamma_k = -1 / r_k
    for its roots r_k.  Ordered by real part, then imaginary part."""
    if n < 1:
        raise ValueError("n must be >= 1")
    r = np.roots([1.0 / math.factorial(j) for j in range(n, -1, -1)])
    g = -1.0 / r.astype(np.complex128)
    return g[np.lexsort((g.imag, g.real))]


def taylor_slice_matrices(K, dk, phi, n):
    """[B~_1, ..., B~_{N_t}] with B~_t = prod_k (1 + gamma_k dk K)
    diag(e^{i phi_t}): the slices of Sec. 8, exp(dk K) replaced by its
    degree-n Taylor polynomial in product form."""
    N = K.shape[0]
    E = np.eye(N, dtype=np.complex128)
    for g in taylor_product_coefficients(n):
        E = (np.eye(N) + g * dk * K) @ E
    return [E * np.exp(1j * phi[t])[None, :] for t in range(phi.shape[0])]


def sparse_logdet_greens(K, dk, phi, n, s):
    """(log det, G) of M~ = 1 + B~_{N_t} ... B~_1 by the method of Sec. 9:
    from P_0 = 1, each slice is applied to the unitary factor X without
    forming B~_t, as x <- diag(e^{i phi_t}) x followed by the n product-form
    steps x <- x + gamma_k dk (K x) of Sec. 8 (each a sparse product when K
    is stored by its nonzeros); every s slices the accumulated X D Y^-1 is
    re-decomposed by a pivoted QR (the sporadic stabilisation), and the
    result is closed by Sec. 7 steps 4-6."""
    Nt, N = phi.shape
    gam = taylor_product_coefficients(n)
    X, D, Yinv = udv_identity(N)
    t = 0
    while t < Nt:
        C = X.astype(np.complex128)
        for row in range(t, min(t + s, Nt)):
            C = np.exp(1j * phi[row])[:, None] * C
            for g in gam:
                C = C + (g * dk) * (K @ C)
        t += s
        Xp, D, Ypinv = _qr_udv(C * D[None, :])
        X, Yinv = Xp, Ypinv @ Yinv
    return udv_close((X, D, Yinv))


# ---------------------------------------------------------------------------
# molecular dynamics (HMC)
# ---------------------------------------------------------------------------

def hmc_hamiltonian(K, dk, phi, pi, dU):
    """H = 1/2 sum pi^2 + sum phi^2 / (2 dU) - 2 Re log det M(phi): unit-mass
    momenta, the Gaussian weight of the auxiliary field and two fermion
    flavours with complex-conjugate determinants (Sec. 3.1 and
    eq. hamiltonian_alg, whose further terms the paper leaves open)."""
    ld = stabilised_logdet_greens(K, dk, phi)[0]
    return 0.5 * float(np.sum(pi * pi)) + float(np.sum(phi * phi)) / (2.0 * dU) - 2.0 * ld.real


def hmc_leapfrog(K, dk, phi, pi, dU, eps, nsteps):
    """Leapfrog integration of the equations of motion of hmc_hamiltonian:
    half kick, nsteps x (drift, kick) with the last kick halved, where the
    kick uses dH/dphi = phi / dU - 2 Re F (F = d log det M / d phi, the
    stabilised force).  Returns (phi, pi, H_end - H_start)."""
    phi = np.array(phi, dtype=float)
    pi = np.array(pi, dtype=float)
    h0 = hmc_hamiltonian(K, dk, phi, pi, dU)

    def grad(f):
        return f / dU - 2.0 * stabilised_force(K, dk, f).real

    pi = pi - 0.5 * eps * grad(phi)
    for n in range(nsteps):
        phi = phi + eps * pi
        pi = pi - (eps if n + 1 < nsteps else 0.5 * eps) * grad(phi)
    return phi, pi, hmc_hamiltonian(K, dk, phi, pi, dU) - h0


def diag_response(F, a=None):
    """Average over the slices of the response to a diagonal operator
    diag(a): (1 / N_t) sum_t sum_x a_x (1 - G~_t)_xx (Sec. 4 shortcut summed
    over every slice), read off the complex force F_{t,x} = i (1 - G~_t)_xx
    as (1 - G~_t)_xx = -i F_{t,x}.  a = None stands for a_x = 1 / N (the
    fermion number)."""
    F = np.asarray(F, dtype=np.complex128)
    Nt, N = F.shape
    w = np.full(N, 1.0 / N) if a is None else np.asarray(a, dtype=float)
    return complex(np.sum((-1j * F) @ w) / Nt)


# ---------------------------------------------------------------------------
# time-displaced Green's function (Sec. 4, matrix element derivatives,
# eq. sausage_all_in_denominator; Sec. 7 steps 7-9)
# ---------------------------------------------------------------------------
# G(t, t0) is block (t, t0) of the inverse of the block fermion matrix
# (1-based slice labels, G(1, 1) = G).  With P the product of the slices
# from row r = t-1 up to (not including) row r0 = t0-1, cyclically, and Q the
# product of the remaining slices from row r0 on (later slices to the left):
#     t >= t0:  G(t, t0) = + (P + Q^{-1})^{-1},  P = B_{t0-1}...B_1 B_{N_t}...B_t,
#                                               Q = B_{t-1}...B_{t0}
#     t <  t0:  G(t, t0) = - (P + Q^{-1})^{-1},  P = B_{t0-1}...B_t,
#                                               Q = B_{t-1}...B_1 B_{N_t}...B_{t0}
# (for t = t0, P is the whole cyclic product from row r and Q = 1).  These
# are eq. sausage_all_in_denominator in the time order of this oracle.

def displaced_split(Nt: int, t: int, t0: int):
    """(P rows start, P length, Q rows start, Q length, sign) for G(t, t0);
    rows are 0-based and taken cyclically."""
    if not (1 <= t <= Nt and 1 <= t0 <= Nt):
        raise ValueError("t and t0 must lie in [1, N_t]")
    r, r0 = t - 1, t0 - 1
    lp = (r0 - r) % Nt
    if lp == 0:
        lp = Nt
    return r, lp, r0, Nt - lp, (-1.0 if t < t0 else 1.0)


def bruteforce_displaced_greens(K, dk, phi, t, t0):
    """G(t, t0): block (t-1, t0-1) of the inverse block fermion matrix (tier 1)."""
    Mb = block_fermion_matrix(K, dk, phi)
    N = phi.shape[1]
    Minv = np.linalg.inv(Mb)
    return Minv[(t - 1) * N:t * N, (t0 - 1) * N:t0 * N].copy()


def _udv_of_rows(U, e, phi, start, length):
    """UDV of the product of `length` slices from row `start` on, cyclically
    (later rows to the left), one uncontracted slice at a time (Sec. 7)."""
    Nt, N = phi.shape
    P = udv_identity(N)
    for q in range(length):
        row = (start + q) % Nt
        P = udv_product(_slice_udv(U, e, np.exp(1j * phi[row])), P)
    return P


def displaced_greens(K, dk, phi, t, t0):
    """G(t, t0) by Sec. 7 steps 7-9: P = X' D' Y'^-1 and
    Q^-1 = Y'' D''^-1 X''^-1 (here from Q = X_Q D_Q Y_Q^-1: Y'' = Y_Q,
    D''^-1 = D_Q^-1, X'' = X_Q); pivoted QR of
    D' (Y'^-1 X'') + (X'^-1 Y'') D''^-1 = Q R; then
    (P + Q^-1)^-1 = X'' R^-1 Q^H X'^-1 (pivot permutation applied to the rows
    of R^-1), times the sign of the split."""
    Nt, N = phi.shape
    ps, pl, qs, ql, sign = displaced_split(Nt, t, t0)
    U, e = _slice_factors(K, dk)
    Xp, Dp, Ypinv = _udv_of_rows(U, e, phi, ps, pl)
    Xq, Dq, Yqinv = _udv_of_rows(U, e, phi, qs, ql)
    Yq = np.linalg.inv(Yqinv)
    mid = Dp[:, None] * (Ypinv @ Xq) + (Xp.conj().T @ Yq) / Dq[None, :]
    Qm, R, piv = sla.qr(mid, pivoting=True)
    # mid[:, piv] = Qm R  =>  mid^-1 = Pi R^-1 Qm^H with (Pi v)[piv] = v
    Z = sla.solve_triangular(R, Qm.conj().T @ Xp.conj().T, lower=False)
    Y = np.empty_like(Z)
    Y[piv, :] = Z
    return sign * (Xq @ Y)


def dsplit_displaced_greens(K, dk, phi, t, t0):
    """G(t, t0) from the same two chains as displaced_greens, closed with the
    scales split (an algebraic identity, not from the paper).  With
    P = X_P D_P T_P, Q = X_Q D_Q T_Q, D_b = max(D, 1) and D_s = min(D, 1):
        P + Q^-1 = X_P D_Pb W D_Qs^-1 X_Q^H,
        W = D_Ps (T_P X_Q) D_Qs + D_Pb^-1 (X_P^H T_Q^-1) D_Qb^-1,
    so G(t, t0) = sign X_Q D_Qs W^-1 D_Pb^-1 X_P^H.  Every factor of W is
    at most one in size, so no row or column of it mixes scales; the
    unsplit middle matrix of Sec. 7 step 8 does, and loses digits at low
    temperature when both chains are long."""
    Nt, N = phi.shape
    ps, pl, qs, ql, sign = displaced_split(Nt, t, t0)
    U, e = _slice_factors(K, dk)
    Xp, Dp, Tp = _udv_of_rows(U, e, phi, ps, pl)
    Xq, Dq, Tq = _udv_of_rows(U, e, phi, qs, ql)
    Dpb, Dps = np.maximum(Dp, 1.0), np.minimum(Dp, 1.0)
    Dqb, Dqs = np.maximum(Dq, 1.0), np.minimum(Dq, 1.0)
    W = (Dps[:, None] * (Tp @ Xq) * Dqs[None, :]
         + (Xp.conj().T @ np.linalg.inv(Tq)) / (Dpb[:, None] * Dqb[None, :]))
    return sign * (Xq * Dqs[None, :]) @ np.linalg.solve(W, Xp.conj().T / Dpb[:, None])
