"""Pins for the CPU oracle: brute force, closed forms, N_t = 1, invariants.

Each test checks the oracle against something other than itself: the block
fermion matrix (paper Sec. 2), the momentum-space closed form of the uniform
field, the textbook single-slice determinant, finite differences, and exact
symmetries of the honeycomb model.
"""
import functools
import math

import numpy as np
import pytest

import oracle as O
from workload import honeycomb_hopping, sample_phi, uniform_phi

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def wrapped_diff(a, b):
    d = complex(a) - complex(b)
    return complex(d.real, math.remainder(d.imag, 2 * math.pi))


def rel_err(a, b):
    return abs(wrapped_diff(a, b)) / max(abs(b), 1e-300)


def case(L, Nt, beta, U=3.0, seed=11):
    K = honeycomb_hopping(L)
    N = K.shape[0]
    dk = beta / Nt
    return K, dk, sample_phi(seed, Nt, N, dk, U)


# --- inputs -----------------------------------------------------------------

def test_honeycomb_spectrum_is_plus_minus_abs_f():
    for L in (2, 3, 4, 6):
        lam = np.sort(np.linalg.eigvalsh(honeycomb_hopping(L)))
        f = np.abs(O.honeycomb_dispersion(L))
        ref = np.sort(np.concatenate([f, -f]))
        assert np.abs(lam - ref).max() < 1e-13


def test_honeycomb_structure():
    K = honeycomb_hopping(3)
    assert np.array_equal(K, K.T)
    assert np.all(K.sum(0) == 3)          # coordination number 3
    assert np.trace(K) == 0
    S = np.diag([(-1.0) ** a for a in range(K.shape[0])])
    assert np.array_equal(S @ K @ S, -K)  # bipartite


def test_phi_sampler_variance():
    phi = sample_phi(5, 256, 128, 0.125, 3.0)
    assert phi.shape == (256, 128)
    assert abs(phi.var() - 0.375) < 0.01
    assert np.array_equal(phi, sample_phi(5, 256, 128, 0.125, 3.0))


# --- the single slice -----------------------------------------------------

def test_slice_exponential_inverse_and_series():
    K = honeycomb_hopping(3)
    dk = 0.125
    E = O.slice_exponential(K, dk)
    Ei = O.slice_exponential(K, -dk)
    assert np.abs(E @ Ei - np.eye(18)).max() < 1e-14
    # power series written out (|dk K| <= 0.375)
    A = dk * K
    S = np.eye(18)
    term = np.eye(18)
    for k in range(1, 30):
        term = term @ A / k
        S = S + term
    assert np.abs(E - S).max() < 1e-14


# --- brute force block matrix vs dense definition ----------------------------

@pytest.mark.parametrize("L,Nt,beta", [(2, 1, 0.5), (2, 4, 1.0), (3, 8, 1.0)])
def test_block_matrix_equals_dense_definition(L, Nt, beta):
    K, dk, phi = case(L, Nt, beta)
    l1, G1 = O.bruteforce_logdet_greens(K, dk, phi)
    l0, G0 = O.dense_logdet_greens(K, dk, phi)
    assert rel_err(l1, l0) < 1e-13
    assert np.abs(G1 - G0).max() < 1e-13


def test_single_slice_textbook():
    """N_t = 1: M = 1 + E diag(e^{i phi}) is one dense matrix."""
    for L in (2, 3, 5):
        K, dk, phi = case(L, 1, 0.4, seed=3)
        N = K.shape[0]
        w, V = np.linalg.eigh(K)
        E = (V * np.exp(dk * w)) @ V.T
        A = np.eye(N) + E * np.exp(1j * phi[0])[None, :]
        sign, la = np.linalg.slogdet(A)
        ref = complex(la, np.angle(sign))
        l2, G2 = O.stabilised_logdet_greens(K, dk, phi)
        assert rel_err(l2, ref) < 1e-13
        # rounding bound of an inverse: a few eps * cond(A) * |A^-1|
        Ainv = np.linalg.inv(A)
        tol = 50 * np.finfo(float).eps * np.linalg.cond(A) * np.abs(Ainv).max()
        assert np.abs(G2 - Ainv).max() < tol


# --- stabilised method vs brute force -------------------------------------------

@pytest.mark.parametrize("L,Nt,beta", [(2, 16, 2.0), (2, 64, 16.0), (3, 16, 2.0), (3, 32, 8.0)])
def test_stabilised_matches_bruteforce(L, Nt, beta):
    K, dk, phi = case(L, Nt, beta)
    l1, G1 = O.bruteforce_logdet_greens(K, dk, phi)
    l2, G2 = O.stabilised_logdet_greens(K, dk, phi)
    assert rel_err(l2, l1) < 1e-13
    assert np.abs(G2 - G1).max() < 1e-12
    for s in (1, 3, 4):
        l3, G3 = O.sporadic_logdet_greens(K, dk, phi, s)
        assert rel_err(l3, l1) < 1e-13
        assert np.abs(G3 - G1).max() < 1e-12


@pytest.mark.slow
def test_stabilised_matches_bruteforce_low_temperature():
    """beta = 32 on the block matrix, which stays well conditioned."""
    K, dk, phi = case(2, 256, 32.0)
    l1, G1 = O.bruteforce_logdet_greens(K, dk, phi)
    l2, G2 = O.sporadic_logdet_greens(K, dk, phi, 8)
    assert rel_err(l2, l1) < 1e-13
    assert np.abs(G2 - G1).max() < 1e-12


def test_time_order_is_later_slices_left():
    """The oracle's G belongs to 1 + B_{N_t}...B_1, not to the reversed order
    (the two share a determinant but not the inverse)."""
    K, dk, phi = case(2, 8, 2.0)
    _, G1 = O.bruteforce_logdet_greens(K, dk, phi)
    _, Grev = O.bruteforce_logdet_greens(K, dk, phi[::-1].copy())
    _, G2 = O.stabilised_logdet_greens(K, dk, phi)
    assert np.abs(G2 - G1).max() < 1e-13
    assert np.abs(G2 - Grev).max() > 1e-3


# --- closed forms ---------------------------------------------------------------

def test_closed_form_matches_dense_at_high_temperature():
    for L in (2, 3, 4):
        K = honeycomb_hopping(L)
        N = K.shape[0]
        Nt, beta = 8, 1.0
        c = np.random.default_rng(L).normal(0, 0.4, Nt)
        phi = uniform_phi(c, N)
        l0, G0 = O.dense_logdet_greens(K, beta / Nt, phi)
        lc = O.uniform_field_logdet(L, beta, c.sum())
        Gc = O.uniform_field_greens(L, beta, c.sum())
        assert rel_err(lc, l0) < 1e-13
        assert np.abs(Gc - G0).max() < 1e-13


@pytest.mark.parametrize("L,beta,Nt,s", [(3, 32.0, 256, 8), (3, 64.0, 512, 16), (6, 32.0, 256, 8)])
def test_stabilised_matches_closed_form_low_temperature(L, beta, Nt, s):
    K = honeycomb_hopping(L)
    N = K.shape[0]
    c = np.random.default_rng(2).normal(0, 0.6, Nt)
    phi = uniform_phi(c, N)
    th = c.sum()
    lc = O.uniform_field_logdet(L, beta, th)
    Gc = O.uniform_field_greens(L, beta, th)
    l2, G2 = O.sporadic_logdet_greens(K, beta / Nt, phi, s)
    assert rel_err(l2, lc) < 1e-13
    assert np.abs(G2 - Gc).max() < 1e-11


def test_free_field_phi_zero():
    """phi = 0: log det = sum_k [a_k + 2 log(1 + e^{-a_k})] on each +-|f| pair."""
    L, beta, Nt = 3, 32.0, 256
    K = honeycomb_hopping(L)
    phi = np.zeros((Nt, K.shape[0]))
    a = beta * np.abs(O.honeycomb_dispersion(L))
    ref = float(np.sum(a + 2.0 * np.log1p(np.exp(-a))))
    l2, G2 = O.sporadic_logdet_greens(K, beta / Nt, phi, 8)
    assert abs(l2.real - ref) / ref < 1e-13 and abs(l2.imag) < 1e-12
    assert np.abs(G2 - G2.conj().T).max() < 1e-12       # Hermitian at phi = 0


# --- invariants -------------------------------------------------------------------

@pytest.mark.parametrize("L,Nt,beta", [(3, 32, 4.0), (4, 64, 8.0)])
def test_phase_invariant_and_half_filling(L, Nt, beta):
    """Bipartite K with tr K = 0: Im log det = sum(phi)/2 (mod pi), Re G_xx = 1/2."""
    K, dk, phi = case(L, Nt, beta, seed=17)
    l2, G2 = O.stabilised_logdet_greens(K, dk, phi)
    d = math.remainder(l2.imag - 0.5 * phi.sum(), math.pi)
    assert abs(d) < 1e-11
    assert np.abs(np.diag(G2).real - 0.5).max() < 1e-12 * max(1.0, np.abs(G2).max())


def test_cyclic_shift():
    """Moving B_1 to the far left keeps log det and maps G -> B_1 G B_1^-1."""
    K, dk, phi = case(3, 16, 4.0)
    l1, G1 = O.stabilised_logdet_greens(K, dk, phi)
    l2, G2 = O.stabilised_logdet_greens(K, dk, np.roll(phi, -1, axis=0))
    B1 = O.slice_matrices(K, dk, phi[:1])[0]
    assert rel_err(l2, l1) < 1e-13
    assert np.abs(G2 - B1 @ G1 @ np.linalg.inv(B1)).max() < 1e-12


def test_dsplit_cross_check():
    K, dk, phi = case(4, 128, 16.0)
    l1, G1 = O.sporadic_logdet_greens(K, dk, phi, 8)
    l2, G2 = O.dsplit_logdet_greens(K, dk, phi, 8)
    assert rel_err(l2, l1) < 1e-13
    assert np.abs(G2 - G1).max() < 1e-12


def test_s_independence():
    K, dk, phi = case(3, 64, 8.0)
    l1, G1 = O.sporadic_logdet_greens(K, dk, phi, 1)
    for s in (2, 4, 8, 16):
        l2, G2 = O.sporadic_logdet_greens(K, dk, phi, s)
        assert rel_err(l2, l1) < 1e-13
        assert np.abs(G2 - G1).max() < 1e-12


# --- force -----------------------------------------------------------------------

@pytest.mark.parametrize("L,Nt,beta", [(2, 8, 1.0), (2, 32, 8.0), (3, 16, 2.0)])
def test_force_matches_bruteforce_jacobi(L, Nt, beta):
    K, dk, phi = case(L, Nt, beta)
    F1 = O.bruteforce_force(K, dk, phi)
    F2 = O.stabilised_force(K, dk, phi)
    assert np.abs(F2 - F1).max() < 1e-12
    assert np.abs(F2.imag - 0.5).max() < 1e-12


def test_force_first_row_is_greens_diagonal():
    K, dk, phi = case(3, 16, 4.0)
    _, G = O.stabilised_logdet_greens(K, dk, phi)
    F = O.stabilised_force_rows(K, dk, phi, [1])
    assert np.abs(F[0] - 1j * (1.0 - np.diag(G))).max() < 1e-12


def test_force_row_is_greens_of_rotated_field():
    """Row t of the force is i(1 - diag G) of the field rotated so that slice
    t acts first: that product is B_{t-1}...B_1 B_{N_t}...B_t.  This is the
    cheap oracle for sampled force rows at the largest sizes."""
    K, dk, phi = case(3, 16, 4.0)
    rows = [1, 6, 16]
    F = O.stabilised_force_rows(K, dk, phi, rows)
    for k, t in enumerate(rows):
        _, Gt = O.sporadic_logdet_greens(K, dk, np.roll(phi, -(t - 1), axis=0), 4)
        assert np.abs(F[k] - 1j * (1.0 - np.diag(Gt))).max() < 1e-12


def test_force_finite_differences():
    K, dk, phi = case(3, 16, 4.0)
    F = O.stabilised_force(K, dk, phi)
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(6):
        t, x = int(rng.integers(16)), int(rng.integers(18))
        pp = phi.copy(); pp[t, x] += h
        pm = phi.copy(); pm[t, x] -= h
        lp = O.stabilised_logdet_greens(K, dk, pp)[0]
        lm = O.stabilised_logdet_greens(K, dk, pm)[0]
        fd = wrapped_diff(lp, lm) / (2 * h)
        assert abs(fd.real - F[t, x].real) < 1e-6
        assert abs(fd.imag - F[t, x].imag) < 1e-6


def test_force_uniform_closed_form():
    L, beta, Nt = 3, 8.0, 64
    K = honeycomb_hopping(L)
    c = np.random.default_rng(4).normal(0, 0.5, Nt)
    phi = uniform_phi(c, K.shape[0])
    rows = [1, 17, 64]
    F = O.stabilised_force_rows(K, beta / Nt, phi, rows)
    ref = O.uniform_field_force(L, beta, c.sum())
    assert np.abs(F - ref).max() < 1e-12


# --- one site: scalar closed form ------------------------------------------

def scalar_site(k0, dk, phi):
    """N = 1: every B_t is the number exp(dk k0 + i phi_t), so P is their
    product, log det M = log(1 + P), G = 1 / (1 + P), and every G~_t = G
    (numbers commute): F_t = i (1 - G) = i P / (1 + P)."""
    P = np.exp(len(phi) * dk * k0 + 1j * np.sum(phi))
    G = 1.0 / (1.0 + P)
    return np.log(1.0 + P), G, np.full((len(phi), 1), 1j * P / (1.0 + P))


@pytest.mark.parametrize("Nt", [1, 2, 5])
def test_scalar_site_all_tiers(Nt):
    K = np.array([[0.7]])
    dk = 0.3
    phi = np.random.default_rng(Nt).normal(0, 0.8, (Nt, 1))
    ld, G, F = scalar_site(0.7, dk, phi[:, 0])
    for lo, Go in (O.bruteforce_logdet_greens(K, dk, phi), O.stabilised_logdet_greens(K, dk, phi)):
        assert abs(wrapped_diff(lo, ld)) <= 1e-14
        assert abs(Go[0, 0] - G) <= 1e-14
    assert np.abs(O.stabilised_force(K, dk, phi) - F).max() <= 1e-14
    assert np.abs(O.bruteforce_force(K, dk, phi) - F).max() <= 1e-14


# --- observables (Sec. 4 shortcut) ------------------------------------------

def test_response_kinetic_is_kappa_derivative_uniform_field():
    """Uniform field: phi_{t,x} = c_t commutes with K, so P = e^{i theta}
    exp(beta kappa K) and d log det M / d(beta kappa) = tr(G P K) =
    tr((1 - G) K) exactly; the derivative is taken by central differences of
    the momentum-space closed form."""
    L, beta, Nt = 3, 4.0, 16
    K = honeycomb_hopping(L)
    c = np.random.default_rng(8).normal(0, 0.4, Nt)
    phi = uniform_phi(c, K.shape[0])
    _, G = O.bruteforce_logdet_greens(K, beta / Nt, phi)
    got = O.response_trace(G, K)
    h = 1e-4
    up = O.uniform_field_logdet(L, beta + h, c.sum())
    dn = O.uniform_field_logdet(L, beta - h, c.sum())
    want = (up - dn) / (2 * h)
    assert abs(got - want) <= 1e-7 * abs(want), (got, want)
    assert abs(got.imag) <= 1e-12 * abs(got)


def test_response_fermion_number_half_filling():
    """Bipartite K with zero diagonal: Re G_xx = 1/2 at any field, so
    Re n = 1/2; A = None is A = 1 / V."""
    K, dk, phi = case(2, 12, 3.0)
    _, G = O.bruteforce_logdet_greens(K, dk, phi)
    n = O.response_trace(G)
    assert abs(n.real - 0.5) <= 1e-13
    assert abs(n - O.response_trace(G, np.eye(K.shape[0]) / K.shape[0])) <= 1e-15
    assert abs(n.imag + np.trace(G).imag / K.shape[0]) <= 1e-15


def test_response_rank_one_operator_picks_one_element():
    """tr((1 - G) e_a e_b^T) = delta_ab - G_ba: the trace of a rank-one
    product is a matrix element (catches a transposed operand)."""
    rng = np.random.default_rng(3)
    G = rng.normal(size=(7, 7)) + 1j * rng.normal(size=(7, 7))
    for a, b in ((0, 0), (2, 5), (6, 1)):
        A = np.zeros((7, 7))
        A[a, b] = 1.0
        assert O.response_trace(G, A) == pytest.approx((a == b) - G[b, a], abs=1e-15)


def test_diag_response_averages_the_shifted_greens_functions():
    """The slice average from the force equals (1 / N_t) sum_t tr((1 - G~_t)
    diag(a)) with every G~_t taken from the block-matrix inverse (the
    diagonal blocks of M_block^{-1} are the G~_t), and, for a = 1 / N, the
    fermion number of G itself (G~_t is similar to G)."""
    K, dk, phi = case(2, 10, 2.5, seed=31)
    Nt, N = phi.shape
    F = O.bruteforce_force(K, dk, phi)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))
    a = np.random.default_rng(4).normal(size=N)
    want = np.mean([np.trace((np.eye(N) - Minv[t * N:(t + 1) * N, t * N:(t + 1) * N]) @ np.diag(a))
                    for t in range(Nt)])
    assert abs(O.diag_response(F, a) - want) <= 1e-12 * max(1.0, abs(want))
    _, G = O.bruteforce_logdet_greens(K, dk, phi)
    assert abs(O.diag_response(F) - O.response_trace(G)) <= 1e-12


def _dense_operator(N, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))


def test_slice_response_matches_block_inverse_diagonal_blocks():
    """tr((1 - G~_t) A) for a dense complex A, every slice, against the
    diagonal blocks of the block-matrix inverse (which are the G~_t)."""
    K, dk, phi = case(2, 10, 2.5, seed=33)
    Nt, N = phi.shape
    A = _dense_operator(N, 5)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))
    want = [np.trace((np.eye(N) - Minv[t * N:(t + 1) * N, t * N:(t + 1) * N]) @ A)
            for t in range(Nt)]
    got = O.slice_response(K, dk, phi, A)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    sub = O.slice_response(K, dk, phi, A, rows=[3, 10])
    assert np.abs(sub - got[[2, 9]]).max() == 0.0


def test_slice_response_diagonal_operator_is_the_brute_force_force():
    """For A = diag(a) the traces are sum_x a_x (-i F_{t,x}) with F the
    brute-force force (Jacobi on the block matrix, off-diagonal blocks)."""
    K, dk, phi = case(2, 12, 3.0, seed=34)
    Nt, N = phi.shape
    a = np.random.default_rng(6).normal(size=N)
    F = O.bruteforce_force(K, dk, phi)
    want = (-1j * F) @ a
    got = O.slice_response(K, dk, phi, np.diag(a))
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_slice_response_uniform_field_closed_form():
    """A space-uniform field makes every slice matrix a phase times E, so all
    cyclic products agree and every G~_t is the closed-form G: each trace is
    tr((1 - G) A), here at beta = 32."""
    L, Nt, beta = 3, 128, 32.0
    K = honeycomb_hopping(L)
    c = np.random.default_rng(7).normal(0, 0.6, Nt)
    phi = uniform_phi(c, 18)
    A = _dense_operator(18, 8)
    Gc = O.uniform_field_greens(L, beta, c.sum())
    want = np.trace((np.eye(18) - Gc) @ A)
    got = O.slice_response(K, beta / Nt, phi, A, rows=[1, 50, 128])
    assert np.abs(got - want).max() <= 1e-10 * max(1.0, abs(want))


def test_slice_response_follows_a_rolled_field():
    """Rolling the field by r slices rolls the per-slice traces by r; a
    transposed operand (tr((1 - G~) A^T)) fails the block inverse."""
    K, dk, phi = case(2, 9, 2.0, seed=35)
    Nt, N = phi.shape
    A = _dense_operator(N, 9)
    base = O.slice_response(K, dk, phi, A)
    rolled = O.slice_response(K, dk, np.roll(phi, -4, axis=0), A)
    assert np.abs(rolled - np.roll(base, -4)).max() <= 1e-12 * np.abs(base).max()
    assert np.abs(O.slice_response(K, dk, phi, A.T) - base).max() > 1e-3


# --- molecular dynamics (Sec. 3.1) -----------------------------------------

def _md_case():
    K, dk, phi = case(2, 12, 3.0, seed=21)
    pi = np.random.default_rng(22).standard_normal(phi.shape)
    return K, dk, phi, pi, dk * 3.0


def test_leapfrog_is_reversible():
    """Leapfrog is time-reversible: run, flip the momenta, run again, and the
    start comes back."""
    K, dk, phi, pi, dU = _md_case()
    p1, q1, d1 = O.hmc_leapfrog(K, dk, phi, pi, dU, 0.05, 4)
    p2, q2, d2 = O.hmc_leapfrog(K, dk, p1, -q1, dU, 0.05, 4)
    assert np.abs(p2 - phi).max() <= 1e-11
    assert np.abs(q2 + pi).max() <= 1e-11
    assert abs(d1 + d2) <= 1e-9


def test_leapfrog_energy_error_is_second_order():
    """At a fixed trajectory length the energy error of leapfrog falls as
    eps^2: halving eps divides dH by about 4.  A wrong sign or factor in the
    force would leave dH of order eps or larger."""
    K, dk, phi, pi, dU = _md_case()
    d1 = O.hmc_leapfrog(K, dk, phi, pi, dU, 0.04, 5)[2]
    d2 = O.hmc_leapfrog(K, dk, phi, pi, dU, 0.02, 10)[2]
    assert abs(d1) < 0.05
    assert 0.18 <= abs(d2 / d1) <= 0.32, (d1, d2)


# --- planted mistakes: each must be caught by a pin above --------------------------

def test_pins_catch_planted_mistakes(monkeypatch):
    """A sign error in the close and a dropped pivot parity must both fail."""
    K, dk, phi = case(2, 8, 2.0)
    l1, G1 = O.bruteforce_logdet_greens(K, dk, phi)
    import oracle.fdet_oracle as fo
    monkeypatch.setattr(fo, "_perm_parity", lambda piv: 0)
    bad = [fo.stabilised_logdet_greens(K, dk, p)[0]
           for p in (phi, phi + 0.3, phi * 1.7)]
    good = [O.bruteforce_logdet_greens(K, dk, p)[0] for p in (phi, phi + 0.3, phi * 1.7)]
    assert any(abs(wrapped_diff(b, g)) > 1.0 for b, g in zip(bad, good))
    monkeypatch.undo()
    orig = fo.udv_identity
    monkeypatch.setattr(fo, "udv_identity", lambda N: (orig(N)[0], -orig(N)[1], orig(N)[2]))
    l3, G3 = fo.stabilised_logdet_greens(K, dk, phi)
    assert np.abs(G3 - G1).max() > 1e-3


# --- worked example: two sites, fixture in tests/golden --------------------

def _golden_two_site():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_site.json")
    with open(path) as f:
        doc = json.load(f)
    for c in doc["cases"]:
        ld = complex(*c["logdet"])
        G = np.array([[complex(*z) for z in row] for row in c["G"]])
        F = np.array([[complex(*z) for z in row] for row in c["F"]])
        yield c["dk"], np.array(c["phi"], dtype=float), ld, G, F


def test_golden_two_site_fixture_matches_closed_form():
    """The stored values are those of the 2 x 2 closed form (regenerate with
    tests/golden/make_two_site.py)."""
    for dk, phi, ld, G, F in _golden_two_site():
        ld2, G2, F2 = O.two_site(dk, phi.tolist())
        assert abs(wrapped_diff(ld2, ld)) <= 1e-15 * abs(ld)
        assert np.abs(G2 - G).max() <= 1e-15
        assert np.abs(F2 - F).max() <= 1e-15


def test_golden_two_site_brute_force_and_stabilised():
    """Block fermion matrix (Sec. 2), stabilised UDV (Sec. 7), sporadic QR
    (Sec. 9) and the force (Sec. 4/5) against the two-site closed form."""
    K = np.array([[0.0, 1.0], [1.0, 0.0]])
    for dk, phi, ld, G, F in _golden_two_site():
        lb, Gb = O.bruteforce_logdet_greens(K, dk, phi)
        ls, Gs = O.stabilised_logdet_greens(K, dk, phi)
        lp, Gp = O.sporadic_logdet_greens(K, dk, phi, 4)
        for l2, G2 in ((lb, Gb), (ls, Gs), (lp, Gp)):
            assert rel_err(l2, ld) <= 1e-12
            assert np.abs(G2 - G).max() <= 1e-12
        assert np.abs(O.bruteforce_force(K, dk, phi) - F).max() <= 1e-12
        assert np.abs(O.stabilised_force(K, dk, phi) - F).max() <= 1e-12
        # Im log det = (1/2) sum phi (mod pi) on the bipartite two-site graph
        d = math.remainder(ld.imag - 0.5 * phi.sum(), math.pi)
        assert abs(d) <= 1e-12


def _golden_two_site_extra():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_site.json")
    with open(path) as f:
        doc = json.load(f)
    cz = lambda z: complex(*z)   # noqa: E731
    for c in doc["cases"]:
        disp = {(d["t"], d["t0"]): np.array([[cz(z) for z in row] for row in d["G"]])
                for d in c["displaced"]}
        tay = (cz(c["taylor4"]["logdet"]),
               np.array([[cz(z) for z in row] for row in c["taylor4"]["G"]]))
        A = np.array([[cz(z) for z in row] for row in c["response"]["A"]])
        tr = np.array([cz(z) for z in c["response"]["traces"]])
        yield c["dk"], np.array(c["phi"], dtype=float), disp, tay, A, tr


def test_golden_two_site_extras_match_closed_forms_and_block_inverse():
    """The stored displaced G, Taylor-slice log det / G and per-slice
    responses are those of the 2 x 2 closed forms, and those closed forms
    agree with the block inverse of the matching slices (the displaced G is
    built there from the block rows, not from eq. sausage_all_in_denominator)."""
    K = np.array([[0.0, 1.0], [1.0, 0.0]])
    for dk, phi, disp, (lt, Gt), A, tr in _golden_two_site_extra():
        Nt = len(phi)
        Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))
        for (t, t0), Gd in disp.items():
            assert np.abs(O.two_site_displaced(dk, phi.tolist(), t, t0) - Gd).max() <= 1e-15
            assert np.abs(Minv[(t - 1) * 2:t * 2, (t0 - 1) * 2:t0 * 2] - Gd).max() \
                <= 1e-12 * max(1.0, np.abs(Gd).max())
        assert len(disp) == Nt * Nt
        l2, G2 = O.two_site_taylor(dk, phi.tolist(), 4)
        assert abs(wrapped_diff(l2, lt)) <= 1e-15 * abs(lt) and np.abs(G2 - Gt).max() <= 1e-15
        Mb = O.block_matrix_of_slices(O.taylor_slice_matrices(K, dk, phi, 4))
        sg, la = np.linalg.slogdet(Mb)
        assert rel_err(complex(la, np.angle(sg)), lt) <= 1e-12
        assert np.abs(np.linalg.inv(Mb)[:2, :2] - Gt).max() <= 1e-12
        assert np.abs(O.two_site_slice_response(dk, phi.tolist(), A) - tr).max() <= 1e-15
        want = [np.trace((np.eye(2) - Minv[t * 2:(t + 1) * 2, t * 2:(t + 1) * 2]) @ A)
                for t in range(Nt)]
        assert np.abs(np.array(want) - tr).max() <= 1e-12 * max(1.0, np.abs(tr).max())


def test_golden_two_site_extras_against_the_oracle():
    """The oracle's displaced G (Sec. 7 steps 7-9 as written and the split
    close), its intermediate-volume variant (Sec. 9, n = 4, QR every 1, 3 and
    5 slices) and its per-slice responses against the stored values."""
    K = np.array([[0.0, 1.0], [1.0, 0.0]])
    for dk, phi, disp, (lt, Gt), A, tr in _golden_two_site_extra():
        for (t, t0), Gd in disp.items():
            bar = 1e-12 * max(1.0, np.abs(Gd).max())
            assert np.abs(O.displaced_greens(K, dk, phi, t, t0) - Gd).max() <= bar, (t, t0)
            assert np.abs(O.dsplit_displaced_greens(K, dk, phi, t, t0) - Gd).max() <= bar, (t, t0)
        for s in (1, 3, 5):
            l2, G2 = O.sparse_logdet_greens(K, dk, phi, 4, s)
            assert rel_err(l2, lt) <= 1e-12 and np.abs(G2 - Gt).max() <= 1e-12
        assert np.abs(O.slice_response(K, dk, phi, A) - tr).max() <= 1e-12 * max(1.0, np.abs(tr).max())


def test_response_pins_catch_planted_mistakes():
    """A transposed operand and a dropped identity must fail the pins above."""
    rng = np.random.default_rng(3)
    G = rng.normal(size=(7, 7)) + 1j * rng.normal(size=(7, 7))
    A = np.zeros((7, 7))
    A[2, 5] = 1.0
    transposed = complex(np.trace((np.eye(7) - G) @ A.T))
    assert abs(transposed - ((2 == 5) - G[5, 2])) > 1e-3
    K, dk, phi = case(2, 12, 3.0)
    _, Gk = O.bruteforce_logdet_greens(K, dk, phi)
    no_identity = complex(-np.trace(Gk) / K.shape[0])
    assert abs(no_identity.real - 0.5) > 1e-3


def test_md_pins_catch_planted_mistakes(monkeypatch):
    """A force with the wrong sign, or the fermion term counted once, breaks
    the eps^2 law above."""
    import oracle.fdet_oracle as fo
    K, dk, phi, pi, dU = _md_case()
    orig = fo.stabilised_force
    for bad in (lambda K_, dk_, f: -orig(K_, dk_, f), lambda K_, dk_, f: 0.5 * orig(K_, dk_, f)):
        monkeypatch.setattr(fo, "stabilised_force", bad)
        d1 = fo.hmc_leapfrog(K, dk, phi, pi, dU, 0.04, 5)[2]
        d2 = fo.hmc_leapfrog(K, dk, phi, pi, dU, 0.02, 10)[2]
        assert not (abs(d1) < 0.05 and 0.18 <= abs(d2 / d1) <= 0.32), (d1, d2)
    monkeypatch.undo()


# ---------------------------------------------------------------------------
# time-displaced Green's function G(t, t0) (eq. sausage_all_in_denominator,
# Sec. 7 steps 7-9)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("beta", [1.5, 6.0])
def test_displaced_matches_block_inverse_every_pair(beta):
    """Every (t, t0) block of the inverse block fermion matrix (L = 2,
    N_t = 12), including both signs of t - t0 and t = t0."""
    K = honeycomb_hopping(2)
    Nt = 12
    dk = beta / Nt
    phi = sample_phi(31, Nt, 8, dk, 3.0)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))
    for t in range(1, Nt + 1):
        for t0 in range(1, Nt + 1):
            Gb = Minv[(t - 1) * 8:t * 8, (t0 - 1) * 8:t0 * 8]
            G = O.displaced_greens(K, dk, phi, t, t0)
            assert np.abs(G - Gb).max() <= 1e-12 * max(1.0, np.abs(Gb).max()), (t, t0)


def test_displaced_block_inverse_helper():
    K = honeycomb_hopping(2)
    phi = sample_phi(32, 6, 8, 0.2, 3.0)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, 0.2, phi))
    assert np.array_equal(O.bruteforce_displaced_greens(K, 0.2, phi, 4, 2), Minv[24:32, 8:16])


def test_displaced_split_ranges():
    """P and Q cover the N_t slices once; P starts at row t - 1."""
    for Nt in (1, 2, 7):
        for t in range(1, Nt + 1):
            for t0 in range(1, Nt + 1):
                ps, pl, qs, ql, sg = O.displaced_split(Nt, t, t0)
                assert ps == t - 1 and qs == t0 - 1 and pl + ql == Nt and pl >= 1
                assert sg == (-1.0 if t < t0 else 1.0)
                rows = {(ps + q) % Nt for q in range(pl)} | {(qs + q) % Nt for q in range(ql)}
                assert rows == set(range(Nt))


def test_displaced_equal_time_is_shifted_greens():
    """G(t, t) is the equal-time Green's function of the field rotated to start
    at slice t; G(1, 1) = G."""
    K = honeycomb_hopping(3)
    Nt, beta = 40, 8.0
    dk = beta / Nt
    phi = sample_phi(33, Nt, 18, dk, 3.0)
    _, G = O.stabilised_logdet_greens(K, dk, phi)
    assert np.abs(O.displaced_greens(K, dk, phi, 1, 1) - G).max() <= 1e-12
    _, Gt = O.stabilised_logdet_greens(K, dk, np.roll(phi, -9, axis=0))
    assert np.abs(O.displaced_greens(K, dk, phi, 10, 10) - Gt).max() <= 1e-12


def test_displaced_row_step():
    """Rows of the block inverse obey the fermion matrix: for t0 != t + 1,
    G(t + 1, t0) = B_t G(t, t0) (B_t the slice between t and t + 1), and
    G(1, t0) = -B_{N_t} G(N_t, t0) across the anti-periodic boundary."""
    K = honeycomb_hopping(3)
    Nt, beta = 24, 12.0
    dk = beta / Nt
    phi = sample_phi(34, Nt, 18, dk, 3.0)
    B = O.slice_matrices(K, dk, phi)
    for t0 in (1, 9, 24):
        for t in range(1, Nt):
            if t + 1 == t0:
                continue
            G1 = O.displaced_greens(K, dk, phi, t + 1, t0)
            G0 = O.displaced_greens(K, dk, phi, t, t0)
            assert np.abs(G1 - B[t - 1] @ G0).max() <= 1e-11 * max(1.0, np.abs(G1).max()), (t, t0)
        if t0 != 1:
            G1 = O.displaced_greens(K, dk, phi, 1, t0)
            GN = O.displaced_greens(K, dk, phi, Nt, t0)
            assert np.abs(G1 + B[Nt - 1] @ GN).max() <= 1e-11 * max(1.0, np.abs(G1).max())


@pytest.mark.parametrize("t,t0", [(1, 1), (200, 17), (17, 200), (256, 1), (1, 256), (129, 128)])
def test_displaced_uniform_closed_form_low_temperature(t, t0):
    """Space-uniform field at beta = 32 (cond of the slice product ~ 1e41):
    the stabilised form against the eigenbasis closed form."""
    L, Nt, beta = 3, 256, 32.0
    K = honeycomb_hopping(L)
    dk = beta / Nt
    c = np.random.default_rng(2).normal(0, 0.6, Nt)
    phi = uniform_phi(c, 18)
    Gc = O.uniform_field_displaced_greens(K, dk, c, t, t0)
    G = O.displaced_greens(K, dk, phi, t, t0)
    assert np.abs(G - Gc).max() <= 1e-11


def test_displaced_pins_catch_planted_mistakes(monkeypatch):
    """A wrong sign for t < t0 or P and Q swapped fail the block inverse."""
    from oracle import fdet_oracle as F
    K = honeycomb_hopping(2)
    Nt, dk = 6, 0.25
    phi = sample_phi(35, Nt, 8, dk, 3.0)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))

    def worst():
        e = 0.0
        for t in range(1, Nt + 1):
            for t0 in range(1, Nt + 1):
                Gb = Minv[(t - 1) * 8:t * 8, (t0 - 1) * 8:t0 * 8]
                e = max(e, np.abs(F.displaced_greens(K, dk, phi, t, t0) - Gb).max())
        return e

    assert worst() < 1e-12
    orig = F.displaced_split
    monkeypatch.setattr(F, "displaced_split",
                        lambda n, t, t0: orig(n, t, t0)[:4] + (1.0,))
    assert worst() > 1e-3
    monkeypatch.setattr(F, "displaced_split",
                        lambda n, t, t0: (lambda r: (r[2], r[3], r[0], r[1], r[4]))(orig(n, t, t0)))
    assert worst() > 1e-3


@functools.lru_cache(maxsize=None)
def _low_temperature_block_inverse():
    """L = 2, N_t = 128, beta = 32: the block inverse (dimension 1024) and the
    field, shared by the low-temperature displaced pins."""
    K = honeycomb_hopping(2)
    Nt, beta = 128, 32.0
    dk = beta / Nt
    phi = sample_phi(8, Nt, 8, dk, 3.0)
    return K, dk, phi, np.linalg.inv(O.block_fermion_matrix(K, dk, phi))


@pytest.mark.parametrize("t,t0", [(1, 1), (70, 3), (3, 70), (128, 1), (1, 128), (40, 39), (39, 40)])
def test_dsplit_displaced_matches_block_inverse_low_temperature(t, t0):
    """The split close of G(t, t0) against the block inverse at beta = 32,
    random field, both chains long."""
    K, dk, phi, Minv = _low_temperature_block_inverse()
    Gb = Minv[(t - 1) * 8:t * 8, (t0 - 1) * 8:t0 * 8]
    G = O.dsplit_displaced_greens(K, dk, phi, t, t0)
    assert np.abs(G - Gb).max() <= 1e-12 * max(1.0, np.abs(Gb).max()), (t, t0)


def test_unsplit_displaced_close_loses_digits_at_low_temperature():
    """The middle matrix of Sec. 7 step 8 taken as written mixes scales in
    its rows and columns: at beta = 32 with both chains long it is off the
    block inverse by far more than rounding, while the split close is not
    (the reason the GPU path and the low-temperature parity reference use
    the split form)."""
    K, dk, phi, Minv = _low_temperature_block_inverse()
    Gb = Minv[69 * 8:70 * 8, 2 * 8:3 * 8]
    assert np.abs(O.displaced_greens(K, dk, phi, 70, 3) - Gb).max() > 1e-9
    assert np.abs(O.dsplit_displaced_greens(K, dk, phi, 70, 3) - Gb).max() < 1e-12


def test_dsplit_displaced_every_pair_and_closed_form():
    """Every pair at L = 2, N_t = 12, beta = 6 against the block inverse, and
    the uniform-field closed form at beta = 32."""
    K = honeycomb_hopping(2)
    Nt, dk = 12, 0.5
    phi = sample_phi(31, Nt, 8, dk, 3.0)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))
    for t in range(1, Nt + 1):
        for t0 in range(1, Nt + 1):
            Gb = Minv[(t - 1) * 8:t * 8, (t0 - 1) * 8:t0 * 8]
            G = O.dsplit_displaced_greens(K, dk, phi, t, t0)
            assert np.abs(G - Gb).max() <= 1e-12 * max(1.0, np.abs(Gb).max()), (t, t0)
    K = honeycomb_hopping(3)
    Nt, beta = 256, 32.0
    dk = beta / Nt
    c = np.random.default_rng(2).normal(0, 0.6, Nt)
    phi = uniform_phi(c, 18)
    for t, t0 in [(200, 17), (17, 200), (1, 1)]:
        Gc = O.uniform_field_displaced_greens(K, dk, c, t, t0)
        assert np.abs(O.dsplit_displaced_greens(K, dk, phi, t, t0) - Gc).max() <= 1e-11


def test_dsplit_displaced_catches_planted_mistakes(monkeypatch):
    """A wrong sign for t < t0, or the P and Q chains swapped, fails the
    block inverse."""
    from oracle import fdet_oracle as F
    K = honeycomb_hopping(2)
    Nt, dk = 8, 0.5
    phi = sample_phi(36, Nt, 8, dk, 3.0)
    Minv = np.linalg.inv(O.block_fermion_matrix(K, dk, phi))

    def worst():
        e = 0.0
        for t in range(1, Nt + 1):
            for t0 in range(1, Nt + 1):
                Gb = Minv[(t - 1) * 8:t * 8, (t0 - 1) * 8:t0 * 8]
                e = max(e, np.abs(F.dsplit_displaced_greens(K, dk, phi, t, t0) - Gb).max())
        return e

    assert worst() < 1e-12
    orig = F.displaced_split
    monkeypatch.setattr(F, "displaced_split", lambda n, t, t0: orig(n, t, t0)[:4] + (1.0,))
    assert worst() > 1e-3
    monkeypatch.setattr(F, "displaced_split",
                        lambda n, t, t0: (lambda r: (r[2], r[3], r[0], r[1], r[4]))(orig(n, t, t0)))
    assert worst() > 1e-3


# ---------------------------------------------------------------------------
# intermediate volume, low temperature: product-form Taylor slices (Sec. 8)
# with sporadic QR (Sec. 9)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", range(1, 9))
def test_taylor_product_expands_to_the_taylor_polynomial(n):
    """prod_k (1 + gamma_k x) multiplied out by hand has the coefficients
    1 / j! of the degree-n Taylor polynomial of exp; the gammas come in
    conjugate pairs (real polynomial)."""
    g = O.taylor_product_coefficients(n)
    assert len(g) == n
    coef = np.zeros(n + 1, dtype=complex)   # coef[j] multiplies x^j
    coef[0] = 1.0
    for gk in g:
        coef[1:] = coef[1:] + gk * coef[:-1]
    want = np.array([1.0 / math.factorial(j) for j in range(n + 1)])
    assert np.abs(coef - want).max() <= 1e-13
    assert np.abs(np.sort_complex(g) - np.sort_complex(g.conj())).max() <= 1e-14


def test_taylor_slices_against_the_series():
    """The product-form slice at x = dk K equals the truncated series
    sum_j (dk K)^j / j! summed by powers."""
    K = honeycomb_hopping(3)
    dk, n = 0.125, 4
    phi = np.zeros((1, 18))
    B = O.taylor_slice_matrices(K, dk, phi, n)[0]
    S = np.zeros((18, 18))
    P = np.eye(18)
    for j in range(n + 1):
        S = S + P / math.factorial(j)
        P = P @ (dk * K)
    assert np.abs(B - S).max() <= 1e-15


@pytest.mark.parametrize("n,s", [(4, 1), (4, 4), (3, 8), (6, 5)])
def test_sparse_variant_matches_block_inverse(n, s):
    """Sec. 9 with product-form slices against log det and the (1, 1) block
    of the inverse of the block matrix built from the same slices (L = 2,
    N_t = 24, beta = 6, s not dividing N_t in one case)."""
    K, dk, phi = case(2, 24, 6.0, seed=40)
    Mb = O.block_matrix_of_slices(O.taylor_slice_matrices(K, dk, phi, n))
    sgn, la = np.linalg.slogdet(Mb)
    lb = complex(la, np.angle(sgn))
    Gb = np.linalg.inv(Mb)[:8, :8]
    ld, G = O.sparse_logdet_greens(K, dk, phi, n, s)
    assert rel_err(ld, lb) <= 1e-12
    assert np.abs(G - Gb).max() <= 1e-12


@pytest.mark.parametrize("L,beta,Nt,n", [(3, 32.0, 256, 4), (4, 64.0, 512, 4), (3, 32.0, 256, 2)])
def test_sparse_variant_uniform_field_closed_form(L, beta, Nt, n):
    """A uniform field at beta = 32 and 64: log det and G against the
    momentum-space closed form of the Taylor slices (cond of the product up
    to ~1e83)."""
    K = honeycomb_hopping(L)
    N = K.shape[0]
    c = np.random.default_rng(9).normal(0, 0.6, Nt)
    dk = beta / Nt
    lc, Gc = O.uniform_field_taylor_logdet_greens(L, dk, Nt, c.sum(), n)
    ld, G = O.sparse_logdet_greens(K, dk, uniform_phi(c, N), n, 16)
    assert rel_err(ld, lc) <= 1e-12
    assert np.abs(G - Gc).max() <= 1e-11


def test_sparse_variant_tends_to_the_exact_slices():
    """With n = 14 the Taylor remainder (0.375^15 / 15! ~ 1e-19 per slice) is
    below rounding: the variant equals the exact stabilised oracle; with
    n = 4 it differs by the truncation, which shrinks as n grows."""
    K, dk, phi = case(3, 32, 4.0, seed=41)
    l0, G0 = O.sporadic_logdet_greens(K, dk, phi, 4)
    l14, G14 = O.sparse_logdet_greens(K, dk, phi, 14, 4)
    assert rel_err(l14, l0) <= 1e-12 and np.abs(G14 - G0).max() <= 1e-11
    errs = [np.abs(O.sparse_logdet_greens(K, dk, phi, n, 4)[1] - G0).max() for n in (3, 4, 5, 6)]
    assert errs[0] > errs[1] > errs[2] > errs[3] > 1e-12


def test_sparse_variant_catches_planted_mistakes(monkeypatch):
    """Applying the field after the hopping factors, or conjugated gammas
    with a flipped sign, fails the block inverse."""
    from oracle import fdet_oracle as F
    K, dk, phi = case(2, 12, 3.0, seed=42)
    Mb = O.block_matrix_of_slices(O.taylor_slice_matrices(K, dk, phi, 4))
    Gb = np.linalg.inv(Mb)[:8, :8]
    assert np.abs(F.sparse_logdet_greens(K, dk, phi, 4, 4)[1] - Gb).max() < 1e-12
    real = F.taylor_product_coefficients
    monkeypatch.setattr(F, "taylor_product_coefficients", lambda n: -real(n).conj())
    assert np.abs(F.sparse_logdet_greens(K, dk, phi, 4, 4)[1] - Gb).max() > 1e-3
    monkeypatch.undo()
    # field after the hopping factors: rotate which factor acts first
    Bwrong = [np.exp(1j * phi[t])[:, None] * O.taylor_slice_matrices(K, dk, np.zeros_like(phi), 4)[t]
              for t in range(phi.shape[0])]
    Gw = np.linalg.inv(O.block_matrix_of_slices(Bwrong))[:8, :8]
    assert np.abs(F.sparse_logdet_greens(K, dk, phi, 4, 4)[1] - Gw).max() > 1e-3
