"""GPU parity of the intermediate-volume low-temperature variant (Sec. 9 with
the product-form Taylor slices of Sec. 8, fd_sparse_greens) against the
oracle's sparse_logdet_greens on the same seeded inputs, the block inverse of
the same slices, and the uniform-field closed form.  Bars as in
test_gpu_parity: relative log det error <= 1e-10 (Im mod 2 pi), max |dG| <=
1e-10 max(1, max |G|)."""
import numpy as np
import pytest

import oracle as O
from workload import honeycomb_hopping, hmc_batch, sample_phi, uniform_phi
from test_gpu_parity import check_G, check_ld, to_dev

pytestmark = pytest.mark.gpu


def gpu_sparse(fd, K, phi, dk, n=4, **kw):
    col, val = fd.ell(to_dev(K))
    ld, G = fd.sparse_greens(col, val, to_dev(phi), dk, n=n, **kw)
    return complex(ld.item()), (G.cpu().numpy() if G is not None else None)


@pytest.mark.parametrize("L,Nt,beta,n,s,seg", [(2, 37, 4.0, 4, 4, 1), (3, 40, 5.0, 4, 8, 3),
                                               (5, 33, 4.0, 6, 16, 2), (6, 64, 8.0, 4, 8, 4),
                                               (7, 24, 3.0, 1, 1, 1), (8, 48, 6.0, 4, 16, 2)])
def test_sparse_vs_oracle(fd, L, Nt, beta, n, s, seg):
    """Every register / LDS class (N = 8 .. 128), N_t not a multiple of s or
    of the segments, Taylor orders 1, 4 and 6."""
    K = honeycomb_hopping(L)
    dk = beta / Nt
    phi = sample_phi(3300 + L, Nt, K.shape[0], dk, 3.0)
    ld, G = gpu_sparse(fd, K, phi, dk, n=n, s=s, segments=seg)
    lo, Go = O.sparse_logdet_greens(K, dk, phi, n, s)
    check_ld(ld, lo)
    check_G(G, Go)
    ld2, G2 = gpu_sparse(fd, K, phi, dk, n=n, s=s, segments=seg, want_g=False)
    assert G2 is None and abs(ld2 - ld) <= 1e-13 * abs(ld)


def test_sparse_vs_block_inverse(fd):
    """L = 2, N_t = 24, beta = 6: against log det and the (1, 1) block of the
    inverse of the block matrix built from the same product-form slices."""
    K = honeycomb_hopping(2)
    Nt, dk = 24, 0.25
    phi = sample_phi(3400, Nt, 8, dk, 3.0)
    Mb = O.block_matrix_of_slices(O.taylor_slice_matrices(K, dk, phi, 4))
    sg, la = np.linalg.slogdet(Mb)
    ld, G = gpu_sparse(fd, K, phi, dk, s=4)
    check_ld(ld, complex(la, np.angle(sg)))
    check_G(G, np.linalg.inv(Mb)[:8, :8])


@pytest.mark.parametrize("L,beta,Nt", [(3, 32.0, 256), (4, 64.0, 512)])
def test_sparse_uniform_closed_form(fd, L, beta, Nt):
    """Space-uniform field at beta = 32 and 64 against the momentum-space
    closed form of the Taylor slices."""
    K = honeycomb_hopping(L)
    N = K.shape[0]
    c = np.random.default_rng(9).normal(0, 0.6, Nt)
    dk = beta / Nt
    lc, Gc = O.uniform_field_taylor_logdet_greens(L, dk, Nt, c.sum(), 4)
    ld, G = gpu_sparse(fd, K, uniform_phi(c, N), dk, s=16, segments=4)
    check_ld(ld, lc)
    check_G(G, Gc)


def test_sparse_generic_rows(fd):
    """A random sparse symmetric K with 1 to 7 nonzeros per row (padded ELL
    rows), N = 45, N_t = 30."""
    rng = np.random.default_rng(3500)
    N = 45
    K = np.zeros((N, N))
    for i in range(N):
        for j in rng.choice(N, size=rng.integers(0, 4), replace=False):
            if j != i:
                K[i, j] = K[j, i] = rng.normal()
    Nt, dk = 30, 0.1
    phi = sample_phi(3501, Nt, N, dk, 3.0)
    ld, G = gpu_sparse(fd, K, phi, dk, s=5, segments=2)
    lo, Go = O.sparse_logdet_greens(K, dk, phi, 4, 5)
    check_ld(ld, lo)
    check_G(G, Go)


@pytest.mark.parametrize("L,Nt,beta,s", [(9, 24, 3.0, 8), (16, 64, 8.0, 16)])
def test_sparse_large_class(fd, L, Nt, beta, s):
    """The blocked class: N = 162 and N = 512."""
    import scipy.sparse as sp
    K = honeycomb_hopping(L)
    dk = beta / Nt
    phi = sample_phi(3600 + L, Nt, K.shape[0], dk, 3.0)
    ld, G = gpu_sparse(fd, K, phi, dk, s=s, segments=2)
    lo, Go = O.sparse_logdet_greens(sp.csr_matrix(K), dk, phi, 4, s)
    check_ld(ld, lo)
    check_G(G, Go)


def test_sparse_full_size(fd):
    """N = 512, N_t = 512, beta = 64, s = 16 (field 0 of the 32-field HMC
    batch), the library's default segments: log det and all of G."""
    import scipy.sparse as sp
    w = hmc_batch()[0]
    K, phi = w.K(), w.phi()
    ld, G = gpu_sparse(fd, K, phi, w.dk, s=16)
    lo, Go = O.sparse_logdet_greens(sp.csr_matrix(K), w.dk, phi, 4, 16)
    check_ld(ld, lo)
    check_G(G, Go)


def test_sparse_batched_mixed(fd):
    """Three problems of different sizes in one call against three single
    calls (the batch runs in the largest class's kernels, whose code for the
    smaller classes may contract multiply-adds differently: equal to
    rounding, not bit for bit)."""
    import ctypes
    import torch
    lib = fd.load_library()
    specs = [(3, 40, 5.0), (6, 24, 3.0), (9, 16, 2.0)]
    probs, hops, keep, singles = [], [], [], []
    for k, (L, Nt, beta) in enumerate(specs):
        K = honeycomb_hopping(L)
        dk = beta / Nt
        phi = to_dev(sample_phi(3700 + k, Nt, K.shape[0], dk, 3.0))
        col, val = fd.ell(to_dev(K))
        keep += [phi, col, val]
        probs.append(fd.FdProblem(K.shape[0], Nt, dk, None, phi.data_ptr()))
        hops.append(fd.FdEll(col.shape[1], col.data_ptr(), val.data_ptr()))
        ld, G = fd.sparse_greens(col, val, phi, dk, s=8, segments=1)
        singles.append((ld.cpu().numpy(), G.cpu().numpy()))
    n = len(specs)
    P = (fd.FdProblem * n)(*probs)
    H = (fd.FdEll * n)(*hops)
    o = fd.FdOptions(8, 0, 1, 0)
    need = lib.fd_sparse_workspace_bytes(P, n, ctypes.byref(o), fd.FD_WHAT_GREENS)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    tot = sum(2 * p.N * p.N for p in probs)
    ld = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    G = torch.empty(tot, dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    rc = lib.fd_sparse_greens_batched(P, n, H, 4, ctypes.byref(o), ld.data_ptr(), G.data_ptr(),
                                      base, need, st.data_ptr(), None)
    assert rc == 0, lib.fd_last_error()
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0] * n
    off = 0
    for k, p in enumerate(probs):
        m = 2 * p.N * p.N
        lk = ld.cpu().numpy()[2 * k:2 * k + 2]
        check_ld(complex(lk[0], lk[1]), complex(singles[k][0]), tol=1e-13)
        got = G.cpu().numpy()[off:off + m].reshape(p.N, p.N, 2)
        check_G(got[..., 0] + 1j * got[..., 1], singles[k][1], tol=1e-13)
        off += m
