"""fd_greens_noalloc (workspace in the library's fixed device array) against
fd_greens with a caller workspace: bit for bit, on two calls in a row, the
second smaller than the first."""
import numpy as np
import pytest

from workload import WORKLOADS, honeycomb_hopping, sample_phi

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def test_greens_noalloc_matches_greens(fd):
    import torch
    w = WORKLOADS["lowT_L6"]
    cases = [(w.K(), w.phi(), w.dk, w.s, 32),                       # N = 72, N_t = 256
             (honeycomb_hopping(3), sample_phi(11, 16, 18, 0.125, 2.0), 0.125, 4, 4)]   # smaller
    for K, phi, dk, s, seg in cases:
        N = K.shape[0]
        Kd, pd = _dev(K), _dev(phi)
        # outputs allocated up front; the call itself allocates nothing
        ld = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda:0")
        G = torch.full((N * N * 2,), float("nan"), dtype=torch.float64, device="cuda:0")
        st = torch.full((1,), 99, dtype=torch.int32, device="cuda:0")
        fd.greens_noalloc(Kd, pd, dk, ld, G, st, s=s, segments=seg)
        torch.cuda.synchronize()
        l0, G0 = fd.greens(Kd, pd, dk, s=s, segments=seg)
        assert int(st.item()) == 0
        assert np.array_equal(torch.view_as_complex(ld).cpu().numpy(), l0.cpu().numpy())
        assert np.array_equal(torch.view_as_complex(G.view(N, N, 2)).cpu().numpy(),
                              G0.cpu().numpy())


def test_greens_noalloc_rejects_oversize(fd):
    """A call that needs more than the fixed array fails before any launch."""
    import torch
    K = _dev(honeycomb_hopping(16))
    phi = _dev(np.zeros((512, 512)))
    ld = torch.empty(2, dtype=torch.float64, device="cuda:0")
    G = torch.empty(512 * 512 * 2, dtype=torch.float64, device="cuda:0")
    st = torch.empty(1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(fd.FdError) as e:
        fd.greens_noalloc(K, phi, 0.125, ld, G, st, s=16, segments=32)
    assert e.value.code == fd.FD_ERR_WORKSPACE
