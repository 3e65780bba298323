"""GPU parity at the full sizes of the named workloads, in the launch
configurations that bench.py times.

* batched_mix (256 configurations, L in {3,5,6,7,8}, N_t in {32..512}, s = 8,
  segments chosen per configuration by the library): one configuration of
  every (L, N_t) pair element by element against the oracle, and every
  configuration bitwise against a single call with the segments the batch
  gave it;
* force_L8 (N = 128, N_t = 256, beta = 32, c = 16): every force row against
  the oracle's per-slice stabilised inversions, log det, G, finite
  differences;
* hmc_batch (N = 512, N_t = 512, beta = 64, s = 16, c = 16), two fields of one
  batched force plan: log det and G of both fields against the oracle, and
  force rows at checkpoints and at the largest carry distances (8 slices
  back, 7 forward, 1 back across the cyclic boundary) against G of the field
  rotated to start at that row: F_t = i (1 - G~_t)_xx, and G~_t is G of the
  rotated field (pinned on the CPU by test_oracle).
"""
import functools
import math

import numpy as np
import pytest

import oracle as O
from workload import WORKLOADS, batched_mix, hmc_batch

pytestmark = pytest.mark.gpu

TOL_LD = 1e-10
TOL_G = 1e-10
TOL_F = 1e-10


def wrapped(a, b):
    d = complex(a) - complex(b)
    return complex(d.real, math.remainder(d.imag, 2 * math.pi))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def check_ld(ld, ref):
    err = abs(wrapped(ld, ref)) / max(abs(ref), 1e-300)
    assert err <= TOL_LD, (complex(ld), complex(ref), err)


def g_bar(ref):
    return TOL_G * max(1.0, float(np.abs(ref).max()))


# ---------------------------------------------------------------------------
# batched_mix: the 256-configuration batch
# ---------------------------------------------------------------------------

def test_batched_mix_full_batch(fd):
    ws = batched_mix(256)
    probs = [(to_dev(w.K()), to_dev(w.phi()), w.dk) for w in ws]
    plan = fd.Plan("greens", probs, s=8)
    plan.launch()
    ld, Gs = plan.results(check=True)
    seg = plan.segments()
    ld = ld.cpu().numpy()
    Gs = [G.cpu().numpy() for G in Gs]
    print(f"segments per configuration: min {min(seg)} max {max(seg)}", flush=True)
    # every configuration against a single call with the batch's segments
    mism = []
    for i, w in enumerate(ws):
        K, phi, dk = probs[i]
        l1, G1 = fd.greens(K, phi, dk, s=8, segments=seg[i])
        if not (complex(l1.item()) == complex(ld[i]) and np.array_equal(G1.cpu().numpy(), Gs[i])):
            mism.append(i)
    assert not mism, f"batched != single call for configurations {mism[:10]}"
    # configurations 0..24 hold every (L, N_t) pair once
    pairs = {(ws[i].L, ws[i].Nt) for i in range(25)}
    assert len(pairs) == 25
    for i in range(25):
        w = ws[i]
        lo, Go = O.sporadic_logdet_greens(w.K(), w.dk, w.phi(), 8)
        check_ld(ld[i], lo)
        err = np.abs(Gs[i] - Go).max()
        assert err <= g_bar(Go), (i, w.L, w.Nt, err)


# ---------------------------------------------------------------------------
# force_L8: every row
# ---------------------------------------------------------------------------

def test_force_L8_every_row(fd):
    w = WORKLOADS["force_L8"]
    K, phi = w.K(), w.phi()
    Kd, pd = to_dev(K), to_dev(phi)
    plan = fd.Plan("force", [(Kd, pd, w.dk)], s=w.s, checkpoint=w.c, want_g=True)
    plan.launch()
    ld, Fs = plan.results(check=True)
    F = Fs[0].cpu().numpy()
    G = plan.greens()[0].cpu().numpy()
    assert np.abs(F.imag - 0.5).max() < 1e-9
    Fo = O.stabilised_force(K, w.dk, phi)
    err = np.abs(F - Fo).max(axis=1)
    assert err.max() <= TOL_F, (int(err.argmax()), float(err.max()))
    lo, Go = O.stabilised_logdet_greens(K, w.dk, phi)
    check_ld(complex(ld[0].item()), lo)
    assert np.abs(G - Go).max() <= g_bar(Go)
    # central finite differences of log det (h = 1e-6: good to about 3e-7 here)
    h = 1e-6
    rng = np.random.default_rng(1)
    for _ in range(3):
        t, x = int(rng.integers(w.Nt)), int(rng.integers(w.N))
        pp = phi.copy(); pp[t, x] += h
        pm = phi.copy(); pm[t, x] -= h
        lp = complex(fd.logdet(Kd, to_dev(pp), w.dk, s=w.s).item())
        lm = complex(fd.logdet(Kd, to_dev(pm), w.dk, s=w.s).item())
        fdv = wrapped(lp, lm) / (2 * h)
        assert abs(fdv.real - F[t, x].real) <= 1e-6
        assert abs(fdv.imag - F[t, x].imag) <= 1e-6


# ---------------------------------------------------------------------------
# hmc_batch: two of the 32 fields
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def _rotated_greens(j, r):
    """log det and G of field j of hmc_batch rotated to start at 0-based row r
    (QR every 8 slices; G of the rotated field is G~ of row r)."""
    w = hmc_batch(2)[j]
    return O.sporadic_logdet_greens(w.K(), w.dk, np.roll(w.phi(), -r, axis=0), 8)


# rows (0-based): checkpoints 0 and 256; 7 slices carried forward from 0;
# 8 back from 16 and from 272; 1 back from 0 across the cyclic boundary
ROWS = {0: (0, 7, 8, 256, 264, 511), 1: (0, 8)}


def test_hmc_batch_two_fields(fd):
    ws = hmc_batch(2)
    probs = [(to_dev(w.K()), to_dev(w.phi()), w.dk) for w in ws]
    plan = fd.Plan("force", probs, s=ws[0].s, checkpoint=ws[0].c, want_g=True)
    plan.launch()
    ld, Fs = plan.results(check=True)
    Gs = plan.greens()
    for j in (0, 1):
        print(f"field {j}", flush=True)
        lo, Go = _rotated_greens(j, 0)
        check_ld(ld[j].item(), lo)
        G = Gs[j].cpu().numpy()
        assert np.abs(G - Go).max() <= g_bar(Go), (j, np.abs(G - Go).max())
        F = Fs[j].cpu().numpy()
        assert np.abs(F.imag - 0.5).max() < 1e-9
        for r in ROWS[j]:
            _, Gt = _rotated_greens(j, r)
            err = np.abs(F[r] - 1j * (1.0 - np.diag(Gt))).max()
            assert err <= TOL_F * max(1.0, np.abs(Gt).max()), (j, r, err)
