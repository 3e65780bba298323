"""GPU tests of the runtime around the hot path: prepared-call plans, graph
replay of a force step, the autograd wrapper and the autotuner.  Each result is
checked against the eager entry point (same kernels, so bit-identical) and, on
one case each, against the CPU oracle to the parity bar."""
import math

import numpy as np
import pytest

import oracle as O
from workload import WORKLOADS, honeycomb_hopping, sample_phi

pytestmark = pytest.mark.gpu

TOL = 1e-10


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def wrapped_err(a, b):
    d = complex(a) - complex(b)
    return abs(complex(d.real, math.remainder(d.imag, 2 * math.pi))) / max(abs(complex(b)), 1e-300)


def small_problem(L=3, Nt=32, beta=4.0, U=3.0, seed=11):
    K = honeycomb_hopping(L)
    dk = beta / Nt
    phi = sample_phi(seed, Nt, K.shape[0], dk, U)
    return K, phi, dk


def test_plan_greens_matches_eager(fd):
    import torch
    K, phi, dk = small_problem()
    Kd, pd = to_dev(K), to_dev(phi)
    ld_e, G_e = fd.greens(Kd, pd, dk, s=4, segments=4)
    plan = fd.Plan("greens", [(Kd, pd, dk)], s=4, segments=4)
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        ld, Gs = plan.results(check=True)
        assert torch.equal(ld[0], ld_e) and torch.equal(Gs[0], G_e)
    lo, Go = O.stabilised_logdet_greens(K, dk, phi)
    assert wrapped_err(ld[0].item(), lo) <= TOL
    assert np.abs(Gs[0].cpu().numpy() - Go).max() <= TOL
    plan.close()


def test_plan_reuse_e_and_in_place_phi(fd):
    """A plan with exp(dk K) precomputed follows in-place updates of phi."""
    import torch
    K, phi, dk = small_problem(L=2, Nt=24, beta=3.0)
    Kd, pd = to_dev(K), to_dev(phi)
    plan = fd.Plan("logdet", [(Kd, pd, dk)], s=4, segments=2, reuse_e=True)
    rng = np.random.default_rng(5)
    for _ in range(3):
        new = phi + 0.1 * rng.normal(size=phi.shape)
        pd.copy_(to_dev(new))
        plan.launch()
        ld, _ = plan.results(check=True)
        ref = fd.logdet(Kd, to_dev(new), dk, s=4, segments=2)
        assert torch.equal(ld[0], ref)
        lo, _ = O.stabilised_logdet_greens(K, dk, new)
        assert wrapped_err(ld[0].item(), lo) <= TOL


def test_plan_batched_force_matches_eager(fd):
    import torch
    probs = []
    for i, (L, Nt) in enumerate([(2, 24), (3, 16), (2, 9)]):
        K = honeycomb_hopping(L)
        phi = sample_phi(50 + i, Nt, K.shape[0], 0.25, 3.0)
        probs.append((to_dev(K), to_dev(phi), 0.25))
    Fs_e, ld_e = fd.force_batched(probs, s=4, checkpoint=8)
    plan = fd.Plan("force", probs, s=4, checkpoint=8)
    plan.launch()
    ld, Fs = plan.results(check=True)
    assert torch.equal(ld, ld_e)
    for a, b in zip(Fs, Fs_e):
        assert torch.equal(a, b)


def test_trajectory_graph_replays(fd):
    """The captured force step, replayed on changing fields with eager work and
    synchronisations in between, reproduces the eager force every time."""
    import torch
    K, phi, dk = small_problem(L=3, Nt=48, beta=6.0)
    Kd = to_dev(K)
    traj = fd.Trajectory(Kd, to_dev(phi), dk, s=4, checkpoint=8)
    rng = np.random.default_rng(9)
    fields = [phi + 0.05 * k * rng.normal(size=phi.shape) for k in range(4)]
    for k, f in enumerate(fields):
        ld, F = traj.step(to_dev(f))
        torch.cuda.synchronize()
        ld, F = ld.clone(), F.clone()
        # unrelated eager work between replays
        junk = torch.randn(512, 512, device="cuda:0", dtype=torch.float64)
        (junk @ junk).sum().item()
        F_e, ld_e = fd.force(Kd, to_dev(f), dk, s=4, checkpoint=8, with_logdet=True)
        assert torch.equal(F, F_e), k
        assert torch.equal(ld, ld_e), k
        if k == len(fields) - 1:
            Fo = O.stabilised_force(K, dk, f)
            assert np.abs(F.cpu().numpy() - Fo).max() <= TOL


def test_logdet_autograd(fd):
    """d Re log det / d phi = Re F and d Im log det / d phi = Im F."""
    import torch
    K, phi, dk = small_problem(L=2, Nt=16, beta=2.0)
    Kd = to_dev(K)
    p = to_dev(phi).requires_grad_(True)
    ld = fd.log_det(p, Kd, dk, s=4, checkpoint=8)
    (g_re,) = torch.autograd.grad(ld.real, p, retain_graph=True)
    (g_im,) = torch.autograd.grad(ld.imag, p)
    Fo = O.stabilised_force(K, dk, phi)
    assert np.abs(g_re.cpu().numpy() - Fo.real).max() <= TOL
    assert np.abs(g_im.cpu().numpy() - Fo.imag).max() <= TOL
    lo, _ = O.stabilised_logdet_greens(K, dk, phi)
    assert wrapped_err(ld.detach().item(), lo) <= TOL
    # a real loss mixing both parts: L = 2 Re - 3 Im
    p2 = to_dev(phi).requires_grad_(True)
    ld2 = fd.log_det(p2, Kd, dk, s=4, checkpoint=8)
    (2.0 * ld2.real - 3.0 * ld2.imag).backward()
    assert np.abs(p2.grad.cpu().numpy() - (2.0 * Fo.real - 3.0 * Fo.imag)).max() <= 5 * TOL
    # without grad the forward is the plain log det
    with torch.no_grad():
        ld3 = fd.log_det(to_dev(phi), Kd, dk, s=4)
    assert wrapped_err(ld3.item(), lo) <= TOL


def test_autotune_and_tuned_defaults(fd, tmp_path):
    import torch
    fd.tune_clear()
    w = WORKLOADS["plain_det_L3"]
    K, phi = to_dev(w.K()), to_dev(w.phi())
    best = fd.autotune([(K, phi, w.dk)], what="greens")
    assert best["s"] in (4, 8, 16) and best["segments"] in (1, 2, 4, 8, 16)
    assert best["ms"] > 0
    # calls with s = segments = 0 now take the tuned values
    ld0, G0 = fd.greens(K, phi, w.dk)
    ld1, G1 = fd.greens(K, phi, w.dk, s=best["s"], segments=best["segments"])
    assert torch.equal(ld0, ld1) and torch.equal(G0, G1)
    lo, Go = O.stabilised_logdet_greens(w.K(), w.dk, w.phi())
    assert wrapped_err(ld0.item(), lo) <= TOL
    assert np.abs(G0.cpu().numpy() - Go).max() <= TOL
    path = str(tmp_path / "tune.txt")
    fd.tune_save(path)
    fd.tune_clear()
    assert fd.tune_load(path) == 1
    fb = fd.autotune([(K, phi, w.dk)], what="force", checkpoint=8)
    assert fb["s"] in (4, 8, 16) and fb["checkpoint"] == 8
    fd.tune_clear()


def test_force_plan_returns_greens(fd):
    """The force step's checkpoint at row 0 is G itself."""
    import torch
    K, phi, dk = small_problem(L=3, Nt=32, beta=4.0)
    Kd, pd = to_dev(K), to_dev(phi)
    plan = fd.Plan("force", [(Kd, pd, dk)], s=4, checkpoint=8, want_g=True)
    plan.launch()
    ld, Fs = plan.results(check=True)
    (G,) = plan.greens()
    lo, Go = O.stabilised_logdet_greens(K, dk, phi)
    assert np.abs(G.cpu().numpy() - Go).max() <= TOL
    assert wrapped_err(ld[0].item(), lo) <= TOL
    F_e = fd.force(Kd, pd, dk, s=4, checkpoint=8)
    assert torch.equal(Fs[0], F_e)


def test_batched_trajectory(fd):
    """A batch of fields in one captured step: log det, G and force of each,
    replayed on new fields, against the eager calls."""
    import torch
    probs, fields = [], []
    for i, (L, Nt) in enumerate([(2, 24), (3, 16), (2, 9)]):
        K = honeycomb_hopping(L)
        phi = sample_phi(70 + i, Nt, K.shape[0], 0.25, 3.0)
        probs.append((to_dev(K), to_dev(phi), 0.25))
        fields.append(phi)
    traj = fd.Trajectory(problems=probs, s=4, checkpoint=8, want_g=True)
    rng = np.random.default_rng(3)
    for rep in range(3):
        new = [f + 0.05 * rep * rng.normal(size=f.shape) for f in fields]
        ld, Fs, Gs = traj.step([to_dev(f) for f in new])
        torch.cuda.synchronize()
        for j, ((Kd, _, dk), f) in enumerate(zip(probs, new)):
            F_e, ld_e = fd.force(Kd, to_dev(f), dk, s=4, checkpoint=8, with_logdet=True)
            assert torch.equal(Fs[j], F_e), (rep, j)
            assert torch.equal(ld[j], ld_e), (rep, j)
            _, G_e = fd.greens(Kd, to_dev(f), dk, s=4, segments=1)
            assert np.abs(Gs[j].cpu().numpy() - G_e.cpu().numpy()).max() <= TOL


# ---------------------------------------------------------------------------
# single launch (default) against one launch per phase: bit-identical
# ---------------------------------------------------------------------------

def _single_vs_phased_cases():
    from workload import WORKLOADS, batched_mix, honeycomb_hopping, sample_phi
    return WORKLOADS, batched_mix, honeycomb_hopping, sample_phi


@pytest.mark.gpu
@pytest.mark.skip(reason="FD_SINGLE_LAUNCH is switched off: its run of force_batch_scans (twelve "
                         "N = 18 force problems, grouped scans) did not finish and the cause is "
                         "not known; lowT_L6, batched_mix64 and force_L8 had matched bit for bit")
@pytest.mark.parametrize("case", ["lowT_L6", "batched_mix64", "force_L8", "force_batch_scans",
                                  "large_mixed"])
def test_single_launch_matches_phase_launches(fd, case):
    """The whole call in one persistent launch (FD_SINGLE_LAUNCH: workgroups
    claim items in a precomputed order and wait on completion flags) gives the
    same bits as one launch per phase, for det / G, a mixed batch, the force
    with cyclic windows and with grouped scans, and a batch in the blocked
    class.  """
    import torch
    WORKLOADS, batched_mix, honeycomb_hopping, sample_phi = _single_vs_phased_cases()
    dev = torch.device("cuda:0")

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    S = fd.FD_SINGLE_LAUNCH
    if case == "lowT_L6":
        w = WORKLOADS[case]
        K, phi = t(w.K()), t(w.phi())
        for seg in (1, 8, 32):
            a = fd.greens(K, phi, w.dk, s=w.s, segments=seg, flags=S)
            b = fd.greens(K, phi, w.dk, s=w.s, segments=seg)
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), seg
    elif case == "batched_mix64":
        probs = [(t(w.K()), t(w.phi()), w.dk) for w in batched_mix(64)]
        a = fd.greens_batched(probs, s=8, flags=S)
        b = fd.greens_batched(probs, s=8)
        assert torch.equal(a[0], b[0])
        assert all(torch.equal(x, y) for x, y in zip(a[1], b[1]))
    elif case == "force_L8":
        w = WORKLOADS[case]
        K, phi = t(w.K()), t(w.phi())
        a, la = fd.force(K, phi, w.dk, s=w.s, checkpoint=w.c, with_logdet=True, flags=S)
        b, lb = fd.force(K, phi, w.dk, s=w.s, checkpoint=w.c, with_logdet=True)
        assert torch.equal(a, b) and torch.equal(la, lb)
    elif case == "force_batch_scans":
        K = honeycomb_hopping(3)
        probs = [(t(K), t(sample_phi(40 + i, 96, 18, 0.125, 3.0)), 0.125) for i in range(12)]
        a = fd.force_batched(probs, s=4, checkpoint=4, flags=fd.FD_FORCE_SCANS | S)
        b = fd.force_batched(probs, s=4, checkpoint=4, flags=fd.FD_FORCE_SCANS)
        assert all(torch.equal(x, y) for x, y in zip(a[0], b[0]))
        assert torch.equal(a[1], b[1])
    else:
        probs = []
        for i, L in enumerate((9, 2, 5, 10)):
            K = honeycomb_hopping(L)
            probs.append((t(K), t(sample_phi(70 + i, 24, K.shape[0], 0.125, 3.0)), 0.125))
        a = fd.greens_batched(probs, s=8, segments=2, flags=S)
        b = fd.greens_batched(probs, s=8, segments=2)
        assert torch.equal(a[0], b[0])
        assert all(torch.equal(x, y) for x, y in zip(a[1], b[1]))
        fa = fd.force_batched(probs, s=8, checkpoint=8, flags=S)
        fb = fd.force_batched(probs, s=8, checkpoint=8)
        assert all(torch.equal(x, y) for x, y in zip(fa[0], fb[0]))


# ---------------------------------------------------------------------------
# FD_KEEP_CHECKPOINTS: log det keeps the checkpoints, the force reuses them
# ---------------------------------------------------------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("L,Nt,beta,s,c,scans", [(3, 64, 8.0, 4, 8, False), (2, 90, 9.0, 4, 4, True),
                                                 (6, 256, 32.0, 8, 16, False), (9, 32, 4.0, 4, 8, False)])
def test_keep_checkpoints_matches_full_force(fd, L, Nt, beta, s, c, scans):
    """fd_logdet with FD_KEEP_CHECKPOINTS, then fd_force with it on the same
    workspace (only the checkpoint items run), gives the bits of one full
    fd_force call: log det, G and every force row; fd_greens with the flag
    gives the force plan's G."""
    import torch
    K = honeycomb_hopping(L)
    dk = beta / Nt
    phi = sample_phi(2200 + L, Nt, K.shape[0], dk, 3.0)
    Kd, pd = to_dev(K), to_dev(phi)
    flags = fd.FD_FORCE_SCANS if scans else 0
    keep = flags | fd.FD_KEEP_CHECKPOINTS
    F_full, ld_full = fd.force(Kd, pd, dk, s=s, checkpoint=c, flags=flags, with_logdet=True)
    ws = fd.Workspace()
    ld_keep = fd.logdet(Kd, pd, dk, s=s, checkpoint=c, flags=keep, ws=ws)
    F_keep, ld_again = fd.force(Kd, pd, dk, s=s, checkpoint=c, flags=keep, ws=ws, with_logdet=True)
    assert torch.equal(ld_keep, ld_full) and torch.equal(ld_again, ld_full)
    assert torch.equal(F_keep, F_full)
    lg, G = fd.greens(Kd, pd, dk, s=s, checkpoint=c, flags=keep)
    plan = fd.Plan("force", [(Kd, pd, dk)], s=s, checkpoint=c, want_g=True, flags=flags)
    plan.launch()
    assert torch.equal(G, plan.greens()[0]) and torch.equal(lg, ld_full)
    lo, Go = O.stabilised_logdet_greens(K, dk, phi)
    assert np.abs(G.cpu().numpy() - Go).max() <= 1e-10 * max(1.0, np.abs(Go).max())
