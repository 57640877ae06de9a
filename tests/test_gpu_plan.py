"""Setup / apply split: a frozen plan replayed as a HIP graph equals the eager
evaluation of the same density, on every replay, with eager work and
synchronisations in between; a density with a wider band is refused."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def evs():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    a, b = pk.Evaluator(quad_tol=1e-12), pk.Evaluator(quad_tol=1e-12)
    yield a, b
    a.close()
    b.close()


def test_plan_apply_replays_equal_eager(evs):
    import torch
    import paper_2310_00889_amd as pk
    ev, ref = evs
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    ev.set_geometry(sc)
    ref.set_geometry(sc)
    tn = np.arange(sc.n_nodes, dtype=np.int64)
    u0, d0 = ev.plan(sc.sigma, None, tn)
    e0, f0 = ref.eval(sc.sigma, None, tn)
    assert np.array_equal(u0, e0) and np.array_equal(d0, f0)
    sig2 = -1.5 * sc.sigma[:, [1, 2, 0]]
    us_ref, ud_ref = ref.eval(sig2, None, tn)
    for k in range(4):
        us, ud = ev.apply(sig2)
        assert np.array_equal(us, us_ref) and np.array_equal(ud, ud_ref), k
        # the program's own eager work between replays
        a = torch.randn(4096, device="cuda")
        (a * a).sum().item()
        ref.eval(sc.sigma, None, tn[:100])
        torch.cuda.synchronize()
    # device arrays
    usd, udd = ev.apply(torch.from_numpy(sig2.copy()).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(usd.cpu().numpy(), us_ref) and np.array_equal(udd.cpu().numpy(), ud_ref)
    # a density with every Fourier mode present exceeds the plan's band
    noisy = sc.sigma + 1e-3 * np.random.default_rng(1).normal(size=sc.sigma.shape)
    with pytest.raises(pk.CsbqError):
        ev.apply(noisy)
    # any other evaluation drops the plan
    ev.eval(sc.sigma, None, tn[:10])
    with pytest.raises(pk.CsbqError):
        ev.apply(sig2)


def test_plan_apply_pipe_with_spheres(evs):
    """The 200-sphere pipe (153,600 targets): replay equals the eager
    evaluation; the replay skips search, classification and host round trips."""
    import torch
    ev, ref = evs
    sc = synth.config2()
    ev.set_geometry(sc)
    ref.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(sc.tgt_node).cuda()
    ev.plan(sig, None, tn)
    sig2 = torch.from_numpy(np.ascontiguousarray(0.5 * sc.sigma[:, [2, 0, 1]])).cuda()
    ref.eval(sig2, None, tn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us_ref, ud_ref = ref.eval(sig2, None, tn)
    torch.cuda.synchronize()
    t_eval = time.perf_counter() - t0
    ev.apply(sig2)
    t0 = time.perf_counter()
    us, ud = ev.apply(sig2)
    torch.cuda.synchronize()
    t_apply = time.perf_counter() - t0
    print(f"eval {1e3 * t_eval:.1f} ms, apply {1e3 * t_apply:.1f} ms", flush=True)
    # the two contexts may have tuned different smooth-sum shapes (summation order)
    for a, b in ((us, us_ref), (ud, ud_ref)):
        assert float((a - b).abs().max() / b.abs().max()) < 1e-13
