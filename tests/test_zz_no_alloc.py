"""The allocation-free step size fcsd_cfl_dt_noalloc (the library's static
per-device scratch) against fcsd_cfl_dt with a workspace, through the C
ABI: equal results on two calls in a row, the second on a smaller input
whose maxima are all below the first's (a scratch not cleared between the
calls would keep the first call's maxima and give a smaller step); more
patches than the scratch holds are refused before any launch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
G = 1.4


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_16076_amd import api
    ctx = api.Context(0)
    yield api, ctx, torch
    ctx.sync()


def _state(ps, mach, seed):
    rng = np.random.default_rng(seed)
    e = synth.mach_state(ps, mach, synth.draw_perturbation(rng))
    u = np.zeros((4, ps.plane), np.float32)
    mu = np.zeros(ps.plane, np.float32)
    for p in range(ps.npatch):
        ps.view(u, p)[...] = ps.view(e, p)
        ps.view(mu, p)[...] = 1e-3 * (1 + p % 3)
    return u, mu


def _both(api, torch, s, ps, u, mu, cfl):
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda:0")
    ud, mud = dev(u), dev(mu)
    a = torch.full((1,), -1.0, device="cuda:0")
    b = torch.full((1,), -1.0, device="cuda:0")
    api.fcsd_cfl_dt(s, ud, mud, cfl, G, a)
    api.fcsd_cfl_dt_noalloc(s, ud, mud, cfl, G, b)
    return float(a.cpu()[0]), float(b.cpu()[0])


def test_noalloc_step_size_equals_workspace_version(env):
    api, ctx, torch = env
    big = synth.uneven_sectors(40, 48, 160, 31)
    small = synth.uneven_sectors(6, 48, 96, 32)
    s1 = api.PatchSet.from_layout(ctx, big)
    s2 = api.PatchSet.from_layout(ctx, small)
    u1, mu1 = _state(big, 5.0, 1)
    u2, mu2 = _state(small, 2.0, 2)
    w1, g1 = _both(api, torch, s1, big, u1, mu1, 0.5)
    w2, g2 = _both(api, torch, s2, small, u2, mu2, 0.5)
    print("dt workspace / static scratch:", w1, g1, "|", w2, g2, flush=True)
    assert g1 == w1 and g2 == w2
    assert w1 > 0 and w2 > w1          # the second input's maxima are smaller
    # again, the large input after the small one
    w3, g3 = _both(api, torch, s1, big, u1, mu1, 0.5)
    assert g3 == w3 == w1
    s1.close()
    s2.close()


def test_noalloc_refuses_more_patches_than_the_scratch_holds(env):
    api, ctx, torch = env
    n = 16385
    n1 = np.full(n, 11, np.int32)
    ps = synth.uneven_sectors(1, 11, 11, 0)
    import dataclasses
    off = np.arange(n, dtype=np.int64) * 128
    many = dataclasses.replace(ps, n1=n1, n2=n1.copy(), C1=np.full(n, ps.C1[0], np.int32),
                               C2=np.full(n, ps.C2[0], np.int32), off=off, plane=int(off[-1]) + 128,
                               htilde=np.full(n, ps.htilde[0]), hhat=np.full(n, ps.hhat[0]),
                               internal=np.zeros((n, 4), np.uint8), metric=None, xy=None)
    s = api.PatchSet.from_layout(ctx, many)
    u = torch.ones(4 * many.plane, device="cuda:0")
    dt = torch.zeros(1, device="cuda:0")
    with pytest.raises(api.FcsdError) as ei:
        api.fcsd_cfl_dt_noalloc(s, u, None, 0.5, G, dt)
    assert "16384" in str(ei.value)
    s.close()
