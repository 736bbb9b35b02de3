"""Request loop on the GPU: every result rendered in the mix (continuous
batching, two workers on two streams, Poisson arrivals, mixed image sizes and
modes) equals the same request rendered alone with one call: bit for bit for
depth-sorted requests and additive requests in the deterministic list order,
to rounding for the other additive requests."""
import numpy as np
import pytest

from paper_1606_04427_amd import serve, synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


def _bank(B, ps, n_looks=3):
    bank = []
    for k in range(n_looks):
        looks, pals = [], []
        for sp in range(2):
            s = ps.scalar[ps.species == sp]
            looks.append(dict(log10=1, brightness=0.02 * (1 + sp) * (1 + 0.5 * k),
                              lo=float(np.log10(s.min())), hi=float(np.log10(s.max()))))
            pals.append(synth.palette((sp + k) % 2))
        bank.append((B.Palettes(pals), looks))
    return bank


def _requests(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(64, 64), (128, 128), (256, 256), (200, 120), (96, 160)]
    out = []
    for k in range(n):
        w, h = sizes[rng.integers(len(sizes))]
        pose = synth.random_poses(1, seed=seed * 100 + k, width=w, height=h)[0]
        mode = 2 if rng.uniform() < 0.2 else 1
        look = int(rng.integers(3))
        det = mode == 1 and rng.uniform() < 0.4
        out.append(serve.Request(k, pose, mode, look=look, deterministic=det))
    return out


def test_results_alone_equal_results_in_the_mix():
    import torch

    from paper_1606_04427_amd import binding as B

    ps = synth.soneira_peebles(300_000, seed=61, absorption=True)
    parts = B.DeviceParticles(ps, "cuda:0")
    bank = _bank(B, ps)
    mix = _requests(48, seed=7)
    tagged = set(range(0, 48, 3))  # 16 tagged requests
    keep = lambda r: r.rid in tagged
    cost = lambda r: serve.request_cost(parts.n, r.pose.width, r.pose.height, r.mode == 2,
                                        ordered=r.deterministic)
    srv = serve.Server(lambda w: serve.GpuExecutor(parts, bank), n_workers=2,
                       budget_bytes=6 * sum(cost(mix[0])), max_views=8, cost=cost,
                       keep=keep).start()
    arrivals = synth.poisson_arrivals(len(mix), rate_per_s=2000.0, seed=5)
    serve.drive(srv, mix, arrivals)
    srv.stop()
    assert all(r.error is None for r in mix), [r.error for r in mix if r.error]
    assert srv.n_batches < len(mix)  # some requests shared a batch
    assert srv.peak_reserved <= srv.budget
    alone = [serve.Request(r.rid, r.pose, r.mode, r.look, r.deterministic) for r in mix
             if r.rid in tagged]
    assert any(a.deterministic for a in alone) and any(a.mode == 1 and not a.deterministic
                                                       for a in alone)
    ex = serve.GpuExecutor(parts, bank)
    serve.one_per_call(ex, alone)
    ex.close()
    torch.cuda.synchronize()
    by_id = {r.rid: r for r in mix}
    for a in alone:
        m = by_id[a.rid]
        x, y = m.image.cpu().numpy(), a.image.cpu().numpy()
        if a.mode == 2 or a.deterministic:
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), a.rid
        else:
            assert rel_l2(x, y) < 1e-6, a.rid
        assert m.stats["n_active"] == a.stats["n_active"]
