"""The serving loop on the GPU: every request's image is the same rendered in a batch of
others (continuous batching over several streams, under a tight memory budget) as rendered
alone, and matches the oracle at sampled pixels; the plain per-request server gives the
same images."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def bank_and_models():
    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.serve import ModelBank
    ms = wl.serving_models(n=6, small=True)
    rng = np.random.default_rng(8)
    models = []
    for m in ms:
        _, mod = wl.grid_init(m["image"], int(round(np.sqrt(m["K"]))),
                              int(round(np.sqrt(m["K"]))), sigma=0.5 * m["side"] /
                              np.sqrt(m["K"]), order=1)
        mod = mod.astype(np.float64)
        K = mod.shape[0]
        # perturb so kernels are anisotropic, rotated and unevenly weighted, like fitted ones
        mod[:, 2] *= np.exp(rng.uniform(-0.4, 0.4, K))
        mod[:, 4] *= np.exp(rng.uniform(-0.4, 0.4, K))
        mod[:, 3] = rng.uniform(-0.5, 0.5, K) * mod[:, 2]
        mod[:, 5] = rng.normal(0.0, 0.3, K)
        mod[:, 9:15] = rng.normal(0.0, 0.01, (K, 6))
        models.append(mod.astype(np.float32))
    del smoe
    return ModelBank(models, 3, 1), models, [m["side"] for m in ms]


def _alone(smoe, bank, r):
    grid = smoe.make_grid(r.width, r.height, r.scale, r.origin_x, r.origin_y)
    img, _, _, _ = smoe.render(bank.rows(r.model), 3, 1, grid)
    return img


@pytest.mark.parametrize("streams,budget_mb", [(2, 4096), (3, 24)])
def test_batched_serving_results_equal_alone(bank_and_models, streams, budget_mb):
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.serve import Server
    bank, models, sides = bank_and_models
    say("serving batched", streams, budget_mb)
    reqs = wl.serving_requests(sides, 48, rate=4000.0, max_side=700, seed=11)
    srv = Server(bank, budget_bytes=budget_mb << 20, streams=streams, max_batch=8)
    res, summ = srv.serve(reqs, keep_outputs=True)
    assert summ["peak_bytes"] <= summ["budget_bytes"]
    assert summ["batches"] < len(reqs) or budget_mb < 100
    for i, r in enumerate(res):
        assert r is not None and r.latency > 0
        assert torch.equal(r.image, _alone(smoe, bank, r.request)), i


def test_plain_and_batched_servers_agree_with_oracle(bank_and_models, record_error):
    import torch

    from paper_2510_05814_amd.serve import PlainServer, Server
    bank, models, sides = bank_and_models
    say("serving plain vs batched vs oracle")
    reqs = wl.serving_requests(sides, 16, rate=1000.0, max_side=512, seed=12)
    rb, sb = Server(bank, streams=2).serve(reqs, keep_outputs=True)
    rp, sp = PlainServer(bank).serve(reqs, keep_outputs=True)
    assert sb["requests"] == sp["requests"] == len(reqs)
    rng = np.random.default_rng(3)
    worst = 0.0
    for a, b in zip(rb, rp):
        assert torch.equal(a.image, b.image)
        q = a.request
        pix = np.stack([rng.integers(0, q.width, 64), rng.integers(0, q.height, 64)], 1)
        y_o, _ = oracle.render(models[q.model].astype(np.float64), 3, 1, q.width, q.height,
                               q.scale, q.origin_x, q.origin_y, pixels=pix)
        got = a.image.cpu().numpy()[pix[:, 1], pix[:, 0]]
        worst = max(worst, float(np.max(np.abs(got - y_o))))
    record_error("serving render abs (sampled)", worst, 1e-5)
    assert worst <= 1e-5


@pytest.mark.parametrize("scale,ox,oy", [(2, 0, 0), (4, 1234, 2345)])
def test_full_size_super_resolution_against_oracle(scale, ox, oy, record_error):
    """A 4096^2 RGB output of the 2048^2, K = 65536 model (the serving workload's largest
    request) through the batched server, at sampled pixels against the oracle."""
    import torch

    from paper_2510_05814_amd.serve import ModelBank, Server
    say("serving full size", scale, ox, oy)
    m = wl.serving_models(n=5)[4]
    assert m["K"] == 65536 and m["side"] == 2048
    _, model = wl.grid_init(m["image"], 256, 256, sigma=4.0, order=1)
    rng = np.random.default_rng(21)
    model = model.astype(np.float64)
    model[:, 2] *= np.exp(rng.uniform(-0.3, 0.3, model.shape[0]))
    model[:, 3] = rng.uniform(-0.4, 0.4, model.shape[0]) * model[:, 2]
    model[:, 9:15] = rng.normal(0.0, 0.01, (model.shape[0], 6))
    model = model.astype(np.float32)
    bank = ModelBank([model], 3, 1)
    req = dict(model=0, scale=scale, width=4096, height=4096, origin_x=ox, origin_y=oy)
    res, summ = Server(bank, streams=1).serve([req, dict(req, origin_x=ox + 7)],
                                               realtime=False, keep_outputs=True)
    pix = np.stack([rng.integers(0, 4096, 1500), rng.integers(0, 4096, 1500)], 1)
    worst = 0.0
    for r in res:
        q = r.request
        y_o, _ = oracle.render(model.astype(np.float64), 3, 1, 4096, 4096, q.scale, q.origin_x,
                               q.origin_y, pixels=pix)
        got = r.image[torch.from_numpy(pix[:, 1]).cuda(), torch.from_numpy(pix[:, 0]).cuda()]
        worst = max(worst, float(np.max(np.abs(got.cpu().numpy() - y_o))))
    record_error(f"serving 4096^2 s={scale} abs (sampled)", worst, 1e-5)
    assert worst <= 1e-5
