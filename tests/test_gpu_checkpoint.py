"""A fit stopped, written to a checkpoint and resumed continues bit for bit as the
uninterrupted fit; a model written to a file serves the same image as the in-memory one."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_resumed_fit_continues_bitwise(tmp_path):
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import checkpoint as ck
    print("[case] checkpoint resume", flush=True)
    w = wl.workload(2)
    t = torch.from_numpy(w.target).cuda()
    raw0 = torch.from_numpy(w.raw0).cuda()
    adam = smoe.AdamConfig(total_steps=2000)
    full = smoe.FitState(t, raw0, 1, adam, max_steps=16)
    part = smoe.FitState(t, raw0, 1, adam, max_steps=16)
    for _ in range(12):
        full.step()
    for _ in range(5):
        part.step()
    p = str(tmp_path / "fit.safetensors")
    ck.save_fit(p, part)
    del part
    res = ck.resume_fit(p, t)
    assert res.steps_done() == 5
    for _ in range(7):
        res.step()
    torch.cuda.synchronize()
    assert res.steps_done() == 12
    assert torch.equal(res.raw, full.raw)
    assert torch.equal(res.m, full.m) and torch.equal(res.v, full.v)
    assert torch.equal(res.model, full.model)
    assert torch.equal(res.loss_history, full.loss_history)


def test_model_file_serves_the_same_image(tmp_path):
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import checkpoint as ck
    from paper_2510_05814_amd.serve import ModelBank, Server
    print("[case] model file", flush=True)
    w = wl.workload(2)
    st = smoe.FitState(torch.from_numpy(w.target).cuda(), torch.from_numpy(w.raw0).cuda(), 1,
                       smoe.AdamConfig(total_steps=20), max_steps=20)
    for _ in range(20):
        st.step()
    p = str(tmp_path / "model.safetensors")
    ck.save_model(p, st.raw, 3, 1, 512, 512)
    rows, infos = ck.load_models_materialized([p])
    assert infos[0]["width"] == 512 and torch.equal(rows[0], st.model)
    bank = ModelBank(rows, 3, 1)
    req = [dict(model=0, scale=2, width=300, height=200, origin_x=17, origin_y=40, arrival=0.0)]
    res, _ = Server(bank).serve(req, realtime=False, keep_outputs=True)
    img, _, _, _ = smoe.render(st.model, 3, 1, smoe.make_grid(300, 200, 2, 17, 40))
    assert torch.equal(res[0].image, img)
