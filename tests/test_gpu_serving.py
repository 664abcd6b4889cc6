"""Serving loop (many scenes on one GPU): a scene's result in the mix equals
its result alone bit for bit, the HBM budget bounds admission, and a served
scene matches the FP64 oracle."""
import numpy as np
import pytest

import workloads as WL
from gpu_common import note

pytestmark = pytest.mark.gpu


def small_stream(count, n_max=2 ** 14, steps=20, seed=3):
    return [WL.c4_scene(seed, i, steps=steps, n_max=n_max, materialize=False) for i in range(count)]


@pytest.mark.parametrize("batched", [True, False])
def test_serving_isolation(gpu_lib, batched):
    from paper_2207_04658_amd.serving import Server
    note(f"serving: 8 scenes mixed vs alone, batched={batched}")
    scenes = small_stream(8)
    mixed = Server(streams=4, steps_per_tick=3, keep_words=True, batched=batched).run(scenes)
    assert set(mixed.latencies_s) == {s["name"] for s in scenes}
    assert mixed.max_active == 8
    for s in scenes:
        # alone, through the other launch path and another tick length
        alone = Server(streams=1, steps_per_tick=7, keep_words=True, batched=not batched).run([s])
        assert np.array_equal(alone.words[s["name"]], mixed.words[s["name"]]), s["name"]
    assert mixed.particle_substeps == sum(s["n"] * s["steps"] for s in scenes)


def test_step_batch_equals_step(gpu_lib):
    """mpmq_step_batch on contexts of different schemes, grids, sizes and
    sort intervals (3D, one of them empty) against mpmq_step on each: words,
    ids and statistics identical, step counters advanced."""
    import torch
    from gpu_common import gpu_context
    note("step_batch vs step: five 3D scenes")
    scenes = [s for s in small_stream(24, n_max=5000) if s["params"]["dim"] == 3][:4]
    assert len(scenes) == 4
    for s, se in zip(scenes, (0, 3, 5, 0)):
        s["params"] = dict(s["params"], sort_every=se)
        s["state"] = WL.c4_state(s)
    empty = dict(scenes[0], name="empty", n=0,
                 state=tuple(a[:, :0] for a in scenes[0]["state"]))
    scenes.append(empty)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = [gpu_context(gpu_lib, s, capacity=max(s["n"], 1)) for s in scenes]
        b = [gpu_context(gpu_lib, s, capacity=max(s["n"], 1)) for s in scenes]
        for c in a:
            c.set_stats(1)
        for c in b:
            c.set_stats(1)
        gpu_lib.step_batch(a, 4)
        gpu_lib.step_batch(a[1:], 3)
        gpu_lib.step_batch(a[:1], 3)
        for c in b:
            c.step(7)
    st.synchronize()
    for s, x, y in zip(scenes, a, b):
        assert x.step_count() == y.step_count() == 7, s["name"]
        if s["n"]:
            assert np.array_equal(x.words(), y.words()), s["name"]
            assert np.array_equal(x.ids(), y.ids()), s["name"]
        sx, sy = x.stats(), y.stats()
        for f in "xvCF":
            assert sx[f] == sy[f], (s["name"], f)
        assert sx["active_nodes"] == sy["active_nodes"] and sx["sorts"] == sy["sorts"], s["name"]
    for c in a + b:
        c.close()


def test_step_batch_rejects(gpu_lib):
    import torch
    from gpu_common import gpu_context
    note("step_batch argument errors")
    s3 = [s for s in small_stream(24, n_max=5000) if s["params"]["dim"] == 3][0]
    s2 = [s for s in small_stream(24, n_max=5000) if s["params"]["dim"] == 2][0]
    for s in (s2, s3):
        s["state"] = WL.c4_state(s)
    c3 = gpu_context(gpu_lib, s3)
    c2 = gpu_context(gpu_lib, s2)
    with pytest.raises(gpu_lib.MpmqError) as e:
        gpu_lib.step_batch([c3, c2], 1)
    assert e.value.status == -1 and "dimension" in str(e.value)
    with pytest.raises(gpu_lib.MpmqError) as e:
        gpu_lib.step_batch([c3, c3], 1)
    assert e.value.status == -1 and "twice" in str(e.value)
    other = torch.cuda.Stream()
    c3b = gpu_lib.Context(s3["scheme"], s3["params"], s3["n"], stream=other)
    with pytest.raises(gpu_lib.MpmqError) as e:
        gpu_lib.step_batch([c3, c3b], 1)
    assert e.value.status == -1 and "stream" in str(e.value)
    assert c3.step_count() == 0 and c2.step_count() == 0
    for c in (c3, c2, c3b):
        c.close()


def test_serving_budget(gpu_lib):
    from paper_2207_04658_amd.serving import Server, scene_bytes
    note("serving: admission under a small HBM budget")
    scenes = small_stream(6)
    need = sorted(scene_bytes(s) for s in scenes)
    budget = need[-1] + need[-2] - 1  # never room for the two largest together
    res = Server(hbm_budget_bytes=budget, streams=2, steps_per_tick=5).run(scenes, arrivals=[0.0] * 6)
    assert len(res.latencies_s) == 6
    assert res.peak_bytes <= max(budget, need[-1])
    assert res.max_active < 6
    assert max(res.queue_wait_s.values()) > 0.0


def test_served_scene_matches_oracle(gpu_lib, orc):
    from paper_2207_04658_amd.serving import Server
    note("serving: one small scene vs the oracle")
    sc = None
    for i in range(64):
        s = WL.c4_scene(5, i, steps=10, n_max=6000)
        if s["params"]["dim"] == 2 and s["params"]["grid_res"] <= 64:
            sc = s
            break
    assert sc is not None
    res = Server(streams=1, steps_per_tick=4, keep_words=True).run([sc])
    w_gpu = res.words[sc["name"]]
    x, v, C, F = sc["state"]
    w0, _ = orc.encode(sc["scheme"], x, v, C, F, 0, 2)
    sim = orc.Sim(sc["scheme"], sc["params"], w0)
    sim.step(sc["steps"])
    xo = orc.decode(sc["scheme"], sim.words())[0]
    xg = orc.decode(sc["scheme"], w_gpu)[0]
    # both sides sort the same decoded positions the same way: slots agree
    assert np.max(np.abs(xg - xo)) <= 1e-4
    sim.close()
