"""The request server: results in a mix of views and edits equal the
oracle's render of the map at each view's edit epoch (so alone == in the
mix), the in-flight budget is never exceeded, and stopping leaves the
newest map in the context."""
import numpy as np
import pytest

import oracle
import synth

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from test_gpu_parity import assert_parity, load  # noqa: E402
from oracle_cache import config_map, host_threads  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = tc.Context(0)
    yield c
    c.close()


def _mixed_requests(F, B, seed, n_views, n_edits, sizes):
    rng = np.random.default_rng(seed)
    H, W = F.shape
    reqs = []
    for k in range(n_views + n_edits):
        if k % max(1, (n_views + n_edits) // max(1, n_edits)) == 3 and n_edits:
            n_edits -= 1
            if rng.random() < 0.7:
                e = synth.crater_list(rng, W, H, int(rng.integers(1, 4)), size=(8, 48),
                                      depth=(10, 80))
            else:
                e = synth.random_set_patches(rng, W, H, 2, max_size=24)
            reqs.append(("edit", e))
        else:
            w, h = sizes[int(rng.integers(0, len(sizes)))]
            if rng.random() < 0.3:
                v = synth.shadow_view(int(rng.integers(0, W - 32)), int(rng.integers(0, H - 32)),
                                      min(w, 96), 35.0, rng.uniform(0, 360))
            else:
                eye = synth.eye_above_floor(F, B, rng.uniform(0, W), rng.uniform(0, H),
                                            dz=float(rng.uniform(1, 30)))
                v = synth.perspective_view(eye, rng.uniform(0, 360), rng.uniform(-60, 10), w, h)
            reqs.append(("view", v))
    return reqs


def _expected(F, B, T, reqs):
    """Oracle result of every view at its epoch."""
    out = {}
    Fk, Bk, Tk = F, B, T
    for i, (kind, x) in enumerate(reqs):
        if kind == "edit":
            Fk, Bk, Tk = oracle.apply_edits(Fk, Bk, Tk, x)
        else:
            out[i] = oracle.render(Fk, Bk, Tk, [x])
    return out, (Fk, Bk, Tk)


@pytest.mark.parametrize("mode,batch,streams", [(0, 16, 4), (2, 8, 3), (0, 1, 1)])
def test_mixed_stream_matches_epochs(ctx, mode, batch, streams):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, mode)
    reqs = _mixed_requests(F, B, 60 + batch, 48, 8, [(64, 48), (17, 33), (128, 96), (8, 8)])
    exp, final = _expected(F, B, T, reqs)
    srv = ctx.tc_server_start(64 << 20, max_batch_views=batch, streams=streams)
    ids = []
    for kind, x in reqs:
        ids.append(srv.tc_server_submit_view(x) if kind == "view" else srv.tc_server_submit_edit(x))
    for rid in ids:
        srv.tc_server_wait(rid, 120.0)
    states, lats = srv.tc_server_poll_many(ids)
    assert np.all(states == 2) and np.all(lats >= 0)
    with pytest.raises(tc.TCError):
        srv.tc_server_poll_many(ids[:3] + [987654321])
    for i, (kind, x) in enumerate(reqs):
        st, lat = srv.tc_server_poll(ids[i])
        assert st == 2 and lat == lats[i]
        if kind == "view":
            n = int(x["width"]) * int(x["height"])
            wg, dg = srv.tc_server_read(ids[i], n)
            assert_parity(wg, dg, exp[i][0], exp[i][1], "request %d" % i)
            srv.tc_server_release(ids[i])
    stats = srv.tc_server_get_stats()
    assert stats["views"] == len(exp) and stats["edits"] == len(reqs) - len(exp)
    assert stats["bytes_in_use"] == 0
    srv.tc_server_stop()
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    # the newest map version is left in the context
    g = ctx.tc_read_columns(0, 0, 256, 256)
    assert np.array_equal(g[0], final[0]) and np.array_equal(g[1], final[1])
    for L in range(1, ctx.tc_pyramid_info() + 1):
        assert np.array_equal(ctx.tc_read_pyramid(L),
                              oracle.pyramid_level_fast(final[0], final[1], final[2], L))
    for L in range(0, ctx.tc_pyramid_info() + 1):
        assert np.array_equal(ctx.tc_read_window(L),
                              oracle.window_level_fast(final[0], final[1], final[2], L))


def test_back_to_back_edits_replay(ctx):
    """Runs of edits with no view between them, then views, then more
    edits: each version buffer catches up by replaying the edit it missed,
    so every view still equals the oracle at its epoch."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(77)
    reqs = []
    for k in range(5):
        for _ in range(int(rng.integers(1, 5))):
            reqs.append(("edit", synth.crater_list(rng, 256, 256, int(rng.integers(1, 3)),
                                                   size=(8, 40), depth=(10, 80))
                         if rng.random() < 0.6 else synth.random_set_patches(rng, 256, 256, 2,
                                                                              max_size=24)))
        for _ in range(int(rng.integers(1, 4))):
            eye = synth.eye_above_floor(F, B, rng.uniform(0, 256), rng.uniform(0, 256), dz=12.0)
            reqs.append(("view", synth.perspective_view(eye, rng.uniform(0, 360), -25, 48, 32)))
    exp, final = _expected(F, B, T, reqs)
    srv = ctx.tc_server_start(64 << 20, max_batch_views=4, streams=2)
    ids = [srv.tc_server_submit_view(x) if k == "view" else srv.tc_server_submit_edit(x)
           for k, x in reqs]
    for rid in ids:
        srv.tc_server_wait(rid, 60.0)
    for i, (kind, x) in enumerate(reqs):
        if kind == "view":
            wg, dg = srv.tc_server_read(ids[i], 48 * 32)
            assert_parity(wg, dg, exp[i][0], exp[i][1], "view %d" % i)
            srv.tc_server_release(ids[i])
    srv.tc_server_stop()
    g = ctx.tc_read_columns(0, 0, 256, 256)
    assert np.array_equal(g[0], final[0]) and np.array_equal(g[1], final[1])
    assert np.array_equal(g[2], final[2])


def test_budget_admission_and_release(ctx):
    """With a budget of three large views, a burst of 20 is admitted as the
    client releases finished results; the pool never exceeds the budget."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(70)
    views = [synth.perspective_view(synth.eye_above_floor(F, B, rng.uniform(0, 256),
                                                          rng.uniform(0, 256)),
                                    rng.uniform(0, 360), -10, 200, 150) for _ in range(20)]
    one = 200 * 150 * 8
    budget = 3 * ((one + 255) // 256 * 256)
    srv = ctx.tc_server_start(budget, max_batch_views=8, streams=2)
    ids = [srv.tc_server_submit_view(v) for v in views]
    pending = list(range(20))
    seen_done = 0
    import time
    t0 = time.time()
    while pending and time.time() - t0 < 60:
        for i in list(pending):
            st, _ = srv.tc_server_poll(ids[i])
            if st == 2:
                w, d = srv.tc_server_read(ids[i], 200 * 150)
                wo, do = oracle.render(F, B, T, [views[i]])
                assert_parity(w, d, wo, do, "budget view %d" % i)
                srv.tc_server_release(ids[i])
                pending.remove(i)
                seen_done += 1
        assert srv.tc_server_get_stats()["bytes_in_use"] <= budget
    assert not pending
    assert srv.tc_server_get_stats()["peak_bytes"] <= budget
    with pytest.raises(tc.TCError) as e:
        srv.tc_server_submit_view(synth.perspective_view((5.5, 5.5, 80.0), 0, -30, 400, 300))
    assert e.value.status == tc.TC_OVER_BUDGET
    srv.tc_server_stop()


def test_server_owns_map_and_auto_release(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    srv = ctx.tc_server_start(16 << 20, flags=tc.TC_SERVER_AUTO_RELEASE)
    v = synth.config_views(1, F, B)[0]
    out = torch.empty((320 * 240, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(tc.TCError):
        ctx.tc_render_views([v], out.data_ptr())
    with pytest.raises(tc.TCError):
        ctx.tc_apply_edit([dict(kind=2, x0=0, y0=0, w=4, h=4, depth=3)])
    ids = [srv.tc_server_submit_view(v) for _ in range(10)]
    for rid in ids:
        srv.tc_server_wait(rid, 60.0)
    assert srv.tc_server_get_stats()["bytes_in_use"] == 0
    with pytest.raises(tc.TCError):
        srv.tc_server_read(ids[0], 320 * 240)     # result was discarded
    with pytest.raises(tc.TCError):
        srv.tc_server_poll(123456789)
    srv.tc_server_stop()
    # the context is usable again
    ctx.tc_render_views([v], out.data_ptr())
    torch.cuda.synchronize()


def test_c5_map_mixed_full(ctx):
    """On the 2048x16384 map: views of the configuration-5 sizes mixed with
    crater edits; every record of each request's whole buffer against the
    oracle's render of the map at its epoch."""
    F, B, T = config_map(5)
    H, W = F.shape
    load(ctx, F, B, T)
    rng = np.random.default_rng(80)
    reqs = []
    for k in range(20):
        if k % 5 == 4:
            reqs.append(("edit", synth.crater_list(rng, W, H, 1, size=(16, 64))))
        else:
            reqs.append(("view", synth.request_view(rng, F, B)))
    srv = ctx.tc_server_start(2 << 30, max_batch_views=8, streams=4)
    ids = [srv.tc_server_submit_view(x) if k == "view" else srv.tc_server_submit_edit(x)
           for k, x in reqs]
    for rid in ids:
        srv.tc_server_wait(rid, 120.0)
    Fk, Bk, Tk = F, B, T
    for i, (kind, x) in enumerate(reqs):
        if kind == "edit":
            Fk, Bk, Tk = oracle.apply_edits(Fk, Bk, Tk, x)
            continue
        w, h = int(x["width"]), int(x["height"])
        wg, dg = srv.tc_server_read(ids[i], w * h)
        wo, do = oracle.render(Fk, Bk, Tk, [x], threads=host_threads())
        assert_parity(wg, dg, wo, do, "c5 request %d (%dx%d)" % (i, w, h))
        srv.tc_server_release(ids[i])
    srv.tc_server_stop()
