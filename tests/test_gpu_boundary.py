"""The C ABI's memory and serving contracts on the GPU: every device
allocation goes through a registered allocator and none is outstanding once
the handles are destroyed and the scratch released; scene options; server
cancellation, per-request failure isolation inside a merged pass, ordering
after the producer's stream, merged FP8 requests."""
import gc

import numpy as np
import pytest
import torch

import paper_2410_14462_amd as lv
from synth import philox, scenes

pytestmark = pytest.mark.gpu


def rel_diff(a, b):
    a, b = a.double().cpu(), b.double().cpu()
    scale = b.abs().max(dim=0).values.clamp_min(1e-30)
    return float(((a - b).abs() / scale).max())


class Counting:
    """A device allocator over torch's caching allocator that records every
    allocation; `fail_above` makes larger allocations fail."""

    def __init__(self, fail_above=None):
        self.live, self.allocs, self.frees, self.refused = {}, 0, 0, 0
        self.fail_above = fail_above

    def alloc(self, nbytes, stream):
        if self.fail_above is not None and nbytes > self.fail_above:
            self.refused += 1
            return 0
        p = torch.cuda.caching_allocator_alloc(max(nbytes, 1), 0, stream or 0)
        self.live[p] = nbytes
        self.allocs += 1
        return p

    def free(self, ptr, nbytes, stream):
        assert self.live.pop(ptr) == nbytes
        self.frees += 1
        torch.cuda.caching_allocator_delete(ptr)


def quiesce():
    gc.collect()
    torch.cuda.synchronize()
    lv.release_scratch()


@pytest.fixture
def counting():
    quiesce()
    assert lv.memory_stats() == (0, 0), "library memory held by earlier objects"
    c = Counting()
    lv.set_allocator(c.alloc, c.free)
    yield c
    quiesce()
    lv.set_allocator(None)


def small_rig(seed=21, n=4000, views=6):
    sc = scenes.make_scene(seed, n, -3.8, 0.5, 0.0, 1.0)
    cams = [scenes.look_at(e, 96, 72, 60.0) for e in scenes.fibonacci_eyes(views, 4.0)]
    return sc, cams


def test_every_device_allocation_goes_through_the_allocator(counting):
    sc, cams = small_rig()
    gs = lv.Scene.from_arrays(sc)
    maps = [torch.as_tensor(philox.normal(5, v, 72 * 96 * 8).reshape(72, 96, 8), device="cuda")
            for v in range(len(cams))]
    f, b = gs.uplift(cams, maps)                                       # structure + blend scratch
    codes, sc8 = zip(*[lv.encode(m, "fp8") for m in maps])            # codec scratch
    f8, _ = gs.uplift(cams, list(codes), dtype="fp8", scales=torch.stack(sc8).contiguous())
    keep = lv.prune_by_weight(b, sc.n // 2)                            # filtering scratch
    G = lv.Graph.knn(gs, f, 8)                                         # graph build + CSR
    out = G.diffuse(f, 3, scene=gs)                                    # diffusion buffers
    acc = lv.Accum(gs, 8, counts=True)
    acc.add(cams, maps)
    srv = lv.Server(workers=2, budget=8 << 30, scratch=1 << 30)       # server passes
    for k in range(4):
        srv.submit(gs, cams[k:k + 2], maps[k:k + 2], tag=k)
    srv.drain()
    done = srv.poll()
    torch.cuda.synchronize()
    assert all(c["status"] == 0 for c in done) and len(done) == 4
    assert rel_diff(f8, f) < 0.1 and int(keep.sum()) == sc.n // 2 and torch.isfinite(out).all()
    held = lv.memory_stats()
    assert held[1] > 0 and len(counting.live) == held[1]
    assert sum(counting.live.values()) == held[0]
    srv.close()
    acc.close()
    G.close()
    gs.close()
    del done, acc, G, gs
    quiesce()
    print(f"allocator: {counting.allocs} allocations, {counting.frees} frees")
    assert counting.allocs > 10 and counting.frees == counting.allocs
    assert counting.live == {} and lv.memory_stats() == (0, 0)


def test_allocator_cannot_change_under_live_handles(counting):
    sc, _ = small_rig(n=500)
    gs = lv.Scene.from_arrays(sc)
    with pytest.raises(lv.LvError):
        lv.set_allocator(None)
    gs.close()


def test_scene_options():
    sc, cams = small_rig(n=500, views=1)
    t = [torch.as_tensor(np.ascontiguousarray(a), device="cuda")
         for a in (sc.means, sc.scales, sc.quats, sc.opacity)]
    g = lv.Scene(*t, opts={})  # every field at its default
    f, _ = g.uplift(cams, [torch.ones((72, 96, 2), device="cuda")])
    torch.cuda.synchronize()
    assert torch.isfinite(f).all()
    for bad in ({"alpha_min": 0.01}, {"t_eps": 1e-3}, {"alpha_max": 0.999}, {"dilation": 0.0},
                {"tile": 8}):
        with pytest.raises(lv.LvError, match="status 4"):
            lv.Scene(*t, opts=bad)


def test_failing_request_in_a_merged_pass_fails_alone():
    """Three requests merged into one pass on one scene; the middle one's
    accumulator cannot be allocated (the allocator refuses it): the pass
    fails, each request runs again alone, and only that one fails."""
    quiesce()
    assert lv.memory_stats() == (0, 0)
    sc, cams = small_rig(n=4000)
    big = 4000  # channels: its accumulator is n x 4000 x 4 = 64 MB
    c = Counting(fail_above=32 << 20)
    lv.set_allocator(c.alloc, c.free)
    try:
        gs = lv.Scene.from_arrays(sc)
        bank = torch.as_tensor(philox.normal(9, 0, 72 * 96 * big).reshape(72, 96, big), device="cuda")
        srv = lv.Server(workers=1, budget=16 << 30, scratch=1 << 30, max_channels=8192)
        # a first request keeps the worker busy while the next three queue up
        srv.submit(gs, cams, [bank[..., :64]] * len(cams), tag=0)
        for tag, D in ((1, 3), (2, big), (3, 5)):
            srv.submit(gs, cams[:3], [bank[..., :D]] * 3, tag=tag)
        srv.drain()
        done = {x["tag"]: x for x in srv.poll()}
        st = srv.stats()
        srv.close()
        assert done[2]["status"] == 2 and c.refused > 0  # LV_ERR_OUT_OF_MEMORY
        for tag, D in ((1, 3), (3, 5)):
            assert done[tag]["status"] == 0
            f, _ = gs.uplift(cams[:3], [bank[..., :D].contiguous()] * 3)
            assert rel_diff(done[tag]["out"], f) < 1e-4
        print(f"isolation: {st['passes']} passes for 4 requests, batch sizes "
              f"{[done[t]['batch_size'] for t in range(4)]}")
        gs.close()
        del gs, done
    finally:
        quiesce()
        lv.set_allocator(None)


def test_cancel_waiting_requests():
    sc, cams = small_rig(n=20000, views=8)
    gs = lv.Scene.from_arrays(sc)
    bank = torch.as_tensor(philox.normal(10, 0, 72 * 96 * 64).reshape(72, 96, 64), device="cuda")
    srv = lv.Server(workers=1, budget=8 << 30, scratch=1 << 30, max_sets=1)
    for tag in range(6):
        srv.submit(gs, cams, [bank] * len(cams), tag=tag)
    cancelled = [t for t in (5, 3) if srv.cancel(t)]
    srv.drain()
    done = {x["tag"]: x for x in srv.poll()}
    st = srv.stats()
    assert not srv.cancel(0) and not srv.cancel(99)  # finished / unknown
    srv.close()
    assert cancelled, "nothing was still waiting"
    assert sorted(done) == list(range(6)) and st["cancelled"] == len(cancelled)
    for t in range(6):
        assert done[t]["status"] == (lv.LV_ERR_CANCELLED if t in cancelled else 0), t
    f, _ = gs.uplift(cams, [bank] * len(cams))
    for t in range(6):
        if t not in cancelled:
            assert rel_diff(done[t]["out"], f) < 1e-4


def test_pass_waits_for_the_producer_stream():
    """The maps are written on a side stream behind a long busy kernel; the
    request is submitted from that stream right away: the pass must see the
    written maps, not the zeros before them."""
    sc, cams = small_rig(n=4000, views=4)
    gs = lv.Scene.from_arrays(sc)
    src = torch.as_tensor(philox.normal(11, 0, 4 * 72 * 96 * 16).reshape(4, 72, 96, 16), device="cuda")
    ref, _ = gs.uplift(cams, [src[v] for v in range(4)])
    srv = lv.Server(workers=2, budget=8 << 30, scratch=1 << 30)
    maps = torch.zeros_like(src)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        torch.cuda._sleep(200_000_000)  # ~0.1 s of spinning before the maps are written
        maps.copy_(src)
        srv.submit(gs, cams, [maps[v] for v in range(4)], tag=1)
    srv.drain()
    (done,) = srv.poll()
    srv.close()
    torch.cuda.synchronize()
    assert done["status"] == 0
    assert rel_diff(done["out"], ref) < 1e-4


def test_fp8_requests_merge():
    sc, cams = small_rig(n=6000, views=8)
    gs = lv.Scene.from_arrays(sc)
    D = 24
    src = [torch.as_tensor(philox.normal(12, v, 72 * 96 * D).reshape(72, 96, D), device="cuda")
           for v in range(8)]
    enc = [lv.encode(m, "fp8") for m in src]
    codes = [e[0] for e in enc]
    scales = torch.stack([e[1] for e in enc]).contiguous()
    srv = lv.Server(workers=1, budget=8 << 30, scratch=1 << 30, max_sets=8)
    reqs = [[0, 1, 2, 3, 4, 5, 6, 7], [1, 3, 5], [6, 2], [4, 0, 7]]
    # a first request keeps the worker busy so that the others merge
    for tag, views in enumerate(reqs):
        srv.submit(gs, [cams[v] for v in views], [codes[v] for v in views], dtype="fp8",
                   scales=scales[views].contiguous(), tag=tag)
    srv.drain()
    done = {x["tag"]: x for x in srv.poll()}
    st = srv.stats()
    srv.close()
    assert st["passes"] < len(reqs), st
    for tag, views in enumerate(reqs):
        f, _ = gs.uplift([cams[v] for v in views], [codes[v] for v in views], dtype="fp8",
                         scales=scales[views].contiguous())
        assert done[tag]["status"] == 0
        assert rel_diff(done[tag]["out"], f) < 1e-4, (tag, done[tag]["batch_size"])
