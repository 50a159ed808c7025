"""Host-side logic of the serving loop that needs no GPU: the arena
allocator used for admission by free HBM."""

import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _serve_module():
    # the allocator module has no imports, so it loads without the GPU library
    path = os.path.join(ROOT, "paper_1605_05436_amd", "arena.py")
    spec = importlib.util.spec_from_file_location("_xsum_arena", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.ArenaAllocator


def test_first_fit_alloc_release_and_coalesce():
    A = _serve_module()
    a = A(4096, align=256)
    o1, l1 = a.alloc(1)
    o2, l2 = a.alloc(300)
    o3, l3 = a.alloc(1000)
    assert (o1, l1) == (0, 256) and (o2, l2) == (256, 512) and (o3, l3) == (768, 1024)
    assert a.alloc(4096)[0] is None          # does not fit: admission waits
    a.release(o2, l2)
    o4, _ = a.alloc(200)
    assert o4 == 256                          # first fit reuses the hole
    a.release(o1, l1)
    a.release(o4, 256)
    a.release(o3, l3)
    assert a.free == [(0, 4096)]              # everything coalesced back


def test_random_alloc_free_never_overlaps():
    import random
    A = _serve_module()
    a = A(1 << 20, align=256)
    rnd = random.Random(0)
    live = []
    for _ in range(5000):
        if live and rnd.random() < 0.45:
            off, ln = live.pop(rnd.randrange(len(live)))
            a.release(off, ln)
        else:
            off, ln = a.alloc(rnd.randint(1, 50_000))
            if off is not None:
                for o, l in live:
                    assert off + ln <= o or o + l <= off
                assert off % 256 == 0 and off + ln <= (1 << 20)
                live.append((off, ln))
    for off, ln in live:
        a.release(off, ln)
    assert a.free == [(0, 1 << 20)]
