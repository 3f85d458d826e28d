"""The autotuner: the library's own timing of candidate launch shapes, the
installed choice, and parity of size-adaptive shapes (rows derived from a
workgroup density)."""
import os

import numpy as np
import pytest

from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth, tune
from gpu_util import to_device, empty_like_device, from_device, ref, first_mismatch, torch_mod

pytestmark = pytest.mark.gpu


def test_tune_times_and_unsupported():
    torch_mod()
    cands = tune.candidates(5, 20) + [B.Variant(0, 1, B.HIST_STREAM, 32, 8)]
    t = B.tune_times(512, 384, 5, 20, cands, reps=2)
    assert len(t) == len(cands)
    assert all(x > 0 for x in t[:-1]) and t[-1] == -1.0
    # streamed rows need r <= 15: every candidate of r = 20 is the wide layout
    t2 = B.tune_times(300, 200, 20, 20, [B.Variant(0, 1, B.HIST_STREAM, 64, 8)], reps=1)
    assert t2 == [-1.0]


def test_ensure_installs_and_stays_exact(tmp_path, monkeypatch):
    torch = torch_mod()
    monkeypatch.setenv("OILPAINT_TUNE_CACHE", str(tmp_path / "tune.json"))
    B.clear_variants()
    try:
        res = tune.ensure([(3, 20), (7, 64)], 640, 480, reps=2)
        assert os.path.exists(tmp_path / "tune.json")
        for (r, L) in [(3, 20), (7, 64)]:
            v = B.pick_variant(640, 480, r, L)
            want = res["%d,%d" % (r, L)]["variant"]
            assert (v.waves, v.hist, v.lanes, v.per_cu) == tuple(want[1:])
            img = synth.make_image(333, 251, seed=r * 7 + L, n_blobs=6, sigma=(4, 30))
            src, _ = to_device(img, pad=1)
            dst, _ = empty_like_device(img, pad=1)
            B.oilpaint_async(src, dst, r, L)
            torch.cuda.synchronize()
            assert first_mismatch(from_device(dst), ref(img, r, L)) is None
        # a second call comes from the cache file
        assert tune.load() >= 2
    finally:
        B.clear_variants()


@pytest.mark.parametrize("per_cu", [1, 3, 8, 64])
def test_density_shapes_exact(per_cu):
    torch_mod()
    img = synth.make_image(517, 389, seed=per_cu, n_blobs=6, sigma=(4, 40))
    for r, L in [(1, 8), (4, 20), (9, 32), (15, 64)]:
        want = ref(img, r, L)
        for v in [B.Variant(0, 1, B.HIST_STREAM, 64, per_cu), B.Variant(0, 2, B.HIST_PACKED, 64, per_cu),
                  B.Variant(0, 4, B.HIST_PACKED, 64, per_cu)]:
            src, _ = to_device(img, pad=2)
            dst, _ = empty_like_device(img, pad=2)
            B.oilpaint_async(src, dst, r, L, variant=v)
            torch_mod().cuda.synchronize()
            assert first_mismatch(from_device(dst), want) is None, (r, L, v)


def test_ensure_median_installs_and_stays_exact(tmp_path, monkeypatch):
    import oracle
    torch = torch_mod()
    monkeypatch.setenv("OILPAINT_TUNE_CACHE", str(tmp_path / "tune.json"))
    try:
        res = tune.ensure_median([3, 12, 24], 640, 480, reps=2)
        for r in (3, 12, 24):
            kind = res[str(r)]["kind"]
            assert kind in tune.median_candidates(r) and B.median_pick_kind(r) == kind
            assert {k for k, _ in res[str(r)]["all"]} == set(tune.median_candidates(r))
            img = synth.make_image(211, 167, seed=r, n_blobs=5, sigma=(3, 30))
            src = torch.from_numpy(img).cuda()
            out = B.median(src, r, 1)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), oracle.median_ref(img, r, 1, nthreads=4)), r
    finally:
        for r in range(128):
            B.median_set_kind(r, B.MEDIAN_AUTO)
