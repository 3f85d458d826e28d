"""GPU parity of the column layout (per-column histograms and per-level
prefix sums across the strip, radius up to 255) against the CPU oracle,
bit-exact, through the C-ABI: every 64-column chunk count, level counts
from 1 to 100, ragged sizes, run lengths, radii clipped by the image, the
paper form, and batches mixing it with the other layouts."""
import numpy as np
import pytest

from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth
from gpu_util import (to_device, empty_like_device, from_device, padding_bytes, ref, ref_pixel,
                      first_mismatch, torch_mod)

pytestmark = pytest.mark.gpu


def run_variant(img, r, L, variant, pad=0):
    torch = torch_mod()
    h, w, _ = img.shape
    src, sbuf = to_device(img, pad=pad, seed=3)
    dst, dbuf = empty_like_device(img, pad=pad, seed=5)
    before = padding_bytes(dbuf, h, w, 3 * w + pad)
    B.oilpaint_async(src, dst, r, L, variant=variant)
    torch.cuda.synchronize()
    assert np.array_equal(before, padding_bytes(dbuf, h, w, 3 * w + pad)), "dst padding was written"
    return from_device(dst)


def image(w, h, seed):
    if w * h > 100:
        return synth.make_image(w, h, seed=seed, n_blobs=5, sigma=(3, 25))
    return synth.make_random(w, h, seed=seed)


# (w, h, radii): radii from 0 to 255, so that every chunk count 1..9 of a
# strip with its halo occurs, some clipped to the image
CASES = [
    ((1, 1), (0, 20)),
    ((65, 40), (0, 3, 15, 16, 31, 32)),
    ((130, 57), (16, 20, 47, 63, 64)),
    ((97, 33), (95, 96, 127, 128)),
    ((300, 21), (159, 160, 191, 192, 223, 224, 255)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_column_matches_oracle(case):
    (w, h), radii = CASES[case]
    img = image(w, h, seed=200 + case)
    for r in radii:
        for L in (1, 8, 20, 33, 64, 100):
            want = ref(img, r, L)
            for rows in (1, 5, 300):
                v = B.Variant(rows, 1, B.HIST_COLUMN, 64)
                try:
                    got = run_variant(img, r, L, v, pad=(w + rows) % 5)
                except B.OilpaintError as e:
                    # only when the column histograms exceed the on-chip budget
                    assert e.status == B.ERR_UNSUPPORTED and (L + 1) * (64 + 2 * min(r, max(w, h) - 1)) * 8 > 150000
                    continue
                mm = first_mismatch(got, want)
                assert mm is None, (w, h, r, L, rows, mm)


# the radius <= 15 form, with one, two and four wavefronts per strip: every
# radius 0..15 (some clipped by the image), both sides of each prefix-word
# bucket edge (9/10, 21/22, 33/34 levels) and 64, run lengths from 1 row
SMALL = [
    ((65, 40), (0, 1, 3, 7)),
    ((130, 57), (8, 11, 15)),
    ((97, 33), (2, 5, 13, 14)),
    ((1, 1), (0,)),
    ((70, 3), (4, 6, 9, 10, 12)),
]


@pytest.mark.parametrize("waves", (1, 2, 4))
@pytest.mark.parametrize("case", range(len(SMALL)))
def test_column15_matches_oracle(case, waves):
    (w, h), radii = SMALL[case]
    img = image(w, h, seed=400 + case)
    for r in radii:
        for L in (1, 9, 10, 21, 22, 33, 34, 64):
            want = ref(img, r, L)
            for rows in (1, 2, 5, 300):
                v = B.Variant(rows, waves, B.HIST_COLUMN, 64)
                got = run_variant(img, r, L, v, pad=(w + rows) % 5)
                mm = first_mismatch(got, want)
                assert mm is None, (w, h, r, L, waves, rows, mm)


@pytest.mark.parametrize("waves", (1, 2, 4))
def test_column15_paper_form_and_bands(waves):
    # the paper form (white level and borders left alone) and a row band,
    # through the registered launch shape
    torch = torch_mod()
    img = image(150, 90, seed=17)
    try:
        for r, L in ((3, 20), (10, 8), (15, 33), (15, 64)):
            assert B.set_variant(r, L, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            src, _ = to_device(img)
            junk = np.random.default_rng(r + L).integers(0, 256, img.shape, dtype=np.uint8)
            dst, _ = to_device(junk)
            B.run(B.Item(src, dst, r, L, flags=B.FLAG_PAPER))
            torch.cuda.synchronize()
            want = ref(img, r, L, paper=True, out=junk.copy())
            mm = first_mismatch(from_device(dst), want)
            assert mm is None, ("paper", r, L, waves, mm)
            dst, _ = to_device(junk)
            B.run(B.Item(src, dst, r, L, row_begin=17, row_end=61))
            torch.cuda.synchronize()
            want = junk.copy()
            want[17:61] = ref(img, r, L)[17:61]
            mm = first_mismatch(from_device(dst), want)
            assert mm is None, ("band", r, L, waves, mm)
    finally:
        B.clear_variants()


# the radius 16..31 form (16-bit counts, 20-bit sums; two or four wavefronts
# per strip): every radius 16..31 (some clipped by the image), both sides of
# each count-word bucket edge (8/9, 20/21, 32/33 levels) and 64, run lengths
# from 1 row, strips from one to three
WIDE = [
    ((65, 70), (16, 17, 18, 19)),
    ((130, 57), (20, 21, 22, 23)),
    ((200, 80), (24, 25, 26, 27)),
    ((97, 100), (28, 29, 30, 31)),
    ((40, 20), (16, 31)),
]


@pytest.mark.parametrize("waves", (2, 4))
@pytest.mark.parametrize("case", range(len(WIDE)))
def test_column31_matches_oracle(case, waves):
    (w, h), radii = WIDE[case]
    img = image(w, h, seed=600 + case)
    for r in radii:
        for L in (1, 8, 9, 20, 21, 32, 33, 64):
            want = ref(img, r, L)
            for rows in (1, 3, 64):
                v = B.Variant(rows, waves, B.HIST_COLUMN, 64)
                got = run_variant(img, r, L, v, pad=(w + rows) % 5)
                mm = first_mismatch(got, want)
                assert mm is None, (w, h, r, L, waves, rows, mm)


@pytest.mark.parametrize("waves", (2, 4))
def test_column31_paper_form_bands_and_batch(waves):
    # the paper form and a row band through the registered launch shape, and
    # a batch of the same jobs (the radius 16..31 form has no persistent
    # kernel: the batch runs them in the generic column classes)
    torch = torch_mod()
    img = image(170, 120, seed=27)
    items, want = [], []
    try:
        for r, L in ((16, 20), (23, 8), (31, 33), (31, 64)):
            assert B.set_variant(r, L, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            src, _ = to_device(img)
            junk = np.random.default_rng(r + L).integers(0, 256, img.shape, dtype=np.uint8)
            dst, _ = to_device(junk)
            B.run(B.Item(src, dst, r, L, flags=B.FLAG_PAPER))
            torch.cuda.synchronize()
            mm = first_mismatch(from_device(dst), ref(img, r, L, paper=True, out=junk.copy()))
            assert mm is None, ("paper", r, L, waves, mm)
            dst, _ = to_device(junk)
            B.run(B.Item(src, dst, r, L, row_begin=21, row_end=99))
            torch.cuda.synchronize()
            wt = junk.copy()
            wt[21:99] = ref(img, r, L)[21:99]
            mm = first_mismatch(from_device(dst), wt)
            assert mm is None, ("band", r, L, waves, mm)
            bdst, _ = empty_like_device(img)
            items.append(B.Item(src, bdst, r, L))
            want.append(ref(img, r, L))
        B.batch(items)
        torch.cuda.synchronize()
        for it, wt in zip(items, want):
            mm = first_mismatch(from_device(it.dst), wt)
            assert mm is None, ("batch", it.radius, it.levels, mm)
    finally:
        B.clear_variants()


def test_column31_full_hd():
    # 1920x1080 at r = 20, 20 levels and r = 31, 64 levels, every byte
    img = synth.fhd_image()
    for r, L, waves in ((20, 20, 4), (31, 64, 4), (24, 32, 2)):
        got = run_variant(img, r, L, B.Variant(0, waves, B.HIST_COLUMN, 64, 4))
        mm = first_mismatch(got, ref(img, r, L))
        assert mm is None, (r, L, waves, mm)


def test_batch_with_column15_shapes():
    # jobs whose registered shape is the r <= 15 column form: a batch runs the
    # paper form in the column layout's one-wavefront classes and the rest in
    # the streamed classes; every output against the oracle, then two replays
    # of a captured plan
    torch = torch_mod()
    cases = [((150, 90), 12, 20, 1), ((130, 70), 15, 33, 1), ((97, 60), 7, 9, 0), ((150, 90), 12, 20, 0),
             ((64, 200), 10, 64, 1), ((200, 40), 15, 21, 0)]
    items, want = [], []
    try:
        for i, ((w, h), r, L, paper) in enumerate(cases):
            assert B.set_variant(r, L, B.Variant(0, 4, B.HIST_COLUMN, 64, 4)) == B.OK
            img = image(w, h, seed=500 + i)
            src, _ = to_device(img)
            junk = np.random.default_rng(i).integers(0, 256, img.shape, dtype=np.uint8)
            dst, _ = to_device(junk)
            items.append(B.Item(src, dst, r, L, flags=B.FLAG_PAPER if paper else 0))
            want.append(ref(img, r, L, paper=bool(paper), out=junk.copy()) if paper else ref(img, r, L))
        B.batch(items)
        torch.cuda.synchronize()
        for (_, r, L, paper), it, wt in zip(cases, items, want):
            mm = first_mismatch(from_device(it.dst), wt)
            assert mm is None, ("batch", r, L, paper, mm)
        plan = B.Plan(items)
        for _ in range(2):
            for (_, r, L, paper), it, wt in zip(cases, items, want):
                if not paper:
                    it.dst.zero_()
            plan.launch()
            torch.cuda.synchronize()
            for (_, r, L, paper), it, wt in zip(cases, items, want):
                mm = first_mismatch(from_device(it.dst), wt)
                assert mm is None, ("plan", r, L, paper, mm)
        plan.close()
    finally:
        B.clear_variants()


def test_column_paper_form():
    torch = torch_mod()
    img = image(150, 90, seed=7)
    for r, L in ((16, 20), (40, 8), (20, 64)):
        src, _ = to_device(img)
        junk = np.random.default_rng(r).integers(0, 256, img.shape, dtype=np.uint8)
        dst, _ = to_device(junk)
        B.run(B.Item(src, dst, r, L, flags=B.FLAG_PAPER))
        torch.cuda.synchronize()
        assert B.pick_variant(150, 90, r, L).hist == B.HIST_COLUMN
        want = ref(img, r, L, paper=True, out=junk.copy())
        mm = first_mismatch(from_device(dst), want)
        assert mm is None, (r, L, mm)


def test_column_large_image_sampled():
    # the library's default for r > 15 on a 1920x1080 image, against the
    # oracle pixel by pixel on a seeded sample (borders and corners included)
    torch = torch_mod()
    img = synth.fhd_image()
    src = torch.from_numpy(img).cuda()
    rng = np.random.default_rng(11)
    for r, L in ((20, 20), (64, 32)):
        assert B.pick_variant(1920, 1080, r, L).hist == B.HIST_COLUMN
        out = from_device(B.oilpaint(src, r, L))
        pts = [(0, 0), (1919, 1079), (0, 1079), (1919, 0), (r, r), (1919 - r, 1079 - r)]
        pts += [(int(rng.integers(0, 1920)), int(rng.integers(0, 1080))) for _ in range(60)]
        for x, y in pts:
            want = ref_pixel(img, x, y, r, L)
            assert np.array_equal(out[y, x], want), (r, L, x, y, out[y, x], want)


def test_batch_mixes_column_jobs():
    torch = torch_mod()
    cases = [((120, 90), 3, 20), ((200, 70), 20, 20), ((90, 130), 70, 8), ((64, 64), 16, 100),
             ((150, 40), 5, 200), ((33, 250), 40, 33)]
    items, imgs = [], []
    for i, ((w, h), r, L) in enumerate(cases):
        img = image(w, h, seed=300 + i)
        src, _ = to_device(img)
        dst, _ = empty_like_device(img)
        items.append(B.Item(src, dst, r, L))
        imgs.append(img)
    B.batch(items)
    torch.cuda.synchronize()
    for (img, ((w, h), r, L)), it in zip(zip(imgs, cases), items):
        mm = first_mismatch(from_device(it.dst), ref(img, r, L))
        assert mm is None, (w, h, r, L, mm)
    plan = B.Plan(items)
    for _ in range(2):
        for it in items:
            it.dst.zero_()
        plan.launch()
        torch.cuda.synchronize()
        for (img, (_, r, L)), it in zip(zip(imgs, cases), items):
            assert first_mismatch(from_device(it.dst), ref(img, r, L)) is None
    plan.close()
