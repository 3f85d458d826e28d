"""Host code under the compilers' sanitizers, on the CPU (no GPU).

* The library's host half -- status strings, the JPEG header parser and the
  host entropy decoder and encoder -- built with AddressSanitizer and
  UndefinedBehaviorSanitizer on its host side (the device code is compiled
  as usual and never run) and driven by `sanitize/host_driver.cpp`: files
  made by PIL (4:2:0, 4:2:2, 4:4:4, grey, restart intervals), every
  truncation near their ends and a spread in between, 3,000 single-byte
  corruptions and 400 deleted or duplicated bytes per file, and random
  coefficients encoded and read back.
* The C oracles built with ASan + UBSan and with ThreadSanitizer (their row
  bands run on threads) and driven by `sanitize/oracle_driver.c`.

Any sanitizer report, or a wrong result the drivers check, fails the test.
The instrumented library objects are cached under _build/sanitize by a hash
of the sources and flags (the first build takes about a minute)."""
import hashlib
import io
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1405_1020_amd import build as pb
from paper_1405_1020_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "sanitize")
ORACLE = os.path.join(ROOT, "oracle")

# host side only: the device code of a sanitized build is not run here
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer"]
LIB_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", pb.CSRC] + pb.DEVICE
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
           "TSAN_OPTIONS": "halt_on_error=1"}


def _key(paths, flags) -> str:
    h = hashlib.sha256(" ".join(flags).encode())
    for p in paths:
        h.update(p.encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise AssertionError("%s -> %d\n%s%s" % (" ".join(cmd), r.returncode, r.stdout[-4000:], r.stderr[-8000:]))
    return r


def _sanitized_objects() -> list[str]:
    """The library's objects, host side instrumented, compiled once per
    source hash (a directory renamed into place, so concurrent test workers
    share it)."""
    srcs = pb.sources()
    headers = sorted(os.path.join(pb.CSRC, f) for f in os.listdir(pb.CSRC) if f.endswith(".h"))
    key = _key(srcs + headers + [os.path.join(ROOT, "include", "oilpaint.h")], LIB_FLAGS + HOST_SAN)
    final = os.path.join(OUT, "lib-" + key)
    if not os.path.isdir(final):
        tmp = final + ".tmp%d" % os.getpid()
        os.makedirs(tmp, exist_ok=True)
        hipcc = pb.hipcc()

        def one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            _run([hipcc] + LIB_FLAGS + HOST_SAN + ["-c", src, "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=8) as ex:
            list(ex.map(one, srcs))
        try:
            os.rename(tmp, final)
        except OSError:  # another worker finished first
            shutil.rmtree(tmp, ignore_errors=True)
    return sorted(os.path.join(final, f) for f in os.listdir(final) if f.endswith(".o"))


def _jpeg_inputs(folder: str) -> list[str]:
    Image = pytest.importorskip("PIL.Image")
    cases = [((203, 117), 75, 2, {}), ((64, 48), 30, 1, {}), ((1, 1), 80, 2, {}), ((33, 17), 100, 0, {}),
             ((150, 71), 80, 2, {"restart_marker_blocks": 3}), ((97, 61), 60, 0, {"restart_marker_rows": 1})]
    paths = []
    for i, ((w, h), q, ss, kw) in enumerate(cases):
        img = synth.make_image(w, h, seed=i + 1, n_blobs=5, sigma=(2, 30))
        b = io.BytesIO()
        Image.fromarray(img).save(b, format="JPEG", quality=q, subsampling=ss, **kw)
        paths.append(os.path.join(folder, "in%d.jpg" % i))
        open(paths[-1], "wb").write(b.getvalue())
    grey = synth.make_image(45, 31, seed=5, n_blobs=4, sigma=(2, 20))[..., 0].copy()
    b = io.BytesIO()
    Image.fromarray(grey).save(b, format="JPEG", quality=70)
    paths.append(os.path.join(folder, "grey.jpg"))
    open(paths[-1], "wb").write(b.getvalue())
    return paths


def test_library_host_code_under_asan_ubsan(tmp_path):
    try:
        hipcc = pb.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    objs = _sanitized_objects()
    drv = os.path.join(HERE, "sanitize", "host_driver.cpp")
    exe = str(tmp_path / "host_driver")
    _run([hipcc, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include")] + pb.DEVICE + HOST_SAN +
         ["-c", drv, "-o", exe + ".o"])
    _run([hipcc, "--offload-arch=" + pb.ARCH] + HOST_SAN + ["-o", exe, exe + ".o"] + objs)
    files = _jpeg_inputs(str(tmp_path))
    r = _run([exe] + files, env={**os.environ, **SAN_ENV}, timeout=600)
    assert r.stdout.strip().endswith("0 failures"), r.stdout[-2000:]
    assert "variants parsed" in r.stdout


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizers(tmp_path, san):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    extra = ["-fno-sanitize-recover=all"] if san != "thread" else []
    _run([gcc, "-O1", "-g", "-std=c99", "-Wall", "-pthread", "-fsanitize=" + san] + extra +
         [os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ORACLE, "oilpaint_ref.c"),
          os.path.join(ORACLE, "median_ref.c"), "-o", exe])
    r = _run([exe, "4"], env={**os.environ, **SAN_ENV}, timeout=600)
    assert r.stdout.strip().endswith("0 failures"), r.stdout[-2000:]
