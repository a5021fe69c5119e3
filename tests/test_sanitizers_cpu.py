"""Host sanitizer runs (CPU only).

* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every state mode and
  the diffusion coefficients on the 8-species mechanism, with non-physical cells taking the
  error paths (tests/native/oracle_asan_driver.c).
* The serving scheduler under ThreadSanitizer: the mock executor with concurrent
  submitters, waiters that time out and retry, a statistics poller and one failing request,
  under a memory budget that makes admission bind (tests/native/serve_tsan_driver.cpp).

Both builds instrument host code only; a sanitizer report or a non-zero exit fails."""
import os
import shutil
import subprocess

import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def mech_file(tmp_path_factory):
    sp = synth.load_species(synth.FLAME_SPECIES)
    kij = synth.synthetic_kij(len(sp))
    path = tmp_path_factory.mktemp("mech") / "mech8.txt"
    with open(path, "w") as f:
        f.write(f"{len(sp)}\n")
        for s in sp:
            vals = [s[k] for k in ("W", "Tc", "Pc", "Vc", "omega", "dipole", "kappa", "Tmid")]
            vals += list(s["nasa_lo"]) + list(s["nasa_hi"])
            f.write(" ".join(repr(float(v)) for v in vals) + "\n")
        f.write(" ".join(repr(float(x)) for row in kij for x in row) + "\n")
    return str(path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path, mech_file):
    exe = str(tmp_path / "orc_asan")
    rc, out = _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "native", "oracle_asan_driver.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe, mech_file], timeout=120)
    assert rc == 0 and "ERROR" not in out and "runtime error" not in out, out
    assert out.startswith("rc 0"), out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_serving_scheduler_under_thread_sanitizer(tmp_path):
    csrc = os.path.join(ROOT, "paper_2312_04830_amd", "csrc")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=thread",
             "-I", os.path.join(ROOT, "include")]
    objs = []
    for src, lang in ((os.path.join(csrc, "serve.hip"), []), (os.path.join(csrc, "mech.hip"), []),
                      (os.path.join(HERE, "native", "serve_tsan_driver.cpp"), ["-x", "hip"])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        rc, out = _run([HIPCC] + flags + lang + ["-c", src, "-o", obj])
        assert rc == 0, out
        objs.append(obj)
    exe = str(tmp_path / "serve_tsan")
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=thread", "-o", exe] + objs +
                   ["-lpthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, out
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    rc, out = _run([exe], timeout=300, env=env)
    assert rc == 0 and "ThreadSanitizer" not in out, out
    assert "bad 0" in out, out
