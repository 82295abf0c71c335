"""The host code of the library built with AddressSanitizer and with
UndefinedBehaviorSanitizer (device code uninstrumented; CPU only): the
host-only ABI tests (validation before any device call, workspace and plan
sizing, server footprints, option checks) run against each build in a child
process with the sanitizer runtime preloaded, and must pass with no report."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _builder():
    path = os.path.join(ROOT, "paper_1205_4139_amd", "build.py")
    spec = importlib.util.spec_from_file_location("_fcmp_build_san", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("kind", ["address", "undefined"])
def test_host_code_clean_under_sanitizer(kind):
    b = _builder()
    lib = b.build(False, kind)
    env = dict(os.environ)
    env["LD_PRELOAD"] = b.sanitizer_runtime(kind)
    env["FCMP_LIBRARY"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = ("import sys, paper_1205_4139_amd as fc, pytest; "
            f"assert fc.LIB_PATH == {lib!r}, fc.LIB_PATH; "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', 'tests/test_abi_host.py']))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
