"""CPU runs of the host code under the address and undefined-behaviour
sanitizers: the oracle (built with them and loaded into a child process that
preloads the sanitizer runtime) on a small and a contract-edge event, and
the library's geometry builder and its cache (built with them into a small
checker)."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or _runtime() is None,
                                reason="gcc with the address sanitizer runtime is needed")


def _env(extra):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.update(extra)
    return env


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liblst_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-ffp-contract=off", *SAN, "-shared", "-fPIC", "-o", lib,
                           os.path.join(ROOT, "oracle", "lst_oracle.c"), "-lm"])
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import oracle, contract\n"
        "from paper_2407_18231_amd import synth as s\n"
        "g = s.make_geometry('pu200')\n"
        "for ev, geom in ((s.gen_event(g, s.config_pu(20), 7), g),\n"
        "                 (s.gen_event(g, s.config_pu(20, smear=False), 8), contract.shrunk(g, 5.4))):\n"
        "    r = oracle.run(geom, ev)\n"
        "    print({k: len(r[k]) for k in ('md', 'ls', 't3', 't5', 'pt3', 'pt5', 'tc')})\n" % (ROOT, HERE))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                       env=_env({"LD_PRELOAD": _runtime(), "LST_ORACLE_LIB": lib}))
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    assert p.stdout.count("'md'") == 2


@pytest.mark.parametrize("name", ["tiny", "pu200"])
def test_geometry_builder_under_sanitizers(tmp_path, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is needed")
    from paper_2407_18231_amd import lst, synth
    exe = str(tmp_path / "geometry_check")
    csrc = os.path.join(ROOT, "paper_2407_18231_amd", "csrc")
    subprocess.check_call([gxx, "-O1", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           "-o", exe, os.path.join(HERE, "sanitize", "geometry_check.cpp"),
                           os.path.join(csrc, "geometry.cpp")])
    g = synth.make_geometry(name)
    (tmp_path / "mods.bin").write_bytes(lst.module_table(g).tobytes())
    (tmp_path / "params.bin").write_bytes(bytes(lst.default_params()))
    cache = tmp_path / "cache"
    cache.mkdir()
    p = subprocess.run([exe, str(tmp_path / "mods.bin"), str(tmp_path / "params.bin"), str(cache)],
                       capture_output=True, text=True, timeout=600, env=_env({}))
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    assert "runtime error" not in p.stderr, p.stderr[-4000:]
    assert p.stdout.startswith("cache: miss, hit, miss for other parameters\n")
    assert f"modules {len(g.kind)} " in p.stdout
    assert len(list(cache.glob("lst_geometry_*.bin"))) == 2
