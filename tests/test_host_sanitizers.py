"""Host code under AddressSanitizer and UBSan (no GPU).

Builds the library's host C++ (argument checks, layout build, model files,
tuner cache), the CPU oracle and the input generators with
-fsanitize=address,undefined, then reruns the CPU test suites in a child
process with those builds loaded (WEDGE_LIB, WEDGE_ORACLE_LIB,
WEDGE_GEN_LIB) and the sanitizer runtimes preloaded. Any invalid access or
undefined behaviour aborts the child. Device code is not sanitized (GPU
sanitizers are not available); it is the release build's.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           timeout=60).stdout.strip()
    except (OSError, subprocess.SubprocessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _sanitized_env():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not found")
    sys.path.insert(0, ROOT)
    import gen
    import oracle
    from paper_1903_07754_amd import build as libbuild
    if not os.path.exists(os.path.join(ROOT, "paper_1903_07754_amd", "_build", "api.cpp.o")):
        libbuild.build()
    env = dict(os.environ)
    env.update({
        "WEDGE_LIB": libbuild.build_sanitized(),
        "WEDGE_ORACLE_LIB": oracle.build(sanitize=True),
        "WEDGE_GEN_LIB": gen.build(sanitize=True),
        "LD_PRELOAD": f"{asan} {ubsan}",
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    return env


def test_cpu_suites_under_asan_and_ubsan():
    env = _sanitized_env()
    # the child must really have the sanitized builds loaded
    probe = ("import sys; sys.path.insert(0, %r); import gen, oracle, paper_1903_07754_amd as W; "
             "W.lib(); oracle._load(); gen._load(); maps = open('/proc/self/maps').read(); "
             "print(all(x in maps for x in ('libwedge_asan.so', 'liboracle_asan.so', "
             "'libwedgegen_asan.so', 'libasan')))" % ROOT)
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip().splitlines()[-1] == "True"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", "tests/test_abi_host.py",
                        "tests/test_oracle_pins.py", "tests/test_mlp_pins.py"],
                       env=env, capture_output=True, text=True, timeout=1200, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_tune_cache_parser_under_asan(tmp_path):
    # the tuner's cache file is read by host code: valid lines load, malformed
    # ones are skipped; entries are keyed by the device's compute unit count
    # (0 without a GPU), so the child writes the file for its own device
    env = _sanitized_env()
    path = tmp_path / "tune.txt"
    env["WEDGE_TUNE_CACHE"] = str(path)
    code = """
import json, sys
sys.path.insert(0, %r)
import torch
import paper_1903_07754_amd as W
cus = torch.cuda.get_device_properties(0).multi_processor_count if torch.cuda.is_available() else 0
open(%r, "w").write("wedge-tune-v1\\n"
    f"0 1 20 {cus} 32 0 0 8\\n"     # single source, 2^20 edges
    f"1 64 22 {cus} 16 1 2 0\\n"    # multi-source, persistent
    "garbage line\\n"
    f"0 1 21 {cus} 48 0 0 8\\n"     # not a power of two: skipped
    f"9 1 20 {cus} 32 0 0 8\\n"     # unknown kind: skipped
    f"2 1 20 {cus + 1} 32 0 0 8\\n")  # another device: not used here
print(json.dumps([W.tune_lookup("single", 1, 1 << 20), W.tune_lookup("multisource", 64, 1 << 22),
                  W.tune_lookup("single", 1, 1 << 21), W.tune_lookup("batch", 1, 1 << 20)]))
""" % (ROOT, str(path))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    import json
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert got[0] == {"chunk": 32, "persistent": False, "blocks_per_cu": 0, "rows_per_wave": 8}
    assert got[1] == {"chunk": 16, "persistent": True, "blocks_per_cu": 2, "rows_per_wave": 0}
    assert got[2] is None and got[3] is None
