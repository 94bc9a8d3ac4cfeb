"""The serving loop and the batch scheduler on the host, under ASan and UBSan.

The library's `server.cpp`, `exec.cpp`, `desc.cpp` and `mlmc.cpp` are compiled unchanged
for the host only (no device code) and linked against stand-ins for the
device layer (`tests/host/fake_device.cpp`: known per-sample results, solves
of known length, injected device errors) and for the HIP runtime
(`tests/host/fake_hip.cpp`: host memory, immediate execution, tracked
allocations).  Each scenario of `tests/host/server_sim.cpp` checks every
result by sample index and runs in its own process.
"""

import concurrent.futures
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2306_13493_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("exec.cpp", "server.cpp", "desc.cpp", "mlmc.cpp")] + [
    os.path.join(HERE, "host", f) for f in ("fake_hip.cpp", "fake_device.cpp", "server_sim.cpp")]
SCENARIOS = ["batch", "autotune_cache", "mlmc_checkpoint", "serve_mix", "admission", "continuous", "overload", "isolation", "loop_error",
             "destroy_pending"]


def _tool(name):
    p = shutil.which(name) or os.path.join("/opt/rocm/bin", name)
    return p if os.path.exists(p) else None


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    hipcc = _tool("hipcc")
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if hipcc is None or not os.path.exists(clangxx):
        pytest.skip("hipcc / clang++ not available")
    out = tmp_path_factory.mktemp("server_sim")
    # host code only; the sanitizers apply to the host pass
    flags = ["-O1", "-g", "-std=c++17", "--offload-host-only", "-x", "hip", "-fno-omit-frame-pointer",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def compile_one(src):
        obj = str(out / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        r = subprocess.run([hipcc] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    exe = str(out / "server_sim")
    r = subprocess.run([clangxx, "-fsanitize=address,undefined"] + objs + ["-o", exe, "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scenario(sim, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sim, scenario], capture_output=True, text=True, timeout=150, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok " + scenario
