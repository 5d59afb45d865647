"""The kernels' device code under the sanitizers on the CPU (no GPU needed).

tests/devicecheck emulates the HIP device model on the host: a launch runs its workgroups
in sequence with one host thread per lane; __syncthreads, the DPP quad permutes and the
wave shuffles exchange values through barriers.  The library's host code, the rollout,
sampling, update, plant, proposal-noise, tracking-cost and batch kernels are compiled for the
CPU against it (the kernel sources unchanged except that the dynamic-LDS declaration is
renamed so the host compiler can define it), and the launch sequences of the GPU tests
run under
  * AddressSanitizer + UndefinedBehaviorSanitizer: out-of-bounds accesses to device
    buffers (heap), the LDS array and lane-local arrays, integer overflow, bad shifts;
  * MemorySanitizer: reads of memory never written (the caller's workspace and LDS start
    poisoned);
  * ThreadSanitizer: races between lanes on LDS or device memory (a missing barrier).
The batched-serving runtime and its persistent kernels (per-scene and single launch,
graph capture emulated by recording the launches) run under the address and thread
sanitizers; the memory sanitizer run leaves them out (see test_kernels_under_memory_sanitizer).
Every result is also compared with the FP64 oracle.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DC = os.path.join(ROOT, "tests", "devicecheck")
CS = os.path.join(ROOT, "paper_2409_10469_amd", "csrc")
ORC = os.path.join(ROOT, "oracle")
CLANG = "/opt/rocm/llvm/bin/clang++"
CLANG_C = "/opt/rocm/llvm/bin/clang"

KERNELS = ["mppi_kernels.hip", "rollout16.hip", "proposal_kernels.hip", "tracking_kernels.hip"]
HOST = [os.path.join(DC, "emu.cpp"), os.path.join(DC, "driver.cpp"), os.path.join(CS, "mppi_api.cpp"),
        os.path.join(CS, "mppi_policy.cpp"), os.path.join(CS, "mppi_batch.cpp")]
ORACLE = [os.path.join(ORC, "mppi_oracle.c"), os.path.join(ORC, "tracking_oracle.c")]


def _build(tmp, cxx, cc, san, extra=()):
    srcs = []
    for k in KERNELS:
        dst = os.path.join(tmp, k.replace(".hip", ".cpp"))
        with open(os.path.join(CS, k)) as f:
            text = f.read()
        # the only change: the dynamic-LDS declaration gets a name the host compiler can define
        with open(dst, "w") as f:
            f.write(text.replace("extern __shared__", "EMU_DYNAMIC_SHARED"))
        srcs.append(dst)
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}", *extra, "-pthread"]
    inc = ["-I", DC, "-I", os.path.join(ROOT, "include"), "-I", CS, "-I", ORC]
    jobs = [([cxx, "-std=c++17", *flags, "-Wno-unknown-pragmas", "-Wno-attributes", "-Wno-ignored-attributes",
              *inc, "-c", s, "-o", os.path.join(tmp, os.path.basename(s) + ".o")], s) for s in HOST + srcs]
    jobs += [([cc, *flags, "-c", s, "-o", os.path.join(tmp, os.path.basename(s) + ".o")], s) for s in ORACLE]

    def run(job):
        return subprocess.run(job[0], capture_output=True, text=True)

    # three builds run at once (see `runs`), so each takes a third of the cores
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1) // 3)) as ex:
        results = list(ex.map(run, jobs))
    for r, (cmd, src) in zip(results, jobs):
        assert r.returncode == 0, (src, r.stderr[-3000:])
    exe = os.path.join(tmp, "devicecheck")
    objs = [os.path.join(tmp, os.path.basename(s) + ".o") for _, s in jobs]
    r = subprocess.run([cxx, f"-fsanitize={san}", *extra, "-pthread", *objs, "-o", exe, "-lm"], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, mode, env, extra=()):
    r = subprocess.run([exe] + ([mode] if mode else []) + list(extra), capture_output=True, text=True, timeout=1200,
                       env=dict(os.environ, **env))
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "failures: 0" in r.stdout, out[-6000:]
    for marker in ("AddressSanitizer", "runtime error", "MemorySanitizer", "ThreadSanitizer", "emulation:"):
        assert marker not in r.stderr, out[-6000:]
    return r.stdout


def _asan(tmp):
    if shutil.which("g++") is None:
        return "g++ is not available"
    exe = _build(tmp, "g++", "gcc", "address,undefined", ["-fno-sanitize-recover=undefined"])
    out = _run(exe, None, {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert out.count(" ok") >= 13


def _msan(tmp):
    if not os.path.exists(CLANG):
        return "clang is not available"
    exe = _build(tmp, CLANG, CLANG_C, "memory", ["-fsanitize-memory-track-origins"])
    # without the batch case: its runtime's std::map rebalances inside the uninstrumented
    # C++ library, which MemorySanitizer cannot follow (the batch kernels run under the
    # address and thread sanitizers)
    _run(exe, "quick", {}, ["no-batch"])


def _tsan(tmp):
    if shutil.which("g++") is None:
        return "g++ is not available"
    exe = _build(tmp, "g++", "gcc", "thread")
    _run(exe, "quick", {"TSAN_OPTIONS": "halt_on_error=1"})


@pytest.fixture(scope="module")
def runs(tmp_path_factory):
    """The three sanitizer builds and runs, started together (each is a separate process
    tree), so the module takes about as long as the slowest of them."""
    ex = ThreadPoolExecutor(max_workers=3)
    futs = {name: ex.submit(fn, str(tmp_path_factory.mktemp(name))) for name, fn in
            (("asan", _asan), ("msan", _msan), ("tsan", _tsan))}
    yield futs
    ex.shutdown(wait=True)


def _outcome(fut):
    skip = fut.result()  # re-raises the run's assertion
    if skip:
        pytest.skip(skip)


def test_kernels_under_address_and_undefined_behaviour_sanitizers(runs):
    _outcome(runs["asan"])


def test_kernels_under_memory_sanitizer(runs):
    _outcome(runs["msan"])


def test_kernels_under_thread_sanitizer(runs):
    _outcome(runs["tsan"])
