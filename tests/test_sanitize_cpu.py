"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the host sources are compiled again with both sanitizers into a
small driver (tests/sanitize/host_check.cpp) that bit-blasts, splits and
traces seeded query batches of every workload family (exact, without
rewriting, and with 32-bit machine integers), raw random k-SAT batches and
given cubes, and walks the error paths; any memory or UB error aborts it.
The device objects of the normal build are linked unchanged (no GPU call is
made)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2601_21552_amd")
HOST_SRCS = ["api.cpp", "encode.cpp", "split.cpp", "verify.cpp"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _write_queries(path, gens):
    from paper_2601_21552_amd.api import pack_queries
    nodes, nstart, roots, rstart = pack_queries([g.query.arrays()[:2] for g in gens])
    with open(path, "wb") as f:
        for a in (nodes, np.asarray(nstart, np.uint64), np.asarray(roots, np.uint32), np.asarray(rstart, np.uint64)):
            f.write(np.uint64(len(a)).tobytes())
            f.write(np.ascontiguousarray(a).tobytes())


def _write_raw(path, cnfs):
    nv, qs, off, lits = w.concat(cnfs)
    with open(path, "wb") as f:
        for a in (nv, qs, off, lits):
            f.write(np.uint64(len(a)).tobytes())
            f.write(np.ascontiguousarray(a).tobytes())


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    from paper_2601_21552_amd import build
    dev_objs = [os.path.join(build.OBJ, s + ".o") for s in build.HIP_SRCS]
    if not all(os.path.exists(o) for o in dev_objs):
        build.build()
    d = tmp_path_factory.mktemp("san")
    objs = []
    for i, o in enumerate(dev_objs):     # the device objects of the normal build
        dst = str(d / f"kernels{i}.o")
        shutil.copy(o, dst)
        objs.append(dst)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include"]
    procs = []
    for s in HOST_SRCS:
        out = str(d / (s + ".san.o"))
        procs.append(subprocess.Popen(["g++", "-std=c++17", "-O1", "-g", "-fPIC", *SAN, *inc, "-c",
                                       os.path.join(PKG, "csrc", s), "-o", out],
                                      stderr=subprocess.PIPE, text=True))
        objs.append(out)
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err
    exe = str(d / "host_check")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, *inc,
                        os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"), *objs,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


def _run(exe, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", SCUBA_HOST_THREADS="4")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host check ok" in r.stdout


def test_host_code_under_sanitizers(driver):
    exe, d = driver
    rng = np.random.Generator(np.random.PCG64(601))
    inputs = {
        "q1d": w.batch_1d(n=48),
        "q2d": w.batch_2d(n=48, wmax=12),
        "qpart": w.partition_batch(n=32, width=10),
        "qlow": w.batch_lower(n=32),
        "qsingle": [w.single_access(v) for v in ("lt", "none", "le")],
    }
    args = []
    for name, gens in inputs.items():
        path = str(d / f"{name}.bin")
        _write_queries(path, gens)
        args += ["queries", path]
        if name in ("q1d", "qsingle"):
            args += ["norewrite", path]
    wrap = str(d / "wrap.bin")
    _write_queries(wrap, w.batch_wrap(n=24, m=32))
    args += ["wrap32", wrap]
    raw = str(d / "raw.bin")
    _write_raw(raw, [w.random_ksat(n, int(round(4.0 * n)), 3, rng) for n in (12, 20, 30, 40)]
               + [w.pigeonhole(4, 3), w.CNF.from_clauses(3, [], name="empty")])
    args += ["raw", raw]
    _run(exe, args)
