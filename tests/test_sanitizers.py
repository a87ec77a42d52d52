"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The oracle is rebuilt with gcc's sanitizers and driven through its Python
wrapper over small workloads; the library is rebuilt with its host code
(argument checks, topology load, packing, layout, observables) under
clang's sanitizers and the host-only tests run against it.  Device code is
not instrumented (there is no GPU sanitizer here), and no call in these runs
touches a device.  Each run is a child process with the sanitizer runtime
preloaded; a report fails the test.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def _check(proc):
    out = proc.stdout + proc.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert proc.returncode == 0, out[-4000:]


ORACLE_SCRIPT = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle
    from synth import make_config, RunParams
    rng = np.random.default_rng(1)
    for name, kw in (("c0", {{}}), ("c1", {{}}), ("c3", {{"n_traj": 6}})):
        s = make_config(name, **kw)
        o = oracle.OracleSystem(s, RunParams())
        x = s.x + 0.1 * rng.standard_normal(s.x.shape)
        assert np.array_equal(o.pairlist(x), o.pairlist(x, brute=True))
        F, E, fe, st = o.forces(x, step=3)
        assert st == 0
        o.force_scale(x)
        o.force_stiffness(x)
        o.forces_par(x, threads=2)
        o.force_scale_par(x, threads=2)
        o.force_stiffness_par(x, threads=2)
        assert o.run(s.x, 20, energy_every=10)[3] == 0
        assert o.run_par(s.x, 20, energy_every=10, threads=2)[3] == 0
        assert o.run_underdamped(s.x, np.zeros_like(s.x), 20, mass=1.0)[-1] == 0
    print("oracle ok")
""")


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan and shutil.which("gcc")):
        pytest.skip("gcc sanitizer runtimes not found")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp",
                           "-fno-fast-math", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           "-o", lib, os.path.join(ROOT, "oracle", "sop_oracle.c"), "-lm"])
    script = tmp_path / "run_oracle.py"
    script.write_text(ORACLE_SCRIPT.format(root=ROOT))
    env = dict(os.environ, SOP_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    proc = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True,
                          timeout=600)
    _check(proc)
    assert "oracle ok" in proc.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    asan = _clang_asan()
    hipcc = "/opt/rocm/bin/hipcc"
    if not (asan and os.path.exists(hipcc)):
        pytest.skip("hipcc or clang's sanitizer runtime not found")
    sys.path.insert(0, ROOT)
    from paper_1003_1148_amd import build as B
    lib = str(tmp_path / "libsop_san.so")
    flags = [f for f in B.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g"]
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer"):
        flags += ["-Xarch_host", f]
    subprocess.check_call([hipcc] + flags + ["-shared-libsan", "-I", os.path.join(ROOT, "include"),
                                             "-I", B.CSRC] +
                          [os.path.join(B.CSRC, s) for s in B.SOURCES] + ["-o", lib])
    env = dict(os.environ, SOP_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    proc = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                           os.path.join(ROOT, "tests", "test_abi_host.py"),
                           os.path.join(ROOT, "tests", "test_spectroscopy_host.py")],
                          env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    _check(proc)
    probe = subprocess.run([sys.executable, "-c",
                            "import paper_1003_1148_amd as P; print(P.LIB_PATH)"],
                           env=env, capture_output=True, text=True, timeout=300, cwd=ROOT)
    _check(probe)
    assert probe.stdout.strip() == lib
