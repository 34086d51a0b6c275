"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer of the
host code: the oracle, the plan-cache reader and writer (fed malformed
files), and the argument checks of the C-ABI (the host translation units of
libsem.so instrumented, the GPU code unchanged).  Each instrumented build runs
in a child process with the sanitizer runtime preloaded and stops at the
first report.  No GPU is used: every C-ABI call below fails validation before
any HIP call."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_08501_amd", "csrc")
LLVM = "/opt/rocm/llvm"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def asan_runtime():
    found = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    if not found:
        pytest.skip("clang AddressSanitizer runtime not found")
    return found[-1]


def run_child(code, env_extra=None, timeout=600):
    env = dict(os.environ, LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    env.update(env_extra or {})
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    return r.stdout


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    return tmp_path_factory.mktemp("san")


def test_oracle_under_sanitizers(tmp):
    """Every oracle entry point on small inputs (several orders, with and
    without the reference state, boundary faces), instrumented."""
    lib = str(tmp / "libsem_oracle_san.so")
    subprocess.run([os.path.join(LLVM, "bin", "clang"), *SAN, "-ffp-contract=off", "-fPIC",
                    "-shared", "-std=c11", os.path.join(ROOT, "oracle", "sem_oracle.c"), "-o", lib,
                    "-lm"], check=True)
    out = run_child(f"""
        import importlib.util, numpy as np
        import oracle
        oracle._LIB = {lib!r}
        oracle._load()
        spec = importlib.util.spec_from_file_location(
            "sem_inputs", {os.path.join(ROOT, "paper_1604_08501_amd", "inputs.py")!r})
        I = importlib.util.module_from_spec(spec)
        import sys
        sys.modules["sem_inputs"] = I
        spec.loader.exec_module(I)
        for N in (1, 3, 4):
            w = I.warped_workload(N=N, n_side=3, k=500 + N, with_adjoint=True)
            ph = w.phys.as_tuple()
            v = oracle.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, ph)
            v0 = oracle.volume_rhs(w.D, w.geo, w.q, None, None, ph)
            mu = oracle.volume_rhs_adjoint(w.D, w.geo, w.q, w.lam, ph)
            t = I.add_tracers(w)
            for dirs in (3, 7):
                oracle.volume_rhs_ext(t.D, t.geo, t.q, t.rho_ref, t.theta_ref, ph, dirs=dirs)
            s = oracle.surface_rhs(w.geo, w.q, w.nbr, w.theta_ref, ph)
            nbr = w.nbr.copy(); nbr[0, :] = -1; nbr[1, 2] = 10 ** 6
            s2 = oracle.surface_rhs(w.geo, w.q, nbr, None, ph)
            r = oracle.ssp_rk3_step(lambda q: oracle.volume_rhs(w.D, w.geo, q, w.rho_ref,
                                                               w.theta_ref, ph), w.q, 1e-3)
            assert all(np.isfinite(a).all() for a in (v, v0, mu, s, s2, r))
        print("oracle ok")
        """)
    assert "oracle ok" in out


MALFORMED = {
    "empty.json": "",
    "good.json": '{\n  "gfx950/f64/nt512/lds41088/nq8/ne8192": {"epb": 1, "layout": 1, "us": 79.3}\n}\n',
    "huge.json": '{"a": {"epb": 1e300, "layout": -1e300, "us": 1e400}, '
                 '"b": {"epb": 99999999999, "layout": 3, "us": 5}}',
    "nan.json": '{"a": {"epb": nan, "layout": inf, "us": -nan}, "b": {"epb": 2, "layout": 0, "us": nan}}',
    "truncated.json": '{"gfx950/f32/nt256": {"epb": 4, "lay',
    "unbalanced.json": '{"a": }}}} {"b": {{{ "epb": 2, "layout": 1, "us": 3}',
    "quotes.json": '"""""""{"epb": 1}"""' * 50,
    "nonnumeric.json": '{"a": {"epb": "x", "layout": [], "us": {}}}',
    "garbage.bin": bytes(range(256)) * 64,
    "longkey.json": '{"' + "k" * 100000 + '": {"epb": 1, "layout": 0, "us": 1}}',
    "many.json": "{" + ",".join(f'"k{i}": {{"epb": {i % 8 + 1}, "layout": {i % 2}, "us": {i}.5}}'
                                for i in range(5000)) + "}",
}


def test_plan_cache_reader_on_malformed_files(tmp):
    """The plan-cache reader on empty, truncated, unbalanced, non-numeric,
    out-of-range, NaN, binary and oversized files: no sanitizer report,
    entries only within the documented ranges, and a write/read round trip
    that keeps every entry."""
    exe = str(tmp / "plan_cache_harness")
    subprocess.run([os.path.join(LLVM, "bin", "clang++"), *SAN, "-std=c++17", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "sanitize", "plan_cache_harness.cpp"),
                    os.path.join(CSRC, "sem_cache.cpp"), "-o", exe], check=True)
    files = []
    for name, text in MALFORMED.items():
        p = tmp / name
        p.write_bytes(text if isinstance(text, bytes) else text.encode())
        files.append(str(p))
    files.append(str(tmp / "missing.json"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(tmp / "scratch.json"), *files], env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    counts = dict(line.rsplit(": ", 1) for line in r.stdout.splitlines())
    assert counts[str(tmp / "good.json")] == "1 entries"
    assert counts[str(tmp / "huge.json")] == "0 entries"
    assert counts[str(tmp / "nan.json")] == "0 entries"
    assert counts[str(tmp / "longkey.json")] == "0 entries"
    assert counts[str(tmp / "many.json")] == "5000 entries"
    assert counts[str(tmp / "missing.json")] == "0 entries"


HOST_TUS = ("sem_api.cpp", "sem_plan.cpp", "sem_cache.cpp", "batch_static.hip")


@pytest.mark.slow
def test_c_abi_validation_under_sanitizers(tmp):
    """The host translation units of libsem.so built with the sanitizers
    (GPU code unchanged) and linked with the regular kernel objects; the CPU
    argument-check tests of the C-ABI then run against that library."""
    from paper_1604_08501_amd import build as B
    if not all(os.path.exists(os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o"))
               for s in B.SOURCES):
        B.build()
    san_host = [f for flag in SAN for f in ("-Xarch_host", flag)]
    objs = []
    for src in B.SOURCES:
        stem = os.path.splitext(src)[0]
        if src in HOST_TUS:
            o = str(tmp / f"{stem}_san.o")
            subprocess.run([B.hipcc(), *B.HIPCC_FLAGS, *san_host, "-c", os.path.join(CSRC, src),
                            "-o", o], check=True, capture_output=True)
            objs.append(o)
        else:
            objs.append(os.path.join(B.BUILD, stem + ".o"))
    lib = str(tmp / "libsem_san.so")
    subprocess.run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *objs, "-o", lib],
                   check=True, capture_output=True)
    out = run_child(f"""
        import sys, pytest
        from paper_1604_08501_amd import semvol
        semvol.LIB_PATH = {lib!r}
        semvol.lib()
        # (the C-client test builds and runs its own program, not this library)
        sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu",
                              "-k", "not c_client",
                              {os.path.join(ROOT, "tests", "test_abi.py")!r}]))
        """)
    assert "passed" in out
