"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU code paths:
the oracle (oracle.c built with gcc -fsanitize=address,undefined) driven
through its Python front-end on small cases of every PDE, the CFL step, the
FD step, con2prim with the guess fallback and the halo fill; and the
library's host runtime (the .hip sources compiled host-only with
-fsanitize=address,undefined on the host side) driven through every C-ABI
call that needs no GPU: descriptor validation, workspace sizing, the
column-run tables, the tuning-cache file format and the offload checks.
Each runs in a child process with the sanitizer runtime preloaded; any
report fails the test (errors are not recoverable, leaks are not checked:
the interpreter itself is not instrumented)."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()


def _run_child(code, env_extra, tmp_path):
    script = tmp_path / "child.py"
    script.write_text(textwrap.dedent(code))
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, str(script)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "CHILD OK" in r.stdout, out[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fPIC", "-shared",
                           "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    code = f"""
    import sys
    sys.path.insert(0, {ROOT!r})
    sys.path.insert(0, {os.path.join(ROOT, "tests")!r})
    import numpy as np
    import oracle
    oracle._LIB = {str(lib)!r}
    from paper_2608_19273_amd import inputs as I
    # FV: 2D Euler, 3D Euler with ragged patches, both advection forms, SRHD, material field
    oracle.fv_step(I.config0(), cfl=0.4, n_steps=2)
    oracle.fv_step(I.config1(grid=(2, 2, 1), p=8), cfl=0.4, n_steps=2)
    oracle.fv_step(I.adv_var_batch((2, 2, 1), 4), cfl=0.4, n_steps=2)
    oracle.fv_step(I.config3(grid=(2, 1, 1), p=4), cfl=0.4, n_steps=1)
    # FD4 + KO6 + RK4: Euler with a halo of 3 and the linear system
    oracle.fd_step(I.config1(grid=(2, 1, 1), p=4, halo=3), cfl=0.5, sigma=0.1, n_steps=1)
    oracle.fd_step(I.config2(n_patches=3, N=6, sizes=np.array([4, 8, 4], np.int32)), cfl=0.5, sigma=0.1, n_steps=1)
    # con2prim: plain, and a guess that cannot converge in 2 iterations (the fallback)
    cons, p = I.srhd_training_pairs(5, 500)
    oracle.con2prim(cons, tol=1e-12, maxit=50)
    oracle.con2prim(cons, tol=1e-12, maxit=2, p_guess=p * 1e3)
    print("CHILD OK")
    """
    _run_child(code, {"LD_PRELOAD": f"{asan} {ubsan}"}, tmp_path)


def test_host_runtime_under_asan_ubsan(tmp_path):
    rt_dir = "/opt/rocm/lib/llvm/lib/clang"
    rts = []
    if os.path.isdir(rt_dir):
        for v in sorted(os.listdir(rt_dir)):
            for name in ("libclang_rt.asan-x86_64.so", "libclang_rt.ubsan_standalone-x86_64.so"):
                f = os.path.join(rt_dir, v, "lib", "linux", name)
                if os.path.exists(f):
                    rts.append(f)
    if not any("asan" in f for f in rts):
        pytest.skip("clang sanitizer runtime not installed")
    asan = [f for f in rts if "asan" in f][-1]
    sys.path.insert(0, ROOT)
    from paper_2608_19273_amd import build as B
    import concurrent.futures as cf

    def compile_one(src):
        # the device code is built as in the product (the objects must carry
        # their code objects to link); only the host side is instrumented
        obj = tmp_path / (os.path.basename(src) + ".o")
        cmd = [B.HIPCC] + B.DEVICE_FLAGS + ["-g", "-fno-omit-frame-pointer",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all",
               "-I", os.path.join(ROOT, "include"), "-c", src, "-o", str(obj)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return str(obj)

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.sources()))
    lib = tmp_path / "libpatchhip_san.so"
    r = subprocess.run([B.HIPCC, "--offload-arch=" + B.ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", str(lib)] + objs,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    code = f"""
    import sys
    sys.path.insert(0, {ROOT!r})
    sys.path.insert(0, {os.path.join(ROOT, "tests")!r})
    import paper_2608_19273_amd as pb
    pb.LIB_PATH = {str(lib)!r}
    import pytest
    rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", {os.path.join(ROOT, "tests", "test_abi_cpu.py")!r}])
    if rc == 0:
        print("CHILD OK")
    sys.exit(int(rc))
    """
    _run_child(code, {"LD_PRELOAD": asan}, tmp_path)
