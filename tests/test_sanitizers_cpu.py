"""The oracle and the host-copy renderer under AddressSanitizer and
UndefinedBehaviorSanitizer.

Both C libraries are rebuilt here with -fsanitize=address,undefined (plus
float-cast-overflow and float-divide-by-zero, which gcc's "undefined" leaves
out), every finding fatal, and the oracle's pin tests and the host-copy tests
run again in a child interpreter that loads those builds (MM_ORACLE_LIB,
MM_HOSTCOPY_LIB) with the ASan runtime preloaded. The pins that compile
cross-check programs of their own (ATen's and rocRAND's Philox) are left to
the ordinary run. The served form's host scheduling policy has a sanitizer
test of its own (test_sched_cpu.py).

The C ABI library itself is rebuilt with the host side of every source under
the same sanitizers (`-Xarch_host`: the device code is built as always), and
the C ABI tests that need no GPU (argument validation, exported symbols,
status strings) run against it with clang's ASan runtime preloaded (MM_LIB
names that build)."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fsanitize=float-cast-overflow",
       "-fsanitize=float-divide-by-zero", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.slow
def test_oracle_and_hostcopy_pins_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime")
    oracle_lib = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                    "-fexcess-precision=standard", "-fPIC", "-shared", "-Wall", "-Wextra", *SAN,
                    os.path.join(ROOT, "oracle", "mm_oracle.c"), "-o", oracle_lib, "-lm"],
                   check=True, capture_output=True, text=True)
    hc = os.path.join(ROOT, "paper_2504_20937_amd", "hostcopy")
    hostcopy_lib = str(tmp_path / "libmm_hostcopy_san.so")
    subprocess.run([gcc, "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-Wall", *SAN, "-I", hc, os.path.join(hc, "hostcopy.c"),
                    "-o", hostcopy_lib, "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, MM_ORACLE_LIB=oracle_lib, MM_HOSTCOPY_LIB=hostcopy_lib,
               LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = [os.path.join(HERE, f) for f in ("test_oracle_displace.py", "test_oracle_render.py",
                                              "test_oracle_edges.py", "test_oracle_philox.py",
                                              "test_hostcopy_cpu.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", "-k", "not aten and not rocrand", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in r.stdout and "AddressSanitizer" not in out and "runtime error" not in out


@pytest.mark.slow
def test_c_abi_validation_under_host_sanitizers(tmp_path):
    import glob
    from concurrent.futures import ThreadPoolExecutor

    sys.path.insert(0, ROOT)
    from paper_2504_20937_amd import build as mmbuild

    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang ASan runtime")
    host_san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-shared-libsan", "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", flag]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        r = subprocess.run([mmbuild.hipcc(), *mmbuild.HIPFLAGS, *host_san, "-g", "-c", src, "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        objs = list(ex.map(compile_one, mmbuild.sources()))
    lib = str(tmp_path / "libmm_san.so")
    # the sanitizer runtime is the preloaded one, resolved at load time
    r = subprocess.run([mmbuild.hipcc(), "--offload-arch=" + mmbuild.ARCH, "-shared", "-fPIC", *objs,
                        "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    probe = ("import paper_2504_20937_amd as mm; mm.lib(); "
             "print(any('libmm_san' in l for l in open('/proc/self/maps')))")
    env = dict(os.environ, MM_LIB=lib, LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    loaded = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                            text=True, timeout=300)
    assert loaded.stdout.strip() == "True", loaded.stdout + loaded.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(HERE, "test_capi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in r.stdout and "AddressSanitizer" not in out and "runtime error" not in out
