"""Host AddressSanitizer run over the library's argument checks and error paths.

Every library source is compiled with AddressSanitizer on its host side only
(the device code is built as usual), linked into a separate library, and
driven by ``tests/asan/abi_errors.cpp``: invalid meshes, velocity sets, gases,
boundary tables, batches and networks, NULL handles, a missing tuning file,
and one valid case that fails at its first device call here (no GPU).  Each
call must return its documented status with a message, and the sanitizer must
report no invalid access and no leak.  No GPU is touched.
"""

import os
import shutil
import subprocess

import pytest

from paper_2606_15720_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(B.HIPCC) and os.path.exists(CLANG)),
                    reason="hipcc or clang++ not installed")
def test_error_paths_are_clean_under_asan(tmp_path):
    flags = [f for f in B.FLAGS if f not in ("-O3",)] + [
        "-O1", "-g", f"-I{os.path.join(ROOT, 'include')}",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        procs.append(subprocess.Popen([B.HIPCC, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, out.decode()[-2000:]
    lib = str(tmp_path / "libugks_asan.so")
    subprocess.check_call([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                           "-Xarch_host", "-fsanitize=address", *objs, "-o", lib,
                           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    exe = str(tmp_path / "abi_errors")
    subprocess.check_call([CLANG, "-std=c++17", "-g", "-fsanitize=address",
                           f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include",
                           "-D__HIP_PLATFORM_AMD__", os.path.join(HERE, "asan", "abi_errors.cpp"),
                           f"-L{tmp_path}", "-lugks_asan", f"-Wl,-rpath,{tmp_path}",
                           "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "0 unexpected" in r.stdout
