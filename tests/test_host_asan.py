"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs: the library's
error paths and the oracle.

* Every library source is compiled with both sanitizers on its host side
  only (the device code is built as usual), linked into a separate library,
  and driven by ``tests/asan/abi_errors.cpp``: invalid meshes, velocity sets,
  gases, boundary tables, batches and networks, NULL handles, a missing
  tuning file, and one valid case that fails at its first device call here
  (no GPU).  Each call must return its documented status with a message.
* The oracle is compiled with both sanitizers and run by
  ``tests/asan/oracle_cases.cpp`` on small cases covering walls, periodic
  faces, far-field faces, 2-D and 3-D, both reconstruction orders; its final
  state must equal the regular build's.

In both the sanitizers must report no invalid access, no leak and no
undefined behaviour.  No GPU is touched.
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
        "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
        "-Xarch_host", "-fno-omit-frame-pointer"]
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
                           "-Xarch_host", "-fsanitize=address,undefined", *objs, "-o", lib,
                           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    exe = str(tmp_path / "abi_errors")
    subprocess.check_call([CLANG, "-std=c++17", "-g", "-fsanitize=address,undefined",
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
    assert "runtime error" not in r.stderr, r.stderr[-4000:]  # UndefinedBehaviorSanitizer
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "0 unexpected" in r.stdout


def _write_case(path, case, steps, order):
    """The case file read by ``tests/asan/oracle_cases.cpp``, with the final
    W of the regular oracle build after ``steps`` steps."""
    import numpy as np
    from oracle import Oracle

    m = case.mesh.contiguous()
    v, g = case.vel, case.gas
    o = Oracle(case, order=order)
    o.step(steps)
    W = o.state(with_h=False)[0]
    f8 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    arrays = [
        f8(m.cell_volume), f8(m.cell_centroid), np.ascontiguousarray(m.face_cells, dtype=np.int64),
        f8(m.face_area), f8(m.face_normal), f8(m.face_centroid),
        f8(m.face_shift) if m.face_shift is not None else np.zeros(0),
        np.ascontiguousarray(m.face_bc, dtype=np.int32), np.ascontiguousarray(m.face_bc_id, dtype=np.int32),
        f8(v.u), f8(v.w),
        np.array([b.kind for b in case.bcs], dtype=np.int32), f8([b.rho for b in case.bcs]),
        f8([list(b.U) + [0.0] * (3 - len(b.U)) for b in case.bcs]), f8([b.T for b in case.bcs]),
        f8(case.W0), f8(W),
    ]
    hi = np.array([m.dim, m.n_cells, m.n_faces, v.nv, len(case.bcs), g.K, steps, order], dtype=np.int64)
    hd = np.array([g.Pr, g.R, g.T_ref, g.mu_ref, g.omega, g.cfl, g.dt, 0.0], dtype=np.float64)
    with open(path, "wb") as f:
        f.write(hi.tobytes())
        f.write(hd.tobytes())
        for a in arrays:
            b = a.tobytes()
            f.write(np.int64(len(b)).tobytes())
            f.write(b)


def test_oracle_is_clean_under_asan(tmp_path):
    import ugks_cases as uc

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not installed")
    exe = str(tmp_path / "oracle_cases")
    subprocess.check_call([gxx, "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "ugks_oracle.cpp"),
                           os.path.join(HERE, "asan", "oracle_cases.cpp"), "-o", exe])
    cases = [
        ("cavity2d", uc.cavity2d(n=5, nv=6), 4, 2),      # walls, moving lid
        ("couette2d", uc.couette2d(n=5, nv=6), 4, 2),    # periodic faces
        ("channel2d", uc.channel2d(n=4, nv=6), 4, 2),    # far-field faces
        ("sod3d", uc.sod3d_tets(n=2, nv=6), 3, 2),       # tets, 3-D
        ("cavity2d_o1", uc.cavity2d(n=5, nv=6), 3, 1),   # first-order reconstruction
    ]
    files = []
    for name, case, steps, order in cases:
        path = str(tmp_path / f"{name}.bin")
        _write_case(path, case, steps, order)
        files.append(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe, *files], env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]  # UndefinedBehaviorSanitizer
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert f"{len(cases)} cases, 0 failed" in r.stdout
