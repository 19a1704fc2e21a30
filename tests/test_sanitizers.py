"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU:

* the oracle (oracle/oracle.c) on small problems that reach every branch
  (no covariates, a degenerate SNP, h2 at 0 and 1, an indefinite Phi, an
  empty cell list, refused arguments), its outputs compared with the regular
  build's;
* the library's host code (abi.cpp, pipeline.cpp, bed.cpp: argument and
  call-order checks, the genotype-file checks of the reader, the workspace
  carving over some 1400 plan shapes) through tests/sanitize/abi_checks.cpp,
  linked with the regular (unsanitized) device objects and run without a GPU;
* a planted out-of-bounds read and a signed overflow in a throwaway program,
  to show that these flags do report errors.

Only host code is instrumented: on the hipcc lines every -fsanitize= follows
-Xarch_host."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1207_2169_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
HIP_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise AssertionError(f"{' '.join(cmd)} -> {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}")
    return r


def test_sanitizers_report_planted_errors(tmp_path):
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n#include <limits.h>\n"
                   "int main(int argc, char** argv) {\n"
                   "  int* a = malloc(4 * sizeof(int));\n"
                   "  int v = argc > 1 ? a[argc + 3] : 0;\n"   # argc = 2: reads a[5]
                   "  int big = INT_MAX - 1 + argc;\n"          # argc = 3: overflows
                   "  free(a);\n  return v + (big & 1);\n}\n")
    exe = str(tmp_path / "planted")
    _run(["gcc", *GCC_SAN, "-o", exe, str(src)])
    r = subprocess.run([exe, "x"], capture_output=True, text=True, env=ENV)
    # AddressSanitizer or UBSan's object-size check, whichever sees the read first
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr)
    r = subprocess.run([exe, "x", "y"], capture_output=True, text=True, env=ENV)
    assert r.returncode != 0 and "runtime error" in r.stderr


def _problems():
    """(arrays, var_conv, threads) of small problems covering the oracle's branches."""
    rng = np.random.default_rng(41)
    out = []

    def kin(n, rank):
        A = rng.standard_normal((n, rank))
        return A @ A.T / rank + 0.05 * np.eye(n)

    n, pL, ng, nt = 40, 3, 6, 3
    XL = np.c_[np.ones(n), rng.standard_normal((n, pL - 1))]
    G = rng.integers(0, 3, (n, ng)).astype(np.float64)
    G[:, 4] = XL[:, 1]                       # a SNP in span(X_L): flagged degenerate
    Y = rng.standard_normal((n, nt))
    ii, jj = np.meshgrid(np.arange(ng), np.arange(nt), indexing="ij")
    out.append((kin(n, 80), XL, G, Y, np.array([0.0, 1.0, 0.4]), np.array([1.0, 2.0, 0.5]),
                ii.ravel(), jj.ravel(), 0, 2))
    out.append((kin(n, 80), XL, G, Y, np.array([0.3, 0.6, 0.9]), np.ones(3), ii.ravel(), jj.ravel(), 1, 1))
    # no covariates
    out.append((kin(n, 80), np.zeros((n, 0)), G, Y, np.array([0.5, 0.2, 0.7]), np.ones(3), ii.ravel(), jj.ravel(),
                0, 3))
    # an indefinite Phi: M_j not SPD for h2 near 1 (flag 2), fine at h2 = 0
    P = kin(n, 80)
    P[0, 0] = -5.0
    out.append((P, XL, G, Y, np.array([0.0, 0.99, 1.0]), np.ones(3), ii.ravel(), jj.ravel(), 0, 2))
    # an empty cell list
    out.append((kin(n, 80), XL, G, Y, np.ones(3) * 0.5, np.ones(3), np.zeros(0, np.int64), np.zeros(0, np.int64),
                0, 1))
    # a larger problem (the parallel Cholesky path for n - j > 256)
    n2 = 300
    XL2 = np.c_[np.ones(n2), rng.standard_normal(n2)]
    G2 = rng.integers(0, 3, (n2, 2)).astype(np.float64)
    Y2 = rng.standard_normal((n2, 2))
    out.append((kin(n2, 600), XL2, G2, Y2, np.array([0.5, 0.8]), np.array([1.0, 1.5]), np.array([0, 1, 1]),
                np.array([0, 0, 1]), 0, 4))
    return out


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", *GCC_SAN, "-fopenmp", "-std=gnu11", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_checks.c"), "-lm"])
    probs = _problems()
    with open(tmp_path / "in.bin", "wb") as f:
        for Phi, XL, G, Y, h2, s2, snp, tr, vc, thr in probs:
            n, pL = Phi.shape[0], XL.shape[1]
            np.array([n, pL, G.shape[1], Y.shape[1], snp.size, vc, thr], np.int64).tofile(f)
            for a in (Phi, XL, G, Y):
                np.asfortranarray(a, dtype=np.float64).ravel(order="F").tofile(f)
            np.asarray(h2, np.float64).tofile(f)
            np.asarray(s2, np.float64).tofile(f)
            np.asarray(snp, np.int64).tofile(f)
            np.asarray(tr, np.int64).tofile(f)
    r = _run([exe, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")], env=ENV)
    assert f"{len(probs)} problems" in r.stdout
    raw = open(tmp_path / "out.bin", "rb").read()
    off = 0
    seen_flags = set()
    for Phi, XL, G, Y, h2, s2, snp, tr, vc, thr in probs:
        rc = int(np.frombuffer(raw, np.int32, 1, off)[0])
        off += 4
        assert rc == 0
        nc, p = snp.size, XL.shape[1] + 1
        b = np.frombuffer(raw, np.float64, nc * p, off).reshape(nc, p)
        off += 8 * nc * p
        var = np.frombuffer(raw, np.float64, nc * p * p, off).reshape(nc, p, p).transpose(0, 2, 1)
        off += 8 * nc * p * p
        fl = np.frombuffer(raw, np.int32, nc, off)
        off += 4 * nc
        if nc == 0:
            continue
        rb, rv, rf = oracle.gls_cells(Phi, XL, G, Y, h2, s2, snp, tr, var_paper=bool(vc), threads=thr)
        assert np.array_equal(fl, rf)
        assert np.allclose(b, rb, rtol=1e-12, atol=0, equal_nan=True)
        assert np.allclose(var, rv, rtol=1e-12, atol=0, equal_nan=True)
        seen_flags |= set(fl.tolist())
    assert off == len(raw)
    assert seen_flags >= {0, 1, 2}  # solved, degenerate SNP and non-SPD M_j cells all exercised


def _device_objects(tmp_path):
    """The library's regular device objects: the in-tree build's when newer
    than every source, else compiled here with the library's own flags."""
    sys.path.insert(0, ROOT)
    from paper_1207_2169_amd import build as libbuild
    srcs = [s for s in libbuild.SOURCES if s.endswith(".hip")]
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp"))]
    newest = max(os.path.getmtime(f) for f in deps + [os.path.join(ROOT, "include", "clak.h")])
    objs = [os.path.join(libbuild.OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in srcs]
    if all(os.path.exists(o) and os.path.getmtime(o) >= newest for o in objs):
        return objs
    out = []
    for s in srcs:
        obj = str(tmp_path / (os.path.splitext(s)[0] + ".o"))
        _run([libbuild.HIPCC, *libbuild.FLAGS, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", obj])
        out.append(obj)
    return out


@pytest.mark.timeout(900)
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_library_code_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1207_2169_amd import build as libbuild
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in ("abi.cpp", "pipeline.cpp", "bed.cpp", os.path.join(SAN, "abi_checks.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={libbuild.ARCH}", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", *inc, *HIP_SAN, "-c", path, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "abi_checks")
    _run([HIPCC, f"--offload-arch={libbuild.ARCH}", *HIP_SAN, "-o", exe, *objs, *_device_objects(tmp_path),
          "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"])
    scratch = tmp_path / "files"
    scratch.mkdir()
    r = _run([exe, str(scratch)], env=ENV, timeout=300)
    print(r.stdout.strip().splitlines()[-1])
    assert ", 0 failed" in r.stdout
