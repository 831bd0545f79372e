"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle, and the library's host side (argument checks, graph
validation, renumbering and tiling, which run before any device call).
Each build goes to a temporary directory and runs in a child process with
the sanitizer runtime preloaded; a report from either sanitizer fails the
test.  Device code is built as usual (sanitizers are applied to host code
only)."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _runtime(cmd):
    out = subprocess.run(cmd, capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _child(script, preload, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    report = "AddressSanitizer" in r.stderr or "runtime error:" in r.stderr
    assert r.returncode == 0 and not report, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers():
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    ubsan = _runtime(["gcc", "-print-file-name=libubsan.so"])
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "librs_oracle_san.so")
        import oracle
        oracle.build(extra_flags=("-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                  "-fno-sanitize-recover=undefined"), out=lib)
        script = (
            "import numpy as np, oracle\n"
            "from rsgen import random_small, lfr, from_edges\n"
            f"lib = oracle.load({lib!r})\n"
            "for s in range(40):\n"
            "    g = random_small(int(5 + s % 30), 0.3, 1 + s % 5, seed=s)\n"
            "    o = oracle.score(g, lib=lib, rows=True)\n"
            "    oracle.topk(o['R'], 7, lib=lib)\n"
            "    if g.n: oracle.triads(g, 0, lib=lib)\n"
            "g = lfr(3000, 10.0, 120, 0.3, seed=5, cmin=10, cmax=300)\n"
            "o = oracle.score(g, lib=lib, nthreads=2)\n"
            "oracle.score(g, subset=np.arange(0, g.n, 7), lib=lib)\n"
            "oracle.topk(o['R'], 50, lib=lib)\n"
            "bad = from_edges(4, [(0, 1), (1, 2)], [0, 1, 1, 2])\n"
            "bad.col[0] = 3\n"
            "assert oracle.validate(bad, lib=lib) != 0\n"
            "print('ok')\n")
        out = _child(script, f"{asan}:{ubsan}", {"ASAN_OPTIONS": "detect_leaks=0", "OMP_NUM_THREADS": "2"})
        assert out.strip().endswith("ok")


def test_library_host_code_under_sanitizers():
    asan = _runtime([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"])
    if not asan:
        pytest.skip("clang sanitizer runtime not found")
    csrc = os.path.join(ROOT, "paper_2508_01485_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in ("rs_runtime.hip", "rs_kernels.hip", "rs_serve.hip"):
            obj = os.path.join(d, src + ".o")
            cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-c", os.path.join(csrc, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            objs.append(obj)
        lib = os.path.join(d, "librs_san.so")
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                            "-o", lib, *objs], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        script = (
            "import ctypes, numpy as np\n"
            "from rsgen import random_small, lfr, pack_batch\n"
            f"lib = ctypes.CDLL({lib!r})\n"
            "class csr(ctypes.Structure):\n"
            "    _fields_ = [('n', ctypes.c_int64), ('nnz', ctypes.c_int64), ('offset_bytes', ctypes.c_int32),\n"
            "                ('on_device', ctypes.c_int32), ('row_offsets', ctypes.c_void_p),\n"
            "                ('col', ctypes.c_void_p), ('labels', ctypes.c_void_p)]\n"
            "P = ctypes.c_void_p\n"
            "lib.rs_load_graph.argtypes = [ctypes.POINTER(csr), P, ctypes.c_uint32, ctypes.POINTER(P)]\n"
            "lib.rs_load_batch.argtypes = [ctypes.c_int32, P, ctypes.POINTER(csr), P, ctypes.c_uint32, ctypes.POINTER(P)]\n"
            "def mk(off, col, lab, ob=8):\n"
            "    return csr(off.size - 1, col.size, ob, 0, off.ctypes.data, col.ctypes.data, lab.ctypes.data)\n"
            "seen = set()\n"
            "def load(off, col, lab, ob=8):\n"
            "    h = P()\n"
            "    st = lib.rs_load_graph(ctypes.byref(mk(off, col, lab, ob)), None, 0, ctypes.byref(h))\n"
            "    seen.add(st)\n"
            "    assert not h.value or st == 0\n"
            "    return st\n"
            "gs = [random_small(int(2 + s % 40), 0.25, 1 + s % 6, seed=s) for s in range(30)]\n"
            "gs.append(lfr(5000, 12.0, 3000, 0.3, seed=3, cmin=10, cmax=400))\n"
            "for g in gs:\n"
            "    off, col, lab = g.off.astype(np.int64), g.col.astype(np.int32), g.labels.astype(np.int32)\n"
            "    load(off, col, lab)\n"
            "    load(off.astype(np.int32), col, lab, 4)\n"
            "    if g.nnz:\n"
            "        bad = col.copy(); bad[0] = g.n + 5; load(off, bad, lab)\n"
            "        bad = col.copy(); bad[-1] = bad[0]; load(off, bad, lab)\n"
            "        boff = off.copy(); boff[-1] += 3; load(boff, col, lab)\n"
            "    nl = lab.copy()\n"
            "    if g.n: nl[0] = -1; load(off, col, nl)\n"
            "vo, off, col, lab = pack_batch(gs[:8])\n"
            "h = P()\n"
            "vo = np.asarray(vo, np.int64)\n"
            "for o in (off, np.where(np.arange(off.size) == 1, off[-1] + 9, off)):\n"
            "    lib.rs_load_batch(8, vo.ctypes.data, ctypes.byref(mk(o.astype(np.int64), col, lab)), None, 0, ctypes.byref(h))\n"
            "print('ok', sorted(seen))\n")
        out = _child(script, asan, {"ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0",
                                    "UBSAN_OPTIONS": "print_stacktrace=1"})
        assert "ok" in out
