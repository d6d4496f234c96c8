"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no
GPU): a host-sanitised copy of the library (paper_2512_13619_amd/build_san.py) is loaded in a
subprocess that preloads the ASan runtime, and the host paths are exercised there: every
entry point with a NULL context or NULL arguments (argument checks, no device work), the
Hessenberg eigenvalue solver and the harmonic Ritz / Leja ordering on random and degenerate
inputs, and the launch-configuration table read from a JSON file. Any invalid access or
undefined behaviour aborts that process."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc is needed to build the sanitised library")

SCRIPT = textwrap.dedent("""
    import ctypes, sys
    import numpy as np
    sys.path.insert(0, {root!r})
    from paper_2512_13619_amd import hdg
    hdg.LIB_PATH = {lib!r}
    lib = hdg.load()
    # 1. every entry point that takes a context: NULL context and NULL / zero arguments
    n_checked = 0
    for name in hdg.SYMBOLS:
        fn = getattr(lib, name)
        ats = fn.argtypes or []
        if name in ("hdg_hessenberg_eigvals", "hdg_harmonic_ritz", "hdg_last_error", "hdg_local_size",
                    "hdg_solve_opts_default", "hdg_batch_tuned_grid", "hdg_tune_table", "hdg_poly_roots") or not ats:
            continue
        args = []
        for t in ats:
            if t in (ctypes.c_double,):
                args.append(0.0)
            elif t in (ctypes.c_int32, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t):
                args.append(0)
            else:
                args.append(None)
        rc = fn(*args)
        assert rc == -1, (name, rc)
        n_checked += 1
    assert n_checked >= 30, n_checked
    assert lib.hdg_local_size(None) == 0
    # the measured-configuration table is read from HDG_TUNE_CACHE on first use
    tab = hdg.tune_table()
    assert tab["entries"]["face:m32:p32:m20:k0:nb48:S11:nf2^15"] == [256, 2, 612.5], tab
    assert tab["entries"]["face:m64:p64:m20:k1:nb30:S1:nf2^18"] == [128, 1, 40.25], tab
    # 2. the Hessenberg eigenvalue solver on random, triangular and zero matrices
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 7, 16, 40, 64):
        H = np.triu(rng.standard_normal((n, n)), -1)
        got = np.sort_complex(hdg.hessenberg_eigvals(H))
        ref = np.sort_complex(np.linalg.eigvals(H))
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-10 * max(1.0, np.abs(ref).max()))
    assert np.allclose(hdg.hessenberg_eigvals(np.zeros((5, 5))), 0)
    pd = ctypes.POINTER(ctypes.c_double)
    w = np.zeros(4)
    assert lib.hdg_hessenberg_eigvals(0, w.ctypes.data_as(pd), 1, w.ctypes.data_as(pd), w.ctypes.data_as(pd)) != 0
    # 3. harmonic Ritz values and Leja order, including an Arnoldi breakdown (zero subdiagonal)
    for P in (1, 2, 5, 10, 20):
        H = np.triu(rng.standard_normal((P + 1, P)), -1) + 3.0 * np.eye(P + 1, P)
        t = hdg.harmonic_ritz(H)
        assert 1 <= len(t) <= P and np.all(np.isfinite(t))
    H = np.triu(rng.standard_normal((6, 5)), -1) + 3.0 * np.eye(6, 5)
    H[5, 4] = 0.0
    assert np.all(np.isfinite(hdg.harmonic_ritz(H)))
    print("SANITISED_OK", n_checked)
""")


def test_host_code_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2512_13619_amd import build_san
    lib = build_san.build()
    runtime = build_san.asan_runtime()
    assert os.path.exists(runtime), runtime
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cache = tmp_path / "tune.json"
    cache.write_text('{"version": 1, "entries": {\n  "face:m32:p32:m20:k0:nb48:S11:nf2^15": [256, 2, 612.5],'
                     '\n  "face:m64:p64:m20:k1:nb30:S1:nf2^18": [128, 1, 40.25]\n}}\n')
    env["HDG_TUNE_CACHE"] = str(cache)
    script = tmp_path / "san.py"
    script.write_text(SCRIPT.format(root=ROOT, lib=lib))
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "SANITISED_OK" in r.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
